"""Pins of the translation operators (Lemma 3.1, Lemma 5.1, Theorem 5.1)."""
import numpy as np
import pytest
from scipy.special import hankel1, jv

from oracle import contour, operators
from oracle.contour import gamma


def _multipole(beta, k, pt, c):
    p = (beta.size - 1) // 2
    nu = np.arange(-p, p + 1)
    d = np.asarray(pt) - np.asarray(c)
    return np.sum(beta * hankel1(nu, k * np.hypot(*d)) * np.exp(1j * nu * np.arctan2(d[1], d[0])))


def _local(alpha, k, pt, c):
    p = (alpha.size - 1) // 2
    n = np.arange(-p, p + 1)
    d = np.asarray(pt) - np.asarray(c)
    return np.sum(alpha * jv(n, k * np.hypot(*d)) * np.exp(1j * n * np.arctan2(d[1], d[0])))


@pytest.mark.parametrize("xl,xm", [((0.3, -1.0), (2.1, -3.0)), ((5.0, -2.0), (-1.0, -4.5)),
                                   ((0.0, -1.0), (0.0, -1.8))])
def test_graf_translation(rng, xl, xm):
    # brute force: the H-expansion at x_m evaluated directly near x_l against the
    # local expansion alpha = T beta (local order large enough to converge)
    k, p, pbig = 9.0, 6, 40
    beta = rng.standard_normal(2 * p + 1) + 1j * rng.standard_normal(2 * p + 1)
    beta_big = np.zeros(2 * pbig + 1, complex)
    beta_big[pbig - p:pbig + p + 1] = beta
    T = operators.m2l_block(np.array(xl), np.array(xm), k, pbig)
    alpha = T @ beta_big
    for off in [(0.05, 0.03), (-0.1, 0.02), (0.0, -0.12)]:
        pt = np.array(xl) + np.array(off)
        u = _multipole(beta, k, pt, xm)
        ul = _local(alpha, k, pt, xl)
        assert abs(u - ul) < 1e-12 * abs(u)


def test_printed_graf_sign_fails(rng):
    k, p = 9.0, 6
    xl, xm = np.array([0.3, -1.0]), np.array([2.1, -3.0])
    beta = np.zeros(2 * p + 1, complex)
    beta[p + 1] = 1.0                                        # a single H_1 e^{i theta}
    T = operators.m2l_block(xl, xm, k, p)
    n = np.arange(-p, p + 1)
    T_printed = T * ((-1.0) ** (n[:, None] - n[None, :]))   # the extra e^{i n pi}
    pt = xl + np.array([0.05, 0.03])
    u = _multipole(beta, k, pt, xm)
    assert abs(_local(T @ beta, k, pt, xl) - u) < 1e-6 * abs(u)
    assert abs(_local(T_printed @ beta, k, pt, xl) - u) > 1e-2 * abs(u)


def test_m2l_apply_matches_blocks(rng):
    xy = np.array([[0.0, -1.0], [1.1, -2.0], [-0.9, -1.5], [2.5, -3.3]])
    p, k = 4, 9.0
    beta = rng.standard_normal((4, 9)) + 1j * rng.standard_normal((4, 9))
    a = operators.m2l_apply(xy, k, p, beta)
    for l in range(4):
        ref = sum(operators.m2l_block(xy[l], xy[m], k, p) @ beta[m] for m in range(4) if m != l)
        assert np.max(np.abs(a[l] - ref)) < 1e-12 * np.max(np.abs(ref))


def test_jacobi_anger_complex_angle():
    k = 9.0
    lam = np.array([0.5 - 0.2j, 7.0 - 0.2j, 9.3 - 0.2j, 20.0 - 0.2j, -4.0 + 0.2j, 0.1j])
    g = gamma(lam, k)
    X, Y = 0.2, -0.15
    r, th = np.hypot(X, Y), np.arctan2(Y, X)
    nn = np.arange(-80, 81)
    for s in (1, -1):
        terms = ((1j) ** nn[None, :] * ((lam[:, None] - s * g[:, None]) / k) ** nn[None, :]
                 * jv(nn[None, :], k * r) * np.exp(1j * nn[None, :] * th))
        err = np.abs(np.exp(1j * lam * X + s * g * Y) - terms.sum(axis=1))
        assert np.all(err < 1e-13 * np.maximum(1.0, np.abs(terms).max(axis=1)))


def test_s2l_reproduces_layer_field(rng):
    # u_2^t + u_2^b evaluated directly near a particle equals its local expansion
    lam, w = contour.contour(256, 0.2, 32.0, [6.0, 9.0, 12.0])
    k, d, p = 9.0, 8.0, 24
    sp = rng.standard_normal(lam.size) * 1e-2 + 0j
    sm = rng.standard_normal(lam.size) * 1e-2 + 0j
    c = np.array([[0.4, -3.0]])
    alpha = operators.s2l(sp, sm, c, lam, w, k, d, p)[0]
    g = gamma(lam, k)
    for off in [(0.1, 0.05), (-0.07, -0.12)]:
        x, y = c[0] + np.array(off)
        direct = np.sum(w / g * np.exp(1j * lam * x) * (sp * np.exp(g * y) + sm * np.exp(-g * (y + d)))) / (4 * np.pi)
        assert abs(direct - _local(alpha, k, (x, y), c[0])) < 1e-12 * max(1.0, abs(direct))


def test_m2s_spectrum_reproduces_multipoles(rng):
    # the field of several multipoles on y = 0 and y = -d from their spectra P+/P-
    lam, w = contour.contour(96 + 32 * 60, 0.2, 60.0, [6.0, 9.0, 12.0])
    k, d, p = 9.0, 6.0, 5
    xy = np.array([[0.3, -2.0], [-0.8, -3.5], [1.4, -1.2]])
    beta = (rng.standard_normal((3, 2 * p + 1)) + 1j * rng.standard_normal((3, 2 * p + 1))) * 0.1
    Pp, Pm = operators.m2s(beta, xy, lam, k, d)
    g = gamma(lam, k)
    for x in (-0.5, 0.2, 1.7):
        direct_top = sum(_multipole(beta[m], k, (x, 0.0), xy[m]) for m in range(3))
        direct_bot = sum(_multipole(beta[m], k, (x, -d), xy[m]) for m in range(3))
        top = np.sum(w / g * np.exp(1j * lam * x) * Pp) / (4 * np.pi)
        bot = np.sum(w / g * np.exp(1j * lam * x) * Pm) / (4 * np.pi)
        assert abs(top - direct_top) < 1e-11 * abs(direct_top)
        assert abs(bot - direct_bot) < 1e-11 * abs(direct_bot)
