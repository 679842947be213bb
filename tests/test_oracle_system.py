"""Pins of the assembled Schur-complement system (Section 5.4, eq. (49)) and
of the field representation (eq. (36))."""
import numpy as np
import pytest
from scipy.special import hankel1

from oracle import contour, mie, operators, star, system
from synth import rejection_layout


def _problem(k=(6.0, 9.0, 12.0), n=9, p=5, d=6.0, nodes=256, b=0.2, tmax=32.0, shape="disk", seed=5):
    xy, rot = rejection_layout(n, (-3.0, 3.0), (-d + 1.0, -1.0), 0.75, seed)
    if shape == "disk":
        S = np.diag(mie.disk_smatrix(0.25, k[1], 15.0, p))
    else:
        S = star.star_smatrix(0.25, 0.05, 5, k[1], 15.0, p, nb=128)
    lam, w = contour.contour(nodes, b, tmax, list(k))
    return system.Problem(k[0], k[1], k[2], d, p, S, xy, rot, lam, w)


def test_dense_equals_matvec(rng):
    pr = _problem(shape="star")
    x = rng.standard_normal((pr.N, pr.P)) + 1j * rng.standard_normal((pr.N, pr.P))
    K = pr.dense()
    assert np.max(np.abs(K @ x.reshape(-1) - pr.matvec(x).reshape(-1))) < 1e-12 * np.max(np.abs(x))
    tg = [0, 4, 8]
    assert np.max(np.abs(pr.matvec(x, targets=tg) - pr.matvec(x)[tg])) < 1e-13


def test_lu_equals_gmres():
    pr = _problem(shape="star")
    src = np.array([0.3, 1.5])
    b1 = pr.solve_lu(src)
    b2, hist = pr.gmres(src, tol=1e-13)
    assert hist[-1] < 1e-13
    assert np.max(np.abs(b1 - b2.reshape(b1.shape))) < 1e-11 * np.max(np.abs(b1))


def test_free_space_limit_matches_homogeneous_solver():
    # k1 = k2 = k3: the reflection vanishes per node, and on a refined contour the
    # incident local expansions equal Graf's expansion of G itself
    k = 9.0
    pr = _problem(k=(k, k, k), nodes=96 + 32 * 50, tmax=60.0)
    src = np.array([0.4, 2.0])
    beta = pr.solve_lu(src)
    T = np.zeros((pr.N * pr.P,) * 2, complex)
    for l in range(pr.N):
        for m in range(pr.N):
            if m != l:
                T[l * pr.P:(l + 1) * pr.P, m * pr.P:(m + 1) * pr.P] = operators.m2l_block(pr.xy[l], pr.xy[m], k, pr.p)
    Sblk = np.zeros_like(T)
    for l in range(pr.N):
        Sblk[l * pr.P:(l + 1) * pr.P, l * pr.P:(l + 1) * pr.P] = operators.rotated_smatrix(pr.S, pr.rot[l])
    a = operators.incident_local_free(pr.xy, src, k, pr.p).reshape(-1)
    beta_free = np.linalg.solve(np.eye(T.shape[0]) - Sblk @ T, Sblk @ a).reshape(pr.N, pr.P)
    assert np.max(np.abs(beta - beta_free)) < 1e-11 * np.max(np.abs(beta_free))
    x = np.ones((pr.N, pr.P), complex)
    assert np.max(np.abs(pr.matvec_parts(x)[1])) < 1e-14


@pytest.mark.parametrize("shape", ["disk", "star"])
def test_reciprocity(shape):
    pr = _problem(shape=shape)
    xa, xb = np.array([0.5, 2.0]), np.array([-1.3, 1.2])
    G = 0.25j * hankel1(0, pr.k1 * np.hypot(*(xa - xb)))
    ua = pr.field(xa, pr.solve_lu(xa), xb[None])[0] - G
    ub = pr.field(xb, pr.solve_lu(xb), xa[None])[0] - G
    tol = 1e-13 if shape == "disk" else 1e-11
    assert abs(ua - ub) < tol * abs(ua)


def test_field_continuous_across_interfaces():
    # on a refined contour the directly-summed multipoles in layer 2 agree with their
    # Sommerfeld forms carried into layers 1 and 3: u and du/dy are continuous
    pr = _problem(nodes=96 + 32 * 60, tmax=60.0, d=5.0)
    src = np.array([0.2, 1.5])
    beta = pr.solve_lu(src)
    xs = np.linspace(-2.5, 2.5, 5)
    h = 1e-4
    for yi in (0.0, -pr.d):
        f = lambda dy: pr.field(src, beta, np.stack([xs, np.full_like(xs, yi + dy)], 1))
        up0, up1, up2 = f(0.0 + 1e-12 if yi == 0.0 else 1e-12), f(h), f(2 * h)
        dn0, dn1, dn2 = f(-1e-12), f(-h), f(-2 * h)
        scale = np.max(np.abs(up0))
        assert np.max(np.abs(up0 - dn0)) < 1e-10 * scale
        dup = (-3 * up0 + 4 * up1 - up2) / (2 * h)
        ddn = (3 * dn0 - 4 * dn1 + dn2) / (2 * h)
        assert np.max(np.abs(dup - ddn)) < 1e-5 * np.max(np.abs(dup))
