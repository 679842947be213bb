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


def _gl_panels(a, b, breaks, panel):
    """Composite 16-point Gauss-Legendre nodes/weights on [a, b], panels of
    at most `panel`, with the given interior breakpoints."""
    x16, w16 = np.polynomial.legendre.leggauss(16)
    pts = sorted({a, b, *[t for t in breaks if a < t < b]})
    xs, ws = [], []
    for lo, hi in zip(pts[:-1], pts[1:]):
        m = max(1, int(np.ceil((hi - lo) / panel)))
        e = np.linspace(lo, hi, m + 1)
        for u, v in zip(e[:-1], e[1:]):
            xs.append(0.5 * (u + v) + 0.5 * (v - u) * x16)
            ws.append(0.5 * (v - u) * w16)
    return np.concatenate(xs), np.concatenate(ws)


@pytest.mark.parametrize("kinds", [1, 2])
def test_flux_balance_lossless(kinds):
    """Power balance for real wavenumbers: by Green's identity (u and its normal
    derivative continuous across every interface, Delta u + k^2 u = -delta at
    the source), the outgoing flux through any closed contour C around the
    source and the particles is  int_C Im(conj(u) du/dn) ds = Im u(x_s)
    = 1/4 + Im u_s(x_s),  u_s = u - G.  Checked on a rectangle that crosses
    both interfaces, with the solution of the full discrete system.  The
    discrete Sommerfeld contour conserves power only to its own accuracy:
    7e-7 with the 256 nodes of this layout's recipe, 2e-11 with 512 (used
    here), 2e-12 with 1024."""
    from synth import make_workload
    from scipy.special import hankel1
    from oracle import contour as oc, mie
    wl = make_workload("c1")
    lam, w = oc.contour(512, wl.b, wl.t_max, [wl.k1, wl.k2, wl.k3])
    S = np.diag(mie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p))
    if kinds == 1:
        pr = system.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, S, wl.xy, wl.rot, lam, w)
    else:   # two particle types (Section 4.2 Remark): every other disk smaller and softer
        S2 = np.diag(mie.disk_smatrix(0.2, wl.k2, 11.0, wl.p))
        pr = system.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, np.stack([S, S2]), wl.xy, wl.rot, lam, w,
                            types=np.arange(wl.n) % 2)
    src = wl.src[0]
    beta = pr.solve_lu(src)
    xa, xb, ya, yb = -6.0, 6.0, -wl.d - 2.0, 4.0
    h = 5e-4

    def dn(pts, nvec):   # fourth-order central difference along the outward normal
        f = [pr.field(src, beta, pts + s * h * nvec) for s in (-2, -1, 1, 2)]
        return (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)

    flux = 0.0
    yb_breaks = (0.0, -wl.d)
    for side in range(4):
        if side < 2:     # bottom (layer 3), top (layer 1)
            t, wt = _gl_panels(xa, xb, (), 0.25)
            y = ya if side == 0 else yb
            pts = np.stack([t, np.full_like(t, y)], axis=1)
            nvec = np.array([0.0, -1.0 if side == 0 else 1.0])
        else:            # left, right: cross both interfaces
            t, wt = _gl_panels(ya, yb, yb_breaks, 0.25)
            x = xa if side == 2 else xb
            pts = np.stack([np.full_like(t, x), t], axis=1)
            nvec = np.array([-1.0 if side == 2 else 1.0, 0.0])
        u = pr.field(src, beta, pts)
        flux += float(np.sum(wt * np.imag(np.conj(u) * dn(pts, nvec))))
    e = 1e-5
    offs = np.array([[e, 0.0], [-e, 0.0], [0.0, e], [0.0, -e]])
    us = pr.field(src, beta, src[None, :] + offs) - 0.25j * hankel1(0, wl.k1 * e)
    expect = 0.25 + float(np.mean(us).imag)
    assert abs(flux - expect) < 1e-9, (flux, expect)


def test_single_disk_matches_mie_series():
    """One disk in a homogeneous medium (k1 = k2 = k3) lit by the point source:
    the total field outside the disk is G + sum_n S_n a_n H_n(kr) e^{in theta}
    with the Mie coefficients S_n and Graf's incident coefficients
    a_n = (i/4) H_n(k r_s) e^{-in theta_s} (|n| <= 40), independently of the
    layered formulation, its contour and its solver."""
    k, R, kp, d = 9.0, 0.25, 15.0, 8.0
    c = np.array([0.3, -3.0])
    src = np.array([-0.2, 2.0])
    lam, w = contour.contour(96 + 32 * 50, 0.2, 60.0, [k, k, k])
    p = 16
    S = np.diag(mie.disk_smatrix(R, k, kp, p))
    pr = system.Problem(k, k, k, d, p, S, c[None, :], np.zeros(1), lam, w)
    beta = pr.solve_lu(src)
    rng = np.random.default_rng(7)
    ang = rng.uniform(0, 2 * np.pi, 24)
    rad = rng.uniform(0.4, 2.5, 24)
    rcv = c[None, :] + np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    rcv = rcv[np.hypot(rcv[:, 0] - src[0], rcv[:, 1] - src[1]) > 0.3]
    got = pr.field(src, beta, rcv)
    q = 40
    n = np.arange(-q, q + 1)
    rs, ths = np.hypot(*(src - c)), np.arctan2(*(src - c)[::-1])
    a = 0.25j * hankel1(n, k * rs) * np.exp(-1j * n * ths)
    Sq = mie.disk_smatrix(R, k, kp, q)
    r = np.hypot(rcv[:, 0] - c[0], rcv[:, 1] - c[1])
    th = np.arctan2(rcv[:, 1] - c[1], rcv[:, 0] - c[0])
    scat = (hankel1(n[None, :], k * r[:, None]) * np.exp(1j * n[None, :] * th[:, None])) @ (Sq * a)
    exact = 0.25j * hankel1(0, k * np.hypot(rcv[:, 0] - src[0], rcv[:, 1] - src[1])) + scat
    err = np.max(np.abs(got - exact)) / np.max(np.abs(exact))
    assert err < 1e-11, err


def test_types_with_one_matrix_equal_the_single_type_problem():
    from synth import make_workload
    from oracle import contour as oc, mie
    wl = make_workload("c1")
    lam, w = oc.contour(wl.n_nodes, wl.b, wl.t_max, [wl.k1, wl.k2, wl.k3])
    S = np.diag(mie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p))
    a = system.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, S, wl.xy, wl.rot, lam, w)
    b = system.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, np.stack([S, 0 * S]), wl.xy, wl.rot, lam, w,
                       types=np.zeros(wl.n, int))
    x = np.random.default_rng(0).standard_normal((wl.n, wl.P)) + 0j
    assert np.array_equal(a.matvec(x), b.matvec(x))


def test_a_type_that_does_not_scatter_removes_its_particles():
    """Particles whose type has S = 0 radiate nothing: their beta vanish and
    the others solve the problem without them."""
    from synth import make_workload
    from oracle import contour as oc, mie
    wl = make_workload("c1")
    lam, w = oc.contour(wl.n_nodes, wl.b, wl.t_max, [wl.k1, wl.k2, wl.k3])
    S = np.diag(mie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p))
    types = (np.arange(wl.n) % 3 == 0).astype(int)
    mixed = system.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, np.stack([S, 0 * S]), wl.xy, wl.rot, lam, w,
                           types=types)
    keep = types == 0
    sub = system.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, S, wl.xy[keep], wl.rot[keep], lam, w)
    src = wl.src[0]
    b_mixed, b_sub = mixed.solve_lu(src), sub.solve_lu(src)
    assert np.max(np.abs(b_mixed[~keep])) < 1e-14 * np.max(np.abs(b_sub))      # rounding of the dense solve
    assert np.max(np.abs(b_mixed[keep] - b_sub)) < 1e-12 * np.max(np.abs(b_sub))
