"""Pins of the layer-stack oracle (oracle/stack.py)."""
import numpy as np
import pytest
from scipy.special import hankel1

from oracle import contour, mie, system
from oracle.stack import interfaces, stack_problem
from synth import make_workload


def _disks():
    wl = make_workload("c1")
    S = np.diag(mie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p))
    return wl, S


def _contour(ks, n=512):
    return contour.contour(n, 0.2, 32.0, [k.real if isinstance(k, complex) else k for k in ks])


def _rcv(ys, n=40, seed=3):
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.uniform(-5, 5, n), rng.uniform(ys[0], ys[1], n)], axis=1)
    return pts


def test_interfaces():
    y = interfaces([0, 1.5, 8.0, 2.0, 0], 2)
    assert np.allclose(y, [1.5, 0.0, -8.0, -10.0])


def test_three_layers_equal_the_three_layer_oracle(rng):
    wl, S = _disks()
    ks = [wl.k1, wl.k2, wl.k3]
    lam, w = _contour(ks)
    ref = system.Problem(*ks, wl.d, wl.p, S, wl.xy, wl.rot, lam, w)
    st = stack_problem(ks, [0, wl.d, 0], 1, wl.p, S, wl.xy, wl.rot, lam, w)
    x = rng.standard_normal((wl.n, wl.P)) + 1j * rng.standard_normal((wl.n, wl.P))
    a, b = st.matvec(x), ref.matvec(x)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))
    beta = ref.solve_lu(wl.src[0])
    r = _rcv((-11.0, 3.0))
    r = r[np.min(np.hypot(r[:, None, 0] - wl.xy[None, :, 0], r[:, None, 1] - wl.xy[None, :, 1]), axis=1) > 0.3]
    fa, fb = st.field(wl.src[0], beta, r), ref.field(wl.src[0], beta, r)
    assert np.max(np.abs(fa - fb)) < 1e-13 * np.max(np.abs(fb))


@pytest.mark.parametrize("split", ["above", "below"])
def test_interface_between_equal_wavenumbers_changes_nothing(split):
    """A layer of the neighbouring medium's wavenumber inserted as a separate
    layer (an interface with no contrast) leaves the solution unchanged."""
    wl, S = _disks()
    ks3 = [wl.k1, wl.k2, wl.k3]
    lam, w = _contour(ks3)
    ref = stack_problem(ks3, [0, wl.d, 0], 1, wl.p, S, wl.xy, wl.rot, lam, w)
    if split == "above":   # top half-space split at y = 1.2 (source at y = 2 stays above)
        st = stack_problem([wl.k1, wl.k1, wl.k2, wl.k3], [0, 1.2, wl.d, 0], 2, wl.p, S, wl.xy, wl.rot, lam, w)
    else:                  # bottom half-space split 2.5 below the particle layer
        st = stack_problem([wl.k1, wl.k2, wl.k3, wl.k3], [0, wl.d, 2.5, 0], 1, wl.p, S, wl.xy, wl.rot, lam, w)
    src = wl.src[0]
    b_ref, b_st = ref.solve_lu(src), st.solve_lu(src)
    assert np.max(np.abs(b_st - b_ref)) < 1e-11 * np.max(np.abs(b_ref))
    r = _rcv((-12.0, 3.5))
    r = r[np.min(np.hypot(r[:, None, 0] - wl.xy[None, :, 0], r[:, None, 1] - wl.xy[None, :, 1]), axis=1) > 0.3]
    r = r[np.hypot(r[:, 0] - src[0], r[:, 1] - src[1]) > 0.1]
    fa, fb = st.field(src, b_st, r), ref.field(src, b_ref, r)
    assert np.max(np.abs(fa - fb)) < 1e-11 * np.max(np.abs(fb))


def _five_layers(pol="TM"):
    wl, S = _disks()
    if pol == "TE":
        S = np.diag(mie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p, pol="TE"))
    ks = [6.0, 7.5, wl.k2, 11.0, 12.0]
    thick = [0, 1.0, wl.d, 1.5, 0]
    lam, w = _contour(ks, 768)
    return wl, stack_problem(ks, thick, 2, wl.p, S, wl.xy, wl.rot, lam, w, pol=pol)


def test_field_continuous_at_every_interface():
    wl, st = _five_layers()
    src = np.array([0.3, 2.5])
    beta = st.solve_lu(src)
    y = interfaces(st.thick, st.c)
    xs = np.linspace(-5, 5, 9)
    for yi in y:
        e = 1e-9
        ua = st.field(src, beta, np.stack([xs, np.full_like(xs, yi + e)], axis=1))
        ub = st.field(src, beta, np.stack([xs, np.full_like(xs, yi - e)], axis=1))
        assert np.max(np.abs(ua - ub)) < 1e-7 * np.max(np.abs(ua))


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_flux_balance_five_layers(pol):
    """Power balance (as for three layers) on a rectangle crossing all four
    interfaces of a five-layer stack.  TE: the flux density is
    (1/k^2) Im(conj(u) du/dn) with k of the layer it is taken in, and the
    source term carries 1/k_0^2 (the weighted equation div((1/k^2) grad u)
    + u = -(1/k_0^2) delta)."""
    from test_oracle_system import _gl_panels
    wl, st = _five_layers(pol)
    kap = [1.0 if pol == "TM" else 1.0 / k.real ** 2 for k in st.ks]
    src = np.array([0.3, 2.5])
    beta = st.solve_lu(src)
    y = interfaces(st.thick, st.c)
    xa, xb, ya, yb = -6.0, 6.0, y[-1] - 1.5, y[0] + 2.5
    h = 5e-4

    def dn(pts, nvec):
        f = [st.field(src, beta, pts + s * h * nvec) for s in (-2, -1, 1, 2)]
        return (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)

    flux = 0.0
    for side in range(4):
        if side < 2:
            t, wt = _gl_panels(xa, xb, (), 0.25)
            pts = np.stack([t, np.full_like(t, ya if side == 0 else yb)], axis=1)
            nvec = np.array([0.0, -1.0 if side == 0 else 1.0])
        else:
            t, wt = _gl_panels(ya, yb, tuple(y), 0.25)
            pts = np.stack([np.full_like(t, xa if side == 2 else xb), t], axis=1)
            nvec = np.array([-1.0 if side == 2 else 1.0, 0.0])
        u = st.field(src, beta, pts)
        lay = np.sum(pts[:, 1][:, None] < y[None, :], axis=1)
        wk = np.array([kap[j] for j in lay])
        flux += float(np.sum(wk * wt * np.imag(np.conj(u) * dn(pts, nvec))))
    e = 1e-5
    offs = np.array([[e, 0.0], [-e, 0.0], [0.0, e], [0.0, -e]])
    us = st.field(src, beta, src[None, :] + offs) - 0.25j * hankel1(0, st.ks[0].real * e)
    expect = kap[0] * (0.25 + float(np.mean(us).imag))
    assert abs(flux - expect) < 1e-9 * abs(expect), (flux, expect)   # measured 2e-10 (TM), 1e-10 (TE)
