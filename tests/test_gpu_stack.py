"""GPU parity of layer stacks with more than three layers (mpsl_set_layer_stack)
against the stack oracle (dense interface solve per node): matvec, right-hand
side, solve against dense LU, and the field at receivers in every layer.

Tolerances are those of the three-layer parity tests: 1e-12 for FP64
matvec / rhs, 2e-5 for the FP32 matvec, 1e-10 for the FP64 solve and field.
"""
import numpy as np
import pytest

import paper_1407_3868_amd as mp
from gpu_common import coeff_vector, make_workload, prototype_S, rel_err
from oracle import contour as ocontour
from oracle import mie as omie
from oracle import star as ostar
from oracle.stack import interfaces, stack_problem
from synth import receivers

pytestmark = pytest.mark.gpu


def _stack(kind, wl):
    """(wavenumbers, thicknesses, particle layer); the particle layer has the
    workload's k2 and thickness d."""
    d = wl.d
    if kind == "five":
        return [6.0, 7.5, wl.k2, 11.0, 12.0], [0.0, 1.0, d, 1.5, 0.0], 2
    if kind == "top":        # particle layer right under the top half-space
        return [6.0, wl.k2, 4.0, 12.0], [0.0, d, 0.8, 0.0], 1
    if kind == "bottom":     # particle layer right over the bottom half-space
        return [6.0, 3.0, wl.k2, 12.0], [0.0, 0.6, d, 0.0], 2
    if kind == "seven":
        return [3.0, 8.0, 5.0, wl.k2, 6.0, 10.0, 2.0], [0.0, 0.4, 1.3, d, 0.2, 2.5, 0.0], 3
    raise ValueError(kind)


_TE_S = {}


def prototype_S_te(wl):
    """TE prototype scattering matrix from the oracle."""
    key = (wl.shape, wl.shape_params, wl.k2, wl.kp, wl.p)
    if key not in _TE_S:
        if wl.shape == "disk":
            _TE_S[key] = np.diag(omie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p, pol="TE"))
        else:
            a1, a2, a3 = wl.shape_params
            _TE_S[key] = ostar.star_smatrix(a1, a2, a3, wl.k2, wl.kp, wl.p, nb=256, pol="TE")
    return _TE_S[key]


def _setup(name, kind, pol="TM"):
    wl = make_workload(name)
    ks, th, c = _stack(kind, wl)
    # one 16-node panel per interval between branch points, then refinement
    wl.n_nodes = max(wl.n_nodes, 32 * (len(ks) + 4))
    S = prototype_S(wl) if pol == "TM" else prototype_S_te(wl)
    lam, w = ocontour.contour(wl.n_nodes, wl.b, wl.t_max, ks)
    pr = stack_problem(ks, th, c, wl.p, S, wl.xy, wl.rot, lam, w, pol=pol)
    ctx = mp.Context(0)
    if pol == "TE":
        ctx.set_polarization(mp.TE)
    ctx.set_layer_stack(ks, th, c)
    ctx.set_scattering_matrix(wl.p, wl.r_enclose, S)
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    return wl, (ks, th, c), pr, ctx


KINDS = ["five", "top", "bottom", "seven"]


@pytest.mark.parametrize("kind", KINDS)
def test_stack_contour_has_every_branch_point(kind):
    wl, (ks, th, c), pr, ctx = _setup("c1", kind)
    lam, w = ctx.get_contour()
    assert np.max(np.abs(lam - pr.lam)) < 1e-13 * np.max(np.abs(pr.lam))
    assert np.max(np.abs(w - pr.w)) < 1e-13 * np.max(np.abs(pr.w))


@pytest.mark.parametrize("name", ["s70p8", "s150p12"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("prec", [0, 1])
def test_stack_matvec(name, kind, prec):
    wl, _, pr, ctx = _setup(name, kind)
    x = coeff_vector(wl, 6)
    ref = pr.matvec(x)
    got = ctx.apply(prec, x.astype(np.complex128 if prec == 0 else np.complex64))
    err = rel_err(got, ref)
    assert err < (1e-12 if prec == 0 else 2e-5), err


@pytest.mark.parametrize("kind", KINDS)
def test_stack_rhs(kind):
    wl, (ks, th, c), pr, ctx = _setup("s70p8", kind)
    src = np.array([0.3, interfaces(th, c)[0] + 1.1])
    assert rel_err(ctx.rhs(src), pr.rhs(src)) < 1e-12


def _rcv_all_layers(wl, th, c, src, n=160):
    y = interfaces(th, c)
    xs = wl.xy[:, 0]
    return receivers(n, (xs.min() - 1, xs.max() + 1), (y[-1] - 1.5, y[0] + 2.5), wl.xy, 77 + n,
                     particle_excl=wl.r_enclose + 0.05, source=src, source_excl=0.05)


@pytest.mark.parametrize("kind", KINDS)
def test_stack_solve_and_field_match_lu(kind):
    wl, (ks, th, c), pr, ctx = _setup("c1", kind)
    src = np.array([0.4, interfaces(th, c)[0] + 1.0])
    ref = pr.solve_lu(src)
    beta, meta = ctx.solve(src, precision=0, tol=1e-13, maxiter=600)
    assert meta["status"] == 0, meta
    assert rel_err(beta, ref) < 1e-10
    r = _rcv_all_layers(wl, th, c, src)
    lay = np.sum(r[:, 1][:, None] < interfaces(th, c)[None, :], axis=1)
    assert set(lay.tolist()) == set(range(len(ks)))          # a receiver in every layer
    u = ctx.eval_field(src, beta, r)
    assert rel_err(u, pr.field(src, ref, r)) < 1e-10


def test_stack_mixed_solve():
    wl, (ks, th, c), pr, ctx = _setup("c1", "five")
    src = np.array([0.4, interfaces(th, c)[0] + 1.0])
    ref = pr.solve_lu(src)
    beta, meta = ctx.solve(src, precision=1, tol=1e-10, maxiter=600)
    assert meta["status"] == 0, meta
    r = _rcv_all_layers(wl, th, c, src, 64)
    assert rel_err(ctx.eval_field(src, beta, r), pr.field(src, ref, r)) < 1e-6


def test_three_layer_stack_is_set_layers():
    """mpsl_set_layers is the three-layer stack: the same bytes out."""
    wl = make_workload("s70p8")
    S = prototype_S(wl)
    a, b = mp.Context(0), mp.Context(0)
    a.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    b.set_layer_stack([wl.k1, wl.k2, wl.k3], [0.0, wl.d, 0.0], 1)
    for ctx in (a, b):
        ctx.set_scattering_matrix(wl.p, wl.r_enclose, S)
        ctx.set_geometry(wl.xy, wl.rot)
        ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    x = coeff_vector(wl, 2)
    for prec in (0, 1):
        xp = x.astype(np.complex128 if prec == 0 else np.complex64)
        assert np.array_equal(a.apply(prec, xp), b.apply(prec, xp))
    assert np.array_equal(a.rhs(wl.src[0]), b.rhs(wl.src[0]))


def test_stack_arguments_are_checked():
    wl = make_workload("c1")
    ctx = mp.Context(0)
    with pytest.raises(mp.MpslError):
        ctx.set_layer_stack([6.0, 9.0], [0.0, 0.0], 1)                    # two layers
    with pytest.raises(mp.MpslError):
        ctx.set_layer_stack([6.0, 9.0, 12.0, 7.0], [0, 1.0, 2.0, 0], 3)    # half-space as particle layer
    with pytest.raises(mp.MpslError):
        ctx.set_layer_stack([6.0, 9.0, 12.0, 7.0], [0, 1.0, -2.0, 0], 1)   # negative thickness
    ks, th, c = _stack("five", wl)
    ctx.set_layer_stack(ks, th, c)
    ctx.set_scattering_matrix(wl.p, wl.r_enclose, prototype_S(wl))
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    with pytest.raises(mp.MpslError):
        ctx.rhs(np.array([0.0, 0.5]))        # above the particle layer but below the top interface (y = 1)


# ---- TE polarisation: (1/k^2) du/dn continuous ---------------------------------

KINDS_TE = ["three", "five", "seven"]


def _setup_te(name, kind):
    if kind == "three":
        wl = make_workload(name)
        S = prototype_S_te(wl)
        ks, th, c = [wl.k1, wl.k2, wl.k3], [0.0, wl.d, 0.0], 1
        lam, w = ocontour.contour(wl.n_nodes, wl.b, wl.t_max, ks)
        pr = stack_problem(ks, th, c, wl.p, S, wl.xy, wl.rot, lam, w, pol="TE")
        ctx = mp.Context(0)
        ctx.set_polarization(mp.TE)
        ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
        ctx.set_scattering_matrix(wl.p, wl.r_enclose, S)
        ctx.set_geometry(wl.xy, wl.rot)
        ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
        return wl, (ks, th, c), pr, ctx
    return _setup(name, kind, pol="TE")


@pytest.mark.parametrize("name", ["s70p8", "s150p12"])
@pytest.mark.parametrize("kind", KINDS_TE)
@pytest.mark.parametrize("prec", [0, 1])
def test_te_matvec(name, kind, prec):
    wl, _, pr, ctx = _setup_te(name, kind)
    x = coeff_vector(wl, 6, S=pr.S)
    got = ctx.apply(prec, x.astype(np.complex128 if prec == 0 else np.complex64))
    err = rel_err(got, pr.matvec(x))
    assert err < (1e-12 if prec == 0 else 2e-5), err


@pytest.mark.parametrize("kind", KINDS_TE)
def test_te_solve_and_field_match_lu(kind):
    wl, (ks, th, c), pr, ctx = _setup_te("c1", kind)
    src = np.array([0.4, interfaces(th, c)[0] + 1.0])
    ref = pr.solve_lu(src)
    beta, meta = ctx.solve(src, precision=0, tol=1e-13, maxiter=600)
    assert meta["status"] == 0, meta
    assert rel_err(beta, ref) < 1e-10
    r = _rcv_all_layers(wl, th, c, src)
    assert rel_err(ctx.eval_field(src, beta, r), pr.field(src, ref, r)) < 1e-10


def test_te_library_particles_match_oracle():
    """Disk and star matrices computed by the library under TE."""
    ctx = mp.Context(0)
    ctx.set_polarization(mp.TE)
    ctx.set_layers(6.0, 9.0, 12.0, 8.0)
    ctx.set_particle_disk(0.25, 15.0, 8)
    assert np.max(np.abs(ctx.get_scattering_matrix()
                         - np.diag(omie.disk_smatrix(0.25, 9.0, 15.0, 8, pol="TE")))) < 1e-13
    ctx.set_particle_star(0.25, 0.05, 5, 15.0, 12, 256)
    assert np.max(np.abs(ctx.get_scattering_matrix()
                         - ostar.star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 12, nb=256, pol="TE"))) < 1e-12


def test_polarization_change_clears_the_particle():
    wl = make_workload("c1")
    ctx = mp.Context(0)
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_particle_disk(0.25, wl.kp, wl.p)
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    ctx.apply(0, np.zeros((wl.n, wl.P), complex))
    ctx.set_polarization(mp.TE)
    assert ctx.polarization() == mp.TE
    with pytest.raises(mp.MpslError):
        ctx.apply(0, np.zeros((wl.n, wl.P), complex))
    with pytest.raises(mp.MpslError):
        ctx.set_polarization(7)


def test_te_power_balance_through_the_library():
    """Weighted power balance (1/k^2 of each layer on the flux density, 1/k_0^2
    on the source term) for the library's TE solve and field on five layers."""
    from scipy.special import hankel1
    from test_oracle_system import _gl_panels
    wl = make_workload("c1")
    ks, th, c = _stack("five", wl)
    ctx = mp.Context(0)
    ctx.set_polarization(mp.TE)
    ctx.set_layer_stack(ks, th, c)
    ctx.set_particle_disk(wl.shape_params[0], wl.kp, wl.p)
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(768, 0.2, 32.0)
    src = np.array([0.3, 2.5])
    beta, meta = ctx.solve(src, precision=0, tol=1e-13, maxiter=400)
    assert meta["status"] == 0
    kap = [1.0 / k ** 2 for k in ks]
    y = interfaces(th, c)
    xa, xb, ya, yb = -6.0, 6.0, y[-1] - 1.5, y[0] + 2.5
    h = 5e-4
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
        f = [ctx.eval_field(src, beta, pts + s * h * nvec) for s in (-2, -1, 1, 2)]
        du = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
        u = ctx.eval_field(src, beta, pts)
        lay = np.sum(pts[:, 1][:, None] < y[None, :], axis=1)
        flux += float(np.sum(np.array([kap[j] for j in lay]) * wt * np.imag(np.conj(u) * du)))
    e = 1e-5
    offs = np.array([[e, 0.0], [-e, 0.0], [0.0, e], [0.0, -e]])
    us = ctx.eval_field(src, beta, src[None, :] + offs) - 0.25j * hankel1(0, ks[0] * e)
    expect = kap[0] * (0.25 + float(np.mean(us).imag))
    assert abs(flux - expect) < 1e-9 * abs(expect), (flux, expect)


def test_stack_on_span_contour():
    """A five-layer stack on a span-rule contour (breakpoints at every
    layer's wavenumber): nodes and matvec against the stack oracle."""
    wl = make_workload("s150p12")
    ks, th, c = _stack("five", wl)
    X = float(wl.xy[:, 0].max() - wl.xy[:, 0].min())
    b, h = min(0.2, 2.0 / X), 6.0 / X
    lam, w = ocontour.contour_span(b, 24.0, h, ks)
    S = prototype_S(wl)
    pr = stack_problem(ks, th, c, wl.p, S, wl.xy, wl.rot, lam, w)
    ctx = mp.Context(0)
    ctx.set_layer_stack(ks, th, c)
    ctx.set_scattering_matrix(wl.p, wl.r_enclose, S)
    ctx.set_geometry(wl.xy, wl.rot)
    assert ctx.set_contour_span(b, 24.0, h) == lam.size
    x = coeff_vector(wl, 4)
    for prec, tol in ((0, 1e-12), (1, 2e-5)):
        err = rel_err(ctx.apply(prec, x.astype(np.complex128 if prec == 0 else np.complex64)), pr.matvec(x))
        assert err < tol, err
