"""GPU solves against the oracle's dense LU solve of the same discrete system,
and fields at receivers in all three layers."""
import numpy as np
import pytest

from gpu_common import gpu_context, make_workload, oracle_problem, rel_err
from synth import receivers

pytestmark = pytest.mark.gpu


def _rcv(wl, n=96):
    xs = wl.xy[:, 0]
    return receivers(n, (xs.min() - 1, xs.max() + 1), (-wl.d - 1.5, 2.5), wl.xy, 1000 + n,
                     particle_excl=wl.r_enclose + 0.05, source=wl.src[0], source_excl=0.05)


@pytest.mark.parametrize("name", ["c1", "s70p8", "s150p12"])
def test_fp64_solve_matches_lu(name):
    # the stars at k2 = 9, kp = 15 are near-resonant: the s150p12 system has
    # condition number ~6e6 and needs ~500 unrestarted GMRES iterations
    wl = make_workload(name)
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    src = wl.src[0]
    ref = pr.solve_lu(src)
    beta, meta = ctx.solve(src, precision=0, tol=1e-12, maxiter=1200)
    assert meta["status"] == 0 and meta["rel_residual"] < 1e-11
    assert rel_err(beta, ref) < 1e-10
    r = _rcv(wl)
    u_ref = pr.field(src, ref, r)
    u = ctx.eval_field(src, beta, r)
    assert rel_err(u, u_ref) < 1e-10


@pytest.mark.parametrize("name", ["c1", "s70p8"])
def test_mixed_solve_matches_lu(name):
    wl = make_workload(name)
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    src = wl.src[0]
    ref = pr.solve_lu(src)
    beta, meta = ctx.solve(src, precision=1, tol=1e-10, maxiter=1200)
    assert meta["status"] == 0, meta
    assert meta["refinements"] >= 1
    r = _rcv(wl)
    assert rel_err(ctx.eval_field(src, beta, r), pr.field(src, ref, r)) < 1e-6


def test_field_from_oracle_coefficients():
    # a7 alone: the same beta into both field evaluators
    wl = make_workload("s150p12")
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    src = wl.src[0]
    beta = pr.solve_lu(src)
    r = _rcv(wl, 200)
    assert rel_err(ctx.eval_field(src, beta, r), pr.field(src, beta, r)) < 1e-11


def test_receiver_inside_particle_is_nan():
    wl = make_workload("c1")
    ctx = gpu_context(wl)
    beta = np.zeros((wl.n, wl.P), complex)
    r = np.array([[wl.xy[0, 0] + 0.05, wl.xy[0, 1]], [0.0, 1.0]])
    u = ctx.eval_field(wl.src[0], beta, r)
    assert np.isnan(u[0]) and np.isfinite(u[1])


def test_reciprocity_of_gpu_solves():
    wl = make_workload("c1")
    ctx = gpu_context(wl, disk_from_library=True)
    xa, xb = np.array([0.5, 2.0]), np.array([-1.3, 1.2])
    ba, _ = ctx.solve(xa, tol=1e-13)
    bb, _ = ctx.solve(xb, tol=1e-13)
    ua = ctx.eval_field(xa, ba, xb[None])[0]
    ub = ctx.eval_field(xb, bb, xa[None])[0]
    assert abs(ua - ub) < 1e-11 * abs(ua)


def test_bad_inputs_are_rejected():
    import paper_1407_3868_amd as mp
    ctx = mp.Context(0)
    with pytest.raises(mp.MpslError):
        ctx.set_layers(-1.0, 9.0, 12.0, 8.0)
    ctx.set_layers(6.0, 9.0, 12.0, 8.0)
    ctx.set_particle_disk(0.25, 15.0, 8)
    with pytest.raises(mp.MpslError) as e:
        ctx.set_geometry(np.array([[0.0, -2.0], [0.3, -2.0]]))   # enclosing disks overlap
    assert e.value.status == -5
    with pytest.raises(mp.MpslError):
        ctx.set_geometry(np.array([[0.0, -0.1]]))                # crosses y = 0
    with pytest.raises(mp.MpslError):
        ctx.set_contour(100, 0.2, 32.0)                          # not 32 + 32 m
    with pytest.raises(mp.MpslError) as e:
        ctx.apply(0, np.zeros((1, 17), complex))                 # nothing set up yet
    assert e.value.status == -4


def test_flux_balance_of_library_solution():
    """The library's FP64 solve and field evaluation conserve power:
    int_C Im(conj(u) du/dn) ds = 1/4 + Im u_s(x_s) on a rectangle around the
    source and the particles that crosses both interfaces (512 contour nodes,
    where the discrete model conserves power to ~2e-11)."""
    from scipy.special import hankel1
    from test_oracle_system import _gl_panels
    wl = make_workload("c1")
    wl.n_nodes = 512
    ctx = gpu_context(wl, disk_from_library=True)
    src = wl.src[0]
    beta, meta = ctx.solve(src, precision=0, tol=1e-13, maxiter=400)
    assert meta["status"] == 0
    xa, xb, ya, yb = -6.0, 6.0, -wl.d - 2.0, 4.0
    h = 5e-4
    flux = 0.0
    for side in range(4):
        if side < 2:
            t, wt = _gl_panels(xa, xb, (), 0.25)
            pts = np.stack([t, np.full_like(t, ya if side == 0 else yb)], axis=1)
            nvec = np.array([0.0, -1.0 if side == 0 else 1.0])
        else:
            t, wt = _gl_panels(ya, yb, (0.0, -wl.d), 0.25)
            pts = np.stack([np.full_like(t, xa if side == 2 else xb), t], axis=1)
            nvec = np.array([-1.0 if side == 2 else 1.0, 0.0])
        f = [ctx.eval_field(src, beta, pts + s * h * nvec) for s in (-2, -1, 1, 2)]
        du = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
        u = ctx.eval_field(src, beta, pts)
        flux += float(np.sum(wt * np.imag(np.conj(u) * du)))
    e = 1e-5
    offs = np.array([[e, 0.0], [-e, 0.0], [0.0, e], [0.0, -e]])
    us = ctx.eval_field(src, beta, src[None, :] + offs) - 0.25j * hankel1(0, wl.k1 * e)
    expect = 0.25 + float(np.mean(us).imag)
    assert abs(flux - expect) < 1e-9, (flux, expect)
