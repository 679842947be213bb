"""Several particle types (mpsl_set_particle_types / mpsl_set_geometry_typed):
the type-aware scattering-matrix apply, the matvec, the solve and the field
against the oracle with one prototype matrix per type.

Tolerances as for one type: 1e-12 FP64 / 2e-5 FP32 matvec, 1e-10 FP64 solve
and field against LU.
"""
import numpy as np
import pytest

import paper_1407_3868_amd as mp
from gpu_common import make_workload, oracle_problem, prototype_S, rel_err
from oracle import mie, star
from oracle import system as osystem
from oracle.operators import rotated_smatrix
from synth import receivers

pytestmark = pytest.mark.gpu


def _types_setup(name, order):
    """Two or three prototypes on a workload's layout; order 'mixed'
    alternates types particle by particle (every tile holds all of them),
    'sorted' gives contiguous runs."""
    wl = make_workload(name)
    base = prototype_S(wl)
    if wl.shape == "disk":
        Ss = [base, np.diag(mie.disk_smatrix(0.2, wl.k2, 11.0, wl.p))]
        radii = [wl.r_enclose, 0.2]
    else:
        Ss = [base, star.star_smatrix(0.25, -0.03, 5, wl.k2, 15.0, wl.p, nb=256),
              np.diag(mie.disk_smatrix(0.2, wl.k2, 12.0, wl.p))]
        radii = [wl.r_enclose, 0.28, 0.2]
    T = len(Ss)
    types = np.arange(wl.n) % T if order == "mixed" else (np.arange(wl.n) * T) // wl.n
    pr0 = oracle_problem(wl)
    pr = osystem.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, np.stack(Ss), wl.xy, wl.rot, pr0.lam, pr0.w, types=types)
    ctx = mp.Context(0)
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_particle_types(wl.p, radii, np.stack(Ss))
    ctx.set_geometry(wl.xy, wl.rot, types=types)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    return wl, pr, ctx, types


def _coeffs(wl, pr, seed):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((wl.n, wl.P)) + 1j * rng.standard_normal((wl.n, wl.P))
    return np.stack([rotated_smatrix(pr.S_of(l), wl.rot[l]) @ r[l] for l in range(wl.n)])


@pytest.mark.parametrize("name", ["s70p8", "s150p12", "s200p16"])
@pytest.mark.parametrize("order", ["mixed", "sorted"])
@pytest.mark.parametrize("prec", [0, 1])
def test_types_matvec(name, order, prec):
    wl, pr, ctx, _ = _types_setup(name, order)
    x = _coeffs(wl, pr, 3)
    got = ctx.apply(prec, x.astype(np.complex128 if prec == 0 else np.complex64))
    err = rel_err(got, pr.matvec(x))
    assert err < (1e-12 if prec == 0 else 2e-5), err


@pytest.mark.parametrize("prec,nrhs,tol", [(0, 4, 1e-12), (1, 20, 2e-5)])
def test_types_multi_rhs(prec, nrhs, tol):
    import torch
    wl, pr, ctx, _ = _types_setup("s150p12", "mixed")
    X = np.stack([_coeffs(wl, pr, s) for s in range(nrhs)])
    xd = torch.from_numpy(X.astype(np.complex128 if prec == 0 else np.complex64)).cuda()
    yd = torch.zeros_like(xd)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.apply_batch_dev(prec, nrhs, xd, yd)
    torch.cuda.synchronize()
    for r in (0, nrhs - 1):
        assert rel_err(yd[r].cpu().numpy(), pr.matvec(X[r])) < tol


def test_types_solve_and_field_match_lu():
    wl, pr, ctx, _ = _types_setup("c1", "mixed")
    src = wl.src[0]
    ref = pr.solve_lu(src)
    beta, meta = ctx.solve(src, precision=0, tol=1e-13, maxiter=400)
    assert meta["status"] == 0, meta
    assert rel_err(beta, ref) < 1e-10
    xs = wl.xy[:, 0]
    r = receivers(120, (xs.min() - 1, xs.max() + 1), (-wl.d - 1.5, 2.5), wl.xy, 5, particle_excl=wl.r_enclose + 0.05,
                  source=src, source_excl=0.05)
    assert rel_err(ctx.eval_field(src, beta, r), pr.field(src, ref, r)) < 1e-10


def test_one_type_is_the_single_matrix_path():
    wl = make_workload("s70p8")
    S = prototype_S(wl)
    a, b = mp.Context(0), mp.Context(0)
    for ctx in (a, b):
        ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    a.set_scattering_matrix(wl.p, wl.r_enclose, S)
    b.set_particle_types(wl.p, [wl.r_enclose], S[None])
    for ctx in (a, b):
        ctx.set_geometry(wl.xy, wl.rot)
        ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    x = _coeffs(wl, oracle_problem(wl), 1)
    assert np.array_equal(a.apply(0, x), b.apply(0, x))


def test_a_type_that_does_not_scatter():
    wl = make_workload("c1")
    S = prototype_S(wl)
    types = (np.arange(wl.n) % 3 == 0).astype(np.int32)
    ctx = mp.Context(0)
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_particle_types(wl.p, [wl.r_enclose, wl.r_enclose], np.stack([S, 0 * S]))
    ctx.set_geometry(wl.xy, wl.rot, types=types)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    beta, meta = ctx.solve(wl.src[0], precision=0, tol=1e-13, maxiter=400)
    assert meta["status"] == 0
    assert np.max(np.abs(beta[types == 1])) < 1e-14 * np.max(np.abs(beta))


def test_typed_geometry_checks_use_each_radius():
    ctx = mp.Context(0)
    ctx.set_layers(6.0, 9.0, 12.0, 8.0)
    S0 = np.diag(mie.disk_smatrix(0.3, 9.0, 15.0, 4))
    S1 = np.diag(mie.disk_smatrix(0.1, 9.0, 15.0, 4))
    ctx.set_particle_types(4, [0.3, 0.1], np.stack([S0, S1]))
    xy = np.array([[0.0, -2.0], [0.45, -2.0]])
    ctx.set_geometry(xy, types=[0, 1])                       # 0.3 + 0.1 < 0.45
    with pytest.raises(mp.MpslError):
        ctx.set_geometry(xy, types=[0, 0])                   # 0.3 + 0.3 > 0.45
    with pytest.raises(mp.MpslError):
        ctx.set_geometry(xy, types=[0, 2])                   # no type 2
    ctx.set_geometry(np.array([[0.0, -0.15], [3.0, -2.0]]), types=[1, 0])   # small one near y = 0
    with pytest.raises(mp.MpslError):
        ctx.set_geometry(np.array([[0.0, -0.15], [3.0, -2.0]]), types=[0, 1])
    ctx.set_geometry(xy, types=[0, 1])
    ctx.set_contour(256, 0.2, 32.0)
    u = ctx.eval_field(np.array([0.0, 2.0]), np.zeros((2, 9), complex),
                       np.array([[0.45, -2.0 + 0.12], [0.45, -2.0 + 0.08]]))
    assert np.isfinite(u[0]) and np.isnan(u[1])              # outside / inside the 0.1 disk
