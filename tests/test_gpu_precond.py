"""GPU cluster-block preconditioner against the oracle (oracle/precond.py).

- apply: y = M^{-1} x with the device blocks; every cluster's oracle system
  K_c = I - S_c T_cc must map y back to x (backward error, robust to the
  blocks' conditioning), and y must match the oracle's inverses applied to x;
- solves: right-preconditioned FP64 and mixed-precision solves of star
  layouts against the oracle's dense LU solve (coefficients and field), with
  fewer iterations than without the preconditioner;
- the reference fields of the 1000-star recipe and of a 600-star window of
  the 5000-star recipe (tests/golden, written by the oracle's dense LU).

Tolerances: FP64 apply backward error 1e-10 (blocks with condition numbers
up to ~1e10 inverted without pivoting across 64 x 64 steps); FP32 copy 1e-4
forward (FP32 rounding of the inverse entries times the sums' cancellation);
fields 1e-10 (FP64 solve) and 1e-6 (mixed), as for the other solves.
"""
import os

import numpy as np
import pytest

import paper_1407_3868_amd as mp
from gpu_common import gpu_context, make_workload, oracle_problem, rel_err
from oracle import precond as opc
from synth import receivers

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _rcv(wl, n=96):
    xs = wl.xy[:, 0]
    return receivers(n, (xs.min() - 1, xs.max() + 1), (-wl.d - 1.5, 2.5), wl.xy, 1000 + n,
                     particle_excl=wl.r_enclose + 0.05, source=wl.src[0], source_excl=0.05)


@pytest.mark.parametrize("name,size", [("s150p12", 1), ("s150p12", 16), ("s150p12", 40), ("s200p16", 40),
                                       ("s200p16", 7), ("s70p8", 70)])
def test_precond_apply(name, size, torch_dev):
    torch = torch_dev
    wl = make_workload(name)
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.set_preconditioner(mp.PRECOND_CLUSTER, size)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((wl.n, wl.P)) + 1j * rng.standard_normal((wl.n, wl.P))
    xd = torch.from_numpy(x).cuda()
    y64 = torch.zeros_like(xd)
    y32 = torch.zeros_like(xd)
    ctx.precond_apply_dev(0, xd, y64)
    ctx.precond_apply_dev(1, xd, y32)
    torch.cuda.synchronize()
    y64, y32 = y64.cpu().numpy(), y32.cpu().numpy()
    cl = opc.clusters(wl.xy, size)
    info = ctx.precond_info()
    assert info["n_clusters"] == len(cl) and info["replaced"] == 0
    assert info["max_cluster"] == max(len(c) for c in cl)
    worst = 0.0
    inv = []
    for idx in cl:
        K = opc.cluster_matrix(pr, idx)
        r = np.linalg.norm(K @ y64[idx].reshape(-1) - x[idx].reshape(-1)) / np.linalg.norm(x[idx])
        worst = max(worst, r)
        inv.append(np.linalg.inv(K))
    assert worst < 1e-10, worst
    ref = opc.apply(cl, inv, x, wl.P)
    e64, e32 = rel_err(y64, ref), rel_err(y32, ref)
    print(f"{name} size {size}: backward {worst:.2e}, forward FP64 {e64:.2e}, FP32 copy {e32:.2e}")
    assert e64 < 1e-8 and e32 < 1e-4


def test_precond_rebuilds_after_geometry_change(torch_dev):
    torch = torch_dev
    wl = make_workload("s150p12")
    ctx = gpu_context(wl)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.set_preconditioner(mp.PRECOND_CLUSTER, 30)
    x = np.random.default_rng(6).standard_normal((wl.n, wl.P)) + 0j
    xd = torch.from_numpy(x).cuda()
    y = torch.zeros_like(xd)
    ctx.precond_apply_dev(0, xd, y)
    xy = wl.xy.copy()
    xy[:, 0] *= 1.05   # spread the layout: every pair distance changes
    ctx.set_geometry(xy, wl.rot)
    ctx.precond_apply_dev(0, xd, y)
    torch.cuda.synchronize()
    wl2 = make_workload("s150p12")
    wl2.xy = xy
    pr2 = oracle_problem(wl2)
    yy = y.cpu().numpy()
    for idx in opc.clusters(xy, 30):
        K = opc.cluster_matrix(pr2, idx)
        assert np.linalg.norm(K @ yy[idx].reshape(-1) - x[idx].reshape(-1)) < 1e-10 * np.linalg.norm(x[idx])
    # back to no preconditioner: apply is refused, solves run unpreconditioned
    ctx.set_preconditioner(mp.PRECOND_NONE)
    with pytest.raises(mp.MpslError):
        ctx.precond_apply_dev(0, xd, y)


@pytest.mark.parametrize("name,size", [("s150p12", 40), ("s200p16", 40)])
def test_precond_fp64_solve_matches_lu(name, size):
    wl = make_workload(name)
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    src = wl.src[0]
    ref = pr.solve_lu(src)
    _, meta0 = ctx.solve(src, precision=0, tol=1e-12, maxiter=1500)
    ctx.set_preconditioner(mp.PRECOND_CLUSTER, size)
    beta, meta = ctx.solve(src, precision=0, tol=1e-12, maxiter=1500)
    print(f"{name}: {meta0['iterations']} iterations plain, {meta['iterations']} preconditioned "
          f"(blocks {meta['precond_seconds']:.3f} s)")
    assert meta["status"] == 0 and meta["rel_residual"] < 1e-11
    assert meta["iterations"] < 0.7 * meta0["iterations"]
    assert rel_err(beta, ref) < 1e-9
    r = _rcv(wl)
    assert rel_err(ctx.eval_field(src, beta, r), pr.field(src, ref, r)) < 1e-10


@pytest.mark.parametrize("name,size", [("s150p12", 40), ("s200p16", 40), ("s200p16", 200)])
def test_precond_mixed_solve_matches_lu(name, size):
    wl = make_workload(name)
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    ctx.set_preconditioner(mp.PRECOND_CLUSTER, size)
    src = wl.src[0]
    ref = pr.solve_lu(src)
    beta, meta = ctx.solve(src, precision=1, tol=1e-10, maxiter=3000)
    print(f"{name} mixed: {meta['iterations']} iterations, {meta['refinements']} refinements")
    assert meta["status"] == 0, meta
    r = _rcv(wl)
    e = rel_err(ctx.eval_field(src, beta, r), pr.field(src, ref, r))
    print(f"  field error {e:.2e}")
    assert e < 1e-6


def _golden(case):
    path = os.path.join(GOLDEN, f"{case}_lu_field.txt")
    d = np.loadtxt(path)
    return d[:, :2], d[:, 2] + 1j * d[:, 3]


@pytest.mark.parametrize("case,prec,tol", [("c3cut600", 0, 1e-10), ("c3cut600", 1, 1e-6), ("c2", 0, 1e-10),
                                           ("c2", 1, 1e-6)])
def test_solve_matches_golden_lu(case, prec, tol):
    # 600-star window of the 5000-star recipe (p = 16, 1024 nodes) and the
    # 1000-star recipe (p = 12, 512 nodes) against the oracle's dense LU fields
    from gpu_common import prototype_S
    wl = make_workload("c3", cut=600) if case == "c3cut600" else make_workload("c2")
    rcv, u_ref = _golden(case)
    ctx = mp.Context(0)
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_scattering_matrix(wl.p, wl.r_enclose, prototype_S(wl))
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    ctx.set_preconditioner(mp.PRECOND_CLUSTER, 0)
    src = wl.src[0]
    beta, meta = ctx.solve(src, precision=prec, tol=1e-12 if prec == 0 else 1e-10, maxiter=4000)
    u = ctx.eval_field(src, beta, rcv)
    e = rel_err(u, u_ref)
    print(f"{case} prec {prec}: {meta['iterations']} iterations in {meta['seconds']:.2f} s, field error {e:.2e}")
    assert meta["status"] == 0, meta
    assert e < tol
