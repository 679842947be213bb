"""Parity at the benchmark's full size (5000 stars, p = 16, 1024 contour
nodes), in the launch configuration the benchmark times, on outputs the oracle
computes target by target."""
import numpy as np
import pytest

from gpu_common import ENTRY_TOL, coeff_vector, entry_err, gpu_context, make_workload, oracle_problem

pytestmark = pytest.mark.gpu

# 64 seeded rows across the strip, plus both ends and the 64-lane tile edges
TARGETS = sorted(set([0, 1, 63, 64, 2500, 4095, 4999]) |
                 set(np.random.default_rng(64).choice(5000, 57, replace=False).tolist()))


@pytest.fixture(scope="module")
def c3():
    wl = make_workload("c3")
    return wl, oracle_problem(wl), gpu_context(wl)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5)])
def test_matvec_sampled(c3, prec, tol):
    import torch
    wl, pr, ctx = c3
    x = coeff_vector(wl, 11)
    npdt = np.complex128 if prec == 0 else np.complex64
    xd = torch.from_numpy(x.astype(npdt)).cuda()
    yd = torch.zeros_like(xd)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.apply_dev(prec, xd, yd)
    torch.cuda.synchronize()
    got = yd.cpu().numpy()[TARGETS]
    ref = pr.matvec(x, targets=TARGETS)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < tol, err
    etol, eps = ENTRY_TOL[prec]
    e, (row, slot) = entry_err(got, ref, eps)
    assert e < etol, f"worst entry: particle {TARGETS[row]}, slot {slot}: {e:.2e}"
    assert np.all(np.isfinite(yd.cpu().numpy()))


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_checked_in_the_oracle(c3, prec):
    """The benchmark's solve (cluster preconditioner, tol 1e-6) checked in the
    oracle's own operator: the residual b - K beta of the GPU solution at the
    sampled rows, and the oracle's total field (eq. (36)) of the same beta at
    seeded receivers in all three layers against the library's."""
    import paper_1407_3868_amd as mp
    from gpu_common import rel_err
    from synth import receivers
    wl, pr, ctx = c3
    ctx.set_preconditioner(mp.PRECOND_CLUSTER, 160)
    src = wl.src[0]
    beta, meta = ctx.solve(src, precision=prec, tol=1e-6, maxiter=4000, inner_tol=1e-5 if prec else 0.0)
    assert meta["status"] == 0, meta
    b = pr.rhs(src)[TARGETS]
    r = b - pr.matvec(beta, targets=TARGETS)
    res = float(np.linalg.norm(r) / np.linalg.norm(b))
    xs = wl.xy[:, 0]
    rcv = receivers(24, (xs.min() - 2.0, xs.max() + 2.0), (-wl.d - 2.0, 3.0), wl.xy, 1002, particle_excl=0.35,
                    source=src, source_excl=0.05)
    u_gpu = ctx.eval_field(src, beta, rcv)
    u_or = pr.field(src, beta, rcv)
    ferr = rel_err(u_gpu, u_or)
    print(f"prec {prec}: {meta['iterations']} its, GPU residual {meta['rel_residual']:.2e}, "
          f"oracle residual at {len(TARGETS)} rows {res:.2e}, field of the same beta {ferr:.2e}", flush=True)
    assert res < 1e-5, res
    assert ferr < 1e-10, ferr
