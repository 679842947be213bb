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
