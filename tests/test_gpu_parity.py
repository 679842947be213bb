"""GPU parity: every HIP step of the matvec, the matvec itself, the right-hand
side and the solve, against the FP64 oracle on the same seeded inputs.

Tolerances: relative 2-norm over the output, and per entry (gpu_common.ENTRY_TOL:
|got - ref| <= tol (|ref| + eps max|ref| of the particle), worst entry reported):
  FP64 steps      1e-12  (rounding of O(N P) FP64 sums; the oracle uses
                          scipy's AMOS Hankel functions, the library the ROCm
                          device library, both accurate to a few ulp)
  FP32 steps      see FP32_TOL: FP32 unit roundoff 6e-8 times the growth of
                  the Hankel recurrence and the length of the sums
  solve / field   1e-10 relative field error in FP64 mode, 1e-6 in mixed mode
"""
import numpy as np
import pytest

from gpu_common import (ENTRY_TOL, coeff_vector, entry_err, gpu_context, make_workload, max_err, oracle_problem,
                        prototype_S, rel_err)
from oracle import layered as olayered
from oracle import operators as oops

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
# FP32 M2L: the terms h_q beta_nu span many orders of magnitude (|H_q| grows like
# (2q/(e z))^q while beta decays with the scattering matrix), and each output
# sums (N - 1) P of them; 2e-5 is ~300 u_32 and bounds what was measured with
# a 10x margin.
FP32_TOL = 2e-5

SMALL = ["s70p8", "s150p12", "s200p16"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _setup(name):
    wl = make_workload(name)
    return wl, oracle_problem(wl), gpu_context(wl)


def _dev(torch, a, dt):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to("cuda")


def _zeros(torch, shape, dt):
    return torch.zeros(shape, dtype=dt, device="cuda")


@pytest.mark.parametrize("name", SMALL + ["c3"])
def test_contour_nodes_match_oracle(name, torch_dev):
    wl = make_workload(name, n=16 if name == "c3" else None)
    ctx = gpu_context(wl)
    lam, w = ctx.get_contour()
    pr = oracle_problem(wl)
    assert np.max(np.abs(lam - pr.lam)) < 1e-13 * np.max(np.abs(pr.lam))
    assert np.max(np.abs(w - pr.w)) < 1e-13 * np.max(np.abs(pr.w))


def test_disk_matrix_matches_oracle(torch_dev):
    from oracle import mie
    wl = make_workload("c1")
    ctx = gpu_context(wl, disk_from_library=True)
    S = ctx.get_scattering_matrix()
    ref = np.diag(mie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p))
    assert np.max(np.abs(S - ref)) < 1e-13


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("prec", [0, 1])
def test_m2l(name, prec, torch_dev):
    torch = torch_dev
    wl, pr, ctx = _setup(name)
    x = coeff_vector(wl, 1)
    ref = oops.m2l_apply(wl.xy, wl.k2, wl.p, x)
    dt = torch.complex128 if prec == 0 else torch.complex64
    xd = _dev(torch, x, np.complex128 if prec == 0 else np.complex64)
    ad = _zeros(torch, (wl.n, wl.P), dt)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.m2l_dev(prec, xd, ad)
    torch.cuda.synchronize()
    got = ad.cpu().numpy()
    tol = FP64_TOL if prec == 0 else FP32_TOL
    assert rel_err(got, ref) < tol, rel_err(got, ref)
    _assert_entries(got, ref, prec)


def _assert_entries(got, ref, prec):
    tol, eps = ENTRY_TOL[prec]
    e, where = entry_err(got, ref, eps)
    assert e < tol, f"worst entry {where} (row, slot): {e:.2e}"


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("prec", [0, 1])
def test_m2s(name, prec, torch_dev):
    torch = torch_dev
    wl, pr, ctx = _setup(name)
    x = coeff_vector(wl, 2)
    Pp, Pm = oops.m2s(x, wl.xy, pr.lam, wl.k2, wl.d)
    xd = _dev(torch, x, np.complex128 if prec == 0 else np.complex64)
    sd = _zeros(torch, (2, wl.n_nodes), torch.complex128)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.m2s_dev(prec, xd, sd)
    torch.cuda.synchronize()
    got = sd.cpu().numpy()
    ref = np.stack([Pp, Pm])
    tol = FP64_TOL if prec == 0 else FP32_TOL
    assert rel_err(got, ref) < tol, rel_err(got, ref)
    _assert_entries(got, ref, prec)


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("with_particles,with_source", [(True, False), (False, True), (True, True)])
def test_reflect(name, with_particles, with_source, torch_dev):
    # closed-form 2x2 reflection on the GPU against the oracle's 4x4 solve per node
    torch = torch_dev
    wl, pr, ctx = _setup(name)
    rng = np.random.default_rng(3)
    spec = (rng.standard_normal((2, wl.n_nodes)) + 1j * rng.standard_normal((2, wl.n_nodes))) if with_particles else None
    src = np.array([0.7, 1.9]) if with_source else None
    b = np.zeros((wl.n_nodes, 4), complex)
    if spec is not None:
        b += olayered.particle_rhs(pr.lam, wl.k2, spec[0], spec[1])
    if src is not None:
        b += olayered.source_rhs(pr.lam, wl.k1, src[0], src[1])
    ref = olayered.solve_nodes(pr.A, b)[:, 1:3].T
    sd = None if spec is None else _dev(torch, spec, np.complex128)
    out = _zeros(torch, (2, wl.n_nodes), torch.complex128)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.reflect_dev(sd, src, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert rel_err(got, ref) < 1e-13, rel_err(got, ref)


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("prec", [0, 1])
def test_s2l(name, prec, torch_dev):
    torch = torch_dev
    wl, pr, ctx = _setup(name)
    rng = np.random.default_rng(4)
    sig = rng.standard_normal((2, wl.n_nodes)) + 1j * rng.standard_normal((2, wl.n_nodes))
    ref = oops.s2l(sig[0], sig[1], wl.xy, pr.lam, pr.w, wl.k2, wl.d, wl.p)
    sd = _dev(torch, sig, np.complex128)
    dt = torch.complex128 if prec == 0 else torch.complex64
    ad = _zeros(torch, (wl.n, wl.P), dt)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.s2l_dev(prec, sd, ad)
    torch.cuda.synchronize()
    got = ad.cpu().numpy()
    tol = FP64_TOL if prec == 0 else FP32_TOL
    assert rel_err(got, ref) < tol, rel_err(got, ref)
    _assert_entries(got, ref, prec)


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("prec", [0, 1])
def test_sapply(name, prec, torch_dev):
    torch = torch_dev
    wl, pr, ctx = _setup(name)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((wl.n, wl.P)) + 1j * rng.standard_normal((wl.n, wl.P))
    x = rng.standard_normal((wl.n, wl.P)) + 1j * rng.standard_normal((wl.n, wl.P))
    ref = x - pr.apply_S(a)
    npdt = np.complex128 if prec == 0 else np.complex64
    dt = torch.complex128 if prec == 0 else torch.complex64
    yd = _zeros(torch, (wl.n, wl.P), dt)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.sapply_dev(prec, _dev(torch, x, npdt), _dev(torch, a, npdt), yd)
    torch.cuda.synchronize()
    tol = FP64_TOL if prec == 0 else 1e-6
    assert rel_err(yd.cpu().numpy(), ref) < tol
    _assert_entries(yd.cpu().numpy(), ref, prec)


@pytest.mark.parametrize("name", SMALL + ["c1"])
@pytest.mark.parametrize("prec", [0, 1])
def test_matvec(name, prec, torch_dev):
    torch = torch_dev
    wl, pr, ctx = _setup(name)
    x = coeff_vector(wl, 6)
    ref = pr.matvec(x)
    npdt = np.complex128 if prec == 0 else np.complex64
    dt = torch.complex128 if prec == 0 else torch.complex64
    yd = _zeros(torch, (wl.n, wl.P), dt)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.apply_dev(prec, _dev(torch, x, npdt), yd)
    torch.cuda.synchronize()
    tol = FP64_TOL if prec == 0 else FP32_TOL
    err = rel_err(yd.cpu().numpy(), ref)
    assert err < tol, err
    _assert_entries(yd.cpu().numpy(), ref, prec)
    # host-pointer entry point gives the same bytes
    y2 = ctx.apply(prec, x.astype(npdt))
    assert np.array_equal(y2, yd.cpu().numpy())


@pytest.mark.parametrize("name", SMALL + ["c1"])
def test_rhs(name, torch_dev):
    wl, pr, ctx = _setup(name)
    src = np.array([0.3, 2.0])
    assert rel_err(ctx.rhs(src), pr.rhs(src)) < FP64_TOL


def test_free_space_limit_has_no_reflection(torch_dev):
    torch = torch_dev
    wl = make_workload("s150p12")
    ctx = gpu_context(wl, ks=(9.0, 9.0, 9.0))
    rng = np.random.default_rng(7)
    sig_spec = _dev(torch, rng.standard_normal((2, wl.n_nodes)) + 0j, np.complex128)
    out = _zeros(torch, (2, wl.n_nodes), torch.complex128)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.reflect_dev(sig_spec, None, out)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0


@pytest.mark.parametrize("n", [1, 2, 17, 129])
@pytest.mark.parametrize("prec", [0, 1])
def test_small_and_ragged_counts(n, prec, torch_dev):
    # p = 16: the default M2L is the matrix-core form in both precisions (one
    # partial 16-target tile, partial source groups of four)
    wl = make_workload("s200p16", n=n)
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    x = coeff_vector(wl, 8)
    assert ctx.get_tuning(prec)["variant"] == 2
    got = ctx.apply(prec, x.astype(np.complex128 if prec == 0 else np.complex64))
    ref = pr.matvec(x)
    assert rel_err(got, ref) < (FP64_TOL if prec == 0 else FP32_TOL)
    _assert_entries(got, ref, prec)


def test_highest_order(torch_dev):
    wl = make_workload("s70p8")
    wl.p = 20
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    x = coeff_vector(wl, 9)
    assert rel_err(ctx.apply(0, x), pr.matvec(x)) < FP64_TOL


@pytest.mark.parametrize("name", ["s70p8", "s150p12", "s200p16"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("variant,chunks", [(0, 3), (1, 0), (1, 7), (2, 0), (2, 7), (3, 0), (3, 5)])
def test_m2l_variants(name, prec, variant, chunks, torch_dev):
    # every launch shape (whole / output halves through the mirror identity /
    # matrix cores with 16 or 32 targets per wave) and several source-chunk
    # counts give the oracle's translation
    torch = torch_dev
    wl, pr, ctx = _setup(name)
    ctx.set_tuning(prec, variant, chunks)
    x = coeff_vector(wl, 12)
    ref = oops.m2l_apply(wl.xy, wl.k2, wl.p, x)
    dt = torch.complex128 if prec == 0 else torch.complex64
    xd = _dev(torch, x, np.complex128 if prec == 0 else np.complex64)
    ad = _zeros(torch, (wl.n, wl.P), dt)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.m2l_dev(prec, xd, ad)
    torch.cuda.synchronize()
    tol = FP64_TOL if prec == 0 else FP32_TOL
    assert rel_err(ad.cpu().numpy(), ref) < tol
    _assert_entries(ad.cpu().numpy(), ref, prec)
    y = ctx.apply(prec, x.astype(np.complex128 if prec == 0 else np.complex64))
    yref = pr.matvec(x)
    assert rel_err(y, yref) < tol
    _assert_entries(y, yref, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_keeps_results(prec, torch_dev):
    wl, pr, ctx = _setup("s200p16")
    x = coeff_vector(wl, 13)
    npdt = np.complex128 if prec == 0 else np.complex64
    before = ctx.apply(prec, x.astype(npdt))
    ctx.autotune(prec)
    t = ctx.get_tuning(prec)
    assert t["variant"] in (0, 1, 2, 3) and t["chunks"] >= 1 and t["m2l_ms"] > 0
    after = ctx.apply(prec, x.astype(npdt))
    tol = FP64_TOL if prec == 0 else FP32_TOL
    assert rel_err(after, pr.matvec(x)) < tol
    assert rel_err(after, before) < tol


@pytest.mark.parametrize("prec", [0, 1])
def test_m2l_matrix_cores_multi_rhs_and_empty_chunks(prec, torch_dev):
    """The matrix-core M2L over several right-hand sides (grid.z) and with more
    source chunks than fill (trailing chunks empty: their partial slots must
    come out zero), 150 stars at p = 12 (rows 12..15 of each 16-row block
    masked)."""
    torch = torch_dev
    wl, pr, ctx = _setup("s150p12")
    # 149 chunks of 150 sources: the chunk length rounds up to one group of
    # four, so 38 chunks hold sources and the other 111 are empty (49 chunks
    # per right-hand side in the three-source batch: 38 full, 11 empty)
    ctx.set_tuning(prec, 2, 149)
    X = np.stack([coeff_vector(wl, 20 + r) for r in range(3)])
    npdt = np.complex128 if prec == 0 else np.complex64
    xd = torch.from_numpy(X.astype(npdt)).cuda()
    yd = torch.zeros_like(xd)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.apply_batch_dev(prec, 3, xd, yd)
    torch.cuda.synchronize()
    tol = FP64_TOL if prec == 0 else FP32_TOL
    for r in range(3):
        assert rel_err(yd[r].cpu().numpy(), pr.matvec(X[r])) < tol


def test_m2l_matrix_cores_order_limit(torch_dev):
    """p = 20 is beyond the matrix-core form: a stored matrix-core variant
    runs as the one-lane-per-target kernel, and the autotuner skips it."""
    wl = make_workload("s70p8")
    wl.p = 20
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    x = coeff_vector(wl, 9)
    ctx.set_tuning(0, 3, 0)
    assert rel_err(ctx.apply(0, x), pr.matvec(x)) < FP64_TOL
    ctx.autotune(0)
    assert ctx.get_tuning(0)["variant"] in (0, 1)
    assert rel_err(ctx.apply(0, x), pr.matvec(x)) < FP64_TOL
