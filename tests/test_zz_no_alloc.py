"""The allocation-free M2L (mpsl_m2l_dev_noalloc) against mpsl_m2l_dev.

Called through the C ABI twice in a row, the second time with a smaller
problem (the scratch keeps the first call's contents, which must not leak
into the second), in both precisions, to the step's parity bars (relative
2-norm and per entry; the two calls sum different numbers of source chunks,
so they agree to rounding, not bitwise).  Also: sizes beyond the fixed
scratch are refused with MPSL_EINVAL, a context without tables with
MPSL_ESTATE, and the result still matches the oracle.
"""
import numpy as np
import pytest

import paper_1407_3868_amd as mp
from gpu_common import ENTRY_TOL, coeff_vector, entry_err, gpu_context, make_workload, rel_err
from oracle import operators as oops

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 2e-5}


def _m2l(torch, ctx, prec, x, noalloc):
    npdt = np.complex128 if prec == 0 else np.complex64
    xd = torch.from_numpy(x.astype(npdt)).cuda()
    ad = torch.full_like(xd, float("nan"))
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    (ctx.m2l_dev_noalloc if noalloc else ctx.m2l_dev)(prec, xd, ad)
    torch.cuda.synchronize()
    return ad.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_m2l_twice(prec):
    import torch
    assert torch.cuda.is_available()
    for name, n in (("s200p16", None), ("s150p12", 97)):   # second call: smaller input
        wl = make_workload(name, n=n)
        ctx = gpu_context(wl)
        x = coeff_vector(wl, 31)
        ref = _m2l(torch, ctx, prec, x, False)   # builds the tables
        got = _m2l(torch, ctx, prec, x, True)
        etol, eps = ENTRY_TOL[prec]
        assert rel_err(got, ref) < TOL[prec]
        assert entry_err(got, ref, eps)[0] < etol
        ora = oops.m2l_apply(wl.xy, wl.k2, wl.p, x)
        assert rel_err(got, ora) < TOL[prec]
        assert np.all(np.isfinite(got))


def test_noalloc_refusals():
    import torch
    wl = make_workload("s70p8")
    ctx = gpu_context(wl)
    x = torch.zeros((wl.n, wl.P), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(mp.MpslError) as e:   # no tables yet
        ctx.m2l_dev_noalloc(0, x, y)
    assert e.value.status == -4
    # 130000 disks at p = 16: N P = 4.29e6 complex128 is above the 64 MiB scratch
    big = mp.Context(0)
    big.set_layers(6.0, 9.0, 12.0, 170.0)
    big.set_particle_disk(0.25, 15.0, 16)
    g = np.stack(np.meshgrid(np.arange(650) * 0.8, -1.0 - 0.8 * np.arange(200)), -1).reshape(-1, 2)[:130000]
    big.set_geometry(np.ascontiguousarray(g))
    with pytest.raises(mp.MpslError) as e:
        big.m2l_dev_noalloc(0, x, y)
    assert e.value.status == -1
