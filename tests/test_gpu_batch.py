"""Batching: many right-hand sides per launch, and many configurations in
one captured graph; against the oracle and against the unbatched path."""
import numpy as np
import pytest

from gpu_common import coeff_vector, gpu_context, make_workload, oracle_problem, rel_err
from synth import perturbed_layout

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nrhs", [1, 3, 8, 16, 40, 70])
def test_multi_rhs_matvec(prec, nrhs, torch):
    wl = make_workload("s150p12")
    pr = oracle_problem(wl)
    ctx = gpu_context(wl)
    xs = np.stack([coeff_vector(wl, 20 + r) for r in range(nrhs)])
    npdt = np.complex128 if prec == 0 else np.complex64
    xd = torch.from_numpy(xs.astype(npdt)).cuda()
    yd = torch.zeros_like(xd)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    ctx.apply_batch_dev(prec, nrhs, xd, yd)
    torch.cuda.synchronize()
    got = yd.cpu().numpy()
    tol = FP64_TOL if prec == 0 else FP32_TOL
    for r in range(nrhs):
        assert rel_err(got[r], pr.matvec(xs[r])) < tol


def _perturbed(name, seed):
    wl = make_workload(name)
    xy, rot = perturbed_layout(wl.xy, wl.rot, 0.05, seed, 0.75, y_range=(-wl.d + 0.4, -0.4))
    wl.xy, wl.rot = xy, rot
    return wl


def test_graph_batch_of_configurations(torch):
    wls = [make_workload("s70p8"), make_workload("s150p12"), _perturbed("s150p12", 5)]
    items = [(0, 1), (1, 3), (0, 2)]           # (precision, right-hand sides) per configuration
    ctxs = [gpu_context(w) for w in wls]
    stream = torch.cuda.current_stream().cuda_stream
    for c in ctxs:
        c.set_stream(stream)
    xs, ys, refs = [], [], []
    for w, c, (prec, nr) in zip(wls, ctxs, items):
        npdt = np.complex128 if prec == 0 else np.complex64
        x = np.stack([coeff_vector(w, 30 + r) for r in range(nr)]).astype(npdt)
        xd = torch.from_numpy(x).cuda()
        yd = torch.zeros_like(xd)
        c.apply_batch_dev(prec, nr, xd, yd)    # eager reference on the same buffers
        torch.cuda.synchronize()
        refs.append(yd.clone())
        xs.append(xd)
        ys.append(yd)
    import paper_1407_3868_amd as mp
    batch = mp.Batch([(c, prec, nr, x, y) for c, (prec, nr), x, y in zip(ctxs, items, xs, ys)])
    for rep in range(3):
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        batch.launch(stream)
        torch.cuda.synchronize()
        for y, ref in zip(ys, refs):
            assert torch.equal(y, ref), f"replay {rep} differs from the eager result"
        # eager work between replays, on the same contexts
        c0 = ctxs[0]
        scratch = torch.zeros_like(ys[0])
        c0.apply_batch_dev(items[0][0], items[0][1], xs[0], scratch)
        _ = (scratch * 2).sum()
        torch.cuda.synchronize()
    # and the batch agrees with the oracle
    for w, (prec, nr), x, y in zip(wls, items, xs, ys):
        pr = oracle_problem(w)
        tol = FP64_TOL if prec == 0 else FP32_TOL
        for r in range(nr):
            assert rel_err(y[r].cpu().numpy(), pr.matvec(x[r].cpu().numpy().astype(np.complex128))) < tol
    batch.close()
