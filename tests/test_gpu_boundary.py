"""Boundary calls: the field of several sources in one mpsl_eval_field call,
and the per-context HBM budget of mpsl_create."""
import numpy as np
import pytest

from gpu_common import make_workload, oracle_problem, prototype_S, rel_err
from synth import receivers

pytestmark = pytest.mark.gpu


def _configure(ctx, wl):
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_scattering_matrix(wl.p, wl.r_enclose, prototype_S(wl))
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    return ctx


def test_eval_field_of_several_sources():
    """Two sources and their coefficients in one call: each row equals the
    one-source call bitwise, and the oracle's field of the same coefficients
    (eq. (36)) to 1e-10."""
    import paper_1407_3868_amd as mp
    wl = make_workload("c1")
    pr = oracle_problem(wl)
    ctx = _configure(mp.Context(0), wl)
    srcs = np.array([wl.src[0], [1.5, 2.5]])
    betas, meta = ctx.solve(srcs, precision=0, tol=1e-12, maxiter=600)
    assert meta["status"] == 0
    xs = wl.xy[:, 0]
    rcv = receivers(64, (xs.min() - 1, xs.max() + 1), (-wl.d - 1.5, 2.5), wl.xy, 1064,
                    particle_excl=wl.r_enclose + 0.05, source=srcs[0], source_excl=0.05)
    rcv = rcv[np.min(np.hypot(rcv[:, 0] - srcs[1, 0], rcv[:, 1] - srcs[1, 1])[:, None], axis=1) > 0.05]
    both = ctx.eval_field(srcs, betas, rcv)
    assert both.shape == (2, len(rcv))
    for r in range(2):
        one = ctx.eval_field(srcs[r], betas[r], rcv)
        assert np.array_equal(one, both[r])
        assert rel_err(both[r], pr.field(srcs[r], betas[r], rcv)) < 1e-10


def test_eval_field_rejects_a_source_below_the_top_interface():
    import paper_1407_3868_amd as mp
    wl = make_workload("c1")
    ctx = _configure(mp.Context(0), wl)
    beta = np.zeros((2, wl.n, wl.P), np.complex128)
    with pytest.raises(mp.MpslError) as e:
        ctx.eval_field(np.array([[0.0, 2.0], [0.0, -1.0]]), beta, np.array([[0.0, 3.0]]))
    assert e.value.status == -1


def test_hbm_budget_refuses_and_counts():
    """A context whose budget is smaller than its tables refuses the
    allocation with MPSL_ENOMEM and holds no more than the budget; one with
    room computes the same matvec as an unlimited context and reports the
    bytes it holds."""
    import paper_1407_3868_amd as mp
    wl = make_workload("s70p8")
    x = np.random.default_rng(3).standard_normal((wl.n, wl.P)) + 0j
    free = _configure(mp.Context(0), wl)
    ref = free.apply(0, x)
    used_free, budget_free = free.memory()
    assert budget_free == 0 and used_free > 0
    small = mp.Context(0, hbm_budget=64 * 1024)
    with pytest.raises(mp.MpslError) as e:  # the contour tables alone exceed 64 KiB
        _configure(small, wl).apply(0, x)
    assert e.value.status == -2 and "budget" in str(e.value)
    used, budget = small.memory()
    assert budget == 64 * 1024 and used <= budget
    roomy = _configure(mp.Context(0, hbm_budget=2 * used_free), wl)
    y = roomy.apply(0, x)
    used, budget = roomy.memory()
    assert 0 < used <= budget
    assert np.array_equal(y, ref)
    roomy.close()
