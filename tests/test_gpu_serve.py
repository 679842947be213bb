"""Serving: continuous batching of solve requests.  Each result equals the
standalone solve of the same problem bitwise, alone and in a mix, and the
oracle's LU solution to the solve tolerance."""
import numpy as np
import pytest

from gpu_common import gpu_context, make_workload, oracle_problem, prototype_S, rel_err

pytestmark = pytest.mark.gpu


def _req(wl, precision=0, tol=1e-10, maxiter=600, src=None):
    src = wl.src[0] if src is None else src
    if wl.shape == "disk":
        part, shape, S = 0, (wl.shape_params[0],), None
    else:
        part, shape, S = 2, (), prototype_S(wl)
    return dict(k=(wl.k1, wl.k2, wl.k3), d=wl.d, particle=part, shape=shape, kp=wl.kp, p=wl.p, xy=wl.xy,
                rot=wl.rot, n_nodes=wl.n_nodes, b=wl.b, t_max=wl.t_max, src=src, precision=precision, tol=tol,
                maxiter=maxiter, S=S, r_enclose=wl.r_enclose)


def _wait(srv, ticket, timeout=120.0):
    """Wait for one request; a request that never completes fails the test."""
    res = srv.wait(ticket, timeout=timeout)
    assert res is not None, "request still pending after %.0f s" % timeout
    return res


def _standalone(wl, r):
    ctx = gpu_context(wl, disk_from_library=True)
    beta, meta = ctx.solve(r["src"], precision=r["precision"], tol=r["tol"], maxiter=r["maxiter"])
    return beta, meta


def test_results_alone_and_in_mix_are_identical():
    import paper_1407_3868_amd as mp
    wls = [make_workload("c1"), make_workload("s70p8"), make_workload("s150p12"), make_workload("c1", n=9)]
    reqs = [_req(wls[0]), _req(wls[1], precision=1, tol=1e-9), _req(wls[2], tol=1e-8), _req(wls[3], src=(0.5, 1.5))]
    alone = []
    srv = mp.Server(0, hbm_budget=32 << 30, max_active=1)
    for r in reqs:
        alone.append(_wait(srv, srv.submit(**r)))
    srv.close()
    srv = mp.Server(0, hbm_budget=32 << 30, max_active=8)
    tickets = [srv.submit(**r) for r in reqs]
    mix = [_wait(srv, t) for t in tickets]
    srv.close()
    for a, m, wl, r in zip(alone, mix, wls, reqs):
        assert a["status"] == 0 and m["status"] == 0
        assert np.array_equal(a["beta"], m["beta"])           # bitwise, whatever else ran
        assert a["iterations"] == m["iterations"]
        beta, meta = _standalone(wl, r)                        # the library's own solve
        assert np.array_equal(beta, m["beta"])
    # requests really overlapped in the mix
    spans = [(m["t_start"], m["t_finish"]) for m in mix]
    assert any(s2[0] < s1[1] and s1[0] < s2[1] for i, s1 in enumerate(spans) for s2 in spans[i + 1:])


def test_served_solution_matches_oracle():
    import paper_1407_3868_amd as mp
    wl = make_workload("s70p8")
    srv = mp.Server(0)
    res = _wait(srv, srv.submit(**_req(wl, tol=1e-12, maxiter=800)))
    srv.close()
    assert res["status"] == 0
    assert rel_err(res["beta"], oracle_problem(wl).solve_lu(wl.src[0])) < 1e-10


def test_admission_respects_budget_and_errors_are_reported():
    import paper_1407_3868_amd as mp
    wl = make_workload("c1")
    r = _req(wl)
    probe = mp.Server(0, hbm_budget=1 << 40, max_active=4)
    one = _wait(probe, probe.submit(**r))
    probe.close()
    need = one["hbm_bytes"]
    srv = mp.Server(0, hbm_budget=int(need * 1.5), max_active=4)   # room for one request at a time
    tickets = [srv.submit(**r) for _ in range(3)]
    res = [_wait(srv, t) for t in tickets]
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_finish"] - 1e-6                 # admitted only after the previous finished
    with pytest.raises(mp.MpslError) as e:                          # alone larger than the budget
        big = _req(make_workload("s150p12"))
        srv.submit(**big)
    assert e.value.status == -2
    bad = dict(r)
    bad["xy"] = np.array([[0.0, -2.0], [0.1, -2.0]])                # overlapping particles
    bad["rot"] = None
    out = _wait(srv, srv.submit(**bad))
    assert out["status"] == -5 and "beta" not in out
    srv.close()


def test_span_contour_and_preconditioner_requests():
    """Requests on a span-rule contour with the interpolated Sommerfeld sums
    and the cluster preconditioner: bitwise the library's own solve with the
    same settings, alone and in a mix with plain requests, and the oracle's
    LU solution of the same discrete system (star layout, both precisions)."""
    import paper_1407_3868_amd as mp
    wl = make_workload("s150p12")
    X = float(wl.xy[:, 0].max() - wl.xy[:, 0].min())
    b, h = mp.span_contour_params(X, 1e-10)
    assert (b, h) == (min(0.2, 2.0 / X), 6.0 / X)
    extra = dict(contour=1, n_nodes=0, b=b, t_max=24.0, h_max=h, sommerfeld=mp.SOMM_INTERP,
                 precond=mp.PRECOND_CLUSTER, cluster_size=40)
    reqs = [dict(_req(wl, tol=1e-11, maxiter=1500), **extra), dict(_req(wl, precision=1, tol=1e-9), **extra),
            _req(make_workload("c1"))]
    srv = mp.Server(0, hbm_budget=64 << 30, max_active=1)
    alone = [_wait(srv, srv.submit(**r)) for r in reqs]
    srv.close()
    srv = mp.Server(0, hbm_budget=64 << 30, max_active=8)
    mix = [_wait(srv, t) for t in [srv.submit(**r) for r in reqs]]
    srv.close()
    for a, m in zip(alone, mix):
        assert a["status"] == 0 and m["status"] == 0, (a["error"], m["error"])
        assert np.array_equal(a["beta"], m["beta"])
    ctx = mp.Context(0)
    ctx.set_sommerfeld_method(mp.SOMM_INTERP)
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_scattering_matrix(wl.p, wl.r_enclose, prototype_S(wl))
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour_span(b, 24.0, h)
    ctx.set_preconditioner(mp.PRECOND_CLUSTER, 40)
    beta, meta = ctx.solve(wl.src[0], precision=0, tol=1e-11, maxiter=1500)
    assert np.array_equal(beta, mix[0]["beta"])
    from oracle import system as osys
    lam, w = ctx.get_contour()
    pr = osys.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, prototype_S(wl), wl.xy, wl.rot, lam, w)
    ref = pr.solve_lu(wl.src[0])
    assert rel_err(mix[0]["beta"], ref) < 1e-8
    assert rel_err(mix[1]["beta"], ref) < 1e-6
