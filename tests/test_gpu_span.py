"""GPU parity with the span-rule contour (mpsl_set_contour_span): panels of
bounded length so that the Sommerfeld sums resolve e^{i lambda x} over the
layout's lateral extent X.  The library's nodes, matvec and solve against the
oracle on the same contour, at small sizes and at the 5000-particle size with
sampled rows; and the layered part converged against a twice finer contour.

Tolerances: 1e-13 on nodes, 1e-12 FP64 / 2e-5 FP32 matvec (as for the
count-rule contour), 1e-10 FP64 solve against LU.
"""
import numpy as np
import pytest

import paper_1407_3868_amd as mp
from gpu_common import coeff_vector, make_workload, prototype_S, rel_err
from oracle import contour as ocontour
from oracle import system as osystem

pytestmark = pytest.mark.gpu

T_MAX = 24.0


def _extent(wl):
    return float(wl.xy[:, 0].max() - wl.xy[:, 0].min())


def _setup(name, h_factor=6.0):
    wl = make_workload(name)
    X = _extent(wl)
    b, h = min(0.2, 2.0 / X), h_factor / X
    ks = [wl.k1, wl.k2, wl.k3]
    lam, w = ocontour.contour_span(b, T_MAX, h, ks)
    pr = osystem.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, prototype_S(wl), wl.xy, wl.rot, lam, w)
    ctx = mp.Context(0)
    ctx.set_layers(wl.k1, wl.k2, wl.k3, wl.d)
    ctx.set_scattering_matrix(wl.p, wl.r_enclose, prototype_S(wl))
    ctx.set_geometry(wl.xy, wl.rot)
    ns = ctx.set_contour_span(b, T_MAX, h)
    assert ns == lam.size
    return wl, pr, ctx


def test_span_nodes_match_oracle():
    wl, pr, ctx = _setup("s150p12")
    lam, w = ctx.get_contour()
    assert np.max(np.abs(lam - pr.lam)) < 1e-13 * np.max(np.abs(pr.lam))
    assert np.max(np.abs(w - pr.w)) < 1e-13 * np.max(np.abs(pr.w))


@pytest.mark.parametrize("name", ["s150p12", "s200p16"])
@pytest.mark.parametrize("prec", [0, 1])
def test_span_matvec(name, prec):
    wl, pr, ctx = _setup(name)
    x = coeff_vector(wl, 8)
    got = ctx.apply(prec, x.astype(np.complex128 if prec == 0 else np.complex64))
    err = rel_err(got, pr.matvec(x))
    assert err < (1e-12 if prec == 0 else 2e-5), err


def test_span_layered_part_is_converged():
    """The library's matvec on the span contour (h = 6/X) against the oracle's
    on a twice finer one: the difference is the quadrature error of the
    layered part alone, below 1e-8 of it; the workload's fixed 256-node
    contour misses the layered part by more than 1 %."""
    wl, pr, ctx = _setup("s150p12")
    X = _extent(wl)
    fine_lam, fine_w = ocontour.contour_span(min(0.2, 2.0 / X), T_MAX, 3.0 / X, [wl.k1, wl.k2, wl.k3])
    fine = osystem.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, prototype_S(wl), wl.xy, wl.rot, fine_lam, fine_w)
    x = coeff_vector(wl, 9)
    _, layered = fine.matvec_parts(x)
    scale = np.linalg.norm(fine.apply_S(layered))
    err = np.linalg.norm(ctx.apply(0, x) - fine.matvec(x)) / scale
    assert err < 1e-8, err
    count = make_workload("s150p12")
    c = mp.Context(0)
    c.set_layers(count.k1, count.k2, count.k3, count.d)
    c.set_scattering_matrix(count.p, count.r_enclose, prototype_S(count))
    c.set_geometry(count.xy, count.rot)
    c.set_contour(count.n_nodes, count.b, count.t_max)
    assert np.linalg.norm(c.apply(0, x) - fine.matvec(x)) / scale > 1e-2


def test_span_solve_matches_lu():
    wl, pr, ctx = _setup("s70p8")
    src = np.array([0.5, 2.0])
    ref = pr.solve_lu(src)
    beta, meta = ctx.solve(src, precision=0, tol=1e-13, maxiter=800)
    assert meta["status"] == 0, meta
    assert rel_err(beta, ref) < 1e-10


TARGETS = [0, 1, 2500, 4999]


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5)])
def test_span_full_size_sampled(prec, tol):
    """5000 stars, p = 16, span contour with h = 12/X (about 27000 nodes):
    sampled rows against the oracle."""
    wl, pr, ctx = _setup("c3", h_factor=12.0)
    x = coeff_vector(wl, 12)
    got = ctx.apply(prec, x.astype(np.complex128 if prec == 0 else np.complex64))
    assert np.all(np.isfinite(got))
    ref = pr.matvec(x, targets=TARGETS)
    err = rel_err(got[TARGETS], ref)
    assert err < tol, err
