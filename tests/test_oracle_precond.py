"""Pins of the cluster-block preconditioner oracle (oracle/precond.py).

- the bisection rule against layouts whose clusters can be written down by hand
  (points on a line, a 4 x 4 grid, coincident points ordered by index);
- one cluster holding every particle of a homogeneous medium (k1 = k2 = k3, no
  reflected field) gives the whole system matrix, so the preconditioned
  operator is the identity and GMRES stops after one step;
- clusters of one particle give M = I (the paper's own preconditioning);
- on a layered 150-star problem, preconditioned GMRES reaches the LU solution
  with fewer iterations than plain GMRES.
"""
import numpy as np
import pytest

from oracle import precond as opc
from oracle import system as osys
from synth import make_workload
from gpu_common import oracle_problem, prototype_S


def test_bisection_on_a_line():
    rng = np.random.default_rng(0)
    x = rng.uniform(-10, 10, 16)
    xy = np.stack([x, np.zeros(16)], axis=1)
    cl = opc.clusters(xy, 4)
    order = np.argsort(x)
    assert [list(c) for c in cl] == [sorted(order[4 * i:4 * i + 4]) for i in range(4)]


def test_bisection_on_a_grid():
    g = np.array([(x, y) for y in range(4) for x in range(4)], dtype=float)   # index = 4 y + x
    cl = opc.clusters(g, 4)
    quad = lambda xs, ys: sorted(4 * y + x for y in ys for x in xs)
    # x-extent equals y-extent at the top, so the first cut is across x; each
    # half is 2 wide and 4 tall, so the next cut is across y
    assert [list(c) for c in cl] == [quad((0, 1), (0, 1)), quad((0, 1), (2, 3)),
                                     quad((2, 3), (0, 1)), quad((2, 3), (2, 3))]
    assert sorted(len(c) for c in opc.clusters(g, 5)) == [4, 4, 4, 4]
    assert sorted(len(c) for c in opc.clusters(g, 3)) == [2] * 8


def test_bisection_ties_by_index():
    xy = np.zeros((5, 2))
    assert [list(c) for c in opc.clusters(xy, 2)] == [[0, 1], [2], [3, 4]]


def test_bisection_partition_and_sizes():
    wl = make_workload("c3", n=700)
    for size in (1, 7, 40, 160, 700, 1000):
        cl = opc.clusters(wl.xy, size)
        allidx = np.sort(np.concatenate(cl))
        assert np.array_equal(allidx, np.arange(700))
        assert max(len(c) for c in cl) <= size
        # halving keeps the sizes within one of each other at equal depth
        if size < 700:
            assert max(len(c) for c in cl) - min(len(c) for c in cl) <= 1
        lab = opc.cluster_of(wl.xy, size)
        for c, idx in enumerate(cl):
            assert np.all(lab[idx] == c)


def _free_problem(name, n=None):
    wl = make_workload(name, n=n)
    return wl, oracle_problem(wl, ks=(wl.k2, wl.k2, wl.k2))


def test_one_cluster_is_the_free_space_system():
    wl, pr = _free_problem("s70p8", n=24)
    K = pr.dense()
    Kc = opc.cluster_matrix(pr, np.arange(wl.n))
    assert np.max(np.abs(Kc - K)) < 1e-12 * np.max(np.abs(K))
    cl, inv = opc.block_inverses(pr, wl.n)
    assert len(cl) == 1
    b = pr.rhs(wl.src[0]).reshape(-1)
    x, hist = opc.gmres_right(lambda v: pr.matvec(v).reshape(-1), b, 1e-12, 5,
                              lambda v: opc.apply(cl, inv, v, wl.P))
    assert len(hist) == 2 and hist[-1] < 1e-12
    assert np.linalg.norm(x - np.linalg.solve(K, b)) < 1e-11 * np.linalg.norm(x)


def test_single_particle_clusters_are_the_identity():
    wl = make_workload("s150p12", n=30)
    pr = oracle_problem(wl)
    cl, inv = opc.block_inverses(pr, 1)
    assert len(cl) == wl.n
    x = np.random.default_rng(1).standard_normal((wl.n, wl.P)) + 0j
    assert np.array_equal(opc.apply(cl, inv, x, wl.P), x)


def test_cluster_matrix_rows_are_the_operator():
    # K_c applied to x (zero outside the cluster) equals the cluster's rows of the
    # free-space operator I - S T applied to the same x
    wl, pr = _free_problem("s150p12", n=60)
    cl = opc.clusters(wl.xy, 16)
    idx = cl[1]
    x = np.zeros((wl.n, wl.P), complex)
    x[idx] = np.random.default_rng(2).standard_normal((len(idx), wl.P))
    y = pr.matvec(x)[idx].reshape(-1)
    assert np.linalg.norm(opc.cluster_matrix(pr, idx) @ x[idx].reshape(-1) - y) < 1e-12 * np.linalg.norm(y)


def test_preconditioned_gmres_reaches_lu_on_stars():
    wl = make_workload("s150p12")
    pr = oracle_problem(wl)
    K = pr.dense()
    b = pr.rhs(wl.src[0]).reshape(-1)
    ref = np.linalg.solve(K, b)
    cl, inv = opc.block_inverses(pr, 40)
    x, hist = opc.gmres_right(lambda v: K @ v, b, 1e-10, 800, lambda v: opc.apply(cl, inv, v, wl.P))
    _, hist0 = osys.gmres(lambda v: K @ v, b, 1e-10, 800)
    assert hist[-1] < 1e-10
    assert np.linalg.norm(x - ref) < 1e-7 * np.linalg.norm(ref)
    assert len(hist) < 0.6 * len(hist0), (len(hist), len(hist0))
