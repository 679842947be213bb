"""Host-side parts of the library (no device needed) against the oracle:
the disk and star scattering matrices and the contour nodes and weights."""
import numpy as np
import pytest

import paper_1407_3868_amd as mp
from oracle import contour as ocontour
from oracle import mie as omie
from oracle import star as ostar
from oracle import stack as ostack


@pytest.mark.parametrize("R,k2,kp,p", [(0.25, 9.0, 15.0, 8), (0.3, 3.0, 2.0, 12), (0.25, 9.0, 15.0, 20)])
def test_disk_matrix(R, k2, kp, p):
    S = mp.compute_disk_smatrix(R, k2, kp, p)
    assert np.max(np.abs(S - np.diag(omie.disk_smatrix(R, k2, kp, p)))) < 1e-13


@pytest.mark.parametrize("a2,p,nb", [(0.05, 8, 128), (0.05, 12, 256), (0.0, 10, 128), (-0.03, 6, 128)])
def test_star_matrix(a2, p, nb):
    S = mp.compute_star_smatrix(0.25, a2, 5, 9.0, 15.0, p, nb)
    ref = ostar.star_smatrix(0.25, a2, 5, 9.0, 15.0, p, nb=nb)
    assert np.max(np.abs(S - ref)) < 1e-12


def test_star_matrix_is_unitary_and_symmetric():
    S = mp.compute_star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 16, 256)
    U = np.eye(33) + 2 * S
    assert np.max(np.abs(U.conj().T @ U - np.eye(33))) < 1e-11
    assert np.max(np.abs(S - S.T)) < 1e-12


@pytest.mark.parametrize("ks,n,b", [((6, 9, 12), 256, 0.2), ((6, 9, 12), 1024, 0.005), ((9, 9, 9), 512, 0.01),
                                    ((1, 3, 2), 512, 0.2)])
def test_contour(ks, n, b):
    lam, w = mp.compute_contour(*ks, n, b, 32.0)
    rl, rw = ocontour.contour(n, b, 32.0, list(ks))
    assert np.max(np.abs(lam - rl)) < 1e-13 * np.max(np.abs(rl))
    assert np.max(np.abs(w - rw)) < 1e-13 * np.max(np.abs(rw))


def test_bad_host_arguments():
    with pytest.raises(mp.MpslError):
        mp.compute_contour(6, 9, 12, 100, 0.2, 32.0)
    with pytest.raises(mp.MpslError):
        mp.compute_star_smatrix(0.25, 0.3, 5, 9.0, 15.0, 8, 128)   # |a2| >= a1
    with pytest.raises(mp.MpslError):
        mp.compute_disk_smatrix(0.25, 9.0, 15.0, 40)               # order too high


STACKS = [([6.0, 9.0, 12.0], [0, 1.0, 0], 1),
          ([6.0, 7.5, 9.0, 11.0, 12.0], [0, 1.0, 8.0, 1.5, 0], 2),
          ([4.0, 9.0, 5.0, 12.0], [0, 2.0, 0.7, 0], 1),
          ([4.0, 9.0, 5.0, 12.0], [0, 0.3, 3.0, 0], 2),
          ([3.0, 8.0, 5.0, 9.0, 6.0, 10.0, 2.0], [0, 0.4, 1.3, 5.0, 0.2, 2.5, 0], 3),
          ([9.0, 9.0, 9.0, 9.0, 9.0], [0, 1.0, 2.0, 3.0, 0], 2)]


@pytest.mark.parametrize("ks,th,c", STACKS)
def test_layer_map_matches_oracle_node_solve(ks, th, c):
    """The library's generalized reflection / transmission recursion against
    the oracle's dense solve of every interface condition per node, for unit
    particle spectra P+, P- and a unit source wave at the top interface."""
    lam, _ = ocontour.contour(512, 0.05, 40.0, ks)
    got = mp.compute_layer_map(ks, th, c, lam)
    M = ostack.node_system(lam, ks, th, c)
    one = np.ones(lam.size, complex)
    A, B = ostack._col_A(c), ostack._col_B(c)
    ref = np.zeros((lam.size, 6), complex)
    for col, kw in ((0, dict(Pp=one)), (1, dict(Pm=one)), (2, dict(src=(0.0, ostack.interfaces(th, c)[0])))):
        X = np.linalg.solve(M, ostack.rhs(lam, ks, th, c, **kw)[..., None])[..., 0]
        if col < 2:
            ref[:, col], ref[:, 2 + col] = X[:, A], X[:, B]
        else:
            ref[:, 4], ref[:, 5] = X[:, A], X[:, B]
    assert np.max(np.abs(got - ref) / (1 + np.abs(ref))) < 1e-12


def test_layer_map_without_contrast_is_free_space():
    # every layer the same medium: nothing is reflected, the source passes unchanged
    lam, _ = ocontour.contour(256, 0.2, 32.0, [9.0])
    m = mp.compute_layer_map([9.0] * 5, [0, 1.0, 2.0, 3.0, 0], 2, lam)
    g = ocontour.gamma(lam, 9.0)
    assert np.max(np.abs(m[:, :4])) == 0.0 and np.max(np.abs(m[:, 5])) == 0.0
    # the source wave arrives at y = 0 after the 1.0 thick layer above
    assert np.max(np.abs(m[:, 4] - np.exp(-g * 1.0))) < 1e-14


@pytest.mark.parametrize("ks,th,c", [([6.0, 9.0], [0, 0], 1), ([6.0, 9.0, 12.0], [0, 1.0, 0], 0),
                                     ([6.0, 9.0, 12.0], [0, 1.0, 0], 2), ([6.0, 9.0, 12.0], [0, 0.0, 0], 1),
                                     ([6.0, -9.0, 12.0], [0, 1.0, 0], 1), ([6.0, 9.0 + 1j, 12.0], [0, 1.0, 0], 1)])
def test_layer_map_bad_arguments(ks, th, c):
    with pytest.raises(mp.MpslError):
        mp.compute_layer_map(ks, th, c, np.array([1.0 - 0.1j]))


@pytest.mark.parametrize("ks,b,t_max,h_max", [([6, 9, 12], 0.01, 32.0, 0.5), ([6, 9, 12], 2 / 400, 24.0, 6 / 400),
                                              ([3, 8, 5, 9, 6, 10, 2], 0.03, 32.0, 0.2), ([9, 9, 9], 0.2, 32.0, 3.0),
                                              ([1, 3, 1], 0.05, 21.0, 40.0)])
def test_contour_span(ks, b, t_max, h_max):
    lam, w = mp.compute_contour_span(ks, b, t_max, h_max)
    rl, rw = ocontour.contour_span(b, t_max, h_max, ks)
    assert lam.size == rl.size
    assert np.max(np.abs(lam - rl)) < 1e-13 * np.max(np.abs(rl))
    assert np.max(np.abs(w - rw)) < 1e-13 * np.max(np.abs(rw))


@pytest.mark.parametrize("b,t_max,h_max", [(0.0, 32.0, 0.1), (0.1, -1.0, 0.1), (0.1, 32.0, 0.0),
                                           (0.1, 32.0, 1e-5)])          # the last needs > 2^20 nodes
def test_contour_span_bad_arguments(b, t_max, h_max):
    with pytest.raises(mp.MpslError):
        mp.compute_contour_span([6, 9, 12], b, t_max, h_max)


# ---- TE polarisation ------------------------------------------------------------

@pytest.mark.parametrize("R,k2,kp,p", [(0.25, 9.0, 15.0, 8), (0.3, 3.0, 2.0, 12)])
def test_disk_matrix_te(R, k2, kp, p):
    S = mp.compute_disk_smatrix(R, k2, kp, p, polarization=mp.TE)
    assert np.max(np.abs(S - np.diag(omie.disk_smatrix(R, k2, kp, p, pol="TE")))) < 1e-13


@pytest.mark.parametrize("a2,p,nb", [(0.05, 8, 128), (0.05, 12, 256), (0.0, 10, 128)])
def test_star_matrix_te(a2, p, nb):
    S = mp.compute_star_smatrix(0.25, a2, 5, 9.0, 15.0, p, nb, polarization=mp.TE)
    ref = ostar.star_smatrix(0.25, a2, 5, 9.0, 15.0, p, nb=nb, pol="TE")
    assert np.max(np.abs(S - ref)) < 1e-12


@pytest.mark.parametrize("ks,th,c", STACKS)
def test_layer_map_te_matches_oracle_node_solve(ks, th, c):
    lam, _ = ocontour.contour(512, 0.05, 40.0, ks)
    got = mp.compute_layer_map(ks, th, c, lam, polarization=mp.TE)
    M = ostack.node_system(lam, ks, th, c, pol="TE")
    one = np.ones(lam.size, complex)
    A, B = ostack._col_A(c), ostack._col_B(c)
    ref = np.zeros((lam.size, 6), complex)
    for col, kw in ((0, dict(Pp=one)), (1, dict(Pm=one)), (2, dict(src=(0.0, ostack.interfaces(th, c)[0])))):
        X = np.linalg.solve(M, ostack.rhs(lam, ks, th, c, pol="TE", **kw)[..., None])[..., 0]
        if col < 2:
            ref[:, col], ref[:, 2 + col] = X[:, A], X[:, B]
        else:
            ref[:, 4], ref[:, 5] = X[:, A], X[:, B]
    assert np.max(np.abs(got - ref) / (1 + np.abs(ref))) < 1e-12


def test_bad_polarization():
    with pytest.raises(mp.MpslError):
        mp.compute_disk_smatrix(0.25, 9.0, 15.0, 8, polarization=2)


@pytest.mark.parametrize("name,n,size", [("c3", None, 160), ("c3", None, 40), ("c3", 777, 1), ("c5max", 3000, 97),
                                         ("s150p12", None, 150), ("s150p12", None, 1000)])
def test_clusters(name, n, size):
    # recursive coordinate bisection: integer output, bit-exact
    from oracle import precond as opc
    from synth import make_workload
    wl = make_workload(name, n=n)
    lab, nc = mp.compute_clusters(wl.xy, size)
    ref = opc.cluster_of(wl.xy, size)
    assert nc == len(opc.clusters(wl.xy, size))
    assert np.array_equal(lab, ref)


def test_clusters_ties_and_grid():
    from oracle import precond as opc
    g = np.array([(x, y) for y in range(6) for x in range(6)], dtype=float)
    for xy in (np.zeros((9, 2)), g, g[::-1].copy(), np.stack([np.arange(10.0), np.zeros(10)], 1)):
        for size in (1, 2, 3, 4, 5, 100):
            lab, nc = mp.compute_clusters(xy, size)
            assert np.array_equal(lab, opc.cluster_of(xy, size))


def test_clusters_reject_bad_input():
    with pytest.raises(mp.MpslError):
        mp.compute_clusters(np.zeros((3, 2)), 0)
    with pytest.raises(mp.MpslError):
        mp.compute_clusters(np.array([[0.0, np.nan]]), 2)
