"""Host-side parts of the library (no device needed) against the oracle:
the disk and star scattering matrices and the contour nodes and weights."""
import numpy as np
import pytest

import paper_1407_3868_amd as mp
from oracle import contour as ocontour
from oracle import mie as omie
from oracle import star as ostar


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
