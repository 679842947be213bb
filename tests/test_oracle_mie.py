"""Pins of the disk scattering matrix (Section 3.1, eqs. (17)-(18))."""
import numpy as np
import pytest
from scipy.special import hankel1, h1vp, jv, jvp

from oracle import mie


@pytest.mark.parametrize("R,k2,kp,p", [(0.25, 9.0, 15.0, 8), (0.3, 3.0, 2.0, 10), (0.5, 6.0, 6.5, 12)])
def test_closed_form(R, k2, kp, p):
    # eq. (18), denominator read with J_n(kp R)
    n = np.arange(-p, p + 1)
    num = kp * jv(n, k2 * R) * jvp(n, kp * R) - k2 * jvp(n, k2 * R) * jv(n, kp * R)
    den = k2 * h1vp(n, k2 * R) * jv(n, kp * R) - kp * jvp(n, kp * R) * hankel1(n, k2 * R)
    S = mie.disk_smatrix(R, k2, kp, p)
    assert np.max(np.abs(S - num / den)) <= 1e-14 * max(1.0, np.max(np.abs(S)))


def test_no_contrast_is_transparent():
    S = mie.disk_smatrix(0.3, 7.0, 7.0, 10)
    assert np.max(np.abs(S)) < 1e-15


@pytest.mark.parametrize("R,k2,kp", [(0.25, 9.0, 15.0), (0.4, 3.0, 11.0), (0.2, 12.0, 1.5)])
def test_energy_conservation(R, k2, kp):
    # outgoing = (1 + 2 S_n) x incoming for a lossless disk, so |1 + 2 S_n| = 1
    S = mie.disk_smatrix(R, k2, kp, 14)
    assert np.max(np.abs(np.abs(1 + 2 * S) - 1)) < 1e-14


def test_symmetric_orders():
    S = mie.disk_smatrix(0.25, 9.0, 15.0, 8)
    assert np.max(np.abs(S - S[::-1])) < 1e-15


def test_lossy_particle_absorbs():
    S = mie.disk_smatrix(0.3, 6.0, 9.0 + 0.5j, 8)
    assert np.all(np.abs(1 + 2 * S) < 1.0)
