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


# ---- TE polarisation: (1/k^2) du/dn continuous ---------------------------------

@pytest.mark.parametrize("R,k2,kp,p", [(0.25, 9.0, 15.0, 8), (0.3, 3.0, 2.0, 10), (0.5, 6.0, 6.5, 12)])
def test_te_textbook_coefficient(R, k2, kp, p):
    # the H-polarisation cylinder coefficient in relative-index form (m = kp/k2,
    # x = k2 R): a_n = [m J_n(mx) J_n'(x) - J_n'(mx) J_n(x)] / [m J_n(mx) H_n'(x) - J_n'(mx) H_n(x)],
    # scattered field -sum a_n H_n e^{in theta} per unit incoming J_n e^{in theta}
    n = np.arange(-p, p + 1)
    m, x = kp / k2, k2 * R
    a = ((m * jv(n, m * x) * jvp(n, x) - jvp(n, m * x) * jv(n, x))
         / (m * jv(n, m * x) * h1vp(n, x) - jvp(n, m * x) * hankel1(n, x)))
    S = mie.disk_smatrix(R, k2, kp, p, pol="TE")
    assert np.max(np.abs(S + a)) <= 1e-13 * max(1.0, np.max(np.abs(S)))


def test_te_no_contrast_is_transparent():
    assert np.max(np.abs(mie.disk_smatrix(0.3, 7.0, 7.0, 10, pol="TE"))) < 1e-15


@pytest.mark.parametrize("R,k2,kp", [(0.25, 9.0, 15.0), (0.4, 3.0, 11.0), (0.2, 12.0, 1.5)])
def test_te_energy_conservation(R, k2, kp):
    S = mie.disk_smatrix(R, k2, kp, 14, pol="TE")
    assert np.max(np.abs(np.abs(1 + 2 * S) - 1)) < 1e-14


def test_te_differs_from_tm():
    a = mie.disk_smatrix(0.25, 9.0, 15.0, 8, pol="TE")
    b = mie.disk_smatrix(0.25, 9.0, 15.0, 8, pol="TM")
    assert np.max(np.abs(a - b)) > 1e-2
