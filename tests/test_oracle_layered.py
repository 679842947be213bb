"""Pins of the per-node interface system A_lambda (Section 2, eq. (10))."""
import numpy as np

from oracle import layered
from oracle.contour import gamma

LAM = np.array([0.3 - 0.2j, 5.5 - 0.2j, 8.9 - 0.2j, 15.0 - 0.2j, 25.0 - 0.2j, 0.1j, -0.1j, -7.0 + 0.2j])


def test_free_space_no_reflection(rng):
    k, d = 9.0, 5.0
    A = layered.node_matrix(LAM, k, k, k, d)
    Pp = rng.standard_normal(LAM.size) + 1j * rng.standard_normal(LAM.size)
    Pm = rng.standard_normal(LAM.size) + 1j * rng.standard_normal(LAM.size)
    sig = layered.solve_nodes(A, layered.particle_rhs(LAM, k, Pp, Pm))
    assert np.max(np.abs(sig[:, 1:3])) < 1e-13          # no reflected densities
    assert np.max(np.abs(sig[:, 0] - Pp)) < 1e-12        # transmitted up unchanged
    assert np.max(np.abs(sig[:, 3] - Pm)) < 1e-12        # transmitted down unchanged
    xs, ys = 0.7, 2.0
    s = layered.solve_nodes(A, layered.source_rhs(LAM, k, xs, ys))
    g = gamma(LAM, k)
    # layer-2 field of the source is G itself: sigma_2^+ = e^{-i lam xs - g ys}
    assert np.max(np.abs(s[:, 1] - np.exp(-1j * LAM * xs - g * ys))) < 1e-13
    assert np.max(np.abs(s[:, 2])) < 1e-13
    assert np.max(np.abs(s[:, 0])) < 1e-13


def test_fresnel_limit_thick_layer(rng):
    lam = np.array([15.0 - 0.2j, 20.0 - 0.2j, -18.0 + 0.2j])   # evanescent in layer 2
    k1, k2, k3, d = 6.0, 9.0, 12.0, 60.0
    A = layered.node_matrix(lam, k1, k2, k3, d)
    Pp = rng.standard_normal(3) + 0j
    Pm = rng.standard_normal(3) + 0j
    sig = layered.solve_nodes(A, layered.particle_rhs(lam, k2, Pp, Pm))
    g1, g2, g3 = gamma(lam, k1), gamma(lam, k2), gamma(lam, k3)
    assert np.max(np.abs(sig[:, 1] - (g2 - g1) / (g2 + g1) * Pp)) < 1e-13
    assert np.max(np.abs(sig[:, 2] - (g2 - g3) / (g2 + g3) * Pm)) < 1e-13


def test_rows_are_the_interface_conditions(rng):
    # evaluate the four plane-wave amplitudes directly and check [u] = [du/dy] = 0
    k1, k2, k3, d = 6.0, 9.0, 12.0, 4.0
    A = layered.node_matrix(LAM, k1, k2, k3, d)
    Pp = rng.standard_normal(LAM.size) + 1j * rng.standard_normal(LAM.size)
    Pm = rng.standard_normal(LAM.size) + 1j * rng.standard_normal(LAM.size)
    xs, ys = -0.4, 1.5
    b = layered.particle_rhs(LAM, k2, Pp, Pm) + layered.source_rhs(LAM, k1, xs, ys)
    s1, sp, sm, s3 = layered.solve_nodes(A, b).T
    g1, g2, g3 = gamma(LAM, k1), gamma(LAM, k2), gamma(LAM, k3)
    src = np.exp(-1j * LAM * xs - g1 * ys)

    def u1(y):  # source wave (below it) + sigma_1 wave
        return src * np.exp(g1 * y) / g1 + s1 * np.exp(-g1 * y) / g1

    def du1(y):
        return src * np.exp(g1 * y) - s1 * np.exp(-g1 * y)

    def u2(y, above):  # above: particle spectra seen from above the particles
        part = Pp * np.exp(-g2 * y) / g2 if above else Pm * np.exp(g2 * (y + d)) / g2
        return sp * np.exp(g2 * y) / g2 + sm * np.exp(-g2 * (y + d)) / g2 + part

    def du2(y, above):
        part = -Pp * np.exp(-g2 * y) if above else Pm * np.exp(g2 * (y + d))
        return sp * np.exp(g2 * y) - sm * np.exp(-g2 * (y + d)) + part

    def u3(y):
        return s3 * np.exp(g3 * (y + d)) / g3

    def du3(y):
        return s3 * np.exp(g3 * (y + d))

    tol = 1e-12
    assert np.max(np.abs(u1(0.0) - u2(0.0, True))) < tol
    assert np.max(np.abs(du1(0.0) - du2(0.0, True))) < tol
    assert np.max(np.abs(u2(-d, False) - u3(-d))) < tol
    assert np.max(np.abs(du2(-d, False) - du3(-d))) < tol
