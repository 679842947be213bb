"""Pins of the star scattering matrix from Mueller's integral equations (Section 4)."""
import numpy as np
import pytest

from oracle import mie, star


@pytest.fixture(scope="module")
def S_star():
    return star.star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 20, nb=256)


def test_disk_limit_matches_mie():
    S = star.star_smatrix(0.25, 0.0, 5, 9.0, 15.0, 10, nb=128)
    assert np.max(np.abs(S - np.diag(mie.disk_smatrix(0.25, 9.0, 15.0, 10)))) < 1e-13


def test_unitary(S_star):
    U = np.eye(S_star.shape[0]) + 2 * S_star
    assert np.max(np.abs(U.conj().T @ U - np.eye(U.shape[0]))) < 1e-12


def test_fivefold_selection_rule(S_star):
    p = (S_star.shape[0] - 1) // 2
    n = np.arange(-p, p + 1)
    mask = ((n[:, None] - n[None, :]) % 5) != 0
    assert np.max(np.abs(S_star[mask])) < 1e-13
    assert np.abs(S_star[p + 5, p]) > 1e-3      # the allowed coupling is present


def test_mirror_and_reciprocity(S_star):
    p = (S_star.shape[0] - 1) // 2
    n = np.arange(-p, p + 1)
    sgn = (-1.0) ** (n[:, None] + n[None, :])
    # mirror y -> -y: S[l, n] = (-1)^(l+n) S[-l, -n]
    assert np.max(np.abs(S_star - sgn * S_star[::-1, ::-1])) < 1e-13
    # reciprocity: S[l, n] = (-1)^(l+n) S[-n, -l]
    assert np.max(np.abs(S_star - sgn * S_star[::-1, ::-1].T)) < 1e-13


def test_converged_in_boundary_points(S_star):
    S2 = star.star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 20, nb=384)
    assert np.max(np.abs(S_star - S2)) < 1e-13


def test_rotation_by_symmetry_angle_is_identity():
    from oracle.operators import rotated_smatrix
    S = star.star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 8, nb=128)
    assert np.max(np.abs(rotated_smatrix(S, 2 * np.pi / 5) - S)) < 1e-13


def test_rotation_formula_matches_rotated_boundary():
    # a star rotated by psi has r(t) = a1 + a2 cos(a3 (t - psi)); for psi = pi/a3 this
    # is a1 - a2 cos(a3 t), i.e. the star with a2 -> -a2
    from oracle.operators import rotated_smatrix
    S = star.star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 8, nb=128)
    Sm = star.star_smatrix(0.25, -0.05, 5, 9.0, 15.0, 8, nb=128)
    assert np.max(np.abs(rotated_smatrix(S, np.pi / 5) - Sm)) < 1e-13


# ---- TE polarisation -----------------------------------------------------------

@pytest.fixture(scope="module")
def S_star_te():
    return star.star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 16, nb=256, pol="TE")


def test_te_disk_limit_matches_te_mie():
    S = star.star_smatrix(0.25, 0.0, 5, 9.0, 15.0, 10, nb=128, pol="TE")
    assert np.max(np.abs(S - np.diag(mie.disk_smatrix(0.25, 9.0, 15.0, 10, pol="TE")))) < 1e-13


def test_te_unitary_selection_and_reciprocity(S_star_te):
    S = S_star_te
    U = np.eye(S.shape[0]) + 2 * S
    assert np.max(np.abs(U.conj().T @ U - np.eye(U.shape[0]))) < 1e-12
    p = (S.shape[0] - 1) // 2
    n = np.arange(-p, p + 1)
    assert np.max(np.abs(S[((n[:, None] - n[None, :]) % 5) != 0])) < 1e-13
    sgn = (-1.0) ** (n[:, None] + n[None, :])
    assert np.max(np.abs(S - sgn * S[::-1, ::-1].T)) < 1e-13


def test_te_converged_and_distinct_from_tm(S_star_te):
    S2 = star.star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 16, nb=384, pol="TE")
    assert np.max(np.abs(S_star_te - S2)) < 1e-13
    tm = star.star_smatrix(0.25, 0.05, 5, 9.0, 15.0, 16, nb=256)
    assert np.max(np.abs(S_star_te - tm)) > 1e-2
