"""Pins of the Sommerfeld contour (Section 5.1, eq. (37)) and the multipole
plane-wave form of Theorem 5.1 as read here."""
import numpy as np
import pytest
from scipy.special import hankel1

from oracle import contour
from oracle.contour import gamma


@pytest.fixture(scope="module")
def fine():
    return contour.contour(96 + 32 * 60, 0.2, 60.0, [6.0, 9.0, 12.0])


def test_branch():
    lam = np.array([20.0 - 0.1j, 3.0 - 0.1j, -3.0 + 0.1j, 0.05j, -0.05j, 0.0 + 0.0j])
    g = gamma(lam, 9.0)
    assert np.all(g.real >= 0)
    assert np.all(g[np.abs(g.real) < 1e-12].imag <= 0)      # outgoing on the vertical segment
    assert np.allclose(g ** 2, lam ** 2 - 81.0, rtol=0, atol=1e-12)


def test_sizes_and_mirror():
    lam, w = contour.contour(512, 0.01, 32.0, [6.0, 9.0, 12.0])
    assert lam.size == 512 and w.size == 512
    n1 = (512 - 32) // 2
    assert np.array_equal(lam[:n1], -lam[-n1:][::-1])
    assert np.array_equal(w[:n1], w[-n1:][::-1])
    # the chord of the whole path: from -t_max + ib to t_max - ib
    assert abs(np.sum(w) - (64.0 - 0.02j)) < 1e-12


def test_breakpoints_include_branch_points():
    br = contour.panel_breaks(15, 0.01, 32.0, [6.0, 9.0, 12.0])
    ends = {a for a, _ in br} | {c for _, c in br}
    assert {0.0, 6.0, 9.0, 12.0, 32.0} <= ends
    assert len(br) == 15


@pytest.mark.parametrize("X,Y", [(0.7, 1.3), (-2.0, 0.8), (1.5, -1.1), (0.3, -2.5)])
@pytest.mark.parametrize("n", [0, 1, 3, -2, -5, 8])
def test_multipole_plane_wave_form(fine, X, Y, n):
    # (i/4) H_n(kr) e^{in theta} = (1/4pi) int e^{-g|Y|}/g e^{i lam X} (-i)^n ((lam -+ g)/k)^n dlam
    lam, w = fine
    k = 9.0
    g = gamma(lam, k)
    s = np.sign(Y)
    integ = np.sum(w * np.exp(-g * abs(Y)) / g * np.exp(1j * lam * X)
                   * (-1j) ** n * ((lam - s * g) / k) ** n) / (4 * np.pi)
    r = np.hypot(X, Y)
    ref = 0.25j * hankel1(n, k * r) * np.exp(1j * n * np.arctan2(Y, X))
    assert abs(integ - ref) < 1e-12 * max(1.0, abs(ref))


def test_printed_theorem_factor_fails(fine):
    # the printed Theorem 5.1 factor ((g + k^2)/k^2)^n with (-1)^n/(4 pi) does not
    # represent H_1 e^{i theta}; the corrected form above does
    lam, w = fine
    k, X, Y, n = 9.0, 0.7, 1.3, 1
    g = gamma(lam, k)
    printed = (-1) ** n / (4 * np.pi) * np.sum(w * np.exp(-g * Y) / g * np.exp(1j * lam * X)
                                               * ((g + k ** 2) / k ** 2) ** n)
    ref = hankel1(n, k * np.hypot(X, Y)) * np.exp(1j * n * np.arctan2(Y, X))
    assert abs(printed - ref) > 1e-2 * abs(ref)


def test_span_rule_panels():
    pan = contour.span_breaks(0.01, 32.0, 0.5, [6.0, 9.0, 12.0])
    ends = {a for a, _ in pan} | {c for _, c in pan}
    assert {0.0, 6.0, 9.0, 12.0, 32.0} <= ends
    L = np.array([c - a for a, c in pan])
    assert L.max() <= 0.5 + 1e-15
    assert abs(L.sum() - 32.0) < 1e-12                        # the panels tile [0, t_max]
    # graded towards the branch points: the panels touching 9 are b long
    assert min(c - a for a, c in pan if c == 9.0 or a == 9.0) == pytest.approx(0.01)
    lam, w = contour.contour_span(0.01, 32.0, 0.5, [6.0, 9.0, 12.0])
    assert lam.size == 32 + 32 * len(pan)
    assert abs(np.sum(w) - (64.0 - 0.02j)) < 1e-12


@pytest.mark.parametrize("X,Y", [(60.0, 2.0), (-60.0, 1.5), (400.0, 2.0), (400.0, -3.0)])
@pytest.mark.parametrize("n", [0, 3, -5])
def test_span_rule_converges_at_wide_spans(X, Y, n):
    """The plane-wave form of (i/4) H_n(kr) e^{in theta} at lateral distance
    up to 400 with the span rule (b = 2/X, h_max = 6/X) against scipy."""
    k = 9.0
    Xs = abs(X)
    lam, w = contour.contour_span(2.0 / Xs, 24.0, 6.0 / Xs, [6.0, 9.0, 12.0])
    g = gamma(lam, k)
    s = np.sign(Y)
    integ = np.sum(w * np.exp(-g * abs(Y)) / g * np.exp(1j * lam * X)
                   * (-1j) ** n * ((lam - s * g) / k) ** n) / (4 * np.pi)
    ref = 0.25j * hankel1(n, k * np.hypot(X, Y)) * np.exp(1j * n * np.arctan2(Y, X))
    assert abs(integ - ref) < 1e-10 * abs(ref), abs(integ - ref) / abs(ref)


def test_count_rule_does_not_converge_at_wide_spans():
    # the branch-point rule with as many nodes misses the oscillation at X = 400
    k, X, Y = 9.0, 400.0, 2.0
    lam_s, _ = contour.contour_span(2.0 / X, 24.0, 6.0 / X, [6.0, 9.0, 12.0])
    lam, w = contour.contour(lam_s.size, 2.0 / X, 24.0, [6.0, 9.0, 12.0])
    g = gamma(lam, k)
    integ = np.sum(w * np.exp(-g * Y) / g * np.exp(1j * lam * X)) / (4 * np.pi)
    ref = 0.25j * hankel1(0, k * np.hypot(X, Y))
    assert abs(integ - ref) > 1e-3 * abs(ref)
