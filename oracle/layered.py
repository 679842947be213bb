"""Per-node interface system of the three-layer medium (Section 2, eq. (10)).

With the representations (4)-(7) (phase reference x = 0) and the multipoles
of all particles written on the interfaces as in Theorem 5.1, continuity of u
and du/dy at y = 0 and y = -d (eqs. (8)-(9)) gives, for every contour node
lambda, the 4x4 system A_lambda sigma = b_src + b_P of eq. (10):

  rows: u at y = 0, u at y = -d, du/dy at y = 0, du/dy at y = -d
  sigma = (sigma_1, sigma_2^+, sigma_2^-, sigma_3)
  b_src = e^{-i lambda x_s} (-e^{-g1 y_s}/g1, 0, e^{-g1 y_s}, 0)   (point source)
  b_P   = (P+/g2, -P-/g2, P+, -P-)                                 (particles)

where P+ / P- are the plane-wave spectra of all particle multipoles on the
upper / lower interface (``operators.m2s``).  The particle term is not printed
in eq. (10); it is the same continuity conditions with the particle field of
eq. (36) included (stated reading).

Pins (tests/test_oracle_layered.py): k1 = k2 = k3 makes sigma_2^+/- independent
of P+/- and gives sigma_2^+ = e^{-i lambda x_s - g1 y_s}, sigma_2^- = 0 (the
layer-2 field is then exactly G); for d -> infinity the reflection of P+
tends to the Fresnel coefficient (g2 - g1)/(g2 + g1); the assembled field
satisfies both interface conditions pointwise.
"""

import numpy as np

from .contour import gamma


def node_matrix(lam, k1, k2, k3, d):
    """A_lambda of eq. (10) for every node: array (N_S, 4, 4)."""
    lam = np.atleast_1d(np.asarray(lam, dtype=np.complex128))
    g1, g2, g3 = gamma(lam, k1), gamma(lam, k2), gamma(lam, k3)
    E = np.exp(-g2 * d)
    A = np.zeros((lam.size, 4, 4), dtype=np.complex128)
    A[:, 0, 0] = 1 / g1
    A[:, 0, 1] = -1 / g2
    A[:, 0, 2] = -E / g2
    A[:, 1, 1] = E / g2
    A[:, 1, 2] = 1 / g2
    A[:, 1, 3] = -1 / g3
    A[:, 2, 0] = 1
    A[:, 2, 1] = 1
    A[:, 2, 2] = -E
    A[:, 3, 1] = E
    A[:, 3, 2] = -1
    A[:, 3, 3] = -1
    return A


def source_rhs(lam, k1, xs, ys):
    """b_src of eq. (10) for a unit point source at (xs, ys), ys > 0."""
    lam = np.atleast_1d(np.asarray(lam, dtype=np.complex128))
    g1 = gamma(lam, k1)
    e = np.exp(-1j * lam * xs - g1 * ys)
    b = np.zeros((lam.size, 4), dtype=np.complex128)
    b[:, 0] = -e / g1
    b[:, 2] = e
    return b


def particle_rhs(lam, k2, Pp, Pm):
    """b_P: the particle spectra P+ (upper) and P- (lower) moved to the RHS."""
    lam = np.atleast_1d(np.asarray(lam, dtype=np.complex128))
    g2 = gamma(lam, k2)
    b = np.zeros((lam.size, 4), dtype=np.complex128)
    b[:, 0] = Pp / g2
    b[:, 1] = -Pm / g2
    b[:, 2] = Pp
    b[:, 3] = -Pm
    return b


def solve_nodes(A, b):
    """sigma = A^{-1} b per node by Gaussian elimination (LAPACK)."""
    return np.linalg.solve(A, b[..., None])[..., 0]
