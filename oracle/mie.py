"""Scattering matrix of a single dielectric disk (Section 3.1).

Conventions: outgoing waves use the first-kind Hankel function H_n = H_n^(1);
the exterior total field is sum_n alpha_n J_n(k2 r) e^{in theta} +
beta_n H_n(k2 r) e^{in theta}, the interior field gamma_n J_n(kp r) e^{in theta}.

Pins (tests/test_oracle_mie.py): the closed form (18) with the denominator
read as J_n(kp R); no contrast (kp = k2) gives S = 0; energy conservation
|1 + 2 S_n| = 1 for real wavenumbers; mirror symmetry S_n = S_{-n}.
"""

import numpy as np
from scipy.special import hankel1, h1vp, jv, jvp


def disk_smatrix(R, k2, kp, p):
    """Diagonal of the disk scattering matrix, orders n = -p..p.

    Follows Section 3.1: for each mode n, continuity of u and du/dr on
    r = R gives the 2x2 system of eq. (17),

        [ -H_n(k2 R)        J_n(kp R)     ] [beta_n ]   [ alpha_n J_n(k2 R)      ]
        [ -k2 H_n'(k2 R)    kp J_n'(kp R) ] [gamma_n] = [ alpha_n k2 J_n'(k2 R)  ]

    solved here with alpha_n = 1, so beta_n is S_n.  The paper's index set
    "n in N" is read as all integers truncated to |n| <= p.
    Returns complex128 array of length 2p+1 (slot n+p).
    """
    n = np.arange(-p, p + 1)
    S = np.empty(2 * p + 1, dtype=np.complex128)
    for i, nn in enumerate(n):
        A = np.array([[-hankel1(nn, k2 * R), jv(nn, kp * R)],
                      [-k2 * h1vp(nn, k2 * R), kp * jvp(nn, kp * R)]],
                     dtype=np.complex128)
        rhs = np.array([jv(nn, k2 * R), k2 * jvp(nn, k2 * R)], dtype=np.complex128)
        beta, _gamma = np.linalg.solve(A, rhs)
        S[i] = beta
    return S
