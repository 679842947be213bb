"""Scattering matrix of a single dielectric disk (Section 3.1).

Conventions: outgoing waves use the first-kind Hankel function H_n = H_n^(1);
the exterior total field is sum_n alpha_n J_n(k2 r) e^{in theta} +
beta_n H_n(k2 r) e^{in theta}, the interior field gamma_n J_n(kp r) e^{in theta}.

TE polarisation (Section 1 names it beside TM): with the permeability
constant and the permittivity piecewise constant, the field is continuous and
so is (1/eps) du/dn, i.e. (1/k^2) du/dn; the derivative row of the system is
weighted by 1/k^2 of its side.

Pins (tests/test_oracle_mie.py): the closed form (18) with the denominator
read as J_n(kp R); no contrast (kp = k2) gives S = 0; energy conservation
|1 + 2 S_n| = 1 for real wavenumbers (both polarisations); mirror symmetry
S_n = S_{-n}; TE equals the star integral equation's TE result at a2 = 0.
"""

import numpy as np
from scipy.special import hankel1, h1vp, jv, jvp


def disk_smatrix(R, k2, kp, p, pol="TM"):
    """Diagonal of the disk scattering matrix, orders n = -p..p.

    Follows Section 3.1: for each mode n, continuity of u and du/dr on
    r = R gives the 2x2 system of eq. (17),

        [ -H_n(k2 R)        J_n(kp R)     ] [beta_n ]   [ alpha_n J_n(k2 R)      ]
        [ -k2 H_n'(k2 R)    kp J_n'(kp R) ] [gamma_n] = [ alpha_n k2 J_n'(k2 R)  ]

    solved here with alpha_n = 1, so beta_n is S_n.  The paper's index set
    "n in N" is read as all integers truncated to |n| <= p.
    Returns complex128 array of length 2p+1 (slot n+p).
    """
    if pol not in ("TM", "TE"):
        raise ValueError("pol is 'TM' or 'TE'")
    # weight of the derivative condition on each side: 1 (TM), 1/k^2 (TE)
    c2, cp = (1.0, 1.0) if pol == "TM" else (1.0 / k2 ** 2, 1.0 / kp ** 2)
    n = np.arange(-p, p + 1)
    S = np.empty(2 * p + 1, dtype=np.complex128)
    for i, nn in enumerate(n):
        A = np.array([[-hankel1(nn, k2 * R), jv(nn, kp * R)],
                      [-c2 * k2 * h1vp(nn, k2 * R), cp * kp * jvp(nn, kp * R)]],
                     dtype=np.complex128)
        rhs = np.array([jv(nn, k2 * R), c2 * k2 * jvp(nn, k2 * R)], dtype=np.complex128)
        beta, _gamma = np.linalg.solve(A, rhs)
        S[i] = beta
    return S
