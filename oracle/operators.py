"""Translation operators of the multiple-scattering system, written out plainly.

Expansions about a particle centre (Section 3):
  multipole (H-) expansion  sum_n beta_n  H_n(k2 r) e^{in theta}   (eq. (14))
  local (J-) expansion      sum_n alpha_n J_n(k2 r) e^{in theta}   (eq. (16))
orders n = -p..p, stored at slot n + p.

Pins: tests/test_oracle_operators.py (Graf's theorem by direct evaluation
of the multipole near the target; Jacobi-Anger against the plane wave; the
Sommerfeld form of the multipoles against direct Hankel values).
"""

import numpy as np
from scipy.special import hankel1

from .contour import gamma


def orders(p):
    return np.arange(-p, p + 1)


def m2l_block(x_l, x_m, k2, p):
    """T^{ml}: multipole coefficients at x_m -> local coefficients at x_l.

    Section 3.2, Lemma 3.1, with the sign of the printed formula corrected:
      alpha^l_{n'} = sum_n e^{-i n theta_lm} beta^m_{n'-n} H_n(k2 |x_m - x_l|),
    theta_lm = angle of (x_m - x_l) with the x-axis.  (The printed factor
    e^{-i n (theta_lm - pi)} differs by (-1)^n and fails Graf's theorem.)
    Returns T with alpha = T @ beta, shape (2p+1, 2p+1).
    """
    dx = x_m[0] - x_l[0]
    dy = x_m[1] - x_l[1]
    dist = np.hypot(dx, dy)
    theta = np.arctan2(dy, dx)
    P = 2 * p + 1
    T = np.zeros((P, P), dtype=np.complex128)
    for i, n1 in enumerate(orders(p)):          # n'
        for j, nu in enumerate(orders(p)):      # index n' - n of beta
            n = n1 - nu
            T[i, j] = np.exp(-1j * n * theta) * hankel1(n, k2 * dist)
    return T


def m2l_apply(xy, k2, p, beta, targets=None):
    """alpha^l = sum_{m != l} T^{ml} beta^m (eq. (24)), vectorised over sources.

    beta: (N, 2p+1).  targets: iterable of target indices (default all).
    Returns (len(targets), 2p+1).
    """
    xy = np.asarray(xy, dtype=np.float64)
    N = xy.shape[0]
    P = 2 * p + 1
    idx = np.arange(N) if targets is None else np.asarray(list(targets))
    nn = np.arange(-2 * p, 2 * p + 1)
    n1 = orders(p)[:, None]
    nu = orders(p)[None, :]
    sel = (n1 - nu) + 2 * p                      # column of H_n with n = n' - nu
    out = np.zeros((idx.size, P), dtype=np.complex128)
    for a, l in enumerate(idx):
        m = np.r_[0:l, l + 1:N]
        dx = xy[m, 0] - xy[l, 0]
        dy = xy[m, 1] - xy[l, 1]
        dist = np.hypot(dx, dy)
        theta = np.arctan2(dy, dx)
        Hn = hankel1(nn[None, :], k2 * dist[:, None]) * np.exp(-1j * nn[None, :] * theta[:, None])
        T = Hn[:, sel]                            # (M, P, P)
        out[a] = np.einsum("mij,mj->i", T, beta[m])
    return out


def m2s(beta, xy, lam, k2, d):
    """Plane-wave spectra (P+, P-) of all particle multipoles on the interfaces.

    Section 5.3, Theorem 5.1, with the printed factor corrected (derived by
    applying the raising operator d/dx + i d/dy to the Sommerfeld form (3) of
    (i/4) H_0):
      (i/4) H_n(k r) e^{in theta}
          = (1/4pi) int e^{-g |y-y_j|}/g e^{i lambda (x-x_j)} (-i)^n ((lambda -+ g)/k)^n dlambda,
    upper sign for targets above the centre.  Writing the sum of all
    multipoles at y > y_m as (1/4pi) int e^{-g2 y}/g2 e^{i lambda x} P+ dlambda
    and at y < y_m as (1/4pi) int e^{g2 (y+d)}/g2 e^{i lambda x} P- dlambda:
      P+(lambda) = -4i sum_m e^{-i lambda x_m} e^{g2 y_m}        sum_nu beta^m_nu (-i)^nu ((lambda - g2)/k2)^nu
      P-(lambda) = -4i sum_m e^{-i lambda x_m} e^{-g2 (d + y_m)} sum_nu beta^m_nu (-i)^nu ((lambda + g2)/k2)^nu
    """
    beta = np.asarray(beta, dtype=np.complex128)
    P = beta.shape[1]
    p = (P - 1) // 2
    lam = np.asarray(lam, dtype=np.complex128)
    g2 = gamma(lam, k2)
    nu = orders(p)[:, None]
    Wp = (-1j) ** nu * ((lam[None, :] - g2[None, :]) / k2) ** nu   # (P, N_S)
    Wm = (-1j) ** nu * ((lam[None, :] + g2[None, :]) / k2) ** nu
    x = xy[:, 0][:, None]
    y = xy[:, 1][:, None]
    Ep = np.exp(-1j * lam[None, :] * x + g2[None, :] * y)
    Em = np.exp(-1j * lam[None, :] * x - g2[None, :] * (d + y))
    Pp = -4j * np.sum(Ep * (beta @ Wp), axis=0)
    Pm = -4j * np.sum(Em * (beta @ Wm), axis=0)
    return Pp, Pm


def s2l(sig_p, sig_m, xy, lam, w, k2, d, p, targets=None):
    """Local expansions at the particles of the layer-2 Sommerfeld fields.

    Section 5.2.1, Lemma 5.1 / eq. (40), in the exact form of the Jacobi-Anger
    expansion with a complex angle:
      e^{i lambda X + s g Y} = sum_n i^n ((lambda - s g)/k)^n J_n(k r) e^{in theta},
    s = +1 for u_2^t (eq. (5)) and s = -1 for u_2^b (eq. (6)).  Hence
      alpha^l_n = (1/4pi) sum_q (w_q / g2) e^{i lambda_q x_l} i^n
                  [ sigma+_q e^{g2 y_l} ((lambda_q - g2)/k2)^n
                  + sigma-_q e^{-g2 (y_l + d)} ((lambda_q + g2)/k2)^n ].
    """
    lam = np.asarray(lam, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    g2 = gamma(lam, k2)
    xy = np.asarray(xy, dtype=np.float64)
    if targets is not None:
        xy = xy[np.asarray(list(targets))]
    n = orders(p)[None, :]
    Zp = (1j) ** n * ((lam[:, None] - g2[:, None]) / k2) ** n      # (N_S, P)
    Zm = (1j) ** n * ((lam[:, None] + g2[:, None]) / k2) ** n
    c = w / (4 * np.pi * g2)
    x = xy[:, 0][:, None]
    y = xy[:, 1][:, None]
    Fp = np.exp(1j * lam[None, :] * x + g2[None, :] * y)            # (N, N_S)
    Fm = np.exp(1j * lam[None, :] * x - g2[None, :] * (y + d))
    return Fp @ ((c * sig_p)[:, None] * Zp) + Fm @ ((c * sig_m)[:, None] * Zm)


def rotated_smatrix(S, psi):
    """S_psi[l, n] = e^{i (n - l) psi} S[l, n] for a copy rotated CCW by psi (Section 4.1)."""
    P = S.shape[0]
    p = (P - 1) // 2
    n = orders(p)
    return np.exp(1j * (n[None, :] - n[:, None]) * psi) * S


def incident_local_free(xy, src, k, p):
    """Exact local expansion of G_k(x, x_s) = (i/4) H_0(k|x - x_s|) at each centre.

    From Graf's theorem with a single monopole: alpha_n = (i/4) H_{-n}(k rho) e^{-in phi},
    rho, phi = polar form of x_l - x_s.  Used only for free-space checks.
    """
    d = np.asarray(xy) - np.asarray(src)[None, :]
    rho = np.hypot(d[:, 0], d[:, 1])
    phi = np.arctan2(d[:, 1], d[:, 0])
    n = orders(p)[None, :]
    return 0.25j * hankel1(-n, k * rho[:, None]) * np.exp(-1j * n * phi[:, None])
