"""Scattering matrix of a smooth star-shaped dielectric inclusion (Section 4).

The inclusion is eq. (50): x(t) = (a1 + a2 cos(a3 t)) (cos t, sin t).  The
exterior field is u^s = S^{k2} sigma + D^{k2} mu and the interior field
u = S^{kp} sigma + D^{kp} mu (eqs. (26)-(27)).  Continuity of u and du/dn
gives Mueller's second-kind system, eqs. (31)-(32):

    mu + (S2 - Sp) sigma + (D2 - Dp) mu    = -u_inc
   -sigma + (N2 - Np) sigma + (T2 - Tp) mu = -d u_inc / dn

Discretisation (the paper uses Alpert's hybrid Gauss-trapezoidal rule; this
oracle uses an independent high-order Nystrom method): Kress's product
quadrature for the logarithmic part of each kernel, the trapezoidal rule for
the smooth remainder, and Maue's identity
T_k mu = d/ds S_k (d mu/ds) + k^2 n_x . S_k (n_y mu) for the hypersingular
operator, with the tangential derivative taken spectrally.

TE polarisation: (1/k^2) du/dn is continuous instead of du/dn.  With
rho = k2^2 / kp^2 the interior field is represented as
S^{kp} sigma + (1/rho) D^{kp} mu, so that the hypersingular operators still
appear as the difference T2 - Tp:

    (1 + 1/rho)/2 mu + (S2 - Sp) sigma + (D2 - Dp / rho) mu   = -u_inc
   -(1 + rho)/2 sigma + (N2 - rho Np) sigma + (T2 - Tp) mu    = -d u_inc / dn

(rho = 1 is eqs. (31)-(32)); the exterior representation, and hence eq. (35),
is unchanged.

Right-hand sides are the regular waves J_n(k2 r) e^{in theta} on the boundary
(Section 4.1, with k = k2 and r = |y|), and the outgoing coefficients follow
eq. (35) with w read as k2 and the factor i/4 of G = (i/4) H_0 restored:
  beta^n_l = (i/4) int [J_l(k2|y|) e^{-il theta} sigma_n
                        + d/dn_y (J_l(k2|y|) e^{-il theta}) mu_n] ds_y.
S[l, n] = beta^n_l maps the incoming coefficient alpha_n to beta_l.

Pins (tests/test_oracle_star.py): a2 = 0 reproduces the Mie diagonal of
``mie.disk_smatrix``; I + 2S is unitary for real wavenumbers; the a3-fold
selection rule S[l, n] = 0 unless a3 | (l - n); mirror symmetry
S[l, n] = S[-l, -n]; reciprocity S[l, n] = (-1)^(l+n) S[-n, -l];
convergence in the number of boundary points.
"""

import numpy as np
from scipy.special import hankel1, jv, jvp

EULER_GAMMA = 0.57721566490153286061


def star_boundary(a1, a2, a3, nb):
    """Equispaced samples of the boundary of eq. (50): points, derivatives."""
    t = 2.0 * np.pi * np.arange(nb) / nb
    r = a1 + a2 * np.cos(a3 * t)
    rp = -a2 * a3 * np.sin(a3 * t)
    rpp = -a2 * a3 * a3 * np.cos(a3 * t)
    c, s = np.cos(t), np.sin(t)
    x = np.stack([r * c, r * s], axis=1)
    xp = np.stack([rp * c - r * s, rp * s + r * c], axis=1)
    xpp = np.stack([rpp * c - 2 * rp * s - r * c, rpp * s + 2 * rp * c - r * s], axis=1)
    return t, r, x, xp, xpp


def _kress_weights(nb):
    """R_j of Kress's quadrature for int ln(4 sin^2((t-tau)/2)) f(tau) dtau."""
    n = nb // 2
    k = np.arange(nb)
    m = np.arange(1, n)
    Rk = -(2.0 * np.pi / n) * np.sum(np.cos(np.outer(k, m) * np.pi / n) / m, axis=1) \
        - (np.pi / n ** 2) * np.cos(k * np.pi)
    i = np.arange(nb)
    return Rk[(i[:, None] - i[None, :]) % nb]


def _fourier_diff(nb):
    """Spectral derivative d/dt on nb equispaced periodic points (nb even)."""
    i = np.arange(nb)
    diff = i[:, None] - i[None, :]
    h = 2.0 * np.pi / nb
    with np.errstate(divide="ignore"):
        F = 0.5 * (-1.0) ** diff / np.tan(diff * h / 2.0)
    F[diff == 0] = 0.0
    return F


def _layer_matrices(k, x, xp, xpp, t, Rw):
    """Nystrom matrices of S_k, D_k, N_k (= K'_k) and S_k without arc length.

    Each kernel K(t, tau) is split as K1 ln(4 sin^2((t - tau)/2)) + K2 with
    K1, K2 smooth; the discrete operator is Rw*K1 + (2 pi / nb) K2.
    """
    nb = x.shape[0]
    speed = np.hypot(xp[:, 0], xp[:, 1])
    nu = np.stack([xp[:, 1], -xp[:, 0]], axis=1)           # outward, |nu| = speed
    nrm = nu / speed[:, None]
    d = x[:, None, :] - x[None, :, :]                       # x(t_i) - x(t_j)
    r = np.hypot(d[..., 0], d[..., 1])
    off = ~np.eye(nb, dtype=bool)
    rr = np.where(off, r, 1.0)
    tt = t[:, None] - t[None, :]
    logt = np.where(off, np.log(np.where(off, 4.0 * np.sin(tt / 2.0) ** 2, 1.0)), 0.0)
    H0 = hankel1(0, k * rr)
    H1 = hankel1(1, k * rr)
    J0 = jv(0, k * rr)
    J1 = jv(1, k * rr)
    h = 2.0 * np.pi / nb
    diag = np.arange(nb)
    kin = np.einsum("ik,i->i", xpp * nu, 1.0 / speed ** 2)  # nu . x'' / |x'|^2

    # single layer, kernel (i/4) H0(k r) |x'(tau)|
    M = 0.25j * H0 * speed[None, :]
    M1 = -(1.0 / (4 * np.pi)) * J0 * speed[None, :]
    M2 = M - M1 * logt
    M1[diag, diag] = -(1.0 / (4 * np.pi)) * speed
    M2[diag, diag] = (0.25j - EULER_GAMMA / (2 * np.pi)
                      - np.log(k * speed / 2.0) / (2 * np.pi)) * speed
    S = Rw * M1 + h * M2

    # double layer, normal at tau: (ik/4) H1(kr) nu(tau).(x(t)-x(tau)) / r
    nd_y = np.einsum("ijk,jk->ij", d, nu)
    L = 0.25j * k * H1 * nd_y / rr
    L1 = -(k / (4 * np.pi)) * J1 * nd_y / rr
    L2 = L - L1 * logt
    L1[diag, diag] = 0.0
    L2[diag, diag] = kin / (4 * np.pi)
    D = Rw * L1 + h * L2

    # normal derivative of the single layer, normal at t
    nd_x = np.einsum("ijk,ik->ij", d, nrm)
    Lp = -0.25j * k * H1 * nd_x / rr * speed[None, :]
    Lp1 = (k / (4 * np.pi)) * J1 * nd_x / rr * speed[None, :]
    Lp2 = Lp - Lp1 * logt
    Lp1[diag, diag] = 0.0
    Lp2[diag, diag] = kin / (4 * np.pi)
    Np = Rw * Lp1 + h * Lp2

    S0 = S / speed[None, :]                                  # kernel without |x'(tau)|
    return S, D, Np, S0, nrm, speed


def star_smatrix(a1, a2, a3, k2, kp, p, nb=256, return_densities=False, pol="TM"):
    """Prototype scattering matrix S (shape (2p+1, 2p+1), S[l+p, n+p]).

    ``nb`` boundary points (even).  Orientation psi = 0 as in eq. (50).
    """
    if nb % 2:
        raise ValueError("nb must be even")
    if pol not in ("TM", "TE"):
        raise ValueError("pol is 'TM' or 'TE'")
    rho = 1.0 if pol == "TM" else (k2 / kp) ** 2
    t, rad, x, xp, xpp = star_boundary(a1, a2, a3, nb)
    Rw = _kress_weights(nb)
    F = _fourier_diff(nb)
    S2, D2, N2, S02, nrm, speed = _layer_matrices(k2, x, xp, xpp, t, Rw)
    Sp, Dp, Npp, S0p, _, _ = _layer_matrices(kp, x, xp, xpp, t, Rw)
    nn = nrm @ nrm.T
    inv_speed = 1.0 / speed
    # Maue: T_k = (1/|x'|) d/dt S0_k d/dt + k^2 (n_x . n_y) S_k
    Tdiff = (inv_speed[:, None] * (F @ (S02 - S0p) @ F)
             + nn * (k2 ** 2 * S2 - kp ** 2 * Sp))
    I = np.eye(nb)
    A = np.block([[S2 - Sp, 0.5 * (1.0 + 1.0 / rho) * I + D2 - Dp / rho],
                  [-0.5 * (1.0 + rho) * I + N2 - rho * Npp, Tdiff]])

    n = np.arange(-p, p + 1)
    theta = t
    rhat = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    that = np.stack([-np.sin(theta), np.cos(theta)], axis=1)
    n_r = np.einsum("ik,ik->i", nrm, rhat)
    n_t = np.einsum("ik,ik->i", nrm, that)
    Jn = jv(n[None, :], k2 * rad[:, None])
    Jnp = jvp(n[None, :], k2 * rad[:, None])
    ph = np.exp(1j * n[None, :] * theta[:, None])
    uinc = Jn * ph
    dudn = ph * (k2 * Jnp * n_r[:, None] + 1j * n[None, :] / rad[:, None] * Jn * n_t[:, None])
    rhs = np.concatenate([-uinc, -dudn], axis=0)
    sol = np.linalg.solve(A, rhs)
    sigma, mu = sol[:nb], sol[nb:]

    # eq. (35): beta^n_l = (i/4) int [J_l e^{-il theta} sigma + d/dn(J_l e^{-il theta}) mu] ds
    l = n
    phm = np.exp(-1j * l[None, :] * theta[:, None])
    Jl = Jn
    Jlp = Jnp
    f_sig = Jl * phm                                                        # (nb, P)
    f_mu = phm * (k2 * Jlp * n_r[:, None] - 1j * l[None, :] / rad[:, None] * Jl * n_t[:, None])
    wq = (2.0 * np.pi / nb) * speed
    S = 0.25j * ((f_sig * wq[:, None]).T @ sigma + (f_mu * wq[:, None]).T @ mu)
    if return_densities:
        return S, sigma, mu
    return S
