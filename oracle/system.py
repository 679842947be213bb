"""The Schur-complement multiple-scattering system and the field it defines.

Section 5.2 (eq. (38)) couples the interface densities sigma (4 per contour
node) with the particle coefficients beta.  Section 5.4 (eq. (49)) eliminates
sigma node by node and solves for beta alone.  Written in this package's
conventions (see DESIGN notes of the operators):

    beta^l = S_l ( a^l + sum_{m != l} T^{ml} beta^m + C A^{-1} B beta )

so (I - S (T + T_R)) beta = S a with T_R = C A^{-1} B:
  B   : beta -> particle right-hand side b_P of the 4x4 node systems (M2S),
  A   : the block-diagonal 4x4 matrices A_lambda of eq. (10),
  C   : sigma_2^+/- -> local expansions at the particles (S2L),
  a   : C A^{-1} b_src, the local expansion of the source's layer-2 field,
  S_l : the prototype scattering matrix rotated to particle l (Section 4.1).
The paper multiplies by the block-diagonal S as its preconditioner
(Section 3.2); the unknown here is beta, as in eq. (49).

Pins: tests/test_oracle_system.py (free-space limit against the homogeneous
solver, single disk against the Mie series, reciprocity, interface
continuity of the assembled field, dense LU against matrix-free GMRES).
"""

import dataclasses

import numpy as np
from scipy.special import hankel1

from . import layered, operators
from .contour import gamma


@dataclasses.dataclass
class Problem:
    k1: complex
    k2: complex
    k3: complex
    d: float
    p: int
    S: np.ndarray          # prototype scattering matrix, (P, P)
    xy: np.ndarray         # (N, 2)
    rot: np.ndarray        # (N,)
    lam: np.ndarray        # contour nodes (N_S,)
    w: np.ndarray          # contour weights (N_S,)
    types: np.ndarray = None   # several particle types: S is (T, P, P), types[l] in 0..T-1

    def __post_init__(self):
        self.xy = np.asarray(self.xy, dtype=np.float64)
        self.rot = np.asarray(self.rot, dtype=np.float64)
        self.S = np.asarray(self.S, dtype=np.complex128)
        if self.types is not None:
            self.types = np.asarray(self.types, dtype=np.int64)
            if self.S.ndim != 3 or self.types.shape != (self.xy.shape[0],):
                raise ValueError("with types, S is (T, P, P) and types has one entry per particle")
        self.lam = np.asarray(self.lam, dtype=np.complex128)
        self.w = np.asarray(self.w, dtype=np.complex128)
        self.A = layered.node_matrix(self.lam, self.k1, self.k2, self.k3, self.d)

    @property
    def N(self):
        return self.xy.shape[0]

    @property
    def P(self):
        return 2 * self.p + 1

    # -- building blocks -------------------------------------------------
    def S_of(self, l):
        """Prototype matrix of particle l (its type's, Section 4.2 Remark)."""
        return self.S if self.types is None else self.S[self.types[l]]

    def apply_S(self, alpha, targets=None):
        """beta_l = S_{psi_l} alpha_l for each particle (eq. (21), Section 4.1)."""
        idx = np.arange(self.N) if targets is None else np.asarray(list(targets))
        out = np.empty((idx.size, self.P), dtype=np.complex128)
        for a, l in enumerate(idx):
            out[a] = operators.rotated_smatrix(self.S_of(l), self.rot[l]) @ alpha[a]
        return out

    def sigma(self, beta=None, src=None):
        """All four interface densities per node: A^{-1}(b_src + b_P(beta))."""
        b = np.zeros((self.lam.size, 4), dtype=np.complex128)
        if beta is not None:
            Pp, Pm = operators.m2s(beta, self.xy, self.lam, self.k2, self.d)
            b += layered.particle_rhs(self.lam, self.k2, Pp, Pm)
        if src is not None:
            b += layered.source_rhs(self.lam, self.k1, src[0], src[1])
        return layered.solve_nodes(self.A, b)

    def layer_local(self, beta=None, src=None, targets=None):
        """Local expansions at the particles of u_2^t + u_2^b (eqs. (5), (6), (40))."""
        sig = self.sigma(beta, src)
        return operators.s2l(sig[:, 1], sig[:, 2], self.xy, self.lam, self.w,
                             self.k2, self.d, self.p, targets)

    # -- the operator of eq. (49) ------------------------------------------
    def matvec(self, x, targets=None):
        """y = x - S (T + T_R) x, optionally only at some target particles."""
        x = np.asarray(x, dtype=np.complex128).reshape(self.N, self.P)
        alpha = operators.m2l_apply(self.xy, self.k2, self.p, x, targets)
        alpha = alpha + self.layer_local(beta=x, targets=targets)
        xs = x if targets is None else x[np.asarray(list(targets))]
        return xs - self.apply_S(alpha, targets)

    def matvec_parts(self, x, targets=None):
        """(free-space M2L alpha, layered alpha) of x, before S is applied."""
        x = np.asarray(x, dtype=np.complex128).reshape(self.N, self.P)
        return (operators.m2l_apply(self.xy, self.k2, self.p, x, targets),
                self.layer_local(beta=x, targets=targets))

    def rhs(self, src):
        """S a: the scattering matrices applied to the source's local expansions."""
        return self.apply_S(self.layer_local(src=src))

    def dense(self):
        """K = I - S_blk (T + C A^{-1} B) as an (N P) x (N P) matrix."""
        N, P, p = self.N, self.P, self.p
        n = operators.orders(p)
        lam, k2, d = self.lam, self.k2, self.d
        g2 = gamma(lam, k2)
        # T: free-space translations (eq. (25)), block row l
        T = np.zeros((N * P, N * P), dtype=np.complex128)
        nn = np.arange(-2 * p, 2 * p + 1)
        sel = (n[:, None] - n[None, :]) + 2 * p
        for l in range(N):
            m = np.r_[0:l, l + 1:N]
            dx = self.xy[m, 0] - self.xy[l, 0]
            dy = self.xy[m, 1] - self.xy[l, 1]
            dist = np.hypot(dx, dy)
            th = np.arctan2(dy, dx)
            Hn = hankel1(nn[None, :], k2 * dist[:, None]) * np.exp(-1j * nn[None, :] * th[:, None])
            blk = Hn[:, sel]                                   # (N-1, P, P)
            for a, mm in enumerate(m):
                T[l * P:(l + 1) * P, mm * P:(mm + 1) * P] = blk[a]
        # B: unit beta^m_nu -> (P+, P-) -> b_P per node
        Wp = (-1j) ** n[:, None] * ((lam[None, :] - g2[None, :]) / k2) ** n[:, None]
        Wm = (-1j) ** n[:, None] * ((lam[None, :] + g2[None, :]) / k2) ** n[:, None]
        x = self.xy[:, 0][:, None]
        y = self.xy[:, 1][:, None]
        Ep = np.exp(-1j * lam[None, :] * x + g2[None, :] * y)   # (N, N_S)
        Em = np.exp(-1j * lam[None, :] * x - g2[None, :] * (d + y))
        Pp = -4j * (Ep[:, None, :] * Wp[None, :, :]).reshape(N * P, -1).T   # (N_S, NP)
        Pm = -4j * (Em[:, None, :] * Wm[None, :, :]).reshape(N * P, -1).T
        Bm = np.stack([Pp / g2[:, None], -Pm / g2[:, None], Pp, -Pm], axis=1)  # (N_S, 4, NP)
        sig = np.linalg.solve(self.A, Bm)                      # A^{-1} B per node
        # C: sigma_2^+/- -> alpha (eq. (40))
        c = self.w / (4 * np.pi * g2)
        Zp = (1j) ** n[None, :] * ((lam[:, None] - g2[:, None]) / k2) ** n[None, :]
        Zm = (1j) ** n[None, :] * ((lam[:, None] + g2[:, None]) / k2) ** n[None, :]
        Fp = np.exp(1j * lam[None, :] * x + g2[None, :] * y)
        Fm = np.exp(1j * lam[None, :] * x - g2[None, :] * (y + d))
        Cp = (Fp[:, None, :] * (c[:, None] * Zp).T[None, :, :]).reshape(N * P, -1)  # (NP, N_S)
        Cm = (Fm[:, None, :] * (c[:, None] * Zm).T[None, :, :]).reshape(N * P, -1)
        # T + T_R, then the block-diagonal S one block row at a time (the same
        # products as S_blk @ (T + T_R) without forming S_blk)
        K = T
        K += Cp @ sig[:, 1, :]
        K += Cm @ sig[:, 2, :]
        for l in range(N):
            rows = slice(l * P, (l + 1) * P)
            K[rows] = -(operators.rotated_smatrix(self.S_of(l), self.rot[l]) @ K[rows])
        K[np.diag_indices(N * P)] += 1.0
        return K

    def solve_lu(self, src):
        K = self.dense()
        b = self.rhs(src).reshape(-1)
        return np.linalg.solve(K, b).reshape(self.N, self.P)

    def gmres(self, src, tol=1e-12, maxiter=500):
        """Unrestarted GMRES (modified Gram-Schmidt Arnoldi) on eq. (49)."""
        b = self.rhs(src).reshape(-1)
        return gmres(lambda v: self.matvec(v).reshape(-1), b, tol, maxiter)

    # -- field evaluation (eq. (36)) -------------------------------------
    def field(self, src, beta, rcv):
        """Total field at receivers (R, 2); NaN inside no region (caller checks)."""
        rcv = np.asarray(rcv, dtype=np.float64)
        sig = self.sigma(beta, src)
        lam, w = self.lam, self.w
        g1, g2, g3 = gamma(lam, self.k1), gamma(lam, self.k2), gamma(lam, self.k3)
        out = np.zeros(rcv.shape[0], dtype=np.complex128)
        X = rcv[:, 0][:, None]
        Y = rcv[:, 1][:, None]
        ph = np.exp(1j * lam[None, :] * X)
        up = rcv[:, 1] > 0
        lo = rcv[:, 1] < -self.d
        mid = ~(up | lo)
        if up.any():
            r = np.hypot(rcv[up, 0] - src[0], rcv[up, 1] - src[1])
            u1 = (ph[up] * np.exp(-g1[None, :] * Y[up]) / g1[None, :]) @ (w * sig[:, 0])
            out[up] = 0.25j * hankel1(0, self.k1 * r) + u1 / (4 * np.pi)
        if lo.any():
            u3 = (ph[lo] * np.exp(g3[None, :] * (Y[lo] + self.d)) / g3[None, :]) @ (w * sig[:, 3])
            out[lo] = u3 / (4 * np.pi)
        if mid.any():
            Ym = Y[mid]
            u2 = ((ph[mid] * np.exp(g2[None, :] * Ym) / g2[None, :]) @ (w * sig[:, 1])
                  + (ph[mid] * np.exp(-g2[None, :] * (Ym + self.d)) / g2[None, :]) @ (w * sig[:, 2]))
            out[mid] = u2 / (4 * np.pi) + multipole_field(self.xy, beta, self.k2, rcv[mid])
        return out


def multipole_field(xy, beta, k, pts):
    """sum_m sum_nu beta^m_nu H_nu(k r_m) e^{i nu theta_m} at points (R, 2)."""
    P = beta.shape[1]
    p = (P - 1) // 2
    nu = operators.orders(p)
    out = np.zeros(pts.shape[0], dtype=np.complex128)
    for m in range(xy.shape[0]):
        dx = pts[:, 0] - xy[m, 0]
        dy = pts[:, 1] - xy[m, 1]
        r = np.hypot(dx, dy)
        th = np.arctan2(dy, dx)
        out += (hankel1(nu[None, :], k * r[:, None]) * np.exp(1j * nu[None, :] * th[:, None])) @ beta[m]
    return out


def gmres(matvec, b, tol, maxiter):
    """Plain unrestarted GMRES with x0 = 0; returns (x, residual history)."""
    n = b.size
    bn = np.linalg.norm(b)
    if bn == 0:
        return np.zeros_like(b), [0.0]
    V = np.zeros((maxiter + 1, n), dtype=np.complex128)
    H = np.zeros((maxiter + 1, maxiter), dtype=np.complex128)
    V[0] = b / bn
    hist = [1.0]
    for j in range(maxiter):
        wv = matvec(V[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], wv)
            wv = wv - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(wv)
        if H[j + 1, j] != 0:
            V[j + 1] = wv / H[j + 1, j]
        e1 = np.zeros(j + 2, dtype=np.complex128)
        e1[0] = bn
        y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
        res = np.linalg.norm(H[:j + 2, :j + 1] @ y - e1) / bn
        hist.append(res)
        if res < tol or H[j + 1, j] == 0:
            return V[:j + 1].T @ y, hist
    return V[:maxiter].T @ y, hist
