"""Layered medium with any number of layers (TM polarisation), particles in one
finite layer: the extension of Section 2 to an arbitrary layered medium that
the Introduction calls straightforward, written out from the interface
conditions (8)-(9) (u and du/dy continuous across every interface).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Geometry.  Layers j = 0 .. L-1 from top to bottom with wavenumbers k_j;
interface i (i = 0 .. L-2) at height y_i separates layer i (above) from layer
i + 1 (below).  The particles lie in the finite layer c (1 <= c <= L-2),
whose top interface is y = 0 and bottom interface y = -d; the point source
lies in the top half-space (layer 0).

Per contour node lambda (gamma_j = sqrt(lambda^2 - k_j^2), branch of Section
5.1) and with the common factor (1/4 pi) w e^{i lambda x} left out, the field
in each layer is
  layer 0:        g e^{ g0 (y - y_0)}/g0 + B_0 e^{-g0 (y - y_0)}/g0   (source + reflected)
  layer j:        A_j e^{ gj (y - y_{j-1})}/gj + B_j e^{-gj (y - y_j)}/gj
  layer L-1:      A_{L-1} e^{g (y - y_{L-2})}/g
  layer c adds    P+ e^{-gc y}/gc above and P- e^{gc (y + d)}/gc below the
                  particles (their spectra on the two interfaces, Theorem 5.1)
with g = e^{-i lambda x_s - g0 (y_s - y_0)}.  Every exponential is referenced
to its own layer's interface, so all entries of the system are bounded.  The
unknowns X = (B_0, A_1, B_1, ..., A_{L-2}, B_{L-2}, A_{L-1}) solve
  u(above) - u(below) = 0  and  du/dy(above) - du/dy(below) = 0
at every interface, by Gaussian elimination per node.  For L = 3 this is
eq. (10) with (sigma_1, sigma_2^+, sigma_2^-, sigma_3) = (B_0, A_1, B_1, A_2).

TE polarisation: the derivative rows carry the weight 1/k_j^2 of the layer
each term lives in ((1/eps) du/dy continuous); TM has weight 1.

Pins (tests/test_oracle_stack.py): L = 3 against the three-layer oracle;
splitting a layer by an interface between equal wavenumbers changes nothing;
u and du/dy continuous at every interface of the assembled field; power
balance on a rectangle crossing all interfaces.
"""

import numpy as np
from scipy.special import hankel1

from . import operators
from .contour import gamma
from .system import Problem, multipole_field


def interfaces(thick, c):
    """Interface heights y_0 > ... > y_{L-2} from the finite-layer thicknesses
    thick[j] (j = 1 .. L-2; thick[0] and thick[L-1] are ignored) with the
    particle layer c between y = 0 and y = -thick[c]."""
    L = len(thick)
    y = np.zeros(L - 1)
    y[c - 1] = 0.0
    for i in range(c - 2, -1, -1):          # upwards: interface i is the top of layer i + 1
        y[i] = y[i + 1] + thick[i + 1]
    for i in range(c, L - 1):               # downwards: interface i is the bottom of layer i
        y[i] = y[i - 1] - thick[i]
    return y


def _col_A(j):
    return 2 * j - 1            # unknown index of A_j (1 <= j <= L-1)


def _col_B(j):
    return 0 if j == 0 else 2 * j   # unknown index of B_j (0 <= j <= L-2)


def weights(ks, pol):
    """Weight of du/dy in the interface conditions, per layer."""
    if pol not in ("TM", "TE"):
        raise ValueError("pol is 'TM' or 'TE'")
    return [1.0 if pol == "TM" else 1.0 / complex(k) ** 2 for k in ks]


def node_system(lam, ks, thick, c, pol="TM"):
    """Interface matrices per node, (N_S, 2L-2, 2L-2): row 2i is u, row 2i+1
    is (weighted) du/dy, both as (above) - (below) at interface i."""
    lam = np.atleast_1d(np.asarray(lam, dtype=np.complex128))
    L = len(ks)
    kap = weights(ks, pol)
    yint = interfaces(thick, c)
    g = [gamma(lam, k) for k in ks]
    n = 2 * L - 2
    M = np.zeros((lam.size, n, n), dtype=np.complex128)
    for i in range(L - 1):
        up, lo = i, i + 1
        # layer above (index up), evaluated at its bottom interface i
        ku, kl = kap[up], kap[lo]
        if up == 0:
            M[:, 2 * i, _col_B(0)] += 1 / g[0]
            M[:, 2 * i + 1, _col_B(0)] += -ku
        else:
            e = np.exp(-g[up] * (yint[up - 1] - yint[up]))     # A_up at its bottom
            M[:, 2 * i, _col_A(up)] += e / g[up]
            M[:, 2 * i + 1, _col_A(up)] += ku * e
            M[:, 2 * i, _col_B(up)] += 1 / g[up]
            M[:, 2 * i + 1, _col_B(up)] += -ku
        # layer below (index lo), evaluated at its top interface i, subtracted
        M[:, 2 * i, _col_A(lo)] -= 1 / g[lo]
        M[:, 2 * i + 1, _col_A(lo)] -= kl
        if lo < L - 1:
            e = np.exp(-g[lo] * (yint[lo - 1] - yint[lo]))     # B_lo at its top
            M[:, 2 * i, _col_B(lo)] -= e / g[lo]
            M[:, 2 * i + 1, _col_B(lo)] -= -kl * e
    return M


def rhs(lam, ks, thick, c, Pp=None, Pm=None, src=None, pol="TM"):
    """Known terms moved to the right-hand side, (N_S, 2L-2)."""
    lam = np.atleast_1d(np.asarray(lam, dtype=np.complex128))
    L = len(ks)
    kap = weights(ks, pol)
    yint = interfaces(thick, c)
    b = np.zeros((lam.size, 2 * L - 2), dtype=np.complex128)
    if src is not None:                     # layer 0, above interface 0: g/g0, derivative g
        g0 = gamma(lam, ks[0])
        gs = np.exp(-1j * lam * src[0] - g0 * (src[1] - yint[0]))
        b[:, 0] -= gs / g0
        b[:, 1] -= kap[0] * gs
    if Pp is not None:                      # layer c below interface c-1: P+/gc, derivative -P+
        gc = gamma(lam, ks[c])
        i = c - 1
        b[:, 2 * i] += Pp / gc
        b[:, 2 * i + 1] += -kap[c] * Pp
    if Pm is not None:                      # layer c above interface c: P-/gc, derivative +P-
        gc = gamma(lam, ks[c])
        i = c
        b[:, 2 * i] -= Pm / gc
        b[:, 2 * i + 1] -= kap[c] * Pm
    return b


class StackProblem(Problem):
    """Problem of eq. (49) with the layer stack in place of the three layers.
    Build with ``stack_problem``."""

    def sigma(self, beta=None, src=None):
        """All layer amplitudes X per node (see the module docstring)."""
        Pp = Pm = None
        if beta is not None:
            Pp, Pm = operators.m2s(beta, self.xy, self.lam, self.k2, self.d)
        b = rhs(self.lam, self.ks, self.thick, self.c, Pp, Pm, src, self.pol)
        return np.linalg.solve(self.M, b[..., None])[..., 0]

    def layer_local(self, beta=None, src=None, targets=None):
        X = self.sigma(beta, src)
        return operators.s2l(X[:, _col_A(self.c)], X[:, _col_B(self.c)], self.xy, self.lam, self.w,
                             self.k2, self.d, self.p, targets)

    def dense(self):
        """K = I - S_blk (T + T_R), T_R column by column through the node systems."""
        N, P = self.N, self.P
        K = np.zeros((N * P, N * P), dtype=np.complex128)
        for col in range(N * P):
            e = np.zeros(N * P, dtype=np.complex128)
            e[col] = 1.0
            K[:, col] = self.matvec(e).reshape(-1)
        return K

    def field(self, src, beta, rcv):
        """Total field at receivers (R, 2)."""
        rcv = np.asarray(rcv, dtype=np.float64)
        X = self.sigma(beta, src)
        L = len(self.ks)
        yint = interfaces(self.thick, self.c)
        lam, w = self.lam, self.w
        out = np.zeros(rcv.shape[0], dtype=np.complex128)
        ph = np.exp(1j * lam[None, :] * rcv[:, 0][:, None])
        # layer of each receiver: number of interfaces above it
        lay = np.sum(rcv[:, 1][:, None] < yint[None, :], axis=1)
        for j in range(L):
            sel = lay == j
            if not sel.any():
                continue
            gj = gamma(lam, self.ks[j])[None, :]
            Y = rcv[sel, 1][:, None]
            acc = np.zeros((sel.sum(), lam.size), dtype=np.complex128)
            if j == 0:
                acc += np.exp(-gj * (Y - yint[0])) * X[None, :, _col_B(0)]
            else:
                acc += np.exp(gj * (Y - yint[j - 1])) * X[None, :, _col_A(j)]
                if j < L - 1:
                    acc += np.exp(-gj * (Y - yint[j])) * X[None, :, _col_B(j)]
            out[sel] = (ph[sel] * acc / gj) @ w / (4 * np.pi)
            if j == 0:
                r = np.hypot(rcv[sel, 0] - src[0], rcv[sel, 1] - src[1])
                out[sel] += 0.25j * hankel1(0, self.ks[0] * r)
            if j == self.c:
                out[sel] += multipole_field(self.xy, beta, self.k2, rcv[sel])
        return out


def stack_problem(ks, thick, c, p, S, xy, rot, lam, w, pol="TM"):
    """StackProblem for wavenumbers ks (top to bottom), finite-layer
    thicknesses thick (same length; entries 0 and L-1 unused), particle
    layer c and polarisation pol (S must be the matching scattering matrix)."""
    ks = [complex(k) for k in ks]
    thick = [float(t) for t in thick]
    if not (1 <= c <= len(ks) - 2) or len(thick) != len(ks):
        raise ValueError("need 1 <= c <= L-2 and one thickness per layer")
    pr = StackProblem(ks[0], ks[c], ks[-1], thick[c], p, S, xy, rot, lam, w)
    pr.ks, pr.thick, pr.c, pr.pol = ks, thick, c, pol
    pr.M = node_system(pr.lam, ks, thick, c, pol)
    return pr
