"""Cluster-block right preconditioner for the GMRES solve of eq. (49), written
out plainly.  Test infrastructure: the CPU oracle that the library's
preconditioner is checked against.  Nothing in the library imports it.

Section 3.2 multiplies the multiple-scattering system by the block-diagonal
scattering matrices, so that the matrix GMRES sees is I - S T (and with the
layers I - S (T + T_R), eq. (49)).  In that form the diagonal block of one
particle is the identity: the preconditioning is exact for a particle alone.
The Conclusions note that convergence degrades for dense packings of
high-contrast inclusions, where the strongest couplings are between near
neighbours.  The same idea applied to a cluster of nearby particles instead of
one particle: with the particles split into clusters c, let

    K_c = I - S_c T_cc

be the free-space system of the particles of cluster c on their own (T_cc the
translations of Lemma 3.1 between particles of c, S_c their rotated scattering
matrices), and M = blockdiag_c K_c.  GMRES solves the right-preconditioned
system  K M^{-1} u = b  and returns  x = M^{-1} u, which leaves the solution of
K x = b unchanged.  With one particle per cluster M = I (the paper's own form).

Clusters come from recursive coordinate bisection of the particle centres: a
set of more than `size` particles is cut into two halves of floor(n/2) and
ceil(n/2) particles across its longer extent, by the order of that coordinate.

Pins: tests/test_oracle_precond.py.
"""

import numpy as np

from . import operators


def clusters(xy, size):
    """Recursive coordinate bisection of the centres xy (N, 2).

    A set of n > size particles is split along x when its x-extent (max - min
    of the centres) is at least its y-extent, else along y: the particles are
    ordered by that coordinate (equal coordinates by particle index) and the
    first floor(n/2) form the first half.  Halves are split again until every
    set holds at most `size` particles.  Returns the clusters in depth-first
    order, first half before second half, each as a sorted index array.
    """
    xy = np.asarray(xy, dtype=np.float64)
    if size < 1:
        raise ValueError("cluster size must be >= 1")
    out = []

    def split(idx):
        if idx.size <= size:
            out.append(np.sort(idx))
            return
        pts = xy[idx]
        ext = pts.max(axis=0) - pts.min(axis=0)
        axis = 0 if ext[0] >= ext[1] else 1
        order = np.lexsort((idx, pts[:, axis]))   # by coordinate, then index
        h = idx.size // 2
        split(idx[order[:h]])
        split(idx[order[h:]])

    split(np.arange(xy.shape[0]))
    return out


def cluster_of(xy, size):
    """Cluster number of every particle (clusters numbered as clusters() lists them)."""
    lab = np.empty(np.asarray(xy).shape[0], dtype=np.int64)
    for c, idx in enumerate(clusters(xy, size)):
        lab[idx] = c
    return lab


def cluster_matrix(problem, idx):
    """K_c = I - S_c T_cc for the particles idx of a Problem (free space only).

    Row block a, column block b (a != b): -S_{l_a} T^{l_b l_a}, with T the
    translation of Lemma 3.1 from particle l_b to particle l_a.
    """
    P = problem.P
    n = len(idx)
    K = np.eye(n * P, dtype=np.complex128)
    for a, la in enumerate(idx):
        Sa = operators.rotated_smatrix(problem.S_of(la), problem.rot[la])
        for b, lb in enumerate(idx):
            if a != b:
                T = operators.m2l_block(problem.xy[la], problem.xy[lb], problem.k2, problem.p)
                K[a * P:(a + 1) * P, b * P:(b + 1) * P] -= Sa @ T
    return K


def block_inverses(problem, size):
    """(clusters, [K_c^{-1}]) for the cluster size of the rule above."""
    cl = clusters(problem.xy, size)
    return cl, [np.linalg.inv(cluster_matrix(problem, idx)) for idx in cl]


def apply(cl, inv, x, P):
    """y = M^{-1} x for x of shape (N, P) (or flat)."""
    x = np.asarray(x, dtype=np.complex128)
    shape = x.shape
    x = x.reshape(-1, P)
    y = np.empty_like(x)
    for idx, X in zip(cl, inv):
        y[idx] = (X @ x[idx].reshape(-1)).reshape(-1, P)
    return y.reshape(shape)


def gmres_right(matvec, b, tol, maxiter, precond):
    """Unrestarted GMRES on K M^{-1} u = b with x0 = 0; returns (x, history).

    matvec(v) = K v and precond(v) = M^{-1} v on flat vectors; the history is
    the relative residual ||b - K x_j|| / ||b|| of each iterate (exact for the
    right-preconditioned form, whose residual is that of the original system).
    """
    n = b.size
    bn = np.linalg.norm(b)
    if bn == 0:
        return np.zeros_like(b), [0.0]
    V = np.zeros((maxiter + 1, n), dtype=np.complex128)
    H = np.zeros((maxiter + 1, maxiter), dtype=np.complex128)
    V[0] = b / bn
    hist = [1.0]
    y = np.zeros(0, dtype=np.complex128)
    k = 0
    for j in range(maxiter):
        wv = matvec(precond(V[j]))
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], wv)
            wv = wv - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(wv)
        if H[j + 1, j] != 0:
            V[j + 1] = wv / H[j + 1, j]
        e1 = np.zeros(j + 2, dtype=np.complex128)
        e1[0] = bn
        y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
        hist.append(np.linalg.norm(H[:j + 2, :j + 1] @ y - e1) / bn)
        k = j + 1
        if hist[-1] < tol or H[j + 1, j] == 0:
            break
    return precond(V[:k].T @ y), hist
