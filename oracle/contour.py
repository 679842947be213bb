"""Discretised Sommerfeld contour (Section 5.1, eq. (37); parameters of Section 6).

The real line is deformed into three segments: Gamma_3 = {t + ib, t < 0},
Gamma_2 = {it, t in [-b, b]} and Gamma_1 = {t - ib, t > 0}, truncated at
|t| = t_max.  The path runs from -t_max + ib along Gamma_3 to +ib, down
Gamma_2 to -ib, then along Gamma_1 to t_max - ib, so on Gamma_2
lambda = -i s, s in [-b, b], d lambda = -i ds.

Each segment is split into 16-point Gauss-Legendre panels.  Gamma_2 uses the
two panels [-b, 0] and [0, b] in s.  Gamma_1 uses n_pan = (N_S - 32) / 32
panels on [0, t_max]; Gamma_3 is its mirror image lambda -> -lambda with the
same weights.  The panel rule on [0, t_max] (the paper only says
"Gauss-Legendre on each segment", so this is a stated reading):

  1. breakpoints: 0, t_max, and Re k_i for every layer wavenumber with
     0 < Re k_i < t_max (the branch points); one panel per gap;
  2. while fewer than n_pan panels: for each panel [a, c] let
     L = c - a and dist = distance from [a, c] to the nearest Re k_i
     (0 when a breakpoint k_i is an end point); score = L / max(dist, b);
     split the panel with the largest score (ties: smallest a) at
     (a + c) / 2.

gamma_i(lambda) = sqrt(lambda^2 - k_i^2) takes the branch Re gamma >= 0 and,
where Re gamma = 0, Im gamma <= 0 (outgoing / decaying waves).

Span rule (contour_span).  For particles spread over a lateral extent X the
integrands carry e^{i lambda (x_l - x_m)} with |x_l - x_m| up to X, which a
fixed node count cannot resolve once X grows (the paper's node counts of
Section 6 are for compact layouts).  contour_span fixes the panel length
instead of the node count, on [0, t_max]:

  1. breakpoints 0, t_max and Re k_i (0 < Re k_i < t_max), as above;
  2. in each gap [a, c] with midpoint m, an end that is a branch point is
     graded: cuts at a + b 2^j (j = 0, 1, ...) while below m (for a), and at
     c - b 2^j while above m (for c); m itself is a cut when an end is graded;
  3. every piece between cuts splits into ceil(length / h_max) equal panels.

Gamma_2 and Gamma_3 as above.  b ~ 2/X keeps e^{b X} bounded; h_max ~ 6/X
gives about 1e-11 on the layered interaction of two particles X apart
(16-point panels), h_max ~ 12/X about 1e-6.

Pins (tests/test_oracle_contour.py): the quadrature reproduces the Sommerfeld
representation (3) of (i/4) H_0(k r) and of the multipoles of Theorem 5.1 on a
refined contour; Gamma_3 mirrors Gamma_1 exactly; weights sum to the contour's
chord length.
"""

import numpy as np

GL_ORDER = 16
GAMMA2_NODES = 2 * GL_ORDER


def gamma(lam, k):
    """Branch of sqrt(lam^2 - k^2) with Re >= 0, and Im <= 0 when Re == 0."""
    g = np.sqrt(np.asarray(lam, dtype=np.complex128) ** 2 - complex(k) ** 2)
    g = np.where(g.real < 0, -g, g)
    g = np.where((g.real == 0) & (g.imag > 0), -g, g)
    return g


def panel_breaks(n_pan, b, t_max, ks):
    """Panel end points on [0, t_max] for Gamma_1 (rule in the module doc)."""
    sing = sorted({float(np.real(k)) for k in ks if 0.0 < float(np.real(k)) < t_max})
    edges = sorted({0.0, float(t_max), *sing})
    panels = [(edges[i], edges[i + 1]) for i in range(len(edges) - 1)]
    if len(panels) > n_pan:
        raise ValueError("too few contour nodes for the branch-point breakpoints")
    while len(panels) < n_pan:
        best = None
        best_score = -1.0
        for (a, c) in panels:
            L = c - a
            dist = float("inf")
            for s in sing:
                if s < a:
                    dd = a - s
                elif s > c:
                    dd = s - c
                else:
                    dd = 0.0
                dist = min(dist, dd)
            if not sing:
                dist = float("inf")
            score = L / max(dist, b)
            if score > best_score or (score == best_score and a < best[0]):
                best_score = score
                best = (a, c)
        panels.remove(best)
        a, c = best
        m = (a + c) / 2.0
        panels.extend([(a, m), (m, c)])
        panels.sort()
    return panels


def contour(n_nodes, b, t_max, ks):
    """Nodes lambda_q and weights w_q (complex), in path order.

    Order: Gamma_3 (from -t_max + ib to ib), Gamma_2 (ib to -ib),
    Gamma_1 (-ib to t_max - ib).  Returns (lam, w) complex128 arrays.
    """
    if n_nodes % GL_ORDER or n_nodes < 3 * GAMMA2_NODES:
        raise ValueError("n_nodes must be a multiple of 16 and at least 96")
    if (n_nodes - GAMMA2_NODES) % (2 * GL_ORDER):
        raise ValueError("(n_nodes - 32) must be a multiple of 32")
    x, wx = np.polynomial.legendre.leggauss(GL_ORDER)
    n_pan = (n_nodes - GAMMA2_NODES) // (2 * GL_ORDER)
    t1 = []
    w1 = []
    for (a, c) in panel_breaks(n_pan, b, t_max, ks):
        t1.append((a + c) / 2.0 + (c - a) / 2.0 * x)
        w1.append((c - a) / 2.0 * wx)
    t1 = np.concatenate(t1)
    w1 = np.concatenate(w1)
    lam1 = t1 - 1j * b
    lam3 = -lam1[::-1]
    w3 = w1[::-1].astype(np.complex128)
    s2 = np.concatenate([-b / 2.0 + b / 2.0 * x, b / 2.0 + b / 2.0 * x])
    ws2 = np.concatenate([b / 2.0 * wx, b / 2.0 * wx])
    lam2 = -1j * s2
    w2 = -1j * ws2
    lam = np.concatenate([lam3, lam2, lam1]).astype(np.complex128)
    w = np.concatenate([w3, w2, w1.astype(np.complex128)])
    return lam, w


def span_breaks(b, t_max, h_max, ks):
    """Panel end points on [0, t_max] for Gamma_1 under the span rule."""
    sing = sorted({float(np.real(k)) for k in ks if 0.0 < float(np.real(k)) < t_max})
    edges = sorted({0.0, float(t_max), *sing})
    panels = []
    for a, c in zip(edges[:-1], edges[1:]):
        m = (a + c) / 2.0
        cuts = {a, c}
        if a in sing:
            e = b
            while a + e < m:
                cuts.add(a + e)
                e *= 2.0
        if c in sing:
            e = b
            while c - e > m:
                cuts.add(c - e)
                e *= 2.0
        if a in sing or c in sing:
            cuts.add(m)
        pts = sorted(cuts)
        for u, v in zip(pts[:-1], pts[1:]):
            k = int(np.ceil((v - u) / h_max))
            for i in range(k):
                panels.append((u + (v - u) * i / k, u + (v - u) * (i + 1) / k))
    return panels


def contour_span(b, t_max, h_max, ks):
    """Nodes and weights of the span rule, in the path order of ``contour``."""
    if not (b > 0 and t_max > 0 and h_max > 0):
        raise ValueError("b, t_max and h_max must be positive")
    x, wx = np.polynomial.legendre.leggauss(GL_ORDER)
    pan = span_breaks(b, t_max, h_max, ks)
    t1 = np.concatenate([(a + c) / 2.0 + (c - a) / 2.0 * x for a, c in pan])
    w1 = np.concatenate([(c - a) / 2.0 * wx for a, c in pan])
    lam1 = t1 - 1j * b
    lam3 = -lam1[::-1]
    w3 = w1[::-1].astype(np.complex128)
    s2 = np.concatenate([-b / 2.0 + b / 2.0 * x, b / 2.0 + b / 2.0 * x])
    ws2 = np.concatenate([b / 2.0 * wx, b / 2.0 * wx])
    lam = np.concatenate([lam3, -1j * s2, lam1]).astype(np.complex128)
    w = np.concatenate([w3, -1j * ws2, w1.astype(np.complex128)])
    return lam, w
