"""Reference fields of two solves, written by the FP64 oracle alone.

For the 1000-star recipe (c2: p = 12, 512 contour nodes) and for a window of
600 stars cut from the 5000-star recipe (c3: p = 16, 1024 nodes, the 600
particles nearest to x = 0), the discrete system of eq. (49) is assembled
densely and solved by LU (oracle.system.Problem.solve_lu), and the total field
of eq. (36) is evaluated at seeded receivers in all three layers
(oracle.system.Problem.field).  The prototype scattering matrix is the
oracle's star matrix (Section 4, n_bdry = 256).  Imports only oracle/ and
synth/.  Memory: about 3 times the dense matrix (30 GB for c2).

    python tests/golden/make_solve_refs.py c2
    python tests/golden/make_solve_refs.py c3cut600
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import contour as ocontour  # noqa: E402
from oracle import star as ostar  # noqa: E402
from oracle import system as osystem  # noqa: E402
from synth import make_workload, receivers  # noqa: E402

CASES = {
    "c2": dict(name="c2", cut=None, n_rcv=256, seed=2001),
    "c3cut600": dict(name="c3", cut=600, n_rcv=256, seed=2003),
}


def workload(case):
    c = CASES[case]
    return make_workload(c["name"], cut=c["cut"])


def receiver_points(case, wl):
    c = CASES[case]
    xs = wl.xy[:, 0]
    return receivers(c["n_rcv"], (xs.min() - 1, xs.max() + 1), (-wl.d - 1.5, 2.5), wl.xy, c["seed"],
                     particle_excl=wl.r_enclose + 0.05, source=wl.src[0], source_excl=0.05)


def main(case):
    wl = workload(case)
    a1, a2, a3 = wl.shape_params
    t0 = time.time()
    S = ostar.star_smatrix(a1, a2, a3, wl.k2, wl.kp, wl.p, nb=256)
    lam, w = ocontour.contour(wl.n_nodes, wl.b, wl.t_max, [wl.k1, wl.k2, wl.k3])
    pr = osystem.Problem(wl.k1, wl.k2, wl.k3, wl.d, wl.p, S, wl.xy, wl.rot, lam, w)
    src = wl.src[0]
    beta = pr.solve_lu(src)
    rcv = receiver_points(case, wl)
    u = pr.field(src, beta, rcv)
    path = os.path.join(HERE, f"{case}_lu_field.txt")
    with open(path, "w") as fh:
        fh.write(f"# {case}: {wl.n} stars (a1, a2, a3) = {wl.shape_params}, kp = {wl.kp}, p = {wl.p}, "
                 f"k = ({wl.k1}, {wl.k2}, {wl.k3}), d = {wl.d}, {wl.n_nodes} contour nodes, b = {wl.b}, "
                 f"t_max = {wl.t_max}, source ({src[0]:g}, {src[1]:g})\n")
        fh.write("# eq. (49) solved by dense LU, total field of eq. (36); written by "
                 "tests/golden/make_solve_refs.py (oracle only)\n")
        fh.write(f"# |beta|_2 = {np.linalg.norm(beta):.17e}\n")
        fh.write("# x y Re(u) Im(u)\n")
        for (x, y), v in zip(rcv, u):
            fh.write(f"{x:.17e} {y:.17e} {v.real:.17e} {v.imag:.17e}\n")
    print(f"{case}: {wl.n} particles, {time.time() - t0:.0f} s -> {path}")


if __name__ == "__main__":
    main(sys.argv[1])
