"""Shared set-up of the GPU parity tests: one workload, the oracle problem for
it, and an mpsl Context configured with the same inputs."""
import numpy as np

from oracle import contour as ocontour
from oracle import mie as omie
from oracle import star as ostar
from oracle import system as osystem
from synth import make_workload

_S_CACHE = {}


def prototype_S(wl):
    """Prototype scattering matrix from the oracle (the parity input for stars)."""
    key = (wl.shape, wl.shape_params, wl.k2, wl.kp, wl.p)
    if key not in _S_CACHE:
        if wl.shape == "disk":
            _S_CACHE[key] = np.diag(omie.disk_smatrix(wl.shape_params[0], wl.k2, wl.kp, wl.p))
        else:
            a1, a2, a3 = wl.shape_params
            _S_CACHE[key] = ostar.star_smatrix(a1, a2, a3, wl.k2, wl.kp, wl.p, nb=256)
    return _S_CACHE[key]


def oracle_problem(wl, ks=None):
    k1, k2, k3 = ks if ks is not None else (wl.k1, wl.k2, wl.k3)
    lam, w = ocontour.contour(wl.n_nodes, wl.b, wl.t_max, [k1, k2, k3])
    return osystem.Problem(k1, k2, k3, wl.d, wl.p, prototype_S(wl), wl.xy, wl.rot, lam, w)


def gpu_context(wl, ks=None, disk_from_library=False):
    import paper_1407_3868_amd as mp
    ctx = mp.Context(0)
    k1, k2, k3 = ks if ks is not None else (wl.k1, wl.k2, wl.k3)
    ctx.set_layers(k1, k2, k3, wl.d)
    if disk_from_library and wl.shape == "disk":
        ctx.set_particle_disk(wl.shape_params[0], wl.kp, wl.p)
    else:
        ctx.set_scattering_matrix(wl.p, wl.r_enclose, prototype_S(wl))
    ctx.set_geometry(wl.xy, wl.rot)
    ctx.set_contour(wl.n_nodes, wl.b, wl.t_max)
    return ctx


def coeff_vector(wl, seed, S=None):
    """A vector in the range of the scattering matrices (the shape of beta)."""
    rng = np.random.default_rng(seed)
    S = prototype_S(wl) if S is None else S
    r = rng.standard_normal((wl.n, wl.P)) + 1j * rng.standard_normal((wl.n, wl.P))
    from oracle.operators import rotated_smatrix
    return np.stack([rotated_smatrix(S, wl.rot[l]) @ r[l] for l in range(wl.n)])


def rel_err(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def entry_err(got, ref, eps):
    """Worst per-entry error max |got - ref| / (|ref| + eps * max|ref| of its row)
    over an array of rows (particles, or the two interfaces of a spectrum),
    with the (row, column) where it occurs.  eps = 0 makes it the largest
    relative error of any single entry."""
    ref = np.asarray(ref)
    got = np.asarray(got).reshape(ref.shape)
    d = np.abs(got - ref)
    scale = np.abs(ref) + eps * np.abs(ref).max(axis=-1, keepdims=True)
    r = np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), np.where(d > 0, np.inf, 0.0))
    i = np.unravel_index(int(np.argmax(r)), r.shape)
    return float(r[i]), tuple(int(v) for v in i)


# Per-entry bounds of the steps and the matvec (tol, eps of entry_err).  FP64:
# every entry to 1e-11 of itself (measured worst 1.2e-12 over the small
# layouts, M2L / M2S / S2L / matvec); the floor eps keeps exact zeros
# finite.  FP32: 1e-4 with a floor of 1e-3 of the row's largest entry
# (measured worst 3.5e-5 without a floor, 3.0e-5 with it: FP32 rounding of
# the tables and sums of N P terms spanning many decades).
ENTRY_TOL = {0: (1e-11, 1e-9), 1: (1e-4, 1e-3)}


def max_err(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


__all__ = ["make_workload", "prototype_S", "oracle_problem", "gpu_context", "coeff_vector", "rel_err", "max_err",
           "entry_err", "ENTRY_TOL"]
