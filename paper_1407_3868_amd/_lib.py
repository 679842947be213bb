"""ctypes loader of libmpsl.so and the C signatures of include/mpsl.h.

The shared library is built in-tree by ``paper_1407_3868_amd/build.py``.
Loading fails loudly when it is missing: there is no fallback path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpsl.so")


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("restart", ctypes.c_int), ("inner_tol", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("fp64_matvecs", ctypes.c_int), ("refinements", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int),
                ("precond_seconds", ctypes.c_double), ("reorthogonalizations", ctypes.c_int)]


P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double
L = ctypes.c_int64
DP = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes), in header order
SIGNATURES = {
    "mpsl_status_string": (ctypes.c_char_p, [I]),
    "mpsl_last_error": (ctypes.c_char_p, [P]),
    "mpsl_create": (I, [ctypes.POINTER(P), I, ctypes.c_size_t]),
    "mpsl_destroy": (None, [P]),
    "mpsl_get_memory": (I, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "mpsl_set_stream": (I, [P, P]),
    "mpsl_set_layers": (I, [P, c128, c128, c128, D]),
    "mpsl_set_layer_stack": (I, [P, I, P, P, I]),
    "mpsl_set_polarization": (I, [P, I]),
    "mpsl_set_particle_types": (I, [P, I, I, P, P]),
    "mpsl_set_geometry_typed": (I, [P, L, P, P, P]),
    "mpsl_get_polarization": (I, [P]),
    "mpsl_compute_layer_map": (I, [I, P, P, I, I, I, P, P]),
    "mpsl_set_particle_disk": (I, [P, D, c128, I]),
    "mpsl_set_particle_star": (I, [P, D, D, I, c128, I, I]),
    "mpsl_set_scattering_matrix": (I, [P, I, D, P]),
    "mpsl_set_geometry": (I, [P, L, P, P]),
    "mpsl_set_contour": (I, [P, I, D, D]),
    "mpsl_compute_disk_smatrix": (I, [D, c128, c128, I, I, P]),
    "mpsl_compute_star_smatrix": (I, [D, D, I, c128, c128, I, I, I, P]),
    "mpsl_compute_contour": (I, [c128, c128, c128, I, D, D, P, P]),
    "mpsl_set_contour_span": (I, [P, D, D, D]),
    "mpsl_set_sommerfeld_method": (I, [P, I]),
    "mpsl_span_contour_params": (I, [D, D, DP, DP]),
    "mpsl_compute_contour_span": (I, [I, P, D, D, D, I, P, P, P]),
    "mpsl_set_contour_nodes": (I, [P, I, P, P]),
    "mpsl_get_contour": (I, [P, I, P, P]),
    "mpsl_get_scattering_matrix": (I, [P, I, P]),
    "mpsl_get_sizes": (I, [P, ctypes.POINTER(L), ctypes.POINTER(I), ctypes.POINTER(I)]),
    "mpsl_apply": (I, [P, I, P, P]),
    "mpsl_apply_dev": (I, [P, I, P, P]),
    "mpsl_apply_batch_dev": (I, [P, I, I, P, P]),
    "mpsl_batch_create": (I, [ctypes.POINTER(P), I, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(I),
                              ctypes.POINTER(P), ctypes.POINTER(P)]),
    "mpsl_batch_launch": (I, [P, P]),
    "mpsl_batch_destroy": (None, [P]),
    "mpsl_m2l_dev": (I, [P, I, P, P]),
    "mpsl_m2l_dev_noalloc": (I, [P, I, P, P]),
    "mpsl_m2s_dev": (I, [P, I, P, P]),
    "mpsl_reflect_dev": (I, [P, P, P, P]),
    "mpsl_s2l_dev": (I, [P, I, P, P]),
    "mpsl_sapply_dev": (I, [P, I, P, P, P]),
    "mpsl_set_preconditioner": (I, [P, I, I]),
    "mpsl_compute_clusters": (I, [L, P, I, P, ctypes.POINTER(I)]),
    "mpsl_precond_apply_dev": (I, [P, I, P, P]),
    "mpsl_get_precond_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), DP]),
    "mpsl_rhs": (I, [P, P, P]),
    "mpsl_solve": (I, [P, I, P, ctypes.POINTER(Opts), P, ctypes.POINTER(Info)]),
    "mpsl_eval_field": (I, [P, I, P, P, L, P, P]),
    "mpsl_autotune": (I, [P, I]),
    "mpsl_set_tuning": (I, [P, I, I, I]),
    "mpsl_get_tuning": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I), DP]),
    "mpsl_profile": (I, [P, I]),
    "mpsl_profile_read": (I, [P, DP, ctypes.POINTER(I)]),
    "mpsl_set_far_field": (I, [P, I, ctypes.c_double]),
    "mpsl_get_somm_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                               ctypes.POINTER(I)]),
    "mpsl_get_fmm_info": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I), DP, ctypes.POINTER(I),
                              ctypes.POINTER(I), ctypes.POINTER(L), DP]),
}

_lib = None


def _hip_runtimes():
    """Paths of every HIP runtime library mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64.so" in ln})
    except OSError:
        return []


def load():
    """Load libmpsl.so once; raise ImportError when it has not been built.

    torch is imported first: its HIP runtime carries the same soname as the
    one libmpsl.so was linked against, so the library binds to the runtime
    already in the process and torch tensors, streams and the library's
    kernels share one HIP runtime.  Two runtimes in one process are refused.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.isfile(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_1407_3868_amd/build.py (hipcc, gfx950)")
    import torch  # noqa: F401  (loads the process's HIP runtime)
    lib = ctypes.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes are mapped into this process: {rts}")
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class Request(ctypes.Structure):
    _fields_ = [("k1", c128), ("k2", c128), ("k3", c128), ("d", ctypes.c_double), ("particle", ctypes.c_int),
                ("shape", ctypes.c_double * 3), ("kp", c128), ("p", ctypes.c_int), ("n_bdry", ctypes.c_int),
                ("S", ctypes.c_void_p), ("r_enclose", ctypes.c_double), ("n", ctypes.c_int64),
                ("xy", ctypes.c_void_p), ("rot", ctypes.c_void_p), ("n_nodes", ctypes.c_int),
                ("b", ctypes.c_double), ("t_max", ctypes.c_double), ("src", ctypes.c_double * 2),
                ("opts", Opts), ("contour", ctypes.c_int), ("h_max", ctypes.c_double), ("sommerfeld", ctypes.c_int),
                ("precond", ctypes.c_int), ("cluster_size", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n", ctypes.c_int64), ("p", ctypes.c_int),
                ("beta", ctypes.POINTER(c128)), ("iterations", ctypes.c_int), ("fp64_matvecs", ctypes.c_int),
                ("refinements", ctypes.c_int), ("rel_residual", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_finish", ctypes.c_double),
                ("hbm_bytes", ctypes.c_size_t), ("error", ctypes.c_char_p)]


SIGNATURES.update({
    "mpsl_server_create": (I, [ctypes.POINTER(P), I, ctypes.c_size_t, I]),
    "mpsl_server_submit": (I, [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "mpsl_server_poll": (I, [P, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "mpsl_server_wait": (I, [P, ctypes.c_uint64, D, ctypes.POINTER(Result)]),
    "mpsl_server_release": (I, [P, ctypes.c_uint64]),
    "mpsl_server_stats": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(ctypes.c_uint64),
                              ctypes.POINTER(ctypes.c_size_t)]),
    "mpsl_server_destroy": (None, [P]),
})
