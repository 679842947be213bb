"""MI355X library for multi-particle scattering in a three-layer medium.

A thin Python binding of the C ABI in ``include/mpsl.h`` (argument
marshalling only).  Every step of the computation runs in the HIP kernels of
``libmpsl.so``; when the library has not been built, creating a Context
raises.  Device buffers are passed as torch tensors (their data pointers) or
raw integer addresses.
"""

import ctypes

import numpy as np

from . import _lib

FP64 = 0
FP32 = 1
FAR_AUTO, FAR_DIRECT, FAR_FMM = 0, 1, 2
TM, TE = 0, 1
SOMM_DIRECT, SOMM_INTERP = 0, 1
PRECOND_NONE, PRECOND_CLUSTER = 0, 1

STATUS = {0: "MPSL_OK", -1: "MPSL_EINVAL", -2: "MPSL_ENOMEM", -3: "MPSL_EHIP", -4: "MPSL_ESTATE",
          -5: "MPSL_EGEOM", -6: "MPSL_ENOCONV", -7: "MPSL_EUNSUPPORTED", -8: "MPSL_EINSIDE",
          -9: "MPSL_ENUMERIC"}


class MpslError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _c(z):
    z = complex(z)
    return _lib.c128(z.real, z.imag)


def _ptr(a):
    """Data address of a torch tensor, numpy array or integer."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _carr(a, dtype=np.complex128):
    return np.ascontiguousarray(a, dtype=dtype)


def _host_check(rc, what):
    if rc != 0:
        raise MpslError(rc, what)


def compute_disk_smatrix(R, k2, kp, p, polarization=TM):
    """Host: Mie scattering matrix of a disk (mirrors mpsl_compute_disk_smatrix)."""
    lib = _lib.load()
    S = np.zeros((2 * p + 1, 2 * p + 1), np.complex128)
    _host_check(lib.mpsl_compute_disk_smatrix(float(R), _c(k2), _c(kp), int(p), int(polarization), S.ctypes.data),
                "disk matrix")
    return S


def compute_star_smatrix(a1, a2, a3, k2, kp, p, n_bdry=0, polarization=TM):
    """Host: star scattering matrix by the boundary-integral precompute."""
    lib = _lib.load()
    S = np.zeros((2 * p + 1, 2 * p + 1), np.complex128)
    _host_check(lib.mpsl_compute_star_smatrix(float(a1), float(a2), int(a3), _c(k2), _c(kp), int(p), int(n_bdry),
                                              int(polarization), S.ctypes.data), "star matrix")
    return S


def compute_contour(k1, k2, k3, n_nodes, b, t_max):
    """Host: Sommerfeld contour nodes and weights (mirrors mpsl_compute_contour)."""
    lib = _lib.load()
    lam = np.zeros(n_nodes, np.complex128)
    w = np.zeros(n_nodes, np.complex128)
    _host_check(lib.mpsl_compute_contour(_c(k1), _c(k2), _c(k3), int(n_nodes), float(b), float(t_max),
                                         lam.ctypes.data, w.ctypes.data), "contour")
    return lam, w


def compute_contour_span(ks, b, t_max, h_max):
    """Host: span-rule contour nodes and weights (mirrors mpsl_compute_contour_span)."""
    lib = _lib.load()
    kr = np.ascontiguousarray(np.real(np.asarray(ks, dtype=np.complex128)), dtype=np.float64)
    n = ctypes.c_int(0)
    _host_check(lib.mpsl_compute_contour_span(int(kr.size), kr.ctypes.data, float(b), float(t_max), float(h_max),
                                              0, None, None, ctypes.byref(n)), "contour span")
    lam = np.zeros(n.value, np.complex128)
    w = np.zeros(n.value, np.complex128)
    _host_check(lib.mpsl_compute_contour_span(int(kr.size), kr.ctypes.data, float(b), float(t_max), float(h_max),
                                              n.value, lam.ctypes.data, w.ctypes.data, ctypes.byref(n)),
                "contour span")
    return lam, w


def compute_clusters(xy, cluster_size):
    """Host: cluster of every particle under the bisection rule (mirrors mpsl_compute_clusters)."""
    lib = _lib.load()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    lab = np.zeros(xy.shape[0], np.int32)
    nc = ctypes.c_int(0)
    _host_check(lib.mpsl_compute_clusters(int(xy.shape[0]), xy.ctypes.data, int(cluster_size), lab.ctypes.data,
                                          ctypes.byref(nc)), "clusters")
    return lab, nc.value


def span_contour_params(x_extent, tol=1e-10):
    """(b, h_max) of the span rule for a layout of lateral extent x_extent
    (mirrors mpsl_span_contour_params)."""
    lib = _lib.load()
    b, h = ctypes.c_double(), ctypes.c_double()
    _host_check(lib.mpsl_span_contour_params(float(x_extent), float(tol), ctypes.byref(b), ctypes.byref(h)),
                "span contour parameters")
    return b.value, h.value


def compute_layer_map(ks, thickness, particle_layer, lam, polarization=TM):
    """Host: per-node map of a layer stack (mirrors mpsl_compute_layer_map),
    (n_lam, 6): the 2 x 2 reflection map row-major, then the source factors."""
    lib = _lib.load()
    k = _carr(ks)
    t = np.ascontiguousarray(thickness, dtype=np.float64)
    if t.shape != k.shape:
        raise ValueError("one thickness per layer")
    lam = _carr(np.atleast_1d(lam))
    out = np.zeros((lam.size, 6), np.complex128)
    _host_check(lib.mpsl_compute_layer_map(int(k.size), k.ctypes.data, t.ctypes.data, int(particle_layer),
                                           int(polarization), int(lam.size), lam.ctypes.data, out.ctypes.data),
                "layer map")
    return out


class Batch:
    """A captured multi-configuration batch of matvecs (mpsl_batch_*)."""

    def __init__(self, items):
        """items: list of (context, prec, nrhs, x_dev, y_dev)."""
        self.lib = _lib.load()
        n = len(items)
        self._items = items  # keep contexts and buffers alive
        ctxs = (ctypes.c_void_p * n)(*[it[0].h.value for it in items])
        precs = (ctypes.c_int * n)(*[int(it[1]) for it in items])
        nrhs = (ctypes.c_int * n)(*[int(it[2]) for it in items])
        xs = (ctypes.c_void_p * n)(*[_ptr(it[3]) for it in items])
        ys = (ctypes.c_void_p * n)(*[_ptr(it[4]) for it in items])
        h = ctypes.c_void_p()
        rc = self.lib.mpsl_batch_create(ctypes.byref(h), n, ctxs, precs, nrhs, xs, ys)
        if rc != 0:
            raise MpslError(rc, "mpsl_batch_create failed: " + items[0][0].lib.mpsl_last_error(items[0][0].h).decode())
        self.h = h

    def launch(self, stream=None):
        rc = self.lib.mpsl_batch_launch(self.h, ctypes.c_void_p(stream) if stream else None)
        if rc != 0:
            raise MpslError(rc, "mpsl_batch_launch failed")

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpsl_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One mpsl context on a HIP device (mirrors mpsl_create/mpsl_destroy);
    hbm_budget: device bytes it may hold (0: no limit)."""

    def __init__(self, device=0, hbm_budget=0):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        rc = self.lib.mpsl_create(ctypes.byref(h), int(device), int(hbm_budget))
        if rc != 0:
            raise MpslError(rc, "mpsl_create failed (no HIP device?)")
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpsl_destroy(self.h)
            self.h = None

    def memory(self):
        """(device bytes in use, HBM budget) of the context (mpsl_get_memory)."""
        u, b = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.lib.mpsl_get_memory(self.h, ctypes.byref(u), ctypes.byref(b)))
        return u.value, b.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            raise MpslError(rc, self.lib.mpsl_last_error(self.h).decode())
        return rc

    # -- setup ----------------------------------------------------------
    def set_stream(self, stream):
        return self._check(self.lib.mpsl_set_stream(self.h, ctypes.c_void_p(stream)))

    def set_polarization(self, polarization):
        """MPSL_TM or MPSL_TE (mpsl_set_polarization); clears the particle."""
        return self._check(self.lib.mpsl_set_polarization(self.h, int(polarization)))

    def polarization(self):
        return self.lib.mpsl_get_polarization(self.h)

    def set_layers(self, k1, k2, k3, d):
        return self._check(self.lib.mpsl_set_layers(self.h, _c(k1), _c(k2), _c(k3), float(d)))

    def set_layer_stack(self, ks, thickness, particle_layer):
        """Layers top to bottom (mpsl_set_layer_stack): wavenumbers ks, one
        thickness per layer (the half-space entries are ignored), particles in
        layer ``particle_layer``."""
        k = _carr(ks)
        t = np.ascontiguousarray(thickness, dtype=np.float64)
        if t.shape != k.shape:
            raise ValueError("one thickness per layer")
        return self._check(self.lib.mpsl_set_layer_stack(self.h, int(k.size), k.ctypes.data, t.ctypes.data,
                                                         int(particle_layer)))

    def set_particle_disk(self, R, kp, p):
        return self._check(self.lib.mpsl_set_particle_disk(self.h, float(R), _c(kp), int(p)))

    def set_particle_star(self, a1, a2, a3, kp, p, n_bdry=0):
        return self._check(self.lib.mpsl_set_particle_star(self.h, float(a1), float(a2), int(a3), _c(kp), int(p),
                                                           int(n_bdry)))

    def set_scattering_matrix(self, p, r_enclose, S):
        S = _carr(S)
        return self._check(self.lib.mpsl_set_scattering_matrix(self.h, int(p), float(r_enclose), S.ctypes.data))

    def set_geometry(self, xy, rot=None, types=None):
        """Centres, rotations and (with several particle types) a type per particle."""
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        r = None if rot is None else np.ascontiguousarray(rot, dtype=np.float64)
        if types is None:
            return self._check(self.lib.mpsl_set_geometry(self.h, int(xy.shape[0]), xy.ctypes.data,
                                                          None if r is None else r.ctypes.data))
        t = np.ascontiguousarray(types, dtype=np.int32)
        if t.shape != (xy.shape[0],):
            raise ValueError("one type per particle")
        return self._check(self.lib.mpsl_set_geometry_typed(self.h, int(xy.shape[0]), xy.ctypes.data,
                                                            None if r is None else r.ctypes.data, t.ctypes.data))

    def set_particle_types(self, p, r_enclose, S):
        """Several prototype matrices, S of shape (n_types, P, P) (mpsl_set_particle_types)."""
        S = _carr(S)
        r = np.ascontiguousarray(r_enclose, dtype=np.float64)
        if S.ndim != 3 or S.shape[0] != r.size or S.shape[1:] != (2 * p + 1, 2 * p + 1):
            raise ValueError("S is (n_types, P, P) with one radius per type")
        return self._check(self.lib.mpsl_set_particle_types(self.h, int(r.size), int(p), r.ctypes.data,
                                                            S.ctypes.data))

    def set_contour(self, n_nodes, b, t_max):
        return self._check(self.lib.mpsl_set_contour(self.h, int(n_nodes), float(b), float(t_max)))

    def set_contour_span(self, b, t_max, h_max):
        """Span-rule contour (mpsl_set_contour_span); returns the node count."""
        self._check(self.lib.mpsl_set_contour_span(self.h, float(b), float(t_max), float(h_max)))
        return self.sizes()[2]

    def set_sommerfeld_method(self, method):
        """SOMM_DIRECT (default) or SOMM_INTERP (mpsl_set_sommerfeld_method)."""
        return self._check(self.lib.mpsl_set_sommerfeld_method(self.h, int(method)))

    def set_contour_nodes(self, lam, w):
        lam, w = _carr(lam), _carr(w)
        return self._check(self.lib.mpsl_set_contour_nodes(self.h, int(lam.size), lam.ctypes.data, w.ctypes.data))

    def sizes(self):
        n, p, ns = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.mpsl_get_sizes(self.h, ctypes.byref(n), ctypes.byref(p), ctypes.byref(ns)))
        return n.value, p.value, ns.value

    def get_contour(self):
        _, _, ns = self.sizes()
        lam = np.zeros(ns, np.complex128)
        w = np.zeros(ns, np.complex128)
        self._check(self.lib.mpsl_get_contour(self.h, ns, lam.ctypes.data, w.ctypes.data))
        return lam, w

    def get_scattering_matrix(self):
        _, p, _ = self.sizes()
        S = np.zeros((2 * p + 1, 2 * p + 1), np.complex128)
        self._check(self.lib.mpsl_get_scattering_matrix(self.h, p, S.ctypes.data))
        return S

    # -- matvec and its steps ---------------------------------------------
    def apply(self, prec, x):
        n, p, _ = self.sizes()
        dt = np.complex128 if prec == FP64 else np.complex64
        x = _carr(x, dt).reshape(-1)
        y = np.empty_like(x)
        self._check(self.lib.mpsl_apply(self.h, int(prec), x.ctypes.data, y.ctypes.data))
        return y.reshape(n, 2 * p + 1)

    def apply_dev(self, prec, x, y):
        return self._check(self.lib.mpsl_apply_dev(self.h, int(prec), _ptr(x), _ptr(y)))

    def apply_batch_dev(self, prec, nrhs, x, y):
        return self._check(self.lib.mpsl_apply_batch_dev(self.h, int(prec), int(nrhs), _ptr(x), _ptr(y)))

    def m2l_dev(self, prec, beta, alpha):
        return self._check(self.lib.mpsl_m2l_dev(self.h, int(prec), _ptr(beta), _ptr(alpha)))

    def m2l_dev_noalloc(self, prec, beta, alpha):
        """mpsl_m2l_dev without device allocation (fixed 64 MiB library scratch)."""
        return self._check(self.lib.mpsl_m2l_dev_noalloc(self.h, int(prec), _ptr(beta), _ptr(alpha)))

    def m2s_dev(self, prec, beta, spec):
        return self._check(self.lib.mpsl_m2s_dev(self.h, int(prec), _ptr(beta), _ptr(spec)))

    def reflect_dev(self, spec, src, sigma):
        s = None if src is None else np.ascontiguousarray(src, dtype=np.float64)
        self._keep = [s]
        return self._check(self.lib.mpsl_reflect_dev(self.h, _ptr(spec), None if s is None else s.ctypes.data,
                                                     _ptr(sigma)))

    def s2l_dev(self, prec, sigma, alpha):
        return self._check(self.lib.mpsl_s2l_dev(self.h, int(prec), _ptr(sigma), _ptr(alpha)))

    def sapply_dev(self, prec, x, alpha, y):
        return self._check(self.lib.mpsl_sapply_dev(self.h, int(prec), _ptr(x), _ptr(alpha), _ptr(y)))

    # -- preconditioner -------------------------------------------------------
    def set_preconditioner(self, kind, cluster_size=0):
        """PRECOND_NONE or PRECOND_CLUSTER with clusters of at most cluster_size (0: 160)."""
        return self._check(self.lib.mpsl_set_preconditioner(self.h, int(kind), int(cluster_size)))

    def precond_apply_dev(self, prec, x, y):
        return self._check(self.lib.mpsl_precond_apply_dev(self.h, int(prec), _ptr(x), _ptr(y)))

    def precond_info(self):
        nc, mx, m, rep = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        s = ctypes.c_double()
        self._check(self.lib.mpsl_get_precond_info(self.h, ctypes.byref(nc), ctypes.byref(mx), ctypes.byref(m),
                                                   ctypes.byref(rep), ctypes.byref(s)))
        return dict(n_clusters=nc.value, max_cluster=mx.value, block_dim=m.value, replaced=rep.value,
                    setup_seconds=s.value)

    # -- rhs, solve, field ----------------------------------------------------
    def rhs(self, src):
        n, p, _ = self.sizes()
        s = np.ascontiguousarray(src, dtype=np.float64)
        out = np.empty((n, 2 * p + 1), np.complex128)
        self._check(self.lib.mpsl_rhs(self.h, s.ctypes.data, out.ctypes.data))
        return out

    def solve(self, src, precision=FP64, tol=1e-10, maxiter=500, restart=0, inner_tol=0.0):
        n, p, _ = self.sizes()
        s = np.ascontiguousarray(np.atleast_2d(src), dtype=np.float64)
        nr = s.shape[0]
        out = np.empty((nr, n, 2 * p + 1), np.complex128)
        o = _lib.Opts(int(precision), float(tol), int(maxiter), int(restart), float(inner_tol))
        info = _lib.Info()
        rc = self._check(self.lib.mpsl_solve(self.h, nr, s.ctypes.data, ctypes.byref(o), out.ctypes.data,
                                             ctypes.byref(info)), allow=(-6,))
        hist = [info.history[i] for i in range(info.history_len)]
        meta = dict(status=rc, iterations=info.iterations, fp64_matvecs=info.fp64_matvecs,
                    refinements=info.refinements, rel_residual=info.rel_residual, seconds=info.seconds,
                    history=hist, precond_seconds=info.precond_seconds,
                    reorthogonalizations=info.reorthogonalizations)
        return (out[0] if nr == 1 else out), meta

    def eval_field(self, src, beta, rcv):
        """Total field at receivers rcv [R, 2] for one source (src [2], beta [N, P]:
        returns [R]) or several (src [n_rhs, 2], beta [n_rhs, N, P]: returns [n_rhs, R])."""
        s = np.ascontiguousarray(src, dtype=np.float64)
        nrhs = 1 if s.ndim == 1 else s.shape[0]
        b = _carr(beta)
        r = np.ascontiguousarray(rcv, dtype=np.float64)
        u = np.empty((nrhs, r.shape[0]), np.complex128)
        self._check(self.lib.mpsl_eval_field(self.h, int(nrhs), s.ctypes.data, b.ctypes.data, int(r.shape[0]),
                                             r.ctypes.data, u.ctypes.data), allow=(-8,))
        return u[0] if s.ndim == 1 else u

    def autotune(self, prec):
        return self._check(self.lib.mpsl_autotune(self.h, int(prec)))

    def set_tuning(self, prec, variant, chunks=0):
        """M2L launch variant (0 one lane per target, 1 output halves, 2 / 3 matrix cores
        with 16 / 32 targets per wave, p <= 16) and source chunks (0 = default)."""
        return self._check(self.lib.mpsl_set_tuning(self.h, int(prec), int(variant), int(chunks)))

    def get_tuning(self, prec):
        v, c, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(self.lib.mpsl_get_tuning(self.h, int(prec), ctypes.byref(v), ctypes.byref(c), ctypes.byref(ms)))
        return dict(variant=v.value, chunks=c.value, m2l_ms=ms.value)

    def set_far_field(self, method, tol=0.0):
        """Direct all-pairs or FMM far field (FAR_AUTO / FAR_DIRECT / FAR_FMM)."""
        return self._check(self.lib.mpsl_set_far_field(self.h, int(method), float(tol)))

    def somm_info(self):
        v = [ctypes.c_int() for _ in range(5)]
        self._check(self.lib.mpsl_get_somm_info(self.h, *[ctypes.byref(x) for x in v]))
        return dict(active=bool(v[0].value), tiles=v[1].value, intervals=v[2].value, coarse_nodes=v[3].value,
                    direct_nodes=v[4].value)

    def fmm_info(self, prec=FP64):
        a, lv, pl, pt = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        side, work, pairs = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.mpsl_get_fmm_info(self.h, int(prec), ctypes.byref(a), ctypes.byref(lv),
                                               ctypes.byref(side), ctypes.byref(pl), ctypes.byref(pt),
                                               ctypes.byref(pairs), ctypes.byref(work)))
        return dict(active=bool(a.value), levels=lv.value, leaf_side=side.value, p_leaf=pl.value,
                    p_top=pt.value, near_pairs=pairs.value, tree_cmac=work.value)

    def profile(self, enable=True):
        return self._check(self.lib.mpsl_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        ms, cnt = ctypes.c_double(), ctypes.c_int()
        self._check(self.lib.mpsl_profile_read(self.h, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value


PARTICLE_DISK, PARTICLE_STAR, PARTICLE_MATRIX = 0, 1, 2


class Server:
    """Continuous-batching solve server (mpsl_server_*)."""

    def __init__(self, device=0, hbm_budget=64 << 30, max_active=8):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        rc = self.lib.mpsl_server_create(ctypes.byref(h), int(device), int(hbm_budget), int(max_active))
        if rc != 0:
            raise MpslError(rc, "mpsl_server_create failed")
        self.h = h
        self._keep = {}

    def submit(self, k, d, particle, shape, kp, p, xy, rot, n_nodes, b, t_max, src, precision=FP64, tol=1e-10,
               maxiter=500, restart=0, inner_tol=0.0, S=None, r_enclose=0.0, n_bdry=0, contour=0, h_max=0.0,
               sommerfeld=SOMM_DIRECT, precond=PRECOND_NONE, cluster_size=0):
        """Queue one request; returns its ticket (arrays are copied by the library).
        contour 0 = count rule (n_nodes, b, t_max), 1 = span rule (b, t_max, h_max)."""
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        rot = None if rot is None else np.ascontiguousarray(rot, dtype=np.float64)
        Sa = None if S is None else _carr(S)
        r = _lib.Request()
        r.k1, r.k2, r.k3 = _c(k[0]), _c(k[1]), _c(k[2])
        r.d = float(d)
        r.particle = int(particle)
        for i, v in enumerate(list(shape) + [0.0] * (3 - len(shape))):
            r.shape[i] = float(v)
        r.kp = _c(kp)
        r.p = int(p)
        r.n_bdry = int(n_bdry)
        r.S = None if Sa is None else Sa.ctypes.data
        r.r_enclose = float(r_enclose)
        r.n = int(xy.shape[0])
        r.xy = xy.ctypes.data
        r.rot = None if rot is None else rot.ctypes.data
        r.n_nodes, r.b, r.t_max = int(n_nodes), float(b), float(t_max)
        r.src[0], r.src[1] = float(src[0]), float(src[1])
        r.opts = _lib.Opts(int(precision), float(tol), int(maxiter), int(restart), float(inner_tol))
        r.contour, r.h_max, r.sommerfeld = int(contour), float(h_max), int(sommerfeld)
        r.precond, r.cluster_size = int(precond), int(cluster_size)
        t = ctypes.c_uint64()
        rc = self.lib.mpsl_server_submit(self.h, ctypes.byref(r), ctypes.byref(t))
        if rc != 0:
            raise MpslError(rc, "mpsl_server_submit failed")
        return t.value

    @staticmethod
    def _result(res):
        out = dict(status=res.status, iterations=res.iterations, fp64_matvecs=res.fp64_matvecs,
                   refinements=res.refinements, rel_residual=res.rel_residual, t_submit=res.t_submit,
                   t_admit=res.t_admit, t_start=res.t_start, t_finish=res.t_finish, hbm_bytes=res.hbm_bytes,
                   error=(res.error or b"").decode(errors="replace"))
        if res.beta:
            P = 2 * res.p + 1
            arr = np.ctypeslib.as_array(ctypes.cast(res.beta, ctypes.POINTER(ctypes.c_double)),
                                        shape=(res.n * P * 2,))
            out["beta"] = arr.view(np.complex128).reshape(res.n, P).copy()
        return out

    def poll(self, ticket):
        res = _lib.Result()
        rc = self.lib.mpsl_server_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(res))
        if rc == 1:
            return None
        if rc != 0:
            raise MpslError(rc, "mpsl_server_poll failed")
        return self._result(res)

    def wait(self, ticket, timeout=-1.0, release=True):
        res = _lib.Result()
        rc = self.lib.mpsl_server_wait(self.h, ctypes.c_uint64(ticket), float(timeout), ctypes.byref(res))
        if rc == 1:
            return None
        if rc != 0:
            raise MpslError(rc, "mpsl_server_wait failed")
        out = self._result(res)
        if release:
            self.lib.mpsl_server_release(self.h, ctypes.c_uint64(ticket))
        return out

    def stats(self):
        q, a, c, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_uint64(), ctypes.c_size_t()
        self.lib.mpsl_server_stats(self.h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(c), ctypes.byref(b))
        return dict(queued=q.value, active=a.value, completed=c.value, bytes_in_use=b.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpsl_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
