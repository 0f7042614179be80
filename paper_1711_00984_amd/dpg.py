"""Thin ctypes binding of libdpg.so (include/dpg.h).

Argument marshalling only: every step of the integration runs in the HIP
kernels of the library.  PyTorch provides device memory (tensors) and
streams; pointers are passed as plain integers.  If the library is not
built, importing this module raises ImportError: there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpg.so")

H1, HCURL, HDIV, L2 = 0, 1, 2, 3
SPACES = {"H1": H1, "HCURL": HCURL, "HDIV": HDIV, "L2": L2}
FP64, FP32 = 0, 1
TRILINEAR, AFFINE, EXTRUDED = 0, 1, 2
KINDS = {"trilinear": TRILINEAR, "affine": AFFINE, "extruded": EXTRUDED}
GEOM_STRIDE = {TRILINEAR: 24, AFFINE: 12, EXTRUDED: 10}
PATH_AUTO, PATH_GENERAL, PATH_REDUCED = 0, 1, 2
PATHS = {"auto": PATH_AUTO, "general": PATH_GENERAL, "reduced": PATH_REDUCED}
P_MAX = 11

OK, PENDING, EINVAL, ENOMEM, EHIP, EJACOBIAN, EAGAIN, ENOTINIT, ENODEV = 0, 1, -1, -2, -3, -4, -5, -6, -7

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1711_00984_amd.build` "
                      "(or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)


class Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_elem", ctypes.c_int64), ("data", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("path", ctypes.c_int32), ("nq", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("w0", ctypes.c_double), ("w1", ctypes.c_double),
                ("status", ctypes.c_void_p)]


_vp, _i, _i64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
_i32, _u64 = ctypes.c_int32, ctypes.c_uint64


class ServeCfg(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", _i64), ("max_slots", _i64), ("max_inflight", _i32), ("max_queue", _i32),
                ("n_streams", _i32), ("max_merge", _i32), ("test_executor", _i32), ("test_fail_launch", _i32),
                ("test_bytes_per_s", _d), ("test_launch_s", _d)]


class Request(ctypes.Structure):
    _fields_ = [("space", _i32), ("p", _i32), ("dp", _i32), ("prec", _i32), ("path", _i32),
                ("geom_on_host", _i32), ("geom", Geometry), ("w0", _d), ("w1", _d),
                ("pdir", _i32 * 3), ("reserved", _i32)]


class Result(ctypes.Structure):
    _fields_ = [("status", _i32), ("space", _i32), ("p", _i32), ("prec", _i32), ("n_elem", _i64),
                ("packed_len", _i64), ("out", _vp), ("elem_status", _vp), ("t_submit", _d), ("t_admit", _d),
                ("t_done", _d)]


class ServeStats(ctypes.Structure):
    _fields_ = [(n, _i64) for n in ("submitted", "rejected", "admitted", "completed", "failed", "launches",
                                     "cancelled", "queued", "inflight", "elements", "budget_bytes", "admitted_bytes",
                                     "peak_admitted_bytes", "max_concurrent_launches")] + \
               [(n, _d) for n in ("bytes", "t_first_submit", "t_last_done", "lat_p50", "lat_p99", "lat_mean",
                                  "lat_max", "wait_p50", "wait_p99")]


_lib.dpg_opts_default.argtypes = [ctypes.POINTER(Opts)]
_lib.dpg_opts_default.restype = None
_lib.dpg_last_error.argtypes = []
_lib.dpg_last_error.restype = ctypes.c_char_p
_lib.dpg_tables_build.argtypes = [_i, _vp, ctypes.POINTER(_vp)]
_lib.dpg_tables_build.restype = _i
_lib.dpg_ctx_destroy.argtypes = [_vp]
_lib.dpg_ctx_destroy.restype = _i
_lib.dpg_gram_dim.argtypes = [_i, _i]
_lib.dpg_gram_dim.restype = _i64
_lib.dpg_gram_packed_len.argtypes = [_i, _i]
_lib.dpg_gram_packed_len.restype = _i64
_lib.dpg_general_flops.argtypes = [_i, _i]
_lib.dpg_general_flops.restype = _d
_lib.dpg_general_flops_trimmed.argtypes = [_i, _i]
_lib.dpg_general_flops_trimmed.restype = _d
_lib.dpg_gram_integrate.argtypes = [_vp, _i, _i, ctypes.POINTER(Geometry), _vp, ctypes.POINTER(Opts), _vp]
_lib.dpg_gram_integrate.restype = _i
_lib.dpg_gram_integrate_batched.argtypes = [_vp, _vp, _vp, ctypes.POINTER(Geometry), _vp, _vp,
                                            ctypes.POINTER(Opts), _vp]
_lib.dpg_gram_integrate_batched.restype = _i
_lib.dpg_gram_integrate_batched_host.argtypes = [_vp, _vp, _vp, ctypes.POINTER(Geometry), _vp, _vp,
                                                 ctypes.POINTER(Opts), _vp]
_lib.dpg_gram_integrate_batched_host.restype = _i
_lib.dpg_gram_integrate_batched_noalloc.argtypes = [_vp, _vp, _vp, ctypes.POINTER(Geometry), _vp, _vp,
                                                    ctypes.POINTER(Opts), _vp]
_lib.dpg_gram_integrate_batched_noalloc.restype = _i
_lib.dpg_noalloc_max_elements.argtypes = []
_lib.dpg_noalloc_max_elements.restype = _i64
_lib.dpg_autotune.argtypes = [_vp, _i, _i, ctypes.POINTER(Geometry), _vp, ctypes.POINTER(Opts), _vp,
                              ctypes.POINTER(ctypes.c_int)]
_lib.dpg_autotune.restype = _i
_lib.dpg_adjoint_coupling.argtypes = [_vp, _i, _vp, _i, _vp]
_lib.dpg_adjoint_coupling.restype = _i
_lib.dpg_replicate_blocks.argtypes = [_vp, _i64, _i64, _i, _vp, _vp, _i, _vp]
_lib.dpg_replicate_blocks.restype = _i
_lib.dpg_gram_dim_aniso.argtypes = [_i, _vp]
_lib.dpg_gram_dim_aniso.restype = _i64
_lib.dpg_aniso_route.argtypes = [_vp, _i, _vp, _vp]
_lib.dpg_aniso_route.restype = _i
_lib.dpg_gram_integrate_aniso.argtypes = [_vp, _i, _vp, ctypes.POINTER(Geometry), _vp, ctypes.POINTER(Opts), _vp]
_lib.dpg_gram_integrate_aniso.restype = _i
_lib.dpg_cholesky_packed.argtypes = [_vp, _i64, _i64, _vp, _vp, _i, _vp]
_lib.dpg_cholesky_packed.restype = _i
_lib.dpg_cholesky_solve_packed.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _i, _vp]
_lib.dpg_cholesky_solve_packed.restype = _i
_lib.dpg_tune_save.argtypes = [_vp, ctypes.c_char_p]
_lib.dpg_tune_save.restype = _i
_lib.dpg_tune_load.argtypes = [_vp, ctypes.c_char_p]
_lib.dpg_tune_load.restype = _i
_lib.dpg_tune_clear.argtypes = [_vp]
_lib.dpg_tune_clear.restype = _i
_lib.dpg_tune_lookup.argtypes = [_vp, _i, _i, _i, _i, _i64]
_lib.dpg_tune_lookup.restype = _i
_lib.dpg_batch_plans.argtypes = [_vp]
_lib.dpg_batch_plans.restype = _i
_lib.dpg_serve_cfg_default.argtypes = [ctypes.POINTER(ServeCfg)]
_lib.dpg_serve_cfg_default.restype = None
_lib.dpg_serve_create.argtypes = [_vp, ctypes.POINTER(ServeCfg), ctypes.POINTER(_vp)]
_lib.dpg_serve_create.restype = _i
_lib.dpg_serve_submit.argtypes = [_vp, ctypes.POINTER(Request), ctypes.POINTER(_u64)]
_lib.dpg_serve_submit.restype = _i
_lib.dpg_serve_submit_chunked.argtypes = [_vp, ctypes.POINTER(Request), _i64, ctypes.POINTER(_u64),
                                          ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
_lib.dpg_serve_submit_chunked.restype = _i
_lib.dpg_serve_poll.argtypes = [_vp, _u64, ctypes.POINTER(Result)]
_lib.dpg_serve_poll.restype = _i
_lib.dpg_serve_read.argtypes = [_vp, _u64, _vp, _i64, _i64, _vp]
_lib.dpg_serve_read.restype = _i
_lib.dpg_serve_read_status.argtypes = [_vp, _u64, _vp, _i64, _i64, _vp]
_lib.dpg_serve_read_status.restype = _i
_lib.dpg_serve_release.argtypes = [_vp, _u64]
_lib.dpg_serve_release.restype = _i
_lib.dpg_serve_stats_get.argtypes = [_vp, ctypes.POINTER(ServeStats)]
_lib.dpg_serve_stats_get.restype = _i
_lib.dpg_serve_stats_reset.argtypes = [_vp]
_lib.dpg_serve_stats_reset.restype = _i
_lib.dpg_serve_destroy.argtypes = [_vp]
_lib.dpg_serve_destroy.restype = _i
_lib.dpg_host_tables.argtypes = [_i, _i, _vp, _vp, _vp, _vp]
_lib.dpg_host_tables.restype = _i
_lib.dpg_host_ftable.argtypes = [_i, _i, _i, _vp]
_lib.dpg_host_ftable.restype = _i


class DpgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dpg error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise DpgError(rc, _lib.dpg_last_error().decode())
    return rc


def last_error():
    return _lib.dpg_last_error().decode()


def space_id(space):
    return SPACES[space] if isinstance(space, str) else int(space)


def gram_dim(space, p):
    return int(_lib.dpg_gram_dim(space_id(space), p))


def packed_len(space, p):
    return int(_lib.dpg_gram_packed_len(space_id(space), p))


def _orders(p):
    p = [int(x) for x in p]
    if len(p) != 3:
        raise ValueError("need three orders")
    return (ctypes.c_int32 * 3)(*p)


def _dense(t, what):
    if not (t.is_cuda and t.is_contiguous() and t.dtype in (torch.float64, torch.float32)):
        raise ValueError(f"{what} must be a contiguous float64 or float32 CUDA tensor")
    return FP64 if t.dtype == torch.float64 else FP32


def gram_dim_aniso(space, p):
    """Dimension of `space` with orders p = (p1, p2, p3) (dpg_gram_dim_aniso)."""
    return int(_lib.dpg_gram_dim_aniso(space_id(space), _orders(p)))


def general_flops(space, p):
    """Flops of one element's staged contraction, stage xi2 over every (i2, j2)."""
    return float(_lib.dpg_general_flops(space_id(space), p))


def general_flops_trimmed(space, p):
    """The same with stage xi2 of the diagonal pairs over i2 <= j2 only (what the kernels compute)."""
    return float(_lib.dpg_general_flops_trimmed(space_id(space), p))


def default_points(space, p):
    return p if space_id(space) == L2 else p + 1


def host_tables(L, kmax):
    """(zeta, w, chi[kmax+1, L], dchi[kmax+1, L]) as built by the library, float64 numpy."""
    import numpy as np
    z, w = np.zeros(L), np.zeros(L)
    c, d = np.zeros((kmax + 1) * L), np.zeros((kmax + 1) * L)
    _check(_lib.dpg_host_tables(L, kmax, z.ctypes.data, w.ctypes.data, c.ctypes.data, d.ctypes.data))
    return z, w, c.reshape(kmax + 1, L), d.reshape(kmax + 1, L)


def host_ftable(r, s, kmax):
    import numpy as np
    F = np.zeros((kmax + 1) * (kmax + 1))
    _check(_lib.dpg_host_ftable(r, s, kmax, F.ctypes.data))
    return F.reshape(kmax + 1, kmax + 1)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _geometry(geom, kind):
    if not (geom.is_cuda and geom.dtype == torch.float64 and geom.is_contiguous()):
        raise ValueError("geometry must be a contiguous float64 CUDA tensor")
    kind = KINDS.get(kind, kind)
    if kind not in GEOM_STRIDE:
        raise ValueError(f"unknown geometry kind {kind}")
    per = GEOM_STRIDE[kind]
    if geom.numel() % per:
        raise ValueError(f"geometry size {geom.numel()} is not a multiple of {per}")
    return Geometry(kind, 0, geom.numel() // per, geom.data_ptr())


def _opts(prec, path, nq, w0, w1, status):
    o = Opts()
    _lib.dpg_opts_default(ctypes.byref(o))
    o.prec = {"fp64": FP64, "fp32": FP32}.get(prec, prec)
    o.path = PATHS.get(path, path)
    o.nq = nq
    o.w0, o.w1 = float(w0), float(w1)
    if status is not None:
        if not (status.is_cuda and status.dtype == torch.int32):
            raise ValueError("status must be an int32 CUDA tensor")
        o.status = status.data_ptr()
    return o


class Context:
    """Device-resident 1D tables (dpg_tables_build).  tune_table: "default" keeps the
    tuning table the library loads (tune_gfx950.json beside libdpg.so), None starts
    from an empty table, a path replaces it by that file."""

    def __init__(self, p_max=P_MAX, stream=None, tune_table="default"):
        self._h = ctypes.c_void_p()
        _check(_lib.dpg_tables_build(p_max, _stream_ptr(stream), ctypes.byref(self._h)))
        self.p_max = p_max
        if tune_table != "default":
            _check(_lib.dpg_tune_clear(self._h))
            if tune_table is not None:
                _check(_lib.dpg_tune_load(self._h, str(tune_table).encode()))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _check(_lib.dpg_ctx_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gram(self, space, p, geom, kind="trilinear", out=None, prec="fp64", path="auto", nq=0,
             w0=1.0, w1=1.0, status=None, stream=None):
        """Packed Gram matrices of all elements of `geom` (dpg_gram_integrate).

        Returns `out`, a 1D tensor of E * packed_len(space, p) entries
        (float64 or float32), element e at [e * packed_len, (e+1) * packed_len).
        """
        g = _geometry(geom, kind)
        dt = torch.float64 if prec in ("fp64", FP64) else torch.float32
        m = packed_len(space, p)
        if m < 0:
            raise DpgError(EINVAL, f"invalid space/order ({space}, {p})")
        n = g.n_elem * m
        if out is None:
            out = torch.empty(n, dtype=dt, device=geom.device)
        elif out.dtype != dt or out.numel() < n or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or size")
        o = _opts(prec, path, nq, w0, w1, status)
        _check(_lib.dpg_gram_integrate(self._h, space_id(space), p, ctypes.byref(g), out.data_ptr(),
                                       ctypes.byref(o), _stream_ptr(stream)))
        return out

    def autotune(self, space, p, geom, kind="trilinear", out=None, prec="fp64", path="auto", w0=1.0, w1=1.0,
                 stream=None):
        """Time the work decompositions on these elements (dpg_autotune); returns the chosen
        slabs per workgroup.  Blocking."""
        g = _geometry(geom, kind)
        dt = torch.float64 if prec in ("fp64", FP64) else torch.float32
        n = g.n_elem * packed_len(space, p)
        if out is None:
            out = torch.empty(n, dtype=dt, device=geom.device)
        o = _opts(prec, path, 0, w0, w1, None)
        best = ctypes.c_int(0)
        _check(_lib.dpg_autotune(self._h, space_id(space), p, ctypes.byref(g), out.data_ptr(), ctypes.byref(o),
                                 _stream_ptr(stream), ctypes.byref(best)))
        return best.value

    def tune_save(self, path):
        _check(_lib.dpg_tune_save(self._h, str(path).encode()))

    def tune_load(self, path):
        _check(_lib.dpg_tune_load(self._h, str(path).encode()))

    def tune_lookup(self, space, p, prec="fp64", reduced=False, n_elem=1):
        return int(_lib.dpg_tune_lookup(self._h, space_id(space), p, 0 if prec in ("fp64", FP64) else 1,
                                        int(reduced), n_elem))

    def batch_plans(self):
        return int(_lib.dpg_batch_plans(self._h))

    def adjoint_coupling(self, p, prec="fp64", out=None, stream=None):
        """Coupling block C[dim W^p, dim V^p] of the adjoint graph inner product
        (dpg_adjoint_coupling), dense row-major on the device."""
        pr = {"fp64": FP64, "fp32": FP32}.get(prec, prec)
        shape = (gram_dim("H1", p), gram_dim("HDIV", p))
        if min(shape) < 1:
            raise DpgError(EINVAL, f"invalid order p={p}")
        if out is None:
            out = torch.empty(shape, dtype=torch.float64 if pr == FP64 else torch.float32, device="cuda")
        _check(_lib.dpg_adjoint_coupling(self._h, p, out.data_ptr(), pr, _stream_ptr(stream)))
        return out

    def replicate_blocks(self, src, n, copies, prec="fp64", out=None, stream=None):
        """Block-diagonal expansion of packed Grams of dimension n into dimension
        copies * n (dpg_replicate_blocks); src holds n_elem packed Grams."""
        pr = {"fp64": FP64, "fp32": FP32}.get(prec, prec)
        m = n * (n + 1) // 2
        if src.numel() % m:
            raise ValueError(f"source size {src.numel()} is not a multiple of {m}")
        ne = src.numel() // m
        cn = n * copies
        if out is None:
            out = torch.empty(ne * (cn * (cn + 1) // 2), dtype=src.dtype, device="cuda")
        _check(_lib.dpg_replicate_blocks(self._h, ne, n, copies, src.data_ptr(), out.data_ptr(), pr,
                                         _stream_ptr(stream)))
        return out

    def aniso_route(self, space, p, prec="fp64", nq=0, path="auto"):
        """Kernels dpg_gram_integrate_aniso takes: "uniform", "embedded" or "per-direction"."""
        o = _opts(prec, path, nq, 1.0, 1.0, None)
        r = _lib.dpg_aniso_route(self._h, space_id(space), _orders(p), ctypes.byref(o))
        _check(min(r, 0))
        return {0: "per-direction", 1: "uniform", 2: "embedded"}[r]

    def gram_aniso(self, space, p, geom, kind="trilinear", out=None, prec="fp64", nq=0, w0=1.0, w1=1.0,
                   status=None, stream=None, path="auto"):
        """Packed Grams of non-uniform orders p = (p1, p2, p3) (dpg_gram_integrate_aniso);
        path "general" forces the per-direction kernel."""
        g = _geometry(geom, kind)
        dt = torch.float64 if prec in ("fp64", FP64) else torch.float32
        nd = gram_dim_aniso(space, p)
        if nd < 0:
            raise DpgError(EINVAL, f"invalid space/orders ({space}, {tuple(p)})")
        n = g.n_elem * (nd * (nd + 1) // 2)
        if out is None:
            out = torch.empty(n, dtype=dt, device=geom.device)
        elif out.dtype != dt or out.numel() < n or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or size")
        o = _opts(prec, path, nq, w0, w1, status)
        _check(_lib.dpg_gram_integrate_aniso(self._h, space_id(space), _orders(p), ctypes.byref(g),
                                             out.data_ptr(), ctypes.byref(o), _stream_ptr(stream)))
        return out

    def cholesky(self, ap, n, info=None, stream=None):
        """Cholesky factors of packed Grams of dimension n, in place
        (dpg_cholesky_packed); ap is a float64 or float32 CUDA tensor holding
        n_elem packed Grams, info an optional int32 CUDA tensor [n_elem]."""
        pr = _dense(ap, "packed Grams")
        m = n * (n + 1) // 2
        if n < 1 or ap.numel() % m:
            raise ValueError(f"size {ap.numel()} is not a multiple of the packed length {m}")
        ne = ap.numel() // m
        if info is not None and not (info.is_cuda and info.dtype == torch.int32 and info.numel() == ne):
            raise ValueError("info must be an int32 CUDA tensor with one word per element")
        _check(_lib.dpg_cholesky_packed(self._h, ne, n, ap.data_ptr(), None if info is None else info.data_ptr(),
                                        pr, _stream_ptr(stream)))
        return ap

    def cholesky_solve(self, up, n, b, stream=None):
        """b <- G^{-1} b per element (dpg_cholesky_solve_packed); up holds the
        packed factors, b the n_elem column-major n x nrhs blocks (a tensor of
        shape [n_elem, nrhs, n] is that layout)."""
        pr = _dense(up, "packed factors")
        _dense(b, "right-hand sides")
        m = n * (n + 1) // 2
        if n < 1 or up.numel() % m:
            raise ValueError(f"size {up.numel()} is not a multiple of the packed length {m}")
        ne = up.numel() // m
        if b.dtype != up.dtype or (ne and b.numel() % (ne * n)):
            raise ValueError("right-hand sides must match the factor's dtype and hold n x nrhs per element")
        nrhs = b.numel() // (ne * n) if ne else 1
        _check(_lib.dpg_cholesky_solve_packed(self._h, ne, n, up.data_ptr(), nrhs, b.data_ptr(), pr,
                                              _stream_ptr(stream)))
        return b

    def gram_batched(self, space, p, geom, out_offset, out, kind="trilinear", prec="fp64", path="auto",
                     w0=1.0, w1=1.0, status=None, stream=None):
        """Uneven batch (dpg_gram_integrate_batched): int8 space/p, int64 offsets, all on device."""
        g = _geometry(geom, kind)
        for t, dt in ((space, torch.int8), (p, torch.int8), (out_offset, torch.int64)):
            if not (t.is_cuda and t.dtype == dt and t.numel() == g.n_elem):
                raise ValueError("space/p must be int8 and out_offset int64 CUDA tensors of length n_elem")
        o = _opts(prec, path, 0, w0, w1, status)
        _check(_lib.dpg_gram_integrate_batched(self._h, space.data_ptr(), p.data_ptr(), ctypes.byref(g),
                                               out_offset.data_ptr(), out.data_ptr(), ctypes.byref(o),
                                               _stream_ptr(stream)))
        return out

    def gram_batched_host(self, space, p, geom, out_offset, out, kind="trilinear", prec="fp64", path="auto",
                          w0=1.0, w1=1.0, status=None, stream=None):
        """Uneven batch with space/p as host int8 numpy arrays (dpg_gram_integrate_batched_host):
        no read back from the device, no synchronisation on replays."""
        import numpy as np
        g = _geometry(geom, kind)
        for t in (space, p):
            if not (isinstance(t, np.ndarray) and t.dtype == np.int8 and t.flags.c_contiguous and t.size == g.n_elem):
                raise ValueError("space/p must be contiguous int8 numpy arrays of length n_elem")
        if not (out_offset.is_cuda and out_offset.dtype == torch.int64 and out_offset.numel() == g.n_elem):
            raise ValueError("out_offset must be an int64 CUDA tensor of length n_elem")
        o = _opts(prec, path, 0, w0, w1, status)
        _check(_lib.dpg_gram_integrate_batched_host(self._h, space.ctypes.data, p.ctypes.data, ctypes.byref(g),
                                                    out_offset.data_ptr(), out.data_ptr(), ctypes.byref(o),
                                                    _stream_ptr(stream)))
        return out

    def gram_batched_noalloc(self, space, p, geom, out_offset, out, kind="trilinear", prec="fp64", path="auto",
                             w0=1.0, w1=1.0, status=None, stream=None):
        """The uneven batch without allocation (dpg_gram_integrate_batched_noalloc);
        arguments as gram_batched."""
        g = _geometry(geom, kind)
        for t, dt in ((space, torch.int8), (p, torch.int8), (out_offset, torch.int64)):
            if not (t.is_cuda and t.dtype == dt and t.numel() == g.n_elem):
                raise ValueError("space/p must be int8 and out_offset int64 CUDA tensors of length n_elem")
        o = _opts(prec, path, 0, w0, w1, status)
        _check(_lib.dpg_gram_integrate_batched_noalloc(self._h, space.data_ptr(), p.data_ptr(), ctypes.byref(g),
                                                       out_offset.data_ptr(), out.data_ptr(), ctypes.byref(o),
                                                       _stream_ptr(stream)))
        return out


def noalloc_max_elements():
    return int(_lib.dpg_noalloc_max_elements())


class Server:
    """Serving loop (dpg_serve_*): submit requests, poll results, release them.

    ctx may be None only with test_executor=True (the scheduler's timing stub,
    which computes nothing).  Results stay in the server's device memory until
    release(); read() copies elements of a result into a tensor.
    """

    def __init__(self, ctx=None, mem_budget_bytes=1 << 30, max_slots=1 << 18, max_inflight=64, max_queue=4096,
                 n_streams=4, max_merge=32, test_executor=False, test_fail_launch=0, test_bytes_per_s=1e12,
                 test_launch_s=0.0):
        c = ServeCfg()
        _lib.dpg_serve_cfg_default(ctypes.byref(c))
        c.mem_budget_bytes, c.max_slots = int(mem_budget_bytes), int(max_slots)
        c.max_inflight, c.max_queue, c.n_streams, c.max_merge = max_inflight, max_queue, n_streams, max_merge
        c.test_executor, c.test_fail_launch = int(bool(test_executor)), int(test_fail_launch)
        c.test_bytes_per_s, c.test_launch_s = float(test_bytes_per_s), float(test_launch_s)
        self._h = ctypes.c_void_p()
        self._ctx = ctx   # keeps the tables alive while the server runs
        _check(_lib.dpg_serve_create(ctx.handle if ctx is not None else None, ctypes.byref(c),
                                     ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _check(_lib.dpg_serve_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, space, p, geom, dp=0, kind="trilinear", prec="fp64", path="auto", w0=1.0, w1=1.0):
        """Queue one request; returns its ticket.  p: the trial order, or a triple
        (p1, p2, p3) of non-uniform trial orders.  geom: float64 numpy array or
        tensor (host or device) of n_elem * 24 (trilinear), * 12 (affine) or
        * 10 (extruded) values, copied before this returns.  Raises DpgError (code EAGAIN when
        the queue or the element slots are full)."""
        r = self._request(space, p, geom, dp, kind, prec, path, w0, w1)
        t = _u64(0)
        _check(_lib.dpg_serve_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def submit_chunked(self, space, p, geom, dp=0, kind="trilinear", prec="fp64", path="auto", w0=1.0, w1=1.0,
                       max_chunk_bytes=0):
        """Queue a request of any size cut into element chunks (dpg_serve_submit_chunked);
        returns (first ticket, number of chunks, elements per chunk).  Chunk k has the
        ticket first + k and holds elements [k * chunk_elems, ...)."""
        r = self._request(space, p, geom, dp, kind, prec, path, w0, w1)
        t, k, ce = _u64(0), _i64(0), _i64(0)
        _check(_lib.dpg_serve_submit_chunked(self._h, ctypes.byref(r), int(max_chunk_bytes), ctypes.byref(t),
                                             ctypes.byref(k), ctypes.byref(ce)))
        return t.value, k.value, ce.value

    def _request(self, space, p, geom, dp, kind, prec, path, w0, w1):
        kind = KINDS.get(kind, kind)
        per = GEOM_STRIDE.get(kind, 24)
        if isinstance(geom, torch.Tensor):
            if geom.dtype != torch.float64 or not geom.is_contiguous():
                raise ValueError("geometry must be a contiguous float64 tensor")
            ptr, numel, on_host = geom.data_ptr(), geom.numel(), int(not geom.is_cuda)
        else:
            import numpy as np
            if not (isinstance(geom, np.ndarray) and geom.dtype == np.float64 and geom.flags.c_contiguous):
                raise ValueError("geometry must be a C-contiguous float64 array")
            ptr, numel, on_host = geom.ctypes.data, geom.size, 1
        if numel % per:
            raise ValueError(f"geometry size {numel} is not a multiple of {per}")
        pdir = (0, 0, 0)
        if hasattr(p, "__len__"):
            pdir, p = tuple(int(x) for x in p), 0
            if len(pdir) != 3:
                raise ValueError("non-uniform orders need three values")
        return Request(space_id(space), int(p), int(dp), {"fp64": FP64, "fp32": FP32}.get(prec, prec),
                       PATHS.get(path, path), on_host, Geometry(kind, 0, numel // per, ptr), float(w0), float(w1),
                       (_i32 * 3)(*pdir), 0)

    def poll(self, ticket):
        """None while pending; else a dict with status, space, p (Gram order), prec,
        n_elem, packed_len, out / elem_status (device addresses) and the
        timestamps t_submit, t_admit, t_done (seconds since the server started)."""
        r = Result()
        rc = _lib.dpg_serve_poll(self._h, ticket, ctypes.byref(r))
        if rc == PENDING:
            return None
        if rc != OK and r.n_elem == 0:
            raise DpgError(rc, last_error())
        return {f: getattr(r, f) for f, _ in Result._fields_}

    def read(self, ticket, first=0, count=None, out=None, stream=None):
        """Copy elements [first, first+count) of a finished result into out (a
        device tensor by default), asynchronously on stream."""
        r = self.poll(ticket)
        if r is None:
            raise DpgError(EINVAL, f"request {ticket} has not finished")
        count = r["n_elem"] - first if count is None else count
        dt = torch.float64 if r["prec"] == FP64 else torch.float32
        n = count * r["packed_len"]
        if out is None:
            out = torch.empty(n, dtype=dt, device="cuda")
        elif out.dtype != dt or out.numel() < n or not out.is_contiguous():
            raise ValueError("out has the wrong dtype or size")
        _check(_lib.dpg_serve_read(self._h, ticket, out.data_ptr(), first, count, _stream_ptr(stream)))
        return out

    def read_status(self, ticket, first=0, count=None, stream=None):
        """Status words (int32 device tensor) of elements [first, first+count)."""
        r = self.poll(ticket)
        if r is None:
            raise DpgError(EINVAL, f"request {ticket} has not finished")
        count = r["n_elem"] - first if count is None else count
        out = torch.empty(count, dtype=torch.int32, device="cuda")
        _check(_lib.dpg_serve_read_status(self._h, ticket, out.data_ptr(), first, count, _stream_ptr(stream)))
        return out

    def release(self, ticket):
        _check(_lib.dpg_serve_release(self._h, ticket))

    def stats(self):
        s = ServeStats()
        _check(_lib.dpg_serve_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServeStats._fields_}

    def reset_stats(self):
        _check(_lib.dpg_serve_stats_reset(self._h))


def exported_symbols():
    """Names declared in include/dpg.h that the loaded library must export."""
    return [n for n in dir(_lib) if n.startswith("dpg_")]
