"""Python binding of the one-GPU annotated-launch runtime (``liblt.so``).

Argument marshalling only: every planning step runs in the C++ runtime and
every kernel in hand-written HIP.  The functions keep the C-ABI names
(``lt_context_create``, ``lt_array_create``, ``lt_launch``, ``lt_sync``...)
and raise ``LtError`` on a non-zero status.  If the library has not been
built, importing this package raises: there is no fallback.

A small convenience layer (``Context``, ``Array``) sits on top for tests and
the benchmark.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblt.so")

LT_OK = 0
LT_ERR_INVALID = -1
LT_ERR_PARSE = -2
LT_ERR_BUDGET = -3
LT_ERR_OOM = -4
LT_ERR_DEVICE = -5
LT_ERR_TIMEOUT = -6
LT_ERR_UNSUPPORTED = -7
LT_ERR_COMPILE = -8
_ERRNAMES = {-1: "LT_ERR_INVALID", -2: "LT_ERR_PARSE", -3: "LT_ERR_BUDGET", -4: "LT_ERR_OOM",
             -5: "LT_ERR_DEVICE", -6: "LT_ERR_TIMEOUT", -7: "LT_ERR_UNSUPPORTED", -8: "LT_ERR_COMPILE"}
LT_PARAM_CONST = 1

LT_F32, LT_I32, LT_F64, LT_I64, LT_U8 = 0, 1, 2, 3, 4
DTYPES = {LT_F32: np.float32, LT_I32: np.int32, LT_F64: np.float64, LT_I64: np.int64, LT_U8: np.uint8}
NP2LT = {np.dtype(v): k for k, v in DTYPES.items()}

LT_EXEC_PLAIN, LT_EXEC_GROUPED = 0, 1
LT_EVICT_NEXT_USE = 0
LT_EVICT_LRU = 1
LT_ORDER_ROWMAJOR, LT_ORDER_SERPENTINE, LT_ORDER_BANDS = 0, 1, 2
LT_DIST_BLOCK, LT_DIST_CUSTOM, LT_DIST_STENCIL = 0, 1, 2
LT_ARG_ARRAY, LT_ARG_INT, LT_ARG_FLOAT = 0, 1, 2
LT_TASK_EXEC, LT_TASK_COMBINE, LT_TASK_IO = 0, 1, 2


class lt_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("n_compute_streams", C.c_int32), ("exec_mode", C.c_int32),
                ("dry_run", C.c_int32), ("device_budget_bytes", C.c_uint64),
                ("stage_threshold_bytes", C.c_uint64), ("device_arena", C.c_void_p),
                ("arena_bytes", C.c_uint64), ("trace", C.c_int32), ("sb_order", C.c_int32),
                ("drain_workgroups", C.c_int32), ("batch_flush_tasks", C.c_int32), ("drain_vectors", C.c_int32),
                ("evict_policy", C.c_int32), ("sb_band", C.c_int32), ("d2h_kernel", C.c_int32),
                ("host_budget_bytes", C.c_uint64),
                ("spill_dir", C.c_char_p), ("drain_tile", C.c_int64)]


class lt_box(C.Structure):
    _fields_ = [("lo", C.c_int64 * 3), ("hi", C.c_int64 * 3)]


class lt_dist(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nboxes", C.c_int32), ("chunk", C.c_int64 * 3),
                ("boxes", C.POINTER(lt_box)), ("halo", C.c_int64 * 3)]


class lt_arg(C.Structure):
    _fields_ = [("name", C.c_char_p), ("kind", C.c_int32), ("pad", C.c_int32), ("array", C.c_void_p),
                ("i", C.c_int64), ("f", C.c_double)]


class lt_task_info(C.Structure):
    _fields_ = [("id", C.c_uint64), ("launch", C.c_uint64), ("kind", C.c_int32), ("stream", C.c_int32),
                ("ndeps", C.c_int32), ("nregions", C.c_int32), ("sb_lo", C.c_int64 * 3),
                ("sb_hi", C.c_int64 * 3)]


class lt_param(C.Structure):
    _fields_ = [("name", C.c_char_p), ("kind", C.c_int32), ("dtype", C.c_int32), ("ndim", C.c_int32),
                ("flags", C.c_int32)]


class lt_rtc_stats(C.Structure):
    _fields_ = [("compiles", C.c_uint64), ("loads", C.c_uint64), ("compile_seconds", C.c_double)]


class lt_span(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("stream", C.c_int32), ("pad", C.c_int32), ("start_ms", C.c_double),
                ("end_ms", C.c_double)]


class lt_region_info(C.Structure):
    _fields_ = [("arg", C.c_int32), ("mode", C.c_int32), ("op", C.c_int32), ("resolved", C.c_int32),
                ("array_id", C.c_uint64), ("lo", C.c_int64 * 3), ("hi", C.c_int64 * 3)]


class lt_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "launches", "tasks", "dispatches", "bytes_h2d", "bytes_d2h", "bytes_d2d", "copies_h2d",
        "copies_d2h", "copies_d2d", "evictions_clean", "evictions_dirty", "resident_bytes",
        "peak_resident_bytes", "staged_peak_bytes", "throttle_waits", "assembled_regions",
        "direct_regions")] + [("plan_seconds", C.c_double), ("halo_copies", C.c_uint64),
                              ("bytes_disk_write", C.c_uint64), ("bytes_disk_read", C.c_uint64),
                              ("host_spill_bytes", C.c_uint64)]


class lt_trace_rec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("stream", C.c_int32), ("task", C.c_uint64), ("chunk", C.c_uint64),
                ("bytes", C.c_uint64), ("offset", C.c_uint64), ("resident", C.c_uint64)]


class lt_kernel_prof(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("dispatches", C.c_uint64), ("total_ms", C.c_double),
                ("max_ms", C.c_double)]


class lt_server_config(C.Structure):
    _fields_ = [("max_active", C.c_int32), ("keep_resident", C.c_int32), ("admit_bytes", C.c_uint64),
                ("chunk_rows", C.c_int64), ("gemm_tile", C.c_int64), ("lookahead", C.c_int32),
                ("max_bypass", C.c_int32), ("reserved", C.c_int32 * 2)]


class lt_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dataset", C.c_int32), ("size", C.c_int64), ("d", C.c_int64),
                ("K", C.c_int64), ("sweeps", C.c_int32), ("pad", C.c_int32), ("in0", C.c_void_p),
                ("in1", C.c_void_p), ("out", C.c_void_p)]


class lt_completion(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("kind", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("footprint", C.c_uint64),
                ("cache_hit", C.c_int32), ("pad", C.c_int32)]


LT_REQ_JACOBI, LT_REQ_KMEANS, LT_REQ_GEMM = 0, 1, 2

# numpy mirror of lt_arg, for building argument tables without Python loops
ARG_DTYPE = np.dtype([("name", np.uint64), ("kind", np.int32), ("pad", np.int32), ("array", np.uint64),
                      ("i", np.int64), ("f", np.float64)])


class LtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_ERRNAMES.get(status, str(status)), msg))
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError("liblt.so is not built (run __graft_entry__.build() or "
                      "python paper_2202_05549_amd/build.py); there is no fallback path")

_lib = C.CDLL(LIB_PATH)

# (name, restype, argtypes)
_P = C.c_void_p
_SIGS = [
    ("lt_config_init", None, [C.POINTER(lt_config)]),
    ("lt_context_create", C.c_int32, [C.POINTER(lt_config), C.POINTER(_P)]),
    ("lt_context_destroy", C.c_int32, [_P]),
    ("lt_last_error", C.c_char_p, [_P]),
    ("lt_context_configure", C.c_int32, [_P, C.POINTER(lt_config)]),
    ("lt_array_create", C.c_int32, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(lt_dist),
                                    C.POINTER(_P)]),
    ("lt_array_create_host", C.c_int32, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                         C.POINTER(lt_dist), _P, C.POINTER(_P)]),
    ("lt_array_destroy", C.c_int32, [_P, _P]),
    ("lt_array_write", C.c_int32, [_P, _P, _P]),
    ("lt_array_read", C.c_int32, [_P, _P, _P]),
    ("lt_array_fill", C.c_int32, [_P, _P, _P]),
    ("lt_array_write_device", C.c_int32, [_P, _P, _P]),
    ("lt_array_read_device", C.c_int32, [_P, _P, _P]),
    ("lt_array_id", C.c_uint64, [_P]),
    ("lt_host_alloc", C.c_int32, [_P, C.c_uint64, C.POINTER(_P)]),
    ("lt_host_free", C.c_int32, [_P, _P]),
    ("lt_kernel_get", C.c_int32, [_P, C.c_char_p, C.POINTER(_P)]),
    ("lt_kernel_define", C.c_int32, [_P, C.c_char_p, C.c_char_p, C.POINTER(_P)]),
    ("lt_kernel_tune", C.c_int32, [_P, _P, C.c_int32]),
    ("lt_kernel_define_source", C.c_int32, [_P, C.c_char_p, C.c_char_p, C.POINTER(lt_param), C.c_int32,
                                            C.c_char_p, C.POINTER(_P)]),
    ("lt_rtc_stats_get", C.c_int32, [C.POINTER(lt_rtc_stats)]),
    ("lt_launch", C.c_int32, [_P, _P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                              C.POINTER(C.c_int64), C.c_char_p, C.POINTER(lt_arg), C.c_int32,
                              C.POINTER(C.c_uint64)]),
    ("lt_launch_many", C.c_int32, [_P, C.POINTER(_P), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_char_p, C.c_void_p, C.c_int32, C.c_void_p]),
    ("lt_sync", C.c_int32, [_P]),
    ("lt_batch_begin", C.c_int32, [_P]),
    ("lt_batch_end", C.c_int32, [_P]),
    ("lt_batch_end_noalloc", C.c_int32, [_P]),
    ("lt_graph_begin", C.c_int32, [_P]),
    ("lt_graph_end", C.c_int32, [_P, C.POINTER(_P)]),
    ("lt_graph_launch", C.c_int32, [_P, _P]),
    ("lt_graph_destroy", C.c_int32, [_P, _P]),
    ("lt_wait", C.c_int32, [_P, C.c_uint64]),
    ("lt_plan_tasks", C.c_int32, [_P, C.c_uint64, C.POINTER(lt_task_info), C.c_int32, C.POINTER(C.c_int32)]),
    ("lt_plan_regions", C.c_int32, [_P, C.c_uint64, C.POINTER(lt_region_info), C.c_int32,
                                    C.POINTER(C.c_int32)]),
    ("lt_plan_deps", C.c_int32, [_P, C.c_uint64, C.POINTER(C.c_uint64), C.c_int32, C.POINTER(C.c_int32)]),
    ("lt_stats_get", C.c_int32, [_P, C.POINTER(lt_stats)]),
    ("lt_stats_reset", C.c_int32, [_P]),
    ("lt_trace_get", C.c_int32, [_P, C.POINTER(lt_trace_rec), C.c_uint64, C.POINTER(C.c_uint64)]),
    ("lt_trace_clear", C.c_int32, [_P]),
    ("lt_server_create", C.c_int32, [_P, C.POINTER(lt_server_config), C.POINTER(_P)]),
    ("lt_server_submit", C.c_int32, [_P, C.POINTER(lt_request), C.POINTER(C.c_uint64)]),
    ("lt_server_poll", C.c_int32, [_P, C.POINTER(lt_completion), C.c_int32, C.POINTER(C.c_int32)]),
    ("lt_server_drain", C.c_int32, [_P, C.POINTER(lt_completion), C.c_int32, C.POINTER(C.c_int32)]),
    ("lt_server_destroy", C.c_int32, [_P]),
    ("lt_now", C.c_double, []),
    ("lt_profile_enable", C.c_int32, [_P, C.c_int32]),
    ("lt_profile_get", C.c_int32, [_P, C.POINTER(lt_kernel_prof), C.c_int32, C.POINTER(C.c_int32)]),
    ("lt_profile_reset", C.c_int32, [_P]),
    ("lt_profile_spans", C.c_int32, [_P, C.POINTER(lt_span), C.c_uint64, C.POINTER(C.c_uint64)]),
]

for _name, _res, _args in _SIGS:
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


def exported_symbols():
    """Names the binding resolves in liblt.so."""
    return [s[0] for s in _SIGS]


def check(ctx, st):
    if st != LT_OK:
        msg = lt_last_error(ctx)
        raise LtError(st, msg.decode() if msg else "")
    return st


def _i64(vals, n=3, fill=0):
    arr = (C.c_int64 * n)()
    for i in range(n):
        arr[i] = int(vals[i]) if i < len(vals) else fill
    return arr


def make_dist(chunk=None, boxes=None, halo=None):
    """BLOCK distribution with per-axis chunk extents (0 = whole axis), a
    STENCIL distribution (the same cores stored with ``halo`` extra elements
    per side and axis), or a CUSTOM distribution from half-open boxes
    [(lo, hi), ...]."""
    d = lt_dist()
    if boxes is not None:
        arr = (lt_box * len(boxes))()
        for i, (lo, hi) in enumerate(boxes):
            for a in range(3):
                arr[i].lo[a] = lo[a] if a < len(lo) else 0
                arr[i].hi[a] = hi[a] if a < len(hi) else 1
        d.kind = LT_DIST_CUSTOM
        d.nboxes = len(boxes)
        d.boxes = arr
        d._keep = arr
    else:
        d.kind = LT_DIST_BLOCK if halo is None else LT_DIST_STENCIL
        for a in range(3):
            d.chunk[a] = (chunk[a] if chunk is not None and a < len(chunk) else 0)
            d.halo[a] = (halo[a] if halo is not None and a < len(halo) else 0)
    return d


class Array:
    """An lt_array handle with its numpy dtype and shape."""

    def __init__(self, ctx: "Context", handle, dtype, shape, host=None):
        self.ctx = ctx
        self.h = handle
        self.dtype = np.dtype(dtype)
        self.shape = tuple(int(s) for s in shape)
        self.host = host  # keeps a host-backed buffer alive

    @property
    def id(self):
        return int(lt_array_id(self.h))

    @property
    def nbytes(self):
        return int(np.prod(self.shape)) * self.dtype.itemsize

    def write(self, a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=self.dtype)
        assert a.shape == self.shape
        check(self.ctx.h, lt_array_write(self.ctx.h, self.h, a.ctypes.data))

    def read(self) -> np.ndarray:
        out = np.empty(self.shape, self.dtype)
        check(self.ctx.h, lt_array_read(self.ctx.h, self.h, out.ctypes.data))
        return out

    def fill(self, value):
        v = np.array(value, dtype=self.dtype)
        check(self.ctx.h, lt_array_fill(self.ctx.h, self.h, v.ctypes.data))

    def write_device(self, ptr: int):
        check(self.ctx.h, lt_array_write_device(self.ctx.h, self.h, C.c_void_p(ptr)))

    def read_device(self, ptr: int):
        check(self.ctx.h, lt_array_read_device(self.ctx.h, self.h, C.c_void_p(ptr)))

    def destroy(self):
        if self.h:
            check(self.ctx.h, lt_array_destroy(self.ctx.h, self.h))
            self.h = None


class Context:
    """An lt_context with keyword configuration (see lt_config in lt.h)."""

    _FIELDS = None

    @classmethod
    def _check_keys(cls, cfg):
        # ctypes would store an unknown (e.g. misspelt) key as a plain Python
        # attribute and the library would never see it
        if cls._FIELDS is None:
            cls._FIELDS = {f[0] for f in lt_config._fields_} - {"reserved"}
        bad = sorted(set(cfg) - cls._FIELDS)
        if bad:
            raise TypeError("unknown lt_config field(s): %s" % ", ".join(bad))

    def __init__(self, **cfg):
        self._check_keys(cfg)
        c = lt_config()
        lt_config_init(C.byref(c))
        for k, v in cfg.items():
            if k == "device_arena":
                v = C.c_void_p(v)
            if k == "spill_dir" and isinstance(v, str):
                v = v.encode()
            setattr(c, k, v)
        h = _P()
        st = lt_context_create(C.byref(c), C.byref(h))
        if st != LT_OK:
            raise LtError(st, lt_last_error(None).decode())
        self.h = h
        self.cfg = c
        self._kernels = {}

    def configure(self, **cfg):
        """Change tunable fields (exec_mode, stage_threshold_bytes, sb_order,
        sb_band, drain_workgroups, batch_flush_tasks, drain_vectors, drain_tile,
        evict_policy, trace) of the live context."""
        self._check_keys(cfg)
        for k, v in cfg.items():
            setattr(self.cfg, k, v)
        check(self.h, lt_context_configure(self.h, C.byref(self.cfg)))

    def close(self):
        if self.h:
            st = lt_context_destroy(self.h)
            self.h = None
            if st != LT_OK:
                raise LtError(st, "context destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lt_context_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def array(self, shape, dtype=np.float32, chunk=None, boxes=None, halo=None) -> Array:
        shape = tuple(shape)
        dt = NP2LT[np.dtype(dtype)]
        d = make_dist(chunk, boxes, halo)
        h = _P()
        check(self.h, lt_array_create(self.h, dt, len(shape), _i64(shape, len(shape)), C.byref(d), C.byref(h)))
        return Array(self, h, dtype, shape)

    def array_host(self, buf: np.ndarray, chunk=None, boxes=None, halo=None) -> Array:
        """Host-backed array over ``buf`` (kept alive by the handle)."""
        assert buf.flags["C_CONTIGUOUS"]
        dt = NP2LT[buf.dtype]
        d = make_dist(chunk, boxes, halo)
        h = _P()
        check(self.h, lt_array_create_host(self.h, dt, buf.ndim, _i64(buf.shape, buf.ndim), C.byref(d),
                                           C.c_void_p(buf.ctypes.data), C.byref(h)))
        return Array(self, h, buf.dtype, buf.shape, host=buf)

    def pinned(self, shape, dtype=np.float32) -> np.ndarray:
        """A numpy view of pinned host memory owned by the context."""
        nbytes = int(np.prod(shape)) * np.dtype(dtype).itemsize
        p = _P()
        check(self.h, lt_host_alloc(self.h, nbytes, C.byref(p)))
        buf = (C.c_char * nbytes).from_address(p.value)
        return np.frombuffer(buf, dtype=dtype).reshape(shape)

    def kernel(self, name, annotation=None):
        key = (name, annotation)
        if key not in self._kernels:
            k = _P()
            if annotation is None:
                check(self.h, lt_kernel_get(self.h, name.encode(), C.byref(k)))
            else:
                check(self.h, lt_kernel_define(self.h, name.encode(), annotation.encode(), C.byref(k)))
            self._kernels[key] = k
        return self._kernels[key]

    def define_source(self, name, source, function, params, annotation):
        """lt_kernel_define_source: a user __device__ function compiled at run
        time, registered under ``name`` for ``launch``.  ``params``: in order,
        ``(name, "int")``, ``(name, "float")`` (prefix ``"const "`` to bake
        the value into the code), or ``(name, numpy dtype, ndim)`` for an
        array (an optional fourth entry ``"const"`` is rejected by the
        runtime, as for any array)."""
        P = (lt_param * max(1, len(params)))()
        keep = []
        for i, p in enumerate(params):
            nm = p[0].encode()
            keep.append(nm)
            P[i].name = nm
            if isinstance(p[1], str):
                kind = p[1].split()
                P[i].kind = {"int": LT_ARG_INT, "float": LT_ARG_FLOAT}[kind[-1]]
                P[i].flags = LT_PARAM_CONST if kind[0] == "const" else 0
            else:
                P[i].kind = LT_ARG_ARRAY
                P[i].dtype = NP2LT[np.dtype(p[1])]
                P[i].ndim = int(p[2])
                P[i].flags = LT_PARAM_CONST if len(p) > 3 and p[3] == "const" else 0
        k = _P()
        check(self.h, lt_kernel_define_source(self.h, source.encode(), function.encode(), P, len(params),
                                              annotation.encode(), C.byref(k)))
        self._kernels[(name, None)] = k
        return k

    @staticmethod
    def rtc_stats():
        s = lt_rtc_stats()
        check(None, lt_rtc_stats_get(C.byref(s)))
        return {"compiles": int(s.compiles), "loads": int(s.loads), "compile_seconds": float(s.compile_seconds)}

    def tune(self, name, variant, kernel_annotation=None):
        check(self.h, lt_kernel_tune(self.h, self.kernel(name, kernel_annotation), int(variant)))

    def launch(self, name, grid, block, superblock=None, args=(), annotation=None, kernel_annotation=None):
        """Launch built-in ``name``.  ``args`` is a sequence of Array, int or
        float (positional), or (name, value) pairs."""
        k = self.kernel(name, kernel_annotation)
        nd = len(grid)
        A = (lt_arg * max(1, len(args)))()
        for i, a in enumerate(args):
            nm = None
            if isinstance(a, tuple):
                nm, a = a
            A[i].name = nm.encode() if nm else None
            if isinstance(a, Array):
                A[i].kind = LT_ARG_ARRAY
                A[i].array = a.h
            elif isinstance(a, (int, np.integer)):
                A[i].kind = LT_ARG_INT
                A[i].i = int(a)
            else:
                A[i].kind = LT_ARG_FLOAT
                A[i].f = float(a)
        lid = C.c_uint64()
        sb = superblock if superblock is not None else [0] * nd
        check(self.h, lt_launch(self.h, k, nd, _i64(grid, nd), _i64(block, nd), _i64(sb, nd),
                                annotation.encode() if annotation else None, A, len(args), C.byref(lid)))
        return lid.value

    def batch_begin(self):
        check(self.h, lt_batch_begin(self.h))

    def batch_end(self):
        check(self.h, lt_batch_end(self.h))

    def batch_end_noalloc(self):
        """lt_batch_end_noalloc: issue the open batch from the library's fixed
        device scratch, allocating nothing."""
        check(self.h, lt_batch_end_noalloc(self.h))

    def launch_many(self, names, grids, blocks, superblocks, args, annotation=None):
        """Many launches in one call.  ``names``: kernel name per launch (or
        one name); ``grids``/``blocks``/``superblocks``: int arrays (count, ndim);
        ``args``: ARG_DTYPE array (count, nargs) - see ``arg_table``."""
        grids = np.ascontiguousarray(grids, dtype=np.int64)
        count, nd = grids.shape
        blocks = np.ascontiguousarray(np.broadcast_to(blocks, grids.shape), dtype=np.int64)
        sbs = None if superblocks is None else np.ascontiguousarray(np.broadcast_to(superblocks, grids.shape),
                                                                     dtype=np.int64)
        if isinstance(names, str):
            names = [names] * count
        ks = (_P * max(1, count))()
        cache = {}
        for i, nm in enumerate(names):
            if nm not in cache:
                cache[nm] = self.kernel(nm).value
            ks[i] = cache[nm]
        args = np.ascontiguousarray(args)
        assert args.dtype == ARG_DTYPE and args.shape[0] == count
        ids = np.zeros(count, dtype=np.uint64)
        check(self.h, lt_launch_many(self.h, ks, count, nd, grids.ctypes.data, blocks.ctypes.data,
                                     None if sbs is None else sbs.ctypes.data,
                                     annotation.encode() if annotation else None, args.ctypes.data,
                                     args.shape[1], ids.ctypes.data))
        return ids

    @staticmethod
    def arg_table(count, columns):
        """ARG_DTYPE table (count, len(columns)); each column is a list/array of
        Array handles (LT_ARG_ARRAY) or an int array (LT_ARG_INT)."""
        t = np.zeros((count, len(columns)), dtype=ARG_DTYPE)
        for j, col in enumerate(columns):
            if len(col) and isinstance(col[0], Array):
                t["kind"][:, j] = LT_ARG_ARRAY
                t["array"][:, j] = np.array([a.h.value for a in col], dtype=np.uint64)
            else:
                t["kind"][:, j] = LT_ARG_INT
                t["i"][:, j] = np.asarray(col, dtype=np.int64)
        return t

    def graph_begin(self):
        check(self.h, lt_graph_begin(self.h))

    def graph_end(self):
        g = _P()
        check(self.h, lt_graph_end(self.h, C.byref(g)))
        return g

    def graph_launch(self, g):
        check(self.h, lt_graph_launch(self.h, g))

    def graph_destroy(self, g):
        check(self.h, lt_graph_destroy(self.h, g))

    def sync(self):
        check(self.h, lt_sync(self.h))

    def wait(self, launch_id):
        check(self.h, lt_wait(self.h, launch_id))

    def stats(self) -> dict:
        s = lt_stats()
        check(self.h, lt_stats_get(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def reset_stats(self):
        check(self.h, lt_stats_reset(self.h))

    def tasks(self, launch_id):
        n = C.c_int32()
        check(self.h, lt_plan_tasks(self.h, launch_id, None, 0, C.byref(n)))
        buf = (lt_task_info * max(1, n.value))()
        check(self.h, lt_plan_tasks(self.h, launch_id, buf, n.value, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def regions(self, task_id):
        n = C.c_int32()
        check(self.h, lt_plan_regions(self.h, task_id, None, 0, C.byref(n)))
        buf = (lt_region_info * max(1, n.value))()
        check(self.h, lt_plan_regions(self.h, task_id, buf, n.value, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def deps(self, task_id):
        n = C.c_int32()
        check(self.h, lt_plan_deps(self.h, task_id, None, 0, C.byref(n)))
        buf = (C.c_uint64 * max(1, n.value))()
        check(self.h, lt_plan_deps(self.h, task_id, buf, n.value, C.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def trace(self):
        n = C.c_uint64()
        check(self.h, lt_trace_get(self.h, None, 0, C.byref(n)))
        buf = (lt_trace_rec * max(1, n.value))()
        check(self.h, lt_trace_get(self.h, buf, n.value, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def profile(self, on=True, every=1, steps=False):
        """Time dispatches with HIP events: all of them, every ``every``-th
        dispatch of each body, or (``steps``) each stream's run of dispatches
        between two syncs as one interval."""
        check(self.h, lt_profile_enable(self.h, (-1 if steps else int(every)) if on else 0))

    def profile_reset(self):
        check(self.h, lt_profile_reset(self.h))

    def profile_get(self) -> dict:
        n = C.c_int32()
        check(self.h, lt_profile_get(self.h, None, 0, C.byref(n)))
        buf = (lt_kernel_prof * max(1, n.value))()
        check(self.h, lt_profile_get(self.h, buf, n.value, C.byref(n)))
        return {buf[i].name.decode(): {"dispatches": int(buf[i].dispatches), "total_ms": buf[i].total_ms,
                                       "max_ms": buf[i].max_ms} for i in range(n.value)}

    def profile_spans(self):
        """Timed operations since profiling was enabled or reset: a structured
        array of (name, stream, start_ms, end_ms) on the device clock."""
        n = C.c_uint64()
        check(self.h, lt_profile_spans(self.h, None, 0, C.byref(n)))
        buf = (lt_span * max(1, n.value))()
        check(self.h, lt_profile_spans(self.h, buf, n.value, C.byref(n)))
        raw = np.frombuffer(buf, dtype=np.dtype([("name", "S32"), ("stream", np.int32), ("pad", np.int32),
                                                  ("start_ms", np.float64), ("end_ms", np.float64)]))[:n.value]
        return raw[["name", "stream", "start_ms", "end_ms"]].copy()

    def clear_trace(self):
        check(self.h, lt_trace_clear(self.h))
