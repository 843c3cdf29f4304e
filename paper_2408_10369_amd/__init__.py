"""Python binding of libbmlp (Boolean Matrix Logic Programming on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libbmlp.so`` behind the C ABI declared in ``include/bmlp.h``.
PyTorch supplies device memory (``torch.int64`` tensors hold the uint64 bit
words) and the HIP stream (``torch.cuda.current_stream()``).  There is no
fallback: if the library is missing, every call raises.

Bit matrices are 2-D ``torch.int64`` CUDA tensors of shape ``(rows, ld)``,
row-major, column j of a row at bit ``j & 63`` of word ``j >> 6``.  The number
of columns ``n`` is passed explicitly.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbmlp.so")

OK, EINVAL, EALIGN, EALIAS, EPAD, ENOMEM, EDEVICE, EITER, EMODEL = 0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS_NAMES = {0: "BMLP_OK", -1: "BMLP_EINVAL", -2: "BMLP_EALIGN", -3: "BMLP_EALIAS", -4: "BMLP_EPAD",
                -5: "BMLP_ENOMEM", -6: "BMLP_EDEVICE", -7: "BMLP_EITER", -8: "BMLP_EMODEL"}

ARM_AUTO = -1
ARM_PRODUCT_VALU, ARM_PRODUCT_MFMA = 0, 1
ARM_SMP_DENSE, ARM_SMP_SPARSE, ARM_SMP_CLOSURE = 2, 3, 4
ARM_COMPOSE_RMS, ARM_COMPOSE_SEMINAIVE = 5, 6
ARM_SMP_SPARSE_ROUNDS, ARM_SMP_ADAPTIVE = 7, 8
ARM_SMP_CLOSURE_SELECT = 13
ARM_COMPOSE_ROWWISE = 9
ARM_PRODUCT_GATHER = 10
ARM_PRODUCT_SEMINAIVE = 11
ARM_PRODUCT_SEMINAIVE_T = 12
DISPATCH_PLAIN, DISPATCH_LEARNED, DISPATCH_FORCED = 0, 1, 2
N_FEATURES, N_OUTPUTS, N_PARAMS = 16, 4, 5508

EXPORTS = [
    "bmlp_create", "bmlp_destroy", "bmlp_last_error", "bmlp_opts_init", "bmlp_version",
    "bmlp_pack_u8", "bmlp_pack_coo", "bmlp_unpack_coo", "bmlp_unpack_u8",
    "bmlp_or", "bmlp_and", "bmlp_andnot", "bmlp_not", "bmlp_transpose", "bmlp_product",
    "bmlp_rms", "bmlp_smp", "bmlp_compose_linear", "bmlp_compose_two_sided", "bmlp_closure_insert", "bmlp_batched",
    "bmlp_graph_open", "bmlp_graph_query", "bmlp_graph_has_closure", "bmlp_graph_close",
    "bmlp_set_trace", "bmlp_dispatcher_load", "bmlp_dispatcher_save", "bmlp_dispatcher_loaded",
    "bmlp_dispatcher_train", "bmlp_dispatcher_forward", "bmlp_mlp_loss_grad",
    "bmlp_tune_candidates", "bmlp_tune_buckets", "bmlp_tune_bucket_of", "bmlp_tune_get", "bmlp_tune_set",
    "bmlp_autotune", "bmlp_tune_save", "bmlp_tune_load", "bmlp_smp_noalloc",
    "bmlp_pack_coo_async", "bmlp_deferred_error", "bmlp_graph_last_arm", "bmlp_graph_query_sources",
]
TUNE_MAX_CANDIDATES = 8
TUNE_MFMA_PRODUCT, TUNE_VALU_PRODUCT = 0, 1


class Trace(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("call_arm", ctypes.c_int32), ("arm", ctypes.c_int32 * 64),
                ("round_ms", ctypes.c_float * 64), ("features", (ctypes.c_float * 16) * 64),
                ("call_features", ctypes.c_float * 16), ("pred", (ctypes.c_float * 4) * 64),
                ("call_pred", ctypes.c_float * 4), ("total_ms", ctypes.c_float)]

    def as_dict(self):
        import numpy as np
        r = int(self.rounds)
        return {"rounds": r, "call_arm": int(self.call_arm), "arm": [int(a) for a in self.arm[:r]],
                "round_ms": [float(x) for x in self.round_ms[:r]],
                "features": np.array([[float(v) for v in self.features[i]] for i in range(r)], np.float32),
                "call_features": np.array([float(v) for v in self.call_features], np.float32),
                "pred": np.array([[float(v) for v in self.pred[i]] for i in range(r)], np.float32),
                "call_pred": np.array([float(v) for v in self.call_pred], np.float32),
                "total_ms": float(self.total_ms)}


class GraphDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("R1", ctypes.c_void_p), ("closure", ctypes.c_void_p),
                ("ldc", ctypes.c_int64), ("k", ctypes.c_int64), ("ldv", ctypes.c_int64), ("V", ctypes.c_void_p),
                ("Vstar", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("dispatch", ctypes.c_int32), ("product_arm", ctypes.c_int32),
                ("smp_arm", ctypes.c_int32), ("compose_arm", ctypes.c_int32), ("rms_variant", ctypes.c_int32),
                ("smp_reflexive", ctypes.c_int32), ("check_padding", ctypes.c_int32),
                ("workspace_limit", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("products", ctypes.c_int32), ("arm_trace", ctypes.c_int32 * 64),
                ("arm", ctypes.c_int32), ("products_mfma", ctypes.c_int32), ("bool_ops", ctypes.c_uint64),
                ("bytes_moved", ctypes.c_uint64), ("device_ms", ctypes.c_double), ("product_ms", ctypes.c_double),
                ("product_bool_ops", ctypes.c_uint64), ("product_ms_mfma", ctypes.c_double),
                ("product_bool_ops_mfma", ctypes.c_uint64), ("mfma_ops_issued", ctypes.c_uint64),
                ("gathers", ctypes.c_int32), ("gather_ms", ctypes.c_double), ("gather_bytes", ctypes.c_uint64)]

    def as_dict(self):
        tr = [int(a) for a in self.arm_trace if a != -1]
        return {"iterations": int(self.iterations), "products": int(self.products), "arm": int(self.arm),
                "arm_trace": tr, "bool_ops": int(self.bool_ops), "bytes_moved": int(self.bytes_moved),
                "device_ms": float(self.device_ms), "product_ms": float(self.product_ms),
                "product_bool_ops": int(self.product_bool_ops), "products_mfma": int(self.products_mfma),
                "product_ms_mfma": float(self.product_ms_mfma),
                "product_bool_ops_mfma": int(self.product_bool_ops_mfma),
                "mfma_ops_issued": int(self.mfma_ops_issued), "gathers": int(self.gathers),
                "gather_ms": float(self.gather_ms), "gather_bytes": int(self.gather_bytes)}


class BmlpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


_lib = None


def lib():
    """Load libbmlp.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2408_10369_amd/build.py "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    P = ctypes.POINTER
    L.bmlp_create.argtypes = [P(vp), i32]
    L.bmlp_destroy.argtypes = [vp]
    L.bmlp_last_error.restype = ctypes.c_char_p
    L.bmlp_last_error.argtypes = []
    L.bmlp_opts_init.argtypes = [P(Opts)]
    L.bmlp_opts_init.restype = None
    L.bmlp_version.restype = ctypes.c_int32
    L.bmlp_pack_u8.argtypes = [vp, vp, i64, i64, i64, vp, i64, vp]
    L.bmlp_pack_coo.argtypes = [vp, vp, vp, i64, i64, i64, vp, i64, vp]
    L.bmlp_pack_coo_async.argtypes = [vp, vp, vp, i64, i64, i64, vp, i64, vp]
    L.bmlp_deferred_error.argtypes = [vp, vp]
    L.bmlp_graph_last_arm.argtypes = [vp]
    L.bmlp_graph_query_sources.argtypes = [vp, vp, vp, i64, i64, P(Opts), vp, P(Stats)]
    L.bmlp_unpack_u8.argtypes = [vp, vp, i64, i64, i64, vp, i64, vp]
    L.bmlp_unpack_coo.argtypes = [vp, vp, i64, i64, i64, vp, vp, i64, P(ctypes.c_int64), vp]
    for f in (L.bmlp_or, L.bmlp_and, L.bmlp_andnot):
        f.argtypes = [vp, vp, vp, vp, i64, i64, i64, vp]
    L.bmlp_not.argtypes = [vp, vp, vp, i64, i64, i64, vp]
    L.bmlp_transpose.argtypes = [vp, vp, i64, i64, i64, vp, i64, vp]
    L.bmlp_product.argtypes = [vp, vp, i64, vp, i64, vp, vp, i64, i64, i64, i64, P(Opts), vp, P(Stats)]
    L.bmlp_rms.argtypes = [vp, vp, vp, i64, i64, P(Opts), vp, P(Stats)]
    L.bmlp_smp.argtypes = [vp, vp, i64, i64, vp, vp, i64, i64, P(Opts), vp, P(Stats)]
    L.bmlp_smp_noalloc.argtypes = [vp, vp, i64, i64, vp, vp, i64, i64, ctypes.c_int32, vp]
    L.bmlp_compose_linear.argtypes = [vp, vp, vp, vp, i64, i64, P(Opts), vp, P(Stats)]
    L.bmlp_compose_two_sided.argtypes = [vp, vp, vp, vp, vp, i64, i64, P(Opts), vp, P(Stats)]
    L.bmlp_closure_insert.argtypes = [vp, vp, i64, i64, vp, vp, i64, P(Opts), vp, P(Stats)]
    L.bmlp_batched.argtypes = [vp, P(GraphDesc), ctypes.c_int32, P(Opts), vp, P(Stats)]
    fp = ctypes.POINTER(ctypes.c_float)
    L.bmlp_graph_open.argtypes = [vp, vp, i64, i64, vp, P(vp)]
    L.bmlp_graph_query.argtypes = [vp, vp, vp, i64, i64, P(Opts), vp, P(Stats)]
    L.bmlp_graph_has_closure.argtypes = [vp]
    L.bmlp_graph_close.argtypes = [vp]
    L.bmlp_set_trace.argtypes = [vp, P(Trace)]
    L.bmlp_dispatcher_load.argtypes = [vp, ctypes.c_char_p]
    L.bmlp_dispatcher_save.argtypes = [vp, ctypes.c_char_p]
    L.bmlp_dispatcher_loaded.argtypes = [vp]
    L.bmlp_dispatcher_train.argtypes = [vp, fp, fp, fp, i64, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64, fp]
    L.bmlp_dispatcher_forward.argtypes = [vp, fp, i64, fp]
    L.bmlp_mlp_loss_grad.argtypes = [vp, fp, fp, fp, fp, fp, fp, i64, fp, fp]
    L.bmlp_tune_candidates.argtypes = [ctypes.c_int32]
    L.bmlp_tune_buckets.argtypes = [ctypes.c_int32]
    L.bmlp_tune_bucket_of.argtypes = [ctypes.c_int32, i64, i64, i64, ctypes.c_double, ctypes.c_int32]
    L.bmlp_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p, fp]
    L.bmlp_tune_save.argtypes = [vp, ctypes.c_char_p]
    L.bmlp_tune_load.argtypes = [vp, ctypes.c_char_p]
    L.bmlp_tune_get.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32), fp]
    L.bmlp_tune_set.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    for name in EXPORTS:
        f = getattr(L, name)
        if name in ("bmlp_graph_has_closure", "bmlp_dispatcher_loaded", "bmlp_tune_candidates", "bmlp_tune_buckets",
                    "bmlp_tune_bucket_of", "bmlp_graph_last_arm"):
            f.restype = ctypes.c_int32
        elif name not in ("bmlp_last_error", "bmlp_opts_init", "bmlp_version"):
            f.restype = ctypes.c_int
    _lib = L
    return L


def words(n: int) -> int:
    return (n + 63) // 64


def make_opts(**kw) -> Opts:
    o = Opts()
    lib().bmlp_opts_init(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, int(v))
    return o


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _check(rc: int):
    if rc != OK:
        raise BmlpError(rc, lib().bmlp_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _bits_shape(t, rows=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.int64 and t.dim() == 2 and t.is_cuda):
        raise TypeError("bit matrices are 2-D torch.int64 CUDA tensors (rows, ld)")
    if not t.is_contiguous():
        raise ValueError("bit matrix must be contiguous")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"expected {rows} rows, got {t.shape[0]}")
    return t.shape[0], t.shape[1]


class Context:
    """A libbmlp handle bound to one HIP device."""

    def __init__(self, device: int = 0):
        L = lib()
        h = ctypes.c_void_p()
        _check(L.bmlp_create(ctypes.byref(h), int(device)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().bmlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------------------------------------------------------------- allocation helpers
    def zeros(self, rows: int, n: int, ld: int | None = None):
        import torch
        ld = ld if ld is not None else max(words(n), 1)
        return torch.zeros((rows, ld), dtype=torch.int64, device=f"cuda:{self.device}")

    # -------------------------------------------------------------- facts -> matrices
    def pack_coo(self, row, col, rows: int, n: int, ld: int | None = None, out=None, stream=None):
        import torch
        row = row.to(device=f"cuda:{self.device}", dtype=torch.int32).contiguous()
        col = col.to(device=f"cuda:{self.device}", dtype=torch.int32).contiguous()
        if out is None:
            out = self.zeros(rows, n, ld)
        _bits_shape(out, rows)
        _check(lib().bmlp_pack_coo(self._h, _ptr(row), _ptr(col), row.numel(), rows, n, _ptr(out),
                                   out.shape[1], _stream(stream)))
        return out

    def pack_coo_async(self, row, col, rows: int, n: int, out, stream=None):
        """bmlp_pack_coo_async: no synchronisation; row/col must be int32 device tensors, out a bit matrix.
        Out-of-range facts are skipped and reported by deferred_error()."""
        _bits_shape(out, rows)
        _check(lib().bmlp_pack_coo_async(self._h, _ptr(row), _ptr(col), row.numel(), rows, n, _ptr(out),
                                         out.shape[1], _stream(stream)))
        return out

    def deferred_error(self, stream=None):
        _check(lib().bmlp_deferred_error(self._h, _stream(stream)))

    def pack_u8(self, dense, ld: int | None = None, out=None, stream=None):
        rows, n = dense.shape
        if out is None:
            out = self.zeros(rows, n, ld)
        _check(lib().bmlp_pack_u8(self._h, _ptr(dense), rows, n, dense.stride(0), _ptr(out), out.shape[1],
                                  _stream(stream)))
        return out

    def unpack_coo(self, bits, n: int, stream=None):
        """(row, col) int32 device tensors of the set bits, sorted by row then column."""
        import torch
        rows, ld = _bits_shape(bits)
        cnt = ctypes.c_int64(0)
        _check(lib().bmlp_unpack_coo(self._h, _ptr(bits), rows, n, ld, None, None, 0, ctypes.byref(cnt),
                                     _stream(stream)))
        m = int(cnt.value)
        dev = f"cuda:{self.device}"
        r = torch.empty(m, dtype=torch.int32, device=dev)
        c = torch.empty(m, dtype=torch.int32, device=dev)
        if m:
            _check(lib().bmlp_unpack_coo(self._h, _ptr(bits), rows, n, ld, _ptr(r), _ptr(c), m, ctypes.byref(cnt),
                                         _stream(stream)))
        return r, c

    def unpack_u8(self, bits, n: int, stream=None):
        import torch
        rows, ld = _bits_shape(bits)
        out = torch.empty((rows, n), dtype=torch.uint8, device=bits.device)
        _check(lib().bmlp_unpack_u8(self._h, _ptr(bits), rows, n, ld, _ptr(out), n, _stream(stream)))
        return out

    # -------------------------------------------------------------- operators
    def _ew(self, fn, A, B, n, out, stream):
        rows, ld = _bits_shape(A)
        if B is not None:
            _bits_shape(B, rows)
        if out is None:
            out = self.zeros(rows, n, ld)
        if B is None:
            _check(fn(self._h, _ptr(A), _ptr(out), rows, n, ld, _stream(stream)))
        else:
            _check(fn(self._h, _ptr(A), _ptr(B), _ptr(out), rows, n, ld, _stream(stream)))
        return out

    def or_(self, A, B, n, out=None, stream=None):
        return self._ew(lib().bmlp_or, A, B, n, out, stream)

    def and_(self, A, B, n, out=None, stream=None):
        return self._ew(lib().bmlp_and, A, B, n, out, stream)

    def andnot(self, A, B, n, out=None, stream=None):
        return self._ew(lib().bmlp_andnot, A, B, n, out, stream)

    def not_(self, A, n, out=None, stream=None):
        return self._ew(lib().bmlp_not, A, None, n, out, stream)

    def transpose(self, A, cols: int, ldat: int | None = None, out=None, stream=None):
        rows, lda = _bits_shape(A)
        if out is None:
            out = self.zeros(cols, rows, ldat)
        _check(lib().bmlp_transpose(self._h, _ptr(A), rows, cols, lda, _ptr(out), out.shape[1], _stream(stream)))
        return out

    def product(self, A, B, kdim: int, n: int, Cold=None, out=None, opts=None, stream=None, stats=None):
        m, lda = _bits_shape(A)
        _, ldb = _bits_shape(B, kdim)
        if out is None:
            out = self.zeros(m, n)
        st = Stats() if stats is not None else None
        _check(lib().bmlp_product(self._h, _ptr(A), lda, _ptr(B), ldb, _ptr(Cold), _ptr(out), out.shape[1], m,
                                  kdim, n, ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                  ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return out

    # -------------------------------------------------------------- BMLP algorithms
    def rms(self, R1, n: int, out=None, opts=None, stream=None, stats=None):
        rows, ld = _bits_shape(R1, n)
        if out is None:
            out = self.zeros(n, n, ld)
        st = Stats() if stats is not None else None
        _check(lib().bmlp_rms(self._h, _ptr(R1), _ptr(out), n, ld, ctypes.byref(opts) if opts is not None else None,
                              _stream(stream), ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return out

    def smp(self, R1, n: int, V, out=None, opts=None, stream=None, stats=None):
        _, ld = _bits_shape(R1, n)
        k, ldv = _bits_shape(V)
        if out is None:
            out = self.zeros(k, n, ldv)
        st = Stats() if stats is not None else None
        _check(lib().bmlp_smp(self._h, _ptr(R1), n, ld, _ptr(V), _ptr(out), k, ldv,
                              ctypes.byref(opts) if opts is not None else None, _stream(stream),
                              ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return out

    def smp_noalloc(self, R1, n: int, V, out, reflexive: bool = False, stream=None):
        """bmlp_smp_noalloc: the selection with the edge index in the library's fixed device array; the
        caller provides every buffer (``out`` included)."""
        _, ld = _bits_shape(R1, n)
        k, ldv = _bits_shape(V)
        _bits_shape(out, k)
        _check(lib().bmlp_smp_noalloc(self._h, _ptr(R1), n, ld, _ptr(V), _ptr(out), k, ldv,
                                      1 if reflexive else 0, _stream(stream)))
        return out

    def compose_linear(self, Rbase, Rstep, n: int, out=None, opts=None, stream=None, stats=None):
        _, ld = _bits_shape(Rbase, n)
        _bits_shape(Rstep, n)
        if out is None:
            out = self.zeros(n, n, ld)
        st = Stats() if stats is not None else None
        _check(lib().bmlp_compose_linear(self._h, _ptr(Rbase), _ptr(Rstep), _ptr(out), n, ld,
                                         ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                         ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return out

    def compose_two_sided(self, Rbase, Rleft, Rright, n: int, out=None, opts=None, stream=None, stats=None):
        """Least P = Rbase | Rleft . P . Rright (p <- b; p <- l, p, r)."""
        _, ld = _bits_shape(Rbase, n)
        _bits_shape(Rleft, n)
        _bits_shape(Rright, n)
        if out is None:
            out = self.zeros(n, n, ld)
        st = Stats() if stats is not None else None
        _check(lib().bmlp_compose_two_sided(self._h, _ptr(Rbase), _ptr(Rleft), _ptr(Rright), _ptr(out), n, ld,
                                            ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                            ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return out

    def closure_insert(self, Rplus, n: int, src, dst, opts=None, stream=None, stats=None):
        """Rplus (n x n, the closure of some relation) becomes the closure with the edges (src[i], dst[i])
        added, in place."""
        import torch
        _, ld = _bits_shape(Rplus, n)
        src = torch.as_tensor(src).to(device=f"cuda:{self.device}", dtype=torch.int32).contiguous()
        dst = torch.as_tensor(dst).to(device=f"cuda:{self.device}", dtype=torch.int32).contiguous()
        if src.numel() != dst.numel():
            raise ValueError("src and dst must have the same length")
        st = Stats() if stats is not None else None
        _check(lib().bmlp_closure_insert(self._h, _ptr(Rplus), n, ld, _ptr(src), _ptr(dst), src.numel(),
                                         ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                         ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return Rplus

    def batched(self, graphs, opts=None, stream=None, stats=None):
        """One launch over many graphs.  ``graphs``: sequence of dicts with keys
        ``n``, ``R1`` and optionally ``closure`` (output), ``V`` and ``Vstar``
        (output); the outputs are filled in place."""
        arr = (GraphDesc * max(len(graphs), 1))()
        for i, g in enumerate(graphs):
            n = int(g["n"])
            _, ld = _bits_shape(g["R1"], n)
            d = arr[i]
            d.n, d.ld, d.R1 = n, ld, g["R1"].data_ptr()
            clo = g.get("closure")
            if clo is not None:
                _, d.ldc = _bits_shape(clo, n)
                d.closure = clo.data_ptr()
            V = g.get("V")
            if V is not None and V.shape[0] > 0:
                d.k, d.ldv = _bits_shape(V)
                _bits_shape(g["Vstar"], d.k)
                d.V, d.Vstar = V.data_ptr(), g["Vstar"].data_ptr()
        st = Stats() if stats is not None else None
        _check(lib().bmlp_batched(self._h, arr, len(graphs), ctypes.byref(opts) if opts is not None else None,
                                  _stream(stream), ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return graphs

    # -------------------------------------------------------------- the learned dispatcher
    def set_trace(self, trace):
        """Record per-round features and timings into ``trace`` (a Trace) or stop (None)."""
        self._trace = trace
        _check(lib().bmlp_set_trace(self._h, ctypes.byref(trace) if trace is not None else None))

    def dispatcher_loaded(self) -> bool:
        return bool(lib().bmlp_dispatcher_loaded(self._h))

    def dispatcher_load(self, path: str):
        _check(lib().bmlp_dispatcher_load(self._h, os.fsencode(path)))

    def dispatcher_save(self, path: str):
        _check(lib().bmlp_dispatcher_save(self._h, os.fsencode(path)))

    @staticmethod
    def _f32(a, shape):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.shape != shape:
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        return a

    def dispatcher_train(self, X, T, M, epochs=2000, lr=3e-3, seed=0):
        import numpy as np
        X = self._f32(X, (len(X), N_FEATURES))
        T = self._f32(T, (len(X), N_OUTPUTS))
        M = self._f32(M, (len(X), N_OUTPUTS))
        loss = ctypes.c_float(0.0)
        fp = ctypes.POINTER(ctypes.c_float)
        _check(lib().bmlp_dispatcher_train(self._h, X.ctypes.data_as(fp), T.ctypes.data_as(fp), M.ctypes.data_as(fp),
                                           len(X), int(epochs), float(lr), int(seed), ctypes.byref(loss)))
        return float(loss.value)

    def dispatcher_forward(self, X):
        import numpy as np
        X = self._f32(X, (len(X), N_FEATURES))
        Y = np.zeros((len(X), N_OUTPUTS), np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        _check(lib().bmlp_dispatcher_forward(self._h, X.ctypes.data_as(fp), len(X), Y.ctypes.data_as(fp)))
        return Y

    def mlp_loss_grad(self, params, mu, sd, X, T, M):
        import numpy as np
        fp = ctypes.POINTER(ctypes.c_float)
        P = self._f32(params, (N_PARAMS,))
        mu = self._f32(mu, (N_FEATURES,))
        sd = self._f32(sd, (N_FEATURES,))
        X = self._f32(X, (len(X), N_FEATURES))
        T = self._f32(T, (len(X), N_OUTPUTS))
        M = self._f32(M, (len(X), N_OUTPUTS))
        loss = ctypes.c_float(0.0)
        G = np.zeros(N_PARAMS, np.float32)
        _check(lib().bmlp_mlp_loss_grad(self._h, P.ctypes.data_as(fp), mu.ctypes.data_as(fp), sd.ctypes.data_as(fp),
                                        X.ctypes.data_as(fp), T.ctypes.data_as(fp), M.ctypes.data_as(fp), len(X),
                                        ctypes.byref(loss), G.ctypes.data_as(fp)))
        return float(loss.value), G

    # -------------------------------------------------------------- sessions
    # -------------------------------------------------------------- autotuned tile code
    @staticmethod
    def tune_candidates(kernel: int) -> int:
        return int(lib().bmlp_tune_candidates(int(kernel)))

    @staticmethod
    def tune_buckets(kernel: int) -> int:
        return int(lib().bmlp_tune_buckets(int(kernel)))

    @staticmethod
    def tune_bucket_of(kernel: int, m: int, kdim: int, n: int, density: float = -1.0, structured: bool = False) -> int:
        return int(lib().bmlp_tune_bucket_of(int(kernel), int(m), int(kdim), int(n), float(density),
                                             1 if structured else 0))

    def autotune(self, kernel_mask: int = 3, reps: int = 3, cache_out: str | None = None):
        """Time every candidate on every bucket and keep the fastest; returns the report as a nested list
        [kernel][bucket][candidate] of median ms (-1 where not measured)."""
        nk = 2
        nb = self.tune_buckets(0)
        rep = (ctypes.c_float * (nk * nb * TUNE_MAX_CANDIDATES))()
        _check(lib().bmlp_autotune(self._h, int(kernel_mask), int(reps),
                                   cache_out.encode() if cache_out else None, rep))
        return [[[rep[(k * nb + b) * TUNE_MAX_CANDIDATES + v] for v in range(TUNE_MAX_CANDIDATES)]
                 for b in range(nb)] for k in range(nk)]

    def tune_save(self, path: str):
        _check(lib().bmlp_tune_save(self._h, path.encode()))

    def tune_load(self, path: str):
        _check(lib().bmlp_tune_load(self._h, path.encode()))

    def tune_get(self, kernel: int, bucket: int):
        v = ctypes.c_int32()
        ms = ctypes.c_float()
        _check(lib().bmlp_tune_get(self._h, int(kernel), int(bucket), ctypes.byref(v), ctypes.byref(ms)))
        return v.value, ms.value

    def tune_set(self, kernel: int, bucket: int, variant: int):
        _check(lib().bmlp_tune_set(self._h, int(kernel), int(bucket), int(variant)))

    def graph(self, R1, n: int, stream=None):
        return Session(self, R1, n, stream)


class Session:
    """A stream of selections over one relation (closure kept once computed)."""

    def __init__(self, ctx: Context, R1, n: int, stream=None):
        _, ld = _bits_shape(R1, n)
        self.ctx, self.R1, self.n = ctx, R1, n
        g = ctypes.c_void_p()
        _check(lib().bmlp_graph_open(ctx._h, _ptr(R1), n, ld, _stream(stream), ctypes.byref(g)))
        self._g = g

    def query(self, V, out=None, opts=None, stream=None, stats=None):
        k, ldv = _bits_shape(V)
        if out is None:
            out = self.ctx.zeros(k, self.n, ldv)
        st = Stats() if stats is not None else None
        _check(lib().bmlp_graph_query(self._g, _ptr(V), _ptr(out), k, ldv,
                                      ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                      ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return out

    def query_sources(self, src, out, opts=None, stream=None, stats=None):
        """bmlp_graph_query_sources: one-hot queries given by their source indices (int32 device tensor)."""
        k, ldv = _bits_shape(out)
        if src.numel() != k:
            raise ValueError("one source per answer row")
        st = Stats() if stats is not None else None
        _check(lib().bmlp_graph_query_sources(self._g, _ptr(src), _ptr(out), k, ldv,
                                              ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                              ctypes.byref(st) if st is not None else None))
        if st is not None:
            stats.update(st.as_dict())
        return out

    @property
    def has_closure(self) -> bool:
        return bool(lib().bmlp_graph_has_closure(self._g))

    @property
    def last_arm(self) -> int:
        return int(lib().bmlp_graph_last_arm(self._g))

    def close(self):
        if getattr(self, "_g", None):
            lib().bmlp_graph_close(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
