"""Thin ctypes binding of liblagr.so (include/lagr.h).

Argument marshalling only: every step of every operation runs in the HIP
kernels of the shared library.  PyTorch supplies device memory (its caching
allocator is registered as the library's allocator) and the stream.  There
is no CPU fallback: importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblagr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"liblagr.so is not built ({LIB_PATH}); run __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)

MSG_LEN = 256

# codes
SUCCESS, NO_VALUE = 0, 1
NULL_POINTER, INVALID_VALUE, INVALID_INDEX, DOMAIN_MISMATCH = -1, -2, -3, -4
DIMENSION_MISMATCH, INVALID_OBJECT, OUT_OF_MEMORY, PROPERTY_MISSING = -5, -6, -7, -8
NOT_IMPLEMENTED, DEVICE_ERROR, BUDGET_EXCEEDED = -9, -10, -11

# types
BOOL, INT64, FP64, INT32 = 0, 1, 2, 3
# semirings
PLUS_PAIR, ANY_SECONDI, PLUS_FIRST, MIN_PLUS = 0, 1, 2, 3
# binops
NOOP, PLUS, MIN, FIRST, SECOND, TIMES, DIV, ANY = range(8)
# descriptor bits
DESC_DEFAULT, DESC_COMP, DESC_STRUCT, DESC_REPLACE = 0, 1, 2, 4
DESC_TRAN0, DESC_TRAN1, DESC_DETERMINISTIC, DESC_ASSIGN_PARENT = 8, 16, 32, 64
DESC_S = DESC_STRUCT
DESC_RSC = DESC_REPLACE | DESC_STRUCT | DESC_COMP
# vector formats
VEC_SPARSE, VEC_BITMAP, VEC_FULL = 0, 1, 2
# graph kinds
ADJACENCY_UNDIRECTED, ADJACENCY_DIRECTED = 0, 1
# build flags
BUILD_SYMMETRIZE, BUILD_DROP_LOOPS = 1, 2
# bfs flags
BFS_PUSH_ONLY, BFS_ANY_PARENT = 1, 2

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32
_INT = ctypes.c_int
_PP = ctypes.POINTER(ctypes.c_void_p)
_C = ctypes.c_char_p

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)

_PROTOS = {
    "lagr_set_allocator": [ALLOC_FN, FREE_FN, _P, _C],
    "lagr_ctx_new": [_PP, _INT, _P, _C],
    "lagr_ctx_set_stream": [_P, _P, _C],
    "lagr_ctx_free": [_PP],
    "lagr_wait": [_P, _C],
    "lagr_ctx_timing": [_P, _INT, _C],
    "lagr_ctx_kernel_time": [_P, _C, _P, _P, _C],
    "lagr_matrix_new": [_PP, _INT, _I64, _I64, _P, _C],
    "lagr_matrix_wrap_csr": [_PP, _INT, _I64, _I64, _I64, _P, _P, _P, _P, _C],
    "lagr_matrix_build": [_PP, _I64, _I64, _I64, _P, _P, _U32, _P, _C],
    "lagr_matrix_info": [_P, _P, _P, _P, _P, _C],
    "lagr_matrix_extract_csr": [_P, _P, _P, _P, _P, _C],
    "lagr_matrix_nvals": [_P, _P, _P, _C],
    "lagr_select_tril": [_PP, _P, _P, _C],
    "lagr_matrix_free": [_PP],
    "lagr_vector_new": [_PP, _INT, _I64, _P, _C],
    "lagr_vector_wrap_sparse": [_PP, _INT, _I64, _I64, _P, _P, _P, _C],
    "lagr_vector_wrap_bitmap": [_PP, _INT, _I64, _P, _P, _P, _C],
    "lagr_vector_wrap_full": [_PP, _INT, _I64, _P, _P, _C],
    "lagr_vector_info": [_P, _P, _P, _P, _C],
    "lagr_vector_nvals": [_P, _P, _P, _C],
    "lagr_vector_extract_tuples": [_P, _P, _P, _P, _C],
    "lagr_vector_extract_dense": [_P, _P, _P, _P, _P, _C],
    "lagr_vector_free": [_PP],
    "lagr_mxm": [_P, _P, _INT, _INT, _P, _P, _U32, _P, _C],
    "lagr_vxm": [_P, _P, _INT, _INT, _P, _P, _U32, _P, _C],
    "lagr_mxm_reduce": [_P, _P, _INT, _P, _P, _U32, _P, _C],
    "lagr_reduce_scalar": [_P, _INT, _INT, _P, _P, _C],
    "lagr_vector_reduce_scalar": [_P, _INT, _INT, _P, _P, _C],
    "lagr_reduce_rows": [_P, _P, _INT, _INT, _P, _U32, _P, _C],
    "lagr_assign_vector": [_P, _P, _INT, _P, _U32, _P, _C],
    "lagr_assign_scalar": [_P, _P, _INT, _P, _U32, _P, _C],
    "lagr_ewise_add": [_P, _P, _INT, _INT, _P, _P, _U32, _P, _C],
    "lagr_ewise_mult": [_P, _P, _INT, _INT, _P, _P, _U32, _P, _C],
    "lagr_graph_new": [_PP, _PP, _INT, _P, _C],
    "lagr_graph_check": [_P, _P, _C],
    "lagr_property_row_degree": [_P, _P, _C],
    "lagr_property_tc_lower": [_P, _P, _C],
    "lagr_property_at": [_P, _P, _C],
    "lagr_graph_at": [_PP, _P, _C],
    "lagr_graph_matrix": [_PP, _P, _C],
    "lagr_graph_tc_lower": [_PP, _P, _C],
    "lagr_graph_delete_properties": [_P, _P, _C],
    "lagr_graph_ndiag": [_P, _P, _C],
    "lagr_graph_free": [_PP],
    "lagr_tc": [_P, _P, _INT, _P, _C],
    "lagr_tc_adv": [_P, _P, _P, _C],
    "lagr_tc_adv_noalloc": [_P, _P, _P, _C],
    "lagr_bfs": [_PP, _PP, _P, _I64, _U32, _P, _C],
    "lagr_bc": [_PP, _P, _P, _I32, _P, _C],
    "lagr_bc_dir": [_PP, _P, _P, _I32, _U32, _P, _C],
    "lagr_bfs_batch": [_P, _P, _P, _P, _P, _P, _I32, _P, _C],
    "lagr_bfs_autotune": [_P, _P, _P, _P, _I32, _P, _C],
    "lagr_tc_autotune": [_P, _P, _P, _C],
    "lagr_graph_set_tuning": [_P, _I64, _I32, _I32, _P, _C],
    "lagr_graph_get_tuning": [_P, _P, _P, _P, _C],
    "lagr_sssp": [_PP, _P, _I64, ctypes.c_double, _P, _C],
    "lagr_pagerank": [_PP, _P, _P, ctypes.c_double, ctypes.c_double, _I64, _P, _C],
    "lagr_cc": [_PP, _P, _P, _P, _C],
}

_fns = {}
for _name, _args in _PROTOS.items():
    try:
        _f = getattr(_lib, _name)
    except AttributeError:
        continue
    _f.restype = ctypes.c_int
    _f.argtypes = _args
    _fns[_name] = _f


def exported_symbols():
    return set(_fns)


class LagrError(RuntimeError):
    def __init__(self, fn, code, text):
        super().__init__(f"{fn} -> {code}: {text}")
        self.code = code


def call(name, *args):
    """Call an exported function; raise LagrError on a negative code.
    Returns the (non-negative) code."""
    buf = ctypes.create_string_buffer(MSG_LEN)
    rc = _fns[name](*args, buf)
    if rc < 0:
        raise LagrError(name, rc, buf.value.decode(errors="replace"))
    return rc


def call_nomsg(name, *args):
    return _fns[name](*args)


# ------------------------------------------------------------ allocator

_alloc_refs = None
# device allocations made by the library through the registered allocator
alloc_calls = 0


def use_torch_allocator(enable: bool = True):
    """Route the library's device allocations through PyTorch's caching
    allocator on the current device and stream."""
    global _alloc_refs
    if not enable:
        call("lagr_set_allocator", ALLOC_FN(), FREE_FN(), None)
        _alloc_refs = None
        return

    def _alloc(nbytes, user):
        global alloc_calls
        alloc_calls += 1
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None

    def _free(ptr, nbytes, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    a, f = ALLOC_FN(_alloc), FREE_FN(_free)
    call("lagr_set_allocator", a, f, None)
    _alloc_refs = (a, f)


# --------------------------------------------------------------- objects

def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device: int = 0, stream=None):
        torch.cuda.set_device(device)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        self.h = ctypes.c_void_p()
        call("lagr_ctx_new", ctypes.byref(self.h), device, ctypes.c_void_p(s.cuda_stream))

    def wait(self):
        call("lagr_wait", self.h)

    def timing(self, enable: bool):
        call("lagr_ctx_timing", self.h, 1 if enable else 0)

    def kernel_time(self, kernel: str):
        """(total ms, launches) of a library kernel since timing was enabled."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        call("lagr_ctx_kernel_time", self.h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    def free(self):
        if self.h:
            call_nomsg("lagr_ctx_free", ctypes.byref(self.h))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


_TORCH = {BOOL: None, INT64: torch.int64, FP64: torch.float64, INT32: torch.int32}


def _scalar(typ, value=None):
    """A host scalar of the library type typ (int64 for BOOL)."""
    if typ == FP64:
        return ctypes.c_double(value or 0.0)
    if typ == INT32:
        return ctypes.c_int32(value or 0)
    return ctypes.c_int64(value or 0)


def _typ_of(values):
    if values is None:
        return BOOL
    return {torch.float64: FP64, torch.int32: INT32}.get(values.dtype, INT64)


class Matrix:
    """Handle of a lagr_matrix.  Keeps wrapped tensors alive."""

    def __init__(self, h, keep=()):
        self.h = h
        self._keep = keep

    @classmethod
    def new(cls, ctx, typ, nrows, ncols):
        h = ctypes.c_void_p()
        call("lagr_matrix_new", ctypes.byref(h), typ, nrows, ncols, ctx.h)
        return cls(h)

    @classmethod
    def wrap_csr(cls, ctx, nrows, ncols, rowptr, colidx, values=None, typ=None):
        if typ is None:
            typ = _typ_of(values)
        rowptr = rowptr.to(torch.int64).contiguous()
        colidx = colidx.to(torch.int32).contiguous()
        if values is not None:
            values = values.to(_TORCH[typ]).contiguous()
        h = ctypes.c_void_p()
        call("lagr_matrix_wrap_csr", ctypes.byref(h), typ, nrows, ncols, colidx.numel(),
             _ptr(rowptr), _ptr(colidx), _ptr(values), ctx.h)
        return cls(h, (rowptr, colidx, values))

    @classmethod
    def build(cls, ctx, nrows, ncols, src, dst, flags):
        src = src.to(torch.int32).contiguous()
        dst = dst.to(torch.int32).contiguous()
        h = ctypes.c_void_p()
        call("lagr_matrix_build", ctypes.byref(h), nrows, ncols, src.numel(), _ptr(src), _ptr(dst),
             flags, ctx.h)
        return cls(h)

    def info(self):
        t, r, c, nv = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        call("lagr_matrix_info", self.h, ctypes.byref(t), ctypes.byref(r), ctypes.byref(c),
             ctypes.byref(nv))
        return t.value, r.value, c.value, nv.value

    def to_csr(self, ctx):
        typ, nrows, ncols, nvals = self.info()
        dev = torch.device("cuda", torch.cuda.current_device())
        rp = torch.empty(nrows + 1, dtype=torch.int64, device=dev)
        ci = torch.empty(nvals, dtype=torch.int32, device=dev)
        va = None if typ == BOOL else torch.empty(nvals, dtype=_TORCH[typ], device=dev)
        call("lagr_matrix_extract_csr", self.h, _ptr(rp), _ptr(ci), _ptr(va), ctx.h)
        ctx.wait()
        return rp, ci, va

    def free(self):
        if self.h and not getattr(self, "_borrowed", False):
            call_nomsg("lagr_matrix_free", ctypes.byref(self.h))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Vector:
    def __init__(self, h, keep=()):
        self.h = h
        self._keep = keep

    @classmethod
    def new(cls, ctx, typ, n):
        h = ctypes.c_void_p()
        call("lagr_vector_new", ctypes.byref(h), typ, n, ctx.h)
        return cls(h)

    @classmethod
    def wrap_sparse(cls, ctx, n, idx, values=None, typ=None):
        if typ is None:
            typ = _typ_of(values)
        idx = idx.to(torch.int32).contiguous()
        if values is not None:
            values = values.to(_TORCH[typ]).contiguous()
        h = ctypes.c_void_p()
        call("lagr_vector_wrap_sparse", ctypes.byref(h), typ, n, idx.numel(), _ptr(idx),
             _ptr(values), ctx.h)
        return cls(h, (idx, values))

    @classmethod
    def wrap_bitmap(cls, ctx, present, values=None, typ=None):
        if typ is None:
            typ = _typ_of(values)
        present = present.to(torch.uint8).contiguous()
        if values is not None:
            values = values.to(_TORCH[typ]).contiguous()
        h = ctypes.c_void_p()
        call("lagr_vector_wrap_bitmap", ctypes.byref(h), typ, present.numel(), _ptr(present),
             _ptr(values), ctx.h)
        return cls(h, (present, values))

    @classmethod
    def wrap_full(cls, ctx, values):
        typ = _typ_of(values)
        values = values.to(_TORCH[typ]).contiguous()
        h = ctypes.c_void_p()
        call("lagr_vector_wrap_full", ctypes.byref(h), typ, values.numel(), _ptr(values), ctx.h)
        return cls(h, (values,))

    def info(self):
        t, n, f = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int()
        call("lagr_vector_info", self.h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(f))
        return t.value, n.value, f.value

    def nvals(self, ctx):
        nv = ctypes.c_int64()
        call("lagr_vector_nvals", ctypes.byref(nv), self.h, ctx.h)
        return nv.value

    def to_dense(self, ctx, fill=0):
        """-> (present uint8[n], values[n]) device tensors."""
        typ, n, fmt = self.info()
        dev = torch.device("cuda", torch.cuda.current_device())
        pres = torch.empty(n, dtype=torch.uint8, device=dev)
        vt = _TORCH[typ] or torch.int64
        vals = torch.empty(n, dtype=vt, device=dev)
        f = _scalar(typ, fill)
        call("lagr_vector_extract_dense", self.h, _ptr(pres), None if typ == BOOL else _ptr(vals),
             ctypes.byref(f), ctx.h)
        ctx.wait()
        return pres, vals

    def values_full(self, ctx):
        """Values of a FULL vector as a tensor (copy)."""
        return self.to_dense(ctx)[1]

    def to_tuples(self, ctx):
        typ, n, fmt = self.info()
        nv = self.nvals(ctx)
        dev = torch.device("cuda", torch.cuda.current_device())
        idx = torch.empty(nv, dtype=torch.int32, device=dev)
        vals = None if typ == BOOL else torch.empty(nv, dtype=_TORCH[typ], device=dev)
        call("lagr_vector_extract_tuples", self.h, _ptr(idx), _ptr(vals), ctx.h)
        ctx.wait()
        return idx, vals

    def free(self):
        if self.h:
            call_nomsg("lagr_vector_free", ctypes.byref(self.h))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Graph:
    def __init__(self, ctx, A: Matrix, kind=ADJACENCY_UNDIRECTED):
        self.h = ctypes.c_void_p()
        self._keep = A._keep
        call("lagr_graph_new", ctypes.byref(self.h), ctypes.byref(A.h), kind, ctx.h)
        A.h = ctypes.c_void_p()   # moved into the graph (Listing 1)

    def check(self, ctx):
        call("lagr_graph_check", self.h, ctx.h)

    def delete_properties(self, ctx):
        call("lagr_graph_delete_properties", self.h, ctx.h)

    def set_tuning(self, ctx, tc_hubs=-1, bfs_alpha=-1, bfs_beta=-1):
        call("lagr_graph_set_tuning", self.h, tc_hubs, bfs_alpha, bfs_beta, ctx.h)

    def tuning(self):
        h, a, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        call("lagr_graph_get_tuning", ctypes.byref(h), ctypes.byref(a), ctypes.byref(b), self.h)
        return h.value, a.value, b.value

    def _borrowed(self, fn):
        h = ctypes.c_void_p()
        call(fn, ctypes.byref(h), self.h)
        if not h:
            return None
        M = Matrix(h)
        M._borrowed = True
        return M

    def matrix(self):
        """Borrowed handle of the adjacency matrix (owned by the graph)."""
        return self._borrowed("lagr_graph_matrix")

    def tc_lower(self):
        """Borrowed handle of the cached triangle-count operand, or None."""
        return self._borrowed("lagr_graph_tc_lower")

    def property_at(self, ctx):
        call("lagr_property_at", self.h, ctx.h)

    def at(self):
        """Borrowed handle of the transpose (A itself when undirected)."""
        return self._borrowed("lagr_graph_at")

    def ndiag(self):
        v = ctypes.c_int64()
        call("lagr_graph_ndiag", ctypes.byref(v), self.h)
        return v.value

    def free(self):
        if self.h:
            call_nomsg("lagr_graph_free", ctypes.byref(self.h))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------ algorithms

TC_DEFAULT, TC_DOT, TC_MXM = 0, 1, 2


def lagr_tc(G: Graph, ctx: Context, method: int = TC_DEFAULT) -> int:
    t = ctypes.c_int64()
    call("lagr_tc", ctypes.byref(t), G.h, method, ctx.h)
    return t.value


def lagr_tc_adv(G: Graph, ctx: Context) -> int:
    t = ctypes.c_int64()
    call("lagr_tc_adv", ctypes.byref(t), G.h, ctx.h)
    return t.value


def lagr_tc_adv_noalloc(G: Graph, out, ctx: Context):
    """Allocation-free count into `out`, a one-element int64 device tensor;
    queued on ctx's stream, no synchronisation."""
    assert out.dtype == torch.int64 and out.is_cuda and out.numel() >= 1
    call("lagr_tc_adv_noalloc", _ptr(out), G.h, ctx.h)
    return out


def lagr_property_tc_lower(G: Graph, ctx: Context):
    call("lagr_property_tc_lower", G.h, ctx.h)


def lagr_bfs(G: Graph, source: int, ctx: Context, flags: int = 0, want_level=True, want_parent=True):
    lv, pv = ctypes.c_void_p(), ctypes.c_void_p()
    call("lagr_bfs", ctypes.byref(lv) if want_level else None,
         ctypes.byref(pv) if want_parent else None, G.h, source, flags, ctx.h)
    return (Vector(lv) if want_level else None), (Vector(pv) if want_parent else None)


def lagr_sssp(G: Graph, source: int, delta: float, ctx: Context) -> Vector:
    out = ctypes.c_void_p()
    call("lagr_sssp", ctypes.byref(out), G.h, int(source), float(delta), ctx.h)
    return Vector(out)


def lagr_pagerank(G: Graph, ctx: Context, damping=0.85, tol=1e-4, itermax=100):
    """-> (rank Vector, iterations run)."""
    out, it = ctypes.c_void_p(), ctypes.c_int64()
    call("lagr_pagerank", ctypes.byref(out), ctypes.byref(it), G.h, float(damping), float(tol), int(itermax),
         ctx.h)
    return Vector(out), it.value


def lagr_cc(G: Graph, ctx: Context):
    """-> (component label Vector, FastSV iterations run)."""
    out, it = ctypes.c_void_p(), ctypes.c_int64()
    call("lagr_cc", ctypes.byref(out), ctypes.byref(it), G.h, ctx.h)
    return Vector(out), it.value


def lagr_bfs_batch(G: Graph, sources, ctx: Context, want_levels=True):
    """Multi-source BFS: (levels int32 device tensor [ns, n] or None,
    reached, level_sum, depth as int64 numpy arrays)."""
    import numpy as np
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
    ns = src.size
    n = G.matrix().info()[1]
    lev = torch.empty((ns, n), dtype=torch.int32, device="cuda") if want_levels and ns else None
    reached = np.zeros(ns, dtype=np.int64)
    lsum = np.zeros(ns, dtype=np.int64)
    depth = np.zeros(ns, dtype=np.int64)
    call("lagr_bfs_batch", _ptr(lev), reached.ctypes.data_as(ctypes.c_void_p),
         lsum.ctypes.data_as(ctypes.c_void_p), depth.ctypes.data_as(ctypes.c_void_p), G.h,
         src.ctypes.data_as(ctypes.c_void_p), ns, ctx.h)
    return lev, reached, lsum, depth


def lagr_bfs_autotune(G: Graph, sources, ctx: Context):
    import numpy as np
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
    a, b = ctypes.c_int32(), ctypes.c_int32()
    call("lagr_bfs_autotune", ctypes.byref(a), ctypes.byref(b), G.h, src.ctypes.data_as(ctypes.c_void_p),
         src.size, ctx.h)
    return a.value, b.value


def lagr_tc_autotune(G: Graph, ctx: Context) -> int:
    h = ctypes.c_int64()
    call("lagr_tc_autotune", ctypes.byref(h), G.h, ctx.h)
    return h.value


BC_BACKWARD_PUSH_PULL, BC_BACKWARD_PUSH_ONLY = 1, 2


def lagr_bc(G: Graph, sources, ctx: Context, flags: int = 0) -> Vector:
    import numpy as np
    s = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
    out = ctypes.c_void_p()
    if flags:
        call("lagr_bc_dir", ctypes.byref(out), G.h, ctypes.c_void_p(s.ctypes.data), s.size, flags, ctx.h)
    else:
        call("lagr_bc", ctypes.byref(out), G.h, ctypes.c_void_p(s.ctypes.data), s.size, ctx.h)
    return Vector(out)


# ----------------------------------------------------------- operations

def lagr_mxm(C: Matrix, M, accum, semiring, A: Matrix, B: Matrix, desc, ctx: Context):
    return call("lagr_mxm", C.h, None if M is None else M.h, accum, semiring, A.h, B.h, desc, ctx.h)


def lagr_vxm(w: Vector, m, accum, semiring, u: Vector, A: Matrix, desc, ctx: Context):
    return call("lagr_vxm", w.h, None if m is None else m.h, accum, semiring, u.h, A.h, desc, ctx.h)


def lagr_mxm_reduce(M: Matrix, semiring, A: Matrix, B: Matrix, desc, ctx: Context, fp64=False):
    s = ctypes.c_double() if fp64 else ctypes.c_int64()
    call("lagr_mxm_reduce", ctypes.byref(s), M.h, semiring, A.h, B.h, desc, ctx.h)
    return s.value


def lagr_reduce_scalar(A: Matrix, monoid, ctx: Context, accum=NOOP, init=None, fp64=False):
    s = _scalar(A.info()[0], init)
    rc = call("lagr_reduce_scalar", ctypes.byref(s), accum, monoid, A.h, ctx.h)
    return None if rc == NO_VALUE and init is None else s.value


def lagr_vector_reduce_scalar(u: Vector, monoid, ctx: Context, accum=NOOP, init=None, fp64=False):
    s = _scalar(u.info()[0], init)
    rc = call("lagr_vector_reduce_scalar", ctypes.byref(s), accum, monoid, u.h, ctx.h)
    return None if rc == NO_VALUE and init is None else s.value


def lagr_reduce_rows(w: Vector, m, accum, monoid, A: Matrix, desc, ctx: Context):
    return call("lagr_reduce_rows", w.h, None if m is None else m.h, accum, monoid, A.h, desc, ctx.h)


def lagr_assign_vector(w: Vector, m, accum, u: Vector, desc, ctx: Context):
    return call("lagr_assign_vector", w.h, None if m is None else m.h, accum, u.h, desc, ctx.h)


def lagr_assign_scalar(w: Vector, m, accum, s, desc, ctx: Context, fp64=False):
    x = _scalar(w.info()[0], s)
    return call("lagr_assign_scalar", w.h, None if m is None else m.h, accum, ctypes.byref(x), desc,
                ctx.h)


def lagr_ewise_add(C: Matrix, M, accum, op, A: Matrix, B: Matrix, desc, ctx: Context):
    return call("lagr_ewise_add", C.h, None if M is None else M.h, accum, op, A.h, B.h, desc, ctx.h)


def lagr_ewise_mult(C: Matrix, M, accum, op, A: Matrix, B: Matrix, desc, ctx: Context):
    return call("lagr_ewise_mult", C.h, None if M is None else M.h, accum, op, A.h, B.h, desc, ctx.h)


def lagr_select_tril(A: Matrix, ctx: Context) -> Matrix:
    h = ctypes.c_void_p()
    call("lagr_select_tril", ctypes.byref(h), A.h, ctx.h)
    return Matrix(h)


# ------------------------------------------------------ many-graph batch

class Tune(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("row_charge", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]

    def as_dict(self):
        return {"blocks_per_cu": self.blocks_per_cu, "row_charge": self.row_charge,
                "use_graph": self.use_graph}


for _name, _args in {
    "lagr_batch_new": [_PP, _P, _I64, _P, _C],
    "lagr_batch_info": [_P, _P, _P, _P, _C],
    "lagr_batch_autotune": [ctypes.POINTER(Tune), _P, _P, _C],
    "lagr_tc_batched": [_P, _P, ctypes.POINTER(Tune), _P, _C],
    "lagr_batch_free": [_PP],
}.items():
    if hasattr(_lib, _name):
        _f = getattr(_lib, _name)
        _f.restype = ctypes.c_int
        _f.argtypes = _args
        _fns[_name] = _f


class Batch:
    """Packed triangle-count operands of many graphs (lagr_batch)."""

    def __init__(self, ctx: Context, graphs):
        arr = (ctypes.c_void_p * len(graphs))(*[g.h.value for g in graphs])
        self.h = ctypes.c_void_p()
        call("lagr_batch_new", ctypes.byref(self.h), arr, len(graphs), ctx.h)
        self.n = len(graphs)

    def info(self):
        g, r, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        call("lagr_batch_info", self.h, ctypes.byref(g), ctypes.byref(r), ctypes.byref(e))
        return g.value, r.value, e.value

    def autotune(self, ctx: Context) -> Tune:
        t = Tune()
        call("lagr_batch_autotune", ctypes.byref(t), self.h, ctx.h)
        return t

    def tc(self, ctx: Context, tune: Tune = None):
        import numpy as np
        out = np.empty(self.n, dtype=np.int64)
        call("lagr_tc_batched", ctypes.c_void_p(out.ctypes.data), self.h,
             None if tune is None else ctypes.byref(tune), ctx.h)
        return out

    def free(self):
        if self.h:
            call_nomsg("lagr_batch_free", ctypes.byref(self.h))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------ serving

QUERY_TC, QUERY_BFS, QUERY_BC = 0, 1, 2
BUDGET_EXCEEDED = -11


class ServerConfig(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_bfs_batch", ctypes.c_int32),
                ("max_bc_batch", ctypes.c_int32), ("keep_vectors", ctypes.c_int32),
                ("budget_bytes", ctypes.c_int64), ("max_bc_workers", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class Query(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("nsources", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("sources", ctypes.c_int64 * 8), ("arrival", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("kind", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("triangles", ctypes.c_int64), ("reached", ctypes.c_int64),
                ("level_sum", ctypes.c_int64), ("depth", ctypes.c_int64),
                ("bc_sum", ctypes.c_double), ("bc_max", ctypes.c_double),
                ("arrival", ctypes.c_double), ("start", ctypes.c_double),
                ("done", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerCounts(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("batches", ctypes.c_int64 * 3),
                ("queries", ctypes.c_int64 * 3), ("rejected", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("device_peak_bytes", ctypes.c_int64), ("held_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {"completed": self.completed, "batches": list(self.batches),
                "queries": list(self.queries), "rejected": self.rejected,
                "peak_bytes": self.peak_bytes, "pending": self.pending,
                "device_peak_bytes": self.device_peak_bytes, "held_bytes": self.held_bytes}


for _name, _args in {
    "lagr_server_new": [_PP, _P, _I32, ctypes.POINTER(ServerConfig), _P, _C],
    "lagr_server_clock": [_P, ctypes.POINTER(ctypes.c_double), _C],
    "lagr_server_submit": [_P, ctypes.POINTER(Query), _P, _C],
    "lagr_server_poll": [_P, ctypes.POINTER(Result), _I32, _P, _C],
    "lagr_server_wait": [_P, _I64, ctypes.c_double, _C],
    "lagr_server_result_vector": [_P, _I64, _PP, _P, _C],
    "lagr_server_stats": [_P, ctypes.POINTER(ServerCounts), _C],
    "lagr_server_free": [_PP],
}.items():
    if hasattr(_lib, _name):
        _f = getattr(_lib, _name)
        _f.restype = ctypes.c_int
        _f.argtypes = _args
        _fns[_name] = _f


def make_query(kind, graph, sources=(), arrival=0.0) -> Query:
    q = Query()
    q.kind, q.graph, q.nsources, q.arrival = kind, graph, len(sources), float(arrival)
    for i, s in enumerate(sources):
        q.sources[i] = int(s)
    return q


class Server:
    """Continuous-batching query server (lagr_server).  The graphs must
    outlive it; the binding keeps references to them."""

    def __init__(self, ctx: Context, graphs, workers=2, max_bfs_batch=64, max_bc_batch=8,
                 keep_vectors=False, budget_bytes=64 << 30, max_bc_workers=0):
        self._graphs = list(graphs)
        arr = (ctypes.c_void_p * len(graphs))(*[g.h.value for g in graphs])
        cfg = ServerConfig(workers, max_bfs_batch, max_bc_batch, int(bool(keep_vectors)),
                           int(budget_bytes), int(max_bc_workers), 0)
        self.h = ctypes.c_void_p()
        call("lagr_server_new", ctypes.byref(self.h), arr, len(graphs), ctypes.byref(cfg), ctx.h)

    def clock(self) -> float:
        t = ctypes.c_double()
        call("lagr_server_clock", self.h, ctypes.byref(t))
        return t.value

    def submit(self, q: Query) -> int:
        t = ctypes.c_int64()
        call("lagr_server_submit", self.h, ctypes.byref(q), ctypes.byref(t))
        return t.value

    def poll(self, max_results=4096):
        buf = (Result * max_results)()
        n = ctypes.c_int32()
        call("lagr_server_poll", self.h, buf, max_results, ctypes.byref(n))
        return [buf[i] for i in range(n.value)]

    def wait(self, n_completed, timeout_s=60.0) -> bool:
        return call("lagr_server_wait", self.h, n_completed, float(timeout_s)) == 0

    def result_vector(self, ticket, ctx: Context) -> "Vector":
        h = ctypes.c_void_p()
        call("lagr_server_result_vector", self.h, ticket, ctypes.byref(h), ctx.h)
        return Vector(h)

    def stats(self):
        s = ServerCounts()
        call("lagr_server_stats", self.h, ctypes.byref(s))
        return s.as_dict()

    def free(self):
        if self.h:
            call_nomsg("lagr_server_free", ctypes.byref(self.h))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
