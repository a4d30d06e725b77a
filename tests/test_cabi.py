"""Host-side checks of the C ABI (no GPU): the shared library loads, exports
every function include/lagr.h declares, and rejects bad arguments with the
documented codes before any device work (on a validation-only context)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2104_01661_amd", "liblagr.so")
HDR = os.path.join(ROOT, "include", "lagr.h")

NULL_POINTER, INVALID_VALUE, INVALID_INDEX, DOMAIN_MISMATCH = -1, -2, -3, -4
DIMENSION_MISMATCH, PROPERTY_MISSING = -5, -8
BOOL, INT64, FP64 = 0, 1, 2
PLUS_PAIR, ANY_SECONDI, PLUS_FIRST, MIN_PLUS = 0, 1, 2, 3
NOOP, PLUS, MIN, FIRST, SECOND, TIMES, DIV = range(7)


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*int\s+(lagr_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("liblagr.so not built")
    return ctypes.CDLL(LIB)


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) > 40
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


class Api:
    def __init__(self, lib):
        self.lib = lib
        self.msg = ctypes.create_string_buffer(256)

    def __call__(self, name, *args):
        f = getattr(self.lib, name)
        f.restype = ctypes.c_int
        return f(*args, self.msg)

    @property
    def text(self):
        return self.msg.value.decode()


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


@pytest.fixture()
def api(lib):
    return Api(lib)


@pytest.fixture()
def ctx(api):
    c = ctypes.c_void_p()
    assert api("lagr_ctx_new", ctypes.byref(c), -1, None) == 0
    assert api.text == ""
    yield c
    api.lib.lagr_ctx_free(ctypes.byref(c))


def wrap(api, ctx, typ, nrows, ncols, nvals=1):
    h = ctypes.c_void_p()
    rc = api("lagr_matrix_wrap_csr", ctypes.byref(h), typ, ctypes.c_int64(nrows), ctypes.c_int64(ncols),
             ctypes.c_int64(nvals), FAKE, FAKE, None if typ == BOOL else FAKE, ctx)
    assert rc == 0, api.text
    return h


def vec(api, ctx, typ, n):
    h = ctypes.c_void_p()
    assert api("lagr_vector_wrap_sparse", ctypes.byref(h), typ, ctypes.c_int64(n), ctypes.c_int64(1),
               FAKE, None if typ == BOOL else FAKE, ctx) == 0
    return h


def test_mxm_argument_checks(api, ctx):
    A = wrap(api, ctx, BOOL, 3, 4)
    B = wrap(api, ctx, BOOL, 5, 2)
    C = wrap(api, ctx, INT64, 3, 2)
    B4 = wrap(api, ctx, BOOL, 4, 2)
    Cf = wrap(api, ctx, FP64, 3, 2)
    u32 = ctypes.c_uint32
    assert api("lagr_mxm", C, None, NOOP, PLUS_PAIR, A, B, u32(0), ctx) == DIMENSION_MISMATCH
    assert "A'" in api.text
    assert api("lagr_mxm", Cf, None, NOOP, PLUS_PAIR, A, B4, u32(0), ctx) == DOMAIN_MISMATCH
    assert api("lagr_mxm", C, None, NOOP, 9, A, B4, u32(0), ctx) == INVALID_VALUE
    assert api("lagr_mxm", C, None, NOOP, PLUS_PAIR, A, B4, u32(1 << 12), ctx) == INVALID_VALUE
    assert api("lagr_mxm", C, None, DIV, PLUS_PAIR, A, B4, u32(0), ctx) == DOMAIN_MISMATCH
    assert api("lagr_mxm", None, None, NOOP, PLUS_PAIR, A, B4, u32(0), ctx) == NULL_POINTER
    M = wrap(api, ctx, BOOL, 2, 3)
    assert api("lagr_mxm", C, M, NOOP, PLUS_PAIR, A, B4, u32(0), ctx) == DIMENSION_MISMATCH
    # transposes through the descriptor change the checked shapes
    BT = wrap(api, ctx, BOOL, 2, 4)
    assert api("lagr_mxm", Cf, None, NOOP, MIN_PLUS, A, BT, u32(8), ctx) == DIMENSION_MISMATCH
    for h in (A, B, C, B4, Cf, M, BT):
        api.lib.lagr_matrix_free(ctypes.byref(h))


def test_vxm_reduce_assign_checks(api, ctx):
    A = wrap(api, ctx, BOOL, 4, 6)
    u = vec(api, ctx, BOOL, 4)
    w = vec(api, ctx, INT64, 6)
    w5 = vec(api, ctx, INT64, 5)
    u32 = ctypes.c_uint32
    assert api("lagr_vxm", w5, None, NOOP, ANY_SECONDI, u, A, u32(0), ctx) == DIMENSION_MISMATCH
    assert api("lagr_vxm", w, None, NOOP, ANY_SECONDI, u, A, u32(8), ctx) == INVALID_VALUE
    assert api("lagr_vxm", w, None, NOOP, ANY_SECONDI, u, A, u32(64), ctx) == NULL_POINTER
    wf = vec(api, ctx, FP64, 6)
    assert api("lagr_vxm", wf, None, NOOP, ANY_SECONDI, u, A, u32(0), ctx) == DOMAIN_MISMATCH
    # ASSIGN_PARENT writes the parents into the mask, which must be INT64
    mf = vec(api, ctx, FP64, 6)
    assert api("lagr_vxm", w, mf, NOOP, ANY_SECONDI, u, A, u32(64 | 7), ctx) == DOMAIN_MISMATCH
    s = ctypes.c_int64()
    assert api("lagr_reduce_scalar", ctypes.byref(s), NOOP, TIMES, A, ctx) == INVALID_VALUE
    assert api("lagr_reduce_rows", w5, None, NOOP, PLUS, A, u32(0), ctx) == DIMENSION_MISMATCH
    x = ctypes.c_int64(3)
    assert api("lagr_assign_scalar", w, w5, NOOP, ctypes.byref(x), u32(0), ctx) == DIMENSION_MISMATCH
    b = vec(api, ctx, BOOL, 6)
    assert api("lagr_assign_scalar", b, None, NOOP, ctypes.byref(x), u32(0), ctx) == DOMAIN_MISMATCH
    for h in (u, w, w5, wf, b):
        api.lib.lagr_vector_free(ctypes.byref(h))
    api.lib.lagr_matrix_free(ctypes.byref(A))


def test_graph_and_algorithm_checks(api, ctx):
    R = wrap(api, ctx, BOOL, 3, 4)
    G = ctypes.c_void_p()
    assert api("lagr_graph_new", ctypes.byref(G), ctypes.byref(R), 0, ctx) == DIMENSION_MISMATCH
    A = wrap(api, ctx, BOOL, 5, 5)
    assert api("lagr_graph_new", ctypes.byref(G), ctypes.byref(A), 0, ctx) == 0
    assert A.value is None            # moved into the graph (Listing 1)
    lv, pv = ctypes.c_void_p(), ctypes.c_void_p()
    assert api("lagr_bfs", ctypes.byref(lv), ctypes.byref(pv), G, ctypes.c_int64(5), ctypes.c_uint32(0),
               ctx) == INVALID_INDEX
    assert api("lagr_bfs", ctypes.byref(lv), ctypes.byref(pv), G, ctypes.c_int64(-1), ctypes.c_uint32(0),
               ctx) == INVALID_INDEX
    srcs = (ctypes.c_int64 * 2)(0, 7)
    out = ctypes.c_void_p()
    assert api("lagr_bc", ctypes.byref(out), G, srcs, 2, ctx) == INVALID_INDEX
    t = ctypes.c_int64()
    assert api("lagr_tc_adv", ctypes.byref(t), G, ctx) == PROPERTY_MISSING
    assert "tc_lower" in api.text
    api.lib.lagr_graph_free(ctypes.byref(G))
    api.lib.lagr_matrix_free(ctypes.byref(R))


def test_message_cleared_on_success(api, ctx):
    A = wrap(api, ctx, INT64, 2, 2)
    api.msg.value = b"stale"
    t, r, c, nv = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert api("lagr_matrix_info", A, ctypes.byref(t), ctypes.byref(r), ctypes.byref(c), ctypes.byref(nv)) == 0
    assert api.text == "" and (t.value, r.value, c.value) == (INT64, 2, 2)
    api.lib.lagr_matrix_free(ctypes.byref(A))


class ServerConfig(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_bfs_batch", ctypes.c_int32),
                ("max_bc_batch", ctypes.c_int32), ("keep_vectors", ctypes.c_int32),
                ("budget_bytes", ctypes.c_int64), ("max_bc_workers", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


def test_server_checks(api, ctx):
    S = ctypes.c_void_p()
    good = ServerConfig(2, 64, 8, 0, 1 << 30)
    none = (ctypes.c_void_p * 1)(None)
    assert api("lagr_server_new", ctypes.byref(S), none, 1, ctypes.byref(good), ctx) == NULL_POINTER
    assert api("lagr_server_new", ctypes.byref(S), none, 0, ctypes.byref(good), ctx) == INVALID_VALUE
    for bad in (ServerConfig(0, 64, 8, 0, 1 << 30), ServerConfig(17, 64, 8, 0, 1 << 30),
                ServerConfig(2, 65, 8, 0, 1 << 30), ServerConfig(2, 64, 9, 0, 1 << 30),
                ServerConfig(2, 64, 8, 0, 0), ServerConfig(2, 64, 8, 0, 1 << 30, 3),
                ServerConfig(2, 64, 8, 0, 1 << 30, -1)):
        assert api("lagr_server_new", ctypes.byref(S), none, 1, ctypes.byref(bad), ctx) == INVALID_VALUE
    A = wrap(api, ctx, BOOL, 5, 5)
    G = ctypes.c_void_p()
    assert api("lagr_graph_new", ctypes.byref(G), ctypes.byref(A), 1, ctx) == 0   # directed
    one = (ctypes.c_void_p * 1)(G.value)
    assert api("lagr_server_new", ctypes.byref(S), one, 1, ctypes.byref(good), ctx) == -9
    assert S.value is None
    assert api("lagr_server_submit", None, None, None) == NULL_POINTER
    assert api.lib.lagr_server_free(ctypes.byref(ctypes.c_void_p())) == 0
    api.lib.lagr_graph_free(ctypes.byref(G))
