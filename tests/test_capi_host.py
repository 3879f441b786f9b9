"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/countgauss.h declares, and rejects bad arguments
before queueing any GPU work."""
import ctypes
import os
import re

import pytest

from paper_1606_05732_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "countgauss.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(cg_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = L.load()
    declared = _declared_functions()
    assert len(declared) >= 15
    assert sorted(declared) == sorted(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    lib = L.load()
    assert lib.cg_version() >= 100
    for st in range(5):
        assert lib.cg_status_string(st)
    assert lib.cg_status_string(99) == b"unknown status"


def test_opts_struct_matches_header_size():
    # uint32 + 3 int32, then six 8-byte fields
    assert ctypes.sizeof(L.CgOpts) == 64
    assert ctypes.sizeof(L.CgInstance) == 152


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


def _err(status, needle):
    assert status != L.CG_OK
    msg = L.last_error()
    assert needle in msg, msg
    return status


@pytest.mark.parametrize("n,d,m,B,needle", [
    (0, 4, 4, 4, "n ="), (10, 0, 4, 4, "d ="), (10, 4, 0, 4, "m ="),
    (10, 4, 4, 0, "B ="), (10, 4, 4, 1 << 31, "B ="),
])
def test_bad_sizes_are_rejected(n, d, m, B, needle):
    lib = L.load()
    o = L.make_opts()
    st = lib.cg_sketch_dense(FAKE, max(d, 1), L.CG_DTYPE_F32, n, d, m, B, 1, FAKE, ctypes.byref(o))
    assert _err(st, needle) == L.CG_EINVAL


def test_unsupported_and_null_and_space():
    lib = L.load()
    o = L.make_opts()
    st = lib.cg_sketch_dense(FAKE, 2000, L.CG_DTYPE_F32, 10, 2000, 4, 4, 1, FAKE, ctypes.byref(o))
    assert _err(st, "d =") == L.CG_EUNSUPPORTED
    st = lib.cg_sketch_csr(FAKE, FAKE, FAKE, L.CG_DTYPE_F32, 10, 4, 1 << 31, 4, 4, 1, FAKE,
                           ctypes.byref(o))
    assert _err(st, "nnz") == L.CG_EUNSUPPORTED
    st = lib.cg_sketch_dense(None, 4, L.CG_DTYPE_F32, 10, 4, 4, 4, 1, FAKE, ctypes.byref(o))
    assert _err(st, "null") == L.CG_EINVAL
    # valid shapes but no workspace
    st = lib.cg_sketch_dense(FAKE, 4, L.CG_DTYPE_F32, 10, 4, 4, 4, 1, FAKE, ctypes.byref(o))
    assert _err(st, "workspace") == L.CG_ENOSPACE
    o.workspace = 0x100000
    o.workspace_bytes = 16
    st = lib.cg_sketch_dense(FAKE, 4, L.CG_DTYPE_F32, 10, 4, 4, 4, 1, FAKE, ctypes.byref(o))
    assert _err(st, "workspace") == L.CG_ENOSPACE
    o.workspace = 0x100010
    st = lib.cg_sketch_dense(FAKE, 4, L.CG_DTYPE_F32, 10, 4, 4, 4, 1, FAKE, ctypes.byref(o))
    assert _err(st, "aligned") == L.CG_EINVAL


def test_option_validation():
    lib = L.load()
    for field, value, needle in [("precision", 9, "precision"), ("sx_algo", 7, "sx_algo"),
                                 ("kc", 24, "kc"), ("row_offset", -1, "row_offset")]:
        o = L.make_opts()
        setattr(o, field, value)
        st = lib.cg_sketch_dense(FAKE, 4, L.CG_DTYPE_F32, 10, 4, 4, 4, 1, FAKE, ctypes.byref(o))
        _err(st, needle)
    o = L.make_opts()
    o.struct_size = 8
    _err(lib.cg_sketch_dense(FAKE, 4, L.CG_DTYPE_F32, 10, 4, 4, 4, 1, FAKE, ctypes.byref(o)),
         "struct_size")
    o = L.make_opts(precision=L.CG_PREC_BF16)
    _err(lib.cg_sketch_dense(FAKE, 4, L.CG_DTYPE_F64, 10, 4, 4, 4, 1, FAKE, ctypes.byref(o)),
         "FP64")
    _err(lib.cg_sketch_adjoint(FAKE, L.CG_DTYPE_F32, 10, 4, 4, 4, 1, FAKE, 4, ctypes.byref(o)),
         "native")


def test_workspace_query_grows_with_problem():
    lib = L.load()
    o = L.make_opts()
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    L.check(lib.cg_workspace_bytes(L.CG_KIND_CSR, L.CG_DTYPE_F32, 1 << 24, 32, 64, 65536,
                                   27_000_000, ctypes.byref(o), ctypes.byref(a)), "ws")
    assert a.value >= 65536 * 32 * 4
    o.sx_algo = L.CG_SX_SORTED
    L.check(lib.cg_workspace_bytes(L.CG_KIND_CSR, L.CG_DTYPE_F32, 1 << 24, 32, 64, 65536,
                                   27_000_000, ctypes.byref(o), ctypes.byref(b)), "ws")
    assert b.value > a.value + 27_000_000 * 16
    o = L.make_opts()
    c = ctypes.c_size_t(0)
    L.check(lib.cg_workspace_bytes(L.CG_KIND_ADJOINT, L.CG_DTYPE_F64, 100, 3, 5, 1000, 0,
                                   ctypes.byref(o), ctypes.byref(c)), "ws")
    assert c.value >= 1000 * 3 * 8 and c.value % 256 == 0


def test_debug_entry_points_validate():
    lib = L.load()
    _err(lib.cg_debug_hash(1, 0, 0, 10, FAKE, FAKE, None), "B =")
    _err(lib.cg_debug_gaussian(1, 0, 0, 10, 0, FAKE, None), "m =")
    _err(lib.cg_debug_philox(1, FAKE, -1, FAKE, None), "count")


def test_noalloc_rejects_what_the_static_buffer_cannot_hold():
    lib = L.load()
    o = L.make_opts()
    # the FP32-at-scale CSR workload needs far more than the static buffer
    need = ctypes.c_size_t(0)
    L.check(lib.cg_workspace_bytes(L.CG_KIND_CSR, L.CG_DTYPE_F32, 1 << 24, 32, 64, 65536,
                                   27_000_000, ctypes.byref(o), ctypes.byref(need)), "ws")
    assert need.value > L.CG_NOALLOC_SCRATCH_BYTES
    st = lib.cg_sketch_csr_noalloc(FAKE, FAKE, FAKE, L.CG_DTYPE_F32, 1 << 24, 32, 27_000_000, 64,
                                   65536, 1, FAKE, ctypes.byref(o))
    assert _err(st, "static buffer") == L.CG_ENOSPACE
    # the usual argument checks come first, and opts may be NULL
    st = lib.cg_sketch_csr_noalloc(FAKE, FAKE, FAKE, L.CG_DTYPE_F32, 0, 4, 10, 4, 4, 1, FAKE, None)
    assert _err(st, "n =") == L.CG_EINVAL
    st = lib.cg_sketch_csr_noalloc(None, FAKE, FAKE, L.CG_DTYPE_F32, 10, 4, 10, 4, 4, 1, FAKE, None)
    assert _err(st, "null") == L.CG_EINVAL


def test_noalloc_buffer_size_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define CG_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == L.CG_NOALLOC_SCRATCH_BYTES
