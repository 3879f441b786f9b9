"""ctypes declarations of libcountgauss.so (see include/countgauss.h).

The library is loaded on first use.  There is no fallback: if the shared
object is missing or cannot be loaded, every call raises.
"""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcountgauss.so")

CG_OK, CG_EINVAL, CG_ENOSPACE, CG_EUNSUPPORTED, CG_EHIP = 0, 1, 2, 3, 4
CG_DTYPE_F32, CG_DTYPE_F64 = 0, 1
CG_PREC_NATIVE, CG_PREC_BF16, CG_PREC_FP8 = 0, 1, 2
CG_SX_AUTO, CG_SX_ATOMIC, CG_SX_SORTED, CG_SX_BINNED, CG_SX_ROWS, CG_SX_FUSED = 0, 1, 2, 3, 4, 5
CG_KIND_CSR, CG_KIND_DENSE, CG_KIND_ADJOINT, CG_KIND_ADJOINT_CSR = 0, 1, 2, 3
CG_KIND_GAUSSIAN_DENSE, CG_KIND_GAUSSIAN_CSR = 4, 5
CG_KIND_ANCHORS_COUNTGAUSS, CG_KIND_ANCHORS_GAUSSIAN = 6, 7
CG_PROJ_COUNTGAUSS, CG_PROJ_GAUSSIAN = 0, 1
CG_KIND_LEMMA = 8
CG_STREAM_COPY, CG_STREAM_READ, CG_STREAM_WRITE = 0, 1, 2
CG_STREAM_COPY_NT, CG_STREAM_READ_NT, CG_STREAM_WRITE_NT = 3, 4, 5
CG_NORMALS_SINK = 1 << 19

# Every function declared in include/countgauss.h.
EXPORTS = [
    "cg_opts_init", "cg_version", "cg_status_string", "cg_last_error",
    "cg_workspace_bytes", "cg_sketch_csr", "cg_sketch_dense", "cg_sketch_adjoint",
    "cg_sketch_adjoint_csr", "cg_batched_plan", "cg_sketch_batched", "cg_set_tuning",
    "cg_get_tuning", "cg_sketch_csr_noalloc", "cg_gaussian_dense", "cg_gaussian_csr",
    "cg_row_extrema", "cg_anchors_dense", "cg_lemma_stats", "cg_debug_stream", "cg_debug_normals",
    "cg_debug_philox", "cg_debug_hash", "cg_debug_gaussian",
]


class CgOpts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("precision", ctypes.c_int32),
        ("sx_algo", ctypes.c_int32),
        ("kc", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("row_offset", ctypes.c_int64),
        ("sx_out", ctypes.c_void_p),
        ("stage_events", ctypes.c_void_p),
    ]


CG_STAGE_EVENTS = 5

# size of the static scratch buffer behind cg_sketch_csr_noalloc
CG_NOALLOC_SCRATCH_BYTES = 64 << 20


class CgInstance(ctypes.Structure):
    _fields_ = [
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("vals", ctypes.c_void_p),
        ("Y", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("B", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("row_offset", ctypes.c_int64),
        ("ws_off", ctypes.c_int64),
        ("tile_rows", ctypes.c_int64),
        ("tiles", ctypes.c_int32),
        ("ranges", ctypes.c_int32),
        ("bp_shift", ctypes.c_int32),
        ("kc", ctypes.c_int32),
        ("parts", ctypes.c_int32),
        ("gsx_items", ctypes.c_int32),
        ("red_items", ctypes.c_int32),
        ("first_tile", ctypes.c_int32),
        ("first_range", ctypes.c_int32),
        ("first_gsx", ctypes.c_int32),
        ("first_red", ctypes.c_int32),
        ("route", ctypes.c_int32),
    ]


# d classes of the batched tuning table: ceil(log2 d) = 0 .. 10
CG_TUNING_CLASSES = 11


class CountGaussError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} [status {status}]")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t


def load():
    """Load and declare the library (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
            " (there is no CPU fallback)")
    # torch first: its HIP runtime (same soname as the system one) then
    # serves this library too, so torch's stream handles are valid here
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "cg_opts_init": (None, [ctypes.POINTER(CgOpts)]),
        "cg_version": (ctypes.c_int, []),
        "cg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "cg_last_error": (_SZ, [ctypes.c_char_p, _SZ]),
        "cg_workspace_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _I64, _I64, _I64, _I64,
                                              _I64, ctypes.POINTER(CgOpts),
                                              ctypes.POINTER(_SZ)]),
        "cg_sketch_csr": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _I64, _I64, _I64, _I64, _I64,
                                         _U64, _P, ctypes.POINTER(CgOpts)]),
        "cg_sketch_csr_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _I64, _I64, _I64, _I64,
                                                 _I64, _U64, _P, ctypes.POINTER(CgOpts)]),
        "cg_gaussian_dense": (ctypes.c_int, [_P, _I64, ctypes.c_int, _I64, _I64, _I64, _U64, _P,
                                             ctypes.POINTER(CgOpts)]),
        "cg_gaussian_csr": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _I64, _I64, _I64, _I64, _U64,
                                           _P, ctypes.POINTER(CgOpts)]),
        "cg_lemma_stats": (ctypes.c_int, [_P, _P, ctypes.c_int, _I64, _I64, _I64, _P,
                                          ctypes.POINTER(CgOpts)]),
        "cg_row_extrema": (ctypes.c_int, [_P, ctypes.c_int, _I64, _I64, _I64, _P, _P, _P]),
        "cg_anchors_dense": (ctypes.c_int, [_P, _I64, ctypes.c_int, _I64, _I64, _I64, _I64, _U64,
                                            ctypes.c_int, _P, _P, ctypes.POINTER(CgOpts)]),
        "cg_sketch_dense": (ctypes.c_int, [_P, _I64, ctypes.c_int, _I64, _I64, _I64, _I64, _U64,
                                           _P, ctypes.POINTER(CgOpts)]),
        "cg_sketch_adjoint": (ctypes.c_int, [_P, ctypes.c_int, _I64, _I64, _I64, _I64, _U64, _P,
                                             _I64, ctypes.POINTER(CgOpts)]),
        "cg_sketch_adjoint_csr": (ctypes.c_int, [_P, _P, _I64, _P, ctypes.c_int, _I64, _I64, _I64,
                                                 _I64, _U64, _P, ctypes.POINTER(CgOpts)]),
        "cg_batched_plan": (ctypes.c_int, [ctypes.POINTER(CgInstance), _I32,
                                           ctypes.POINTER(CgOpts), ctypes.POINTER(_SZ)]),
        "cg_sketch_batched": (ctypes.c_int, [ctypes.POINTER(CgInstance), _I32,
                                             ctypes.POINTER(CgOpts)]),
        "cg_set_tuning": (ctypes.c_int, [ctypes.POINTER(_I32), ctypes.POINTER(_I32), _I32]),
        "cg_get_tuning": (ctypes.c_int, [ctypes.POINTER(_I32), ctypes.POINTER(_I32), _I32]),
        "cg_debug_stream": (ctypes.c_int, [ctypes.c_int, _P, _P, _I64, _P]),
        "cg_debug_normals": (ctypes.c_int, [_U64, _I64, _I64, _P, _P]),
        "cg_debug_philox": (ctypes.c_int, [_U64, _P, _I64, _P, _P]),
        "cg_debug_hash": (ctypes.c_int, [_U64, _I64, _U64, _I64, _P, _P, _P]),
        "cg_debug_gaussian": (ctypes.c_int, [_U64, _I64, _I64, _I64, ctypes.c_int, _P, _P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error():
    lib = load()
    buf = ctypes.create_string_buffer(1024)
    lib.cg_last_error(buf, len(buf))
    return buf.value.decode(errors="replace")


def check(status, what):
    if status != CG_OK:
        raise CountGaussError(status, f"{what}: {load().cg_status_string(status).decode()}: "
                                      f"{last_error()}")


def make_opts(precision=CG_PREC_NATIVE, sx_algo=CG_SX_AUTO, kc=0, stream=None, workspace=None,
              workspace_bytes=0, row_offset=0, sx_out=None):
    o = CgOpts()
    load().cg_opts_init(ctypes.byref(o))
    o.precision = precision
    o.sx_algo = sx_algo
    o.kc = kc
    o.stream = stream
    o.workspace = workspace
    o.workspace_bytes = workspace_bytes
    o.row_offset = row_offset
    o.sx_out = sx_out
    return o
