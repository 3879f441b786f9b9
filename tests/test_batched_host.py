"""Host-side checks of the batched planner and its tuning table (no GPU:
cg_batched_plan only reads the instance shapes and never touches device
memory, so fake non-NULL pointers are enough)."""
import ctypes

import pytest

from paper_1606_05732_amd import _lib as L

FAKE = 0x1000   # never dereferenced by the planner


def _table(shapes):
    t = (L.CgInstance * len(shapes))()
    for i, (n, d, nnz, m, B) in enumerate(shapes):
        c = t[i]
        c.row_ptr, c.col_idx, c.vals, c.Y = FAKE, FAKE, FAKE, FAKE
        c.n, c.d, c.nnz, c.m, c.B = n, d, nnz, m, B
        c.seed = 77 + i
    return t


def _plan(t):
    lib = L.load()
    nbytes = ctypes.c_size_t(0)
    st = lib.cg_batched_plan(t, len(t), None, ctypes.byref(nbytes))
    return st, nbytes.value


@pytest.fixture(autouse=True)
def _default_tuning():
    L.load().cg_set_tuning(None, None, 0)
    yield
    L.load().cg_set_tuning(None, None, 0)


def _ceil(a, b):
    return -(-a // b)


def _rows_route(n, d, nnz, m, B):
    """The planner's route rule, restated: work per column of G (a nonempty
    row, or a bucket) is m normals plus 13 per 16x16x4 MFMA (one per 16
    columns of X and 64 rows of G); the S X route adds 3 per S X element and
    6 per entry, the rows route 4 per entry; nonempty rows <= min(n, nnz)."""
    col = m + 13.0 * _ceil(d, 16) * _ceil(m, 64)
    return min(n, nnz) * col + 4.0 * nnz < B * (col + 3.0 * d) + 6.0 * nnz


def test_plan_fields_follow_the_shapes():
    shapes = [(1, 1, 0, 1, 1), (100000, 8, 5000, 32, 2048), (40000, 64, 90000, 70, 10000),
              (16384, 32, 26000, 32, 32768), (16385, 16, 1, 5, 7)]
    t = _table(shapes)
    st, ws = _plan(t)
    assert st == L.CG_OK, L.last_error()
    first = {"tile": 0, "range": 0, "gsx": 0, "red": 0}
    prev_off = 0
    routes = [_rows_route(*sh) for sh in shapes]
    assert routes == [True, False, False, True, True]   # both routes are covered
    for i, (n, d, nnz, m, B) in enumerate(shapes):
        c = t[i]
        assert c.route == int(routes[i])
        if routes[i]:
            # rows route: no S X work; parts of 4 kc rows, kc = 2048 rows per
            # wavefront in a batch
            assert (c.tile_rows, c.tiles, c.ranges, c.bp_shift) == (0, 0, 0, 0)
            assert c.kc == 2048 and c.parts == _ceil(n, 4 * 2048)
        else:
            # tuning defaults: 16384 rows per tile, kc 512
            assert c.tile_rows == 16384
            assert c.tiles == _ceil(n, 16384)
            # ranges of 2^bp_shift buckets, 2^bp_shift * d <= 8192 (64 KB of int64 cells)
            assert (1 << c.bp_shift) * d <= 8192 < (2 << c.bp_shift) * d or c.bp_shift == 30
            assert c.ranges == _ceil(B, 1 << c.bp_shift)
            assert c.kc == 512 and c.parts == _ceil(B, 4 * 512)
        assert c.gsx_items == c.parts * _ceil(m, 64) * _ceil(d, 64)
        assert c.red_items == _ceil(m * d, 64)
        assert (c.first_tile, c.first_range, c.first_red) == \
            (first["tile"], first["range"], first["red"])
        first["tile"] += c.tiles
        first["range"] += c.ranges
        first["red"] += c.red_items
        assert c.ws_off % 256 == 0 and c.ws_off > prev_off
        prev_off = c.ws_off
    # the contraction queue holds the items of each MFMA width (16-column
    # blocks: ceil(d / 16) below d = 64, else 4) together, in increasing width
    width = lambda d: _ceil(d, 16) if d < 64 else 4
    order = sorted(range(len(shapes)), key=lambda i: (width(shapes[i][1]), i))
    q = 0
    for i in order:
        assert t[i].first_gsx == q
        q += t[i].gsx_items
    # the last instance's scratch (rows route: its partials) fits in the workspace
    n, d, nnz, m, B = shapes[-1]
    assert ws >= t[-1].ws_off + 4 * t[-1].parts * m * d
    # and an S X instance's (items, S X, partials)
    n, d, nnz, m, B = shapes[2]
    assert t[3].ws_off >= t[2].ws_off + 8 * nnz + 4 * B * d + 4 * t[2].parts * m * d


@pytest.mark.parametrize("n,d,nnz,m,B", [
    (16777216, 32, 26847020, 64, 65536), (500000, 64, 64000, 32, 125000), (100000, 16, 800000, 32, 8192),
    (100000, 16, 8000, 32, 8192), (1000000, 8, 16000, 32, 2048), (1000000, 8, 400000, 32, 2048),
    (3000, 130, 9000, 100, 50000), (5, 3, 2, 70, 3),
])
def test_route_follows_the_cost_rule(n, d, nnz, m, B):
    t = _table([(n, d, nnz, m, B)])
    st, _ = _plan(t)
    assert st == L.CG_OK, L.last_error()
    assert t[0].route == int(_rows_route(n, d, nnz, m, B))


def test_tuning_table_drives_the_plan():
    lib = L.load()
    rows = (ctypes.c_int32 * 11)(*([4096] * 11))
    kc = (ctypes.c_int32 * 11)(*([128] * 11))
    assert lib.cg_set_tuning(rows, kc, 11) == L.CG_OK
    t = _table([(100000, 16, 800000, 32, 8192)])   # S X route
    st, _ = _plan(t)
    assert st == L.CG_OK
    assert t[0].route == 0 and t[0].tile_rows == 4096 and t[0].tiles == _ceil(100000, 4096)
    assert t[0].kc == 128 and t[0].parts == _ceil(8192, 512)
    got_r, got_k = (ctypes.c_int32 * 11)(), (ctypes.c_int32 * 11)()
    assert lib.cg_get_tuning(got_r, got_k, 11) == L.CG_OK
    assert list(got_r) == [4096] * 11 and list(got_k) == [128] * 11
    # one column only: the other stays
    kc2 = (ctypes.c_int32 * 5)(*([256] * 5))
    assert lib.cg_set_tuning(None, kc2, 5) == L.CG_OK
    assert lib.cg_get_tuning(got_r, got_k, 11) == L.CG_OK
    assert list(got_k) == [256] * 5 + [128] * 6 and list(got_r) == [4096] * 11
    assert lib.cg_set_tuning(None, None, 0) == L.CG_OK
    assert lib.cg_get_tuning(got_r, got_k, 11) == L.CG_OK
    assert list(got_r) == [16384] * 11 and list(got_k) == [512] * 11


@pytest.mark.parametrize("rows,kc,classes,needle", [
    (1000, 512, 1, "rows_per_item[0]"), (0, 512, 1, "rows_per_item[0]"),
    (4096, 100, 1, "kc_per_item[0]"), (4096, 0, 1, "kc_per_item[0]"),
    (4096, 512, 12, "classes"), (4096, 512, 0, "classes"),
])
def test_bad_tuning_is_rejected(rows, kc, classes, needle):
    lib = L.load()
    k = max(classes, 1)
    r = (ctypes.c_int32 * k)(*([rows] * k))
    c = (ctypes.c_int32 * k)(*([kc] * k))
    assert lib.cg_set_tuning(r, c, classes) == L.CG_EINVAL
    assert needle in L.last_error()


@pytest.mark.parametrize("field,value,status,needle", [
    ("row_ptr", None, L.CG_EINVAL, "row_ptr"), ("Y", None, L.CG_EINVAL, "Y is NULL"),
    ("col_idx", None, L.CG_EINVAL, "col_idx"), ("n", 0, L.CG_EINVAL, "n ="),
    ("d", 0, L.CG_EINVAL, "d ="), ("d", 2000, L.CG_EUNSUPPORTED, "d ="),
    ("m", 0, L.CG_EINVAL, "m ="), ("B", 0, L.CG_EINVAL, "B ="),
    ("nnz", -1, L.CG_EINVAL, "nnz ="), ("row_offset", -5, L.CG_EINVAL, "row_offset"),
])
def test_bad_instances_are_rejected_by_name(field, value, status, needle):
    t = _table([(1000, 8, 10, 4, 64), (1000, 8, 10, 4, 64), (1000, 8, 10, 4, 64)])
    setattr(t[1], field, value)
    st, _ = _plan(t)
    assert st == status
    msg = L.last_error()
    assert "instance 1" in msg and needle in msg, msg


def test_empty_instances_need_no_column_arrays():
    t = _table([(50, 4, 0, 3, 9)])
    t[0].col_idx, t[0].vals = None, None
    st, _ = _plan(t)
    assert st == L.CG_OK, L.last_error()


def test_launch_rejects_stale_plans_and_missing_workspace():
    lib = L.load()
    t = _table([(1000, 8, 10, 4, 64)])
    st, ws = _plan(t)
    assert st == L.CG_OK
    o = L.make_opts(workspace=None, workspace_bytes=0)
    assert lib.cg_sketch_batched(t, 1, None) == L.CG_EINVAL          # no opts
    assert lib.cg_sketch_batched(t, 1, ctypes.byref(o)) == L.CG_ENOSPACE
    o = L.make_opts(workspace=0x100000, workspace_bytes=ws - 256)
    assert lib.cg_sketch_batched(t, 1, ctypes.byref(o)) == L.CG_ENOSPACE
    t[0].kc = 64                                                       # edited after planning
    o = L.make_opts(workspace=0x100000, workspace_bytes=ws)
    assert lib.cg_sketch_batched(t, 1, ctypes.byref(o)) == L.CG_EINVAL
    assert "planned fields differ" in L.last_error()
    o = L.make_opts(precision=L.CG_PREC_BF16, workspace=0x100000, workspace_bytes=ws)
    assert lib.cg_sketch_batched(t, 1, ctypes.byref(o)) == L.CG_EUNSUPPORTED
