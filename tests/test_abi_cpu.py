"""The C-ABI on the CPU: the library loads, exports every function the
header declares, and rejects invalid calls before any device work (so these
calls are safe without a GPU; the pointers below are never dereferenced)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "streamblas.h")


@pytest.fixture(scope="module")
def L():
    import paper_2108_02025_amd as sb
    if not os.path.exists(sb.lib_path):
        from paper_2108_02025_amd import build
        build.build(verbose=False)
    return sb.load()


@pytest.fixture()
def h(L):
    hd = ctypes.c_void_p()
    assert L.sb_handle_create(None, 0, None, ctypes.byref(hd)) == 0
    yield hd
    L.sb_handle_destroy(hd)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sb_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_version_and_status_strings(L):
    assert L.sb_version() == 100
    assert L.sb_status_string(0) == b"success"
    assert L.sb_status_string(-1) == b"invalid argument"
    assert L.sb_status_string(-2) == b"workspace too small"
    assert L.sb_status_string(-4) == b"unsupported combination"
    assert L.sb_status_string(7) == b"unknown status"


FAKE = 1 << 40          # 16-byte aligned fake device addresses, never touched
A_, X_, C_ = FAKE, FAKE + (1 << 36), FAKE + (2 << 36)


def gemv(L, h, dt=0, layout=0, op=0, m=10, n=10, A=A_, lda=10, x=X_, c=C_):
    return L.sb_gemv(h, dt, layout, op, m, n, A, lda, x, c)


def test_gemv_validation(L, h):
    assert gemv(L, None) == -1
    assert gemv(L, h, dt=2) == -4 and gemv(L, h, dt=3) == -4
    assert gemv(L, h, dt=9) == -1
    assert gemv(L, h, layout=2) == -1 and gemv(L, h, op=5) == -1
    assert gemv(L, h, m=-1) == -1 and gemv(L, h, n=-3) == -1
    assert gemv(L, h, lda=9) == -1                      # row-major needs lda >= n
    assert gemv(L, h, layout=1, m=12, n=5, lda=11) == -1  # column-major needs lda >= m
    assert b"lda" in L.sb_last_error(h)
    assert gemv(L, h, A=None) == -1 and gemv(L, h, x=None) == -1 and gemv(L, h, c=None) == -1
    assert gemv(L, h, A=A_ + 4) == -1                   # not 8-byte aligned for binary64
    assert gemv(L, h, c=A_ + 80) == -1                  # c inside A
    assert gemv(L, h, c=X_ + 8) == -1                   # c overlaps x
    assert gemv(L, h, m=1 << 40, n=1 << 40, lda=1 << 40) == -1  # extent overflow
    # empty outputs / reductions return before any launch, null pointers allowed
    assert gemv(L, h, m=0, A=None, x=None, c=None) == 0
    assert gemv(L, h, n=0, lda=1, A=None, x=None) == 0
    assert gemv(L, h, op=1, m=0, c=None, A=None, x=None) == 0


def test_workspace_sizing_and_enomem(L, h):
    ws = L.sb_workspace_bytes
    assert ws(None, 0, 0, 0, 0, 1024, 1024) == 0          # x fits in LDS: no split
    # few long rows (operand >= 32 MiB): columns split until there are 16
    # waves per compute unit, in chunks of at least 16 KiB
    assert ws(None, 0, 0, 0, 0, 1024, 16384) == 4 * 1024 * 8
    assert ws(None, 0, 0, 0, 0, 512, 16384) == 8 * 512 * 8
    assert ws(None, 0, 0, 0, 0, 4096, 16384) == 0
    assert ws(None, 0, 0, 0, 0, 1024, 4095) == 0          # 32 MiB minus a column: not split
    assert ws(None, 0, 0, 1, 1, 16384, 1024) == 4 * 1024 * 8   # column-major T: same plan
    short_wide = ws(None, 0, 0, 0, 0, 256, 262144)
    assert short_wide > 0 and short_wide % (256 * 8) == 0
    assert ws(None, 0, 0, 1, 1, 262144, 256) == short_wide  # column-major T: same kernel and plan
    assert ws(None, 0, 2, 0, 0, 5, 5) == (1 << 64) - 1      # narrow dtype is not a plain GEMV
    assert ws(None, 1, 0, 0, 0, 1, 1 << 28) > 0            # DOT partial sums
    assert ws(None, 2, 0, 0, 0, 100, 100) == 0             # GER needs none
    assert ws(None, 4, 1, 0, 0, 1, 1 << 27) == 2 * ws(None, 1, 1, 0, 0, 1, 1 << 27)
    # no workspace on the handle: calls that need it fail before launching
    assert gemv(L, h, m=256, n=262144, lda=262144, x=X_, c=C_) == -2
    assert b"workspace" in L.sb_last_error(h)
    assert L.sb_dot(h, 0, 1 << 20, X_, A_, C_) == -2
    assert L.sb_dot2_f32(h, 1 << 20, X_, A_, C_) == -2


def test_small_problem_plans(L, h):
    """Below the cutoffs DOT, Dot2 and GEMV-T run as one launch without
    workspace; just above they use the two-stage form.  Cutoffs are per
    handle and settable."""
    ws = L.sb_workspace_bytes
    v = ctypes.c_int64()
    assert L.sb_get_cutoff(None, 0, ctypes.byref(v)) == 0 and v.value == 256 * 1024
    assert L.sb_get_cutoff(None, 1, ctypes.byref(v)) == 0 and v.value == 2
    cut64, cut32 = 16384, 32768                       # 256 KiB of x and y together
    assert ws(None, 1, 0, 0, 0, 1, cut64) == 0 and ws(None, 1, 0, 0, 0, 1, cut64 + 1) > 0
    assert ws(None, 1, 1, 0, 0, 1, cut32) == 0 and ws(None, 1, 1, 0, 0, 1, cut32 + 1) > 0
    assert ws(None, 4, 1, 0, 0, 1, cut32) == 0 and ws(None, 4, 1, 0, 0, 1, cut32 + 1) > 0
    # row-major T, 16384 columns (128 column blocks of binary64): a 2-way row
    # split (128 <= rows < 192) is replaced by one workgroup of 16 waves per
    # column block
    assert ws(None, 0, 0, 0, 1, 127, 16384) == 0     # no split anyway
    assert ws(None, 0, 0, 0, 1, 128, 16384) == 0
    assert ws(None, 0, 0, 0, 1, 191, 16384) == 0
    assert ws(None, 0, 0, 0, 1, 192, 16384) == 3 * 16384 * 8
    assert ws(None, 0, 0, 1, 0, 16384, 150) == 0     # column-major N: the same kernel
    assert ws(None, 0, 0, 0, 1, 1024, 1024) == 16 * 1024 * 8
    # per-handle overrides
    assert L.sb_set_cutoff(h, 0, 0) == 0 and ws(h, 1, 0, 0, 0, 1, 100) > 0
    assert L.sb_set_cutoff(h, 0, 1 << 30) == 0 and ws(h, 1, 0, 0, 0, 1, 1 << 20) == 0
    assert L.sb_get_cutoff(h, 0, ctypes.byref(v)) == 0 and v.value == 1 << 30
    assert L.sb_set_cutoff(h, 1, 0) == 0 and ws(h, 0, 0, 0, 1, 150, 16384) == 2 * 16384 * 8
    assert L.sb_set_cutoff(h, 1, 16) == 0 and ws(h, 0, 0, 0, 1, 1024, 1024) == 0
    assert L.sb_set_cutoff(h, 1, -1) == -1 and L.sb_set_cutoff(h, 7, 1) == -1
    assert L.sb_set_cutoff(None, 0, 1) == -1 and L.sb_get_cutoff(h, 0, None) == -1


def test_gemv2_validation_and_workspace(L, h):
    Y_, D_ = FAKE + (3 << 36), FAKE + (4 << 36)

    def g2(dt=0, layout=0, m=10, n=12, A=A_, lda=12, x=X_, y=Y_, c=C_, d=D_):
        return L.sb_gemv2(h, dt, layout, m, n, A, lda, x, y, c, d)
    assert L.sb_gemv2(None, 0, 0, 1, 1, A_, 1, X_, Y_, C_, D_) == -1
    assert g2(dt=2) == -4 and g2(dt=5) == -4 and g2(dt=9) == -1 and g2(layout=3) == -1
    assert g2(m=-1) == -1 and g2(lda=11) == -1 and g2(layout=1, lda=9) == -1
    assert g2(A=None) == -1 and g2(y=None) == -1 and g2(d=None) == -1
    assert g2(d=A_ + 8) == -1                      # d inside A
    assert g2(c=D_ + 16) == -1                     # c overlaps d
    assert g2(c=Y_) == -1 and g2(d=X_ + 8) == -1   # outputs overlap inputs
    assert g2(m=4096, n=4096, lda=4096, y=X_) == -2   # x and y may alias; no workspace here
    assert g2(m=0, A=None, x=None, y=None, c=None, d=None) == 0
    assert g2(n=0, lda=1, A=None, x=None, y=None, c=None, d=None) == 0
    ws = L.sb_workspace_bytes
    # 16384 x 16384 binary64: 8 column bands of 2048 and 32 row bands of 512
    # 8-wave bands of 1024 columns (16 bands), 16 row bands of 1024 rows
    assert ws(None, 6, 0, 0, 0, 16384, 16384) == 16 * 16384 * 8 + 16 * 16384 * 8
    assert ws(None, 6, 0, 1, 0, 16384, 16384) == ws(None, 6, 0, 0, 0, 16384, 16384)
    assert ws(None, 6, 0, 0, 0, 64, 64) == 0       # one band each way: direct update
    assert ws(None, 6, 2, 0, 0, 64, 64) == (1 << 64) - 1


def test_mx_validation_and_workspace(L, h):
    S_ = FAKE + (5 << 36)
    qz = L.sb_quantize_mx
    assert qz(h, 3, 4, 64, A_, 64, C_, 64, S_, 2) == -1      # not an MX type
    assert qz(h, 4, 4, 64, A_, 63, C_, 64, S_, 2) == -1      # lda < n
    assert qz(h, 4, 4, 64, A_, 64, C_, 48, S_, 2) == -1      # ldq below the row bytes
    assert qz(h, 5, 4, 64, A_, 64, C_, 40, S_, 2) == -1      # ldq not a multiple of 16
    assert qz(h, 5, 4, 64, A_, 64, C_, 32, S_, 1) == -1      # lds below ceil(n/32)
    assert qz(h, 5, 4, 64, A_, 64, C_ + 8, 32, S_, 2) == -1  # Q not 16-byte aligned
    assert qz(h, 4, 4, 64, A_, 64, A_ + 64, 64, S_, 2) == -1  # Q overlaps A
    assert qz(h, 4, 0, 64, None, 64, None, 64, None, 2) == 0
    gm = L.sb_gemv_mx
    assert gm(h, 2, 4, 64, C_, 64, S_, 2, X_, A_) == -1
    assert gm(h, 4, 4, 64, C_, 64, S_, 2, X_, S_ + 2) == -1   # c overlaps S
    assert gm(h, 5, 4, 64, C_, 32, S_, 2, None, A_) == -1
    assert gm(h, 5, 4, 0, None, 16, None, 1, None, A_) == 0   # empty rows: c unchanged
    # rows of 40000 binary32 x values are split in 8192-column chunks
    assert L.sb_workspace_bytes(None, 7, 4, 0, 0, 1000, 40000) == 5 * 1000 * 4
    assert L.sb_workspace_bytes(None, 7, 5, 0, 0, 1000, 16384) == 0
    assert L.sb_workspace_bytes(None, 7, 3, 0, 0, 1000, 100) == (1 << 64) - 1
    assert gm(h, 4, 1000, 40000, C_, 40000, S_, 1250, X_, A_) == -2   # no workspace
    assert L.sb_gemv(h, 4, 0, 0, 4, 4, A_, 4, X_, C_) == -4          # MX types are storage only


def test_plan_validation(L, h):
    import paper_2108_02025_amd as sb
    p = ctypes.c_void_p()
    arr = (sb.sb_gemv_desc * 1)(_desc(sb, 1, 100, 100, A_, C_))
    assert L.sb_plan_create(h, arr, 1, None) == -1
    assert L.sb_plan_create(None, arr, 1, ctypes.byref(p)) == -1
    assert L.sb_plan_create(h, arr, 1, ctypes.byref(p)) == -2 and not p.value   # no workspace
    bad = (sb.sb_gemv_desc * 1)(_desc(sb, 1, 10, 10, A_, C_, group=3))
    assert L.sb_plan_create(h, bad, 1, ctypes.byref(p)) == -1
    empty = (sb.sb_gemv_desc * 1)(_desc(sb, 1, 0, 10, 0, 0, x=0))
    assert L.sb_plan_create(h, empty, 1, ctypes.byref(p)) == 0 and p.value
    assert L.sb_plan_run(p) == 0               # nothing to launch
    assert L.sb_plan_destroy(p) == 0
    assert L.sb_plan_run(None) == -1 and L.sb_plan_destroy(None) == 0


def test_dot_ger_quant_validation(L, h):
    assert L.sb_dot(h, 0, -1, X_, A_, C_) == -1
    assert L.sb_dot(h, 0, 10, X_, A_, None) == -1
    assert L.sb_dot(h, 0, 10, X_, A_, X_ + 16) == -1       # alpha inside x
    assert L.sb_dot(h, 2, 10, X_, A_, C_) == -4
    assert L.sb_dot(h, 0, 0, None, None, C_) == 0           # empty: alpha unchanged, no launch
    assert L.sb_ger(h, 0, 0, 4, 5, X_, A_, C_, 4) == -1     # ldc < n
    assert L.sb_ger(h, 0, 0, 4, 5, C_ + 8, A_, C_, 5) == -1  # x inside C
    assert L.sb_ger(h, 0, 0, 0, 5, None, None, None, 5) == 0
    assert L.sb_quantize_rows(h, 0, 4, 4, A_, 4, C_, 4, X_) == -1   # q must be narrow
    assert L.sb_quantize_rows(h, 2, 4, 4, A_, 3, C_, 4, X_) == -1   # lda < n
    assert L.sb_quantize_rows(h, 2, 4, 4, A_, 4, A_, 4, X_) == -1   # Aq overlaps A
    assert L.sb_gemv_q(h, 1, 4, 4, A_, 4, X_, X_, C_) == -1          # q must be narrow
    assert L.sb_gemv_q(h, 3, 4, 4, A_, 4, X_, X_ + 64, X_ + 4) == -1  # c overlaps scales
    assert L.sb_dot2_f32(h, 5, X_ + 2, A_, C_) == -1                 # misaligned x


def test_handle_errors(L):
    assert L.sb_handle_create(None, 16, None, None) == -1
    hd = ctypes.c_void_p()
    assert L.sb_handle_create(None, 16, None, ctypes.byref(hd)) == -1
    assert b"workspace" in L.sb_last_error(None)
    assert L.sb_set_stream(None, None) == -1
    assert L.sb_handle_destroy(None) == 0


def _desc(sbmod, dtype, m, n, A, c, x=X_, lda=None, scales=0, layout=0, op=0, **cfg):
    d = sbmod.sb_gemv_desc()
    d.dtype, d.m, d.n, d.lda = dtype, m, n, lda or max(n if layout == 0 else m, 1)
    d.A, d.x, d.c, d.scales = A, x, c, scales or None
    d.group, d.rows_per_tile, d.split = cfg.get("group", 0), cfg.get("rows_per_tile", 0), cfg.get("split", 0)
    d.layout, d.op = layout, op
    return d


def test_batched_resolve_encode_on_host(L):
    """Descriptor resolution and table encoding are pure host work."""
    import struct

    import paper_2108_02025_amd as sb
    arr = (sb.sb_gemv_desc * 3)()
    arr[0] = _desc(sb, 1, 1000, 16384, A_, C_)                      # binary32: x fits one 64 KiB chunk
    arr[1] = _desc(sb, 0, 64, 20000, A_ + (1 << 30), C_ + (1 << 20))  # binary64: needs 3 chunks
    arr[2] = _desc(sb, 2, 5, 7, A_ + (2 << 30), C_ + (2 << 20), scales=X_ + 4096, group=8, rows_per_tile=32)
    out = (sb.sb_gemv_desc * 3)()
    assert L.sb_gemv_batched_resolve(arr, 3, out) == 0
    assert out[0].split == 1 and out[1].split == 3
    assert (out[2].group, out[2].rows_per_tile, out[2].split) == (8, 32, 1)
    # codes whose rows are not 16-byte aligned read x from two shifted
    # copies: chunks of at most 8192 columns, a given split raised to that
    odd = (sb.sb_gemv_desc * 3)(_desc(sb, 2, 100, 8191, A_, C_, scales=X_, split=1),
                                _desc(sb, 2, 100, 12289, A_ + (1 << 30), C_ + (1 << 20), scales=X_ + 4096, split=1),
                                _desc(sb, 2, 100, 12288, A_ + (2 << 30), C_ + (2 << 20), scales=X_ + 8192, split=1))
    odd_out = (sb.sb_gemv_desc * 3)()
    assert L.sb_gemv_batched_resolve(odd, 3, odd_out) == 0
    assert [odd_out[k].split for k in range(3)] == [1, 2, 1]
    for k in range(3):
        assert out[k].group in (4, 8, 16, 32, 64) and out[k].rows_per_tile % (4 * 64 // out[k].group) == 0
    img = ctypes.c_size_t(0)
    total = L.sb_gemv_batched_table_bytes(arr, 3, ctypes.byref(img))
    assert total >= img.value > 64 + 3 * 144
    buf = (ctypes.c_ubyte * img.value)()
    dev_table = 1 << 44
    assert L.sb_gemv_batched_encode(arr, 3, ctypes.c_void_p(dev_table), buf, img.value) == 0
    count, ntiles, total_cost = struct.unpack_from("<qqq", buf, 0)
    tiles, cost = [], 0
    for k in range(3):
        rec = 64 + 144 * k
        dtype, G, RT, S = struct.unpack_from("<iiii", buf, rec)
        m, n, lda, KC, tile0, rtiles, cost0, tile_cost = struct.unpack_from("<qqqqqqqq", buf, rec + 16)
        assert (dtype, G, RT, S) == (arr[k].dtype, out[k].group, out[k].rows_per_tile, out[k].split)
        assert KC % 16 == 0 and KC * S >= n and rtiles == -(-m // RT)
        assert cost0 == cost and tile_cost >= 37      # every tile carries its fixed 0.37 us (10 ns units)
        cost += tile_cost * rtiles * S
        tiles.append((tile0, rtiles * S))
    assert count == 3 and tiles[0][0] == 0 and total_cost == cost
    assert tiles[1][0] == tiles[0][1] and tiles[2][0] == tiles[1][0] + tiles[1][1]
    assert ntiles == sum(t for _, t in tiles)
    # work items: every tile of every problem exactly once, dealt to the
    # workgroups so that no workgroup's cost exceeds both its even share and
    # the lightest one's plus the largest item (the largest-first greedy rule)
    nitems, items_off, lists_off, grid = struct.unpack_from("<qqqi", buf, 24)
    assert items_off == 64 + 3 * 144 and lists_off == items_off + 16 * nitems and grid == 1024
    lists = struct.unpack_from(f"<{grid + 1}i", buf, lists_off)
    assert lists[0] == 0 and lists[-1] == nitems and all(a <= b for a, b in zip(lists, lists[1:]))
    costs = [struct.unpack_from("<q", buf, 64 + 144 * k + 16 + 56)[0] for k in range(3)]
    seen = [set() for _ in range(3)]
    loads, biggest = [], 0
    for b in range(grid):
        load = 0
        for j in range(lists[b], lists[b + 1]):
            prob, cnt, first = struct.unpack_from("<iiq", buf, items_off + 16 * j)
            assert cnt >= 1 and not seen[prob] & set(range(first, first + cnt))
            seen[prob] |= set(range(first, first + cnt))
            load += cnt * costs[prob]
            biggest = max(biggest, cnt * costs[prob])
        loads.append(load)
    assert [len(t) for t in seen] == [t for _, t in tiles]
    share = -(-total_cost // grid)
    assert max(loads) <= max(share, min(loads) + biggest)


def test_batched_items_dealt_evenly_large_batch(L):
    """A batch with more work items than workgroups: the items are dealt in
    alternating rounds, largest first; every tile is run exactly once and no
    workgroup ends above another by more than the largest item.  The deal is
    exactly the snake over the items ordered by (-cost, creation index)."""
    import struct

    import numpy as np

    import paper_2108_02025_amd as sb
    rng = np.random.default_rng(3)
    count = 300
    arr = (sb.sb_gemv_desc * count)()
    for k in range(count):
        m, n = (int(v) for v in np.exp(rng.uniform(np.log(64), np.log(8192), 2)))
        dt = 1 if k % 2 else 2
        arr[k] = _desc(sb, dt, m, n, A_ + (k << 31), C_ + (k << 20), scales=(X_ + (k << 20)) if dt == 2 else 0)
    img = ctypes.c_size_t(0)
    L.sb_gemv_batched_table_bytes(arr, count, ctypes.byref(img))
    buf = (ctypes.c_ubyte * img.value)()
    assert L.sb_gemv_batched_encode(arr, count, ctypes.c_void_p(1 << 44), buf, img.value) == 0
    _, ntiles, total_cost, nitems, items_off, lists_off, grid = struct.unpack_from("<qqqqqqi", buf, 0)
    assert nitems > grid == 1024
    lists = struct.unpack_from(f"<{grid + 1}i", buf, lists_off)
    recs = [struct.unpack_from("<iiii8q", buf, 64 + 144 * k) for k in range(count)]
    tiles = [r[9] * r[3] for r in recs]          # row tiles x splits
    cost = [r[11] for r in recs]                 # per-tile cost
    seen = [np.zeros(t, dtype=np.int32) for t in tiles]
    loads, biggest, dealt = [], 0, {}
    for b in range(grid):
        load, prev = 0, (-1, -1)
        for j in range(lists[b], lists[b + 1]):
            prob, cnt, first = struct.unpack_from("<iiq", buf, items_off + 16 * j)
            assert (prob, first) > prev            # problem and tile order within a group
            prev = (prob, first)
            dealt[prob, first] = (cnt, b)
            seen[prob][first:first + cnt] += 1
            load += cnt * cost[prob]
            biggest = max(biggest, cnt * cost[prob])
        loads.append(load)
    assert all(np.all(v == 1) for v in seen) and sum(tiles) == ntiles
    assert sum(loads) == total_cost and max(loads) - min(loads) <= biggest
    created = sorted(dealt)                        # creation order: problem, then tile
    order = sorted(range(len(created)), key=lambda j: (-dealt[created[j]][0] * cost[created[j][0]], j))
    for k, j in enumerate(order):
        rnd, pos = divmod(k, grid)
        assert dealt[created[j]][1] == (grid - 1 - pos if rnd & 1 else pos)


def test_fill_counter_range(L, h):
    """Binary32 fills take two values per counter pair, so their counter
    range may not wrap past 2^64; binary64 fills may."""
    out = ctypes.c_void_p(FAKE)
    top = (1 << 64) - 1
    assert L.sb_fill_uniform(h, 1, out, 2, ctypes.c_uint64(top), ctypes.c_uint64(top)) == -1
    assert b"wrap" in L.sb_last_error(h)
    assert L.sb_fill_uniform(h, 1, out, 0, ctypes.c_uint64(0), ctypes.c_uint64(top)) == 0


def test_batched_validation(L):
    import paper_2108_02025_amd as sb
    bad = [
        _desc(sb, 1, 10, 10, A_, C_, group=3),                 # group not a power of two in 4..64
        _desc(sb, 1, 10, 10, A_, C_, group=64, rows_per_tile=3),  # not a multiple of 4 rows
        _desc(sb, 0, 10, 10000, A_, C_, split=1),              # binary64 chunk of 10000 > 4096 columns
        _desc(sb, 1, 10, 10, A_, C_, lda=5),                   # lda < n
        _desc(sb, 2, 10, 10, A_, C_),                          # codes without scales
        _desc(sb, 7, 10, 10, A_, C_),                          # bad dtype
    ]
    for d in bad:
        arr = (sb.sb_gemv_desc * 1)(d)
        assert L.sb_gemv_batched_table_bytes(arr, 1, None) == (1 << 64) - 1
    two = (sb.sb_gemv_desc * 2)(_desc(sb, 1, 10, 10, A_, C_), _desc(sb, 1, 10, 10, A_, C_ + 20))
    assert L.sb_gemv_batched_resolve(two, 2, (sb.sb_gemv_desc * 2)()) == -1  # outputs overlap
    assert b"overlap" in L.sb_last_error(None)
    empty = (sb.sb_gemv_desc * 1)(_desc(sb, 1, 0, 10, 0, 0, x=0))
    # header, one record, no items, 1025 list offsets, rounded up to 64
    assert L.sb_gemv_batched_table_bytes(empty, 1, None) == (64 + 144 + 4 * 1025 + 63) // 64 * 64


def test_dot2_tree_matches_library_plan(L):
    """The tests' statement of the compensated DOT's tree (tests/dot2_tree.py)
    launches the same number of workgroups as the library (read back through
    the workspace it asks for: one (sum, error) pair of binary32 per
    workgroup, none for the single-workgroup form)."""
    import dot2_tree
    for n in (1, 1000, 32768, 32769, 65536, 100003, 1 << 20, (1 << 24) - 5, 1 << 24, 1 << 27, 3 << 27):
        p = dot2_tree.plan(n)
        ws = L.sb_workspace_bytes(None, 4, 1, 0, 0, 1, n)
        assert ws == (0 if p["small"] else 8 * p["nblocks"]), n
        if not p["small"]:
            assert p["chunk"] % 1024 == 0 and (p["nblocks"] - 1) * p["chunk"] < n <= p["nblocks"] * p["chunk"]
    assert dot2_tree.plan(1 << 27)["nblocks"] == 1024 and dot2_tree.plan(1 << 27)["chunk"] == 131072
    # 128 vectors per lane (+1 tail), 3 + 6 + 3 in the workgroup, 4 + 6 + 3 in
    # the second stage, alpha and its final sum
    assert dot2_tree.path_length(1 << 27) == 129 + 12 + 13 + 2


def test_gemv_noalloc_checks_before_any_hip_call(L, h):
    """sb_gemv_noalloc validates like sb_gemv and refuses a shape whose split
    partial sums exceed its static scratch (4 MiB) before any HIP call."""
    A, X, C = 1 << 44, 1 << 45, (1 << 45) + (1 << 40)
    assert L.sb_gemv_noalloc(h, 0, 0, 0, 65536, 262144, A, 262144, X, C) == -2
    assert b"static scratch" in L.sb_last_error(h)
    assert L.sb_workspace_bytes(h, 0, 0, 0, 0, 65536, 262144) > (4 << 20)
    assert L.sb_gemv_noalloc(h, 2, 0, 0, 10, 10, A, 10, X, C) == -4      # narrow storage
    assert L.sb_gemv_noalloc(h, 9, 0, 0, 10, 10, A, 10, X, C) == -1      # bad dtype
    assert L.sb_gemv_noalloc(h, 0, 0, 0, 10, 10, A, 9, X, C) == -1       # lda below n
    assert L.sb_gemv_noalloc(h, 0, 0, 0, 10, 10, A, 10, X, A + 8) == -1  # c overlaps A
    assert b"sb_gemv_noalloc" in L.sb_last_error(h)
    assert L.sb_gemv_noalloc(h, 0, 0, 0, 0, 10, A, 10, X, C) == 0        # empty output: nothing to do
    assert L.sb_gemv_noalloc(None, 0, 0, 0, 10, 10, A, 10, X, C) == -1


def test_stream_update_validation(L, h):
    C = 1 << 40
    assert L.sb_stream_update(None, C, 4, 4, 4) == -1
    assert L.sb_stream_update(h, C, 4, 8, 4) == -1          # ldc below cols
    assert L.sb_stream_update(h, C, -1, 4, 4) == -1
    assert L.sb_stream_update(h, C + 4, 4, 4, 4) == -1      # not 8-byte aligned
    assert L.sb_stream_update(h, None, 4, 4, 4) == -1
    assert L.sb_stream_update(h, None, 0, 4, 4) == 0        # empty: nothing launched


def test_batched_layouts_resolve_and_encode_on_host(L):
    """(row-major, T) and (column-major, N) are column axpys over the stored
    rows, (column-major, T) a row dot: the records carry the stored shape,
    the form, column blocks of one wave's width and the row chunking."""
    import struct

    import paper_2108_02025_amd as sb
    arr = (sb.sb_gemv_desc * 4)()
    arr[0] = _desc(sb, 1, 1000, 3000, A_, C_, layout=0, op=1)                        # 1000 stored rows of 3000
    arr[1] = _desc(sb, 0, 3000, 70, A_ + (1 << 30), C_ + (1 << 20), layout=1, op=0)  # 70 stored rows of 3000
    arr[2] = _desc(sb, 1, 500, 20000, A_ + (2 << 30), C_ + (2 << 20), layout=1, op=1)  # row dot, 20000 rows of 500
    arr[3] = _desc(sb, 1, 1000, 3001, A_ + (3 << 30), C_ + (3 << 20), layout=0, op=1, rows_per_tile=100)
    out = (sb.sb_gemv_desc * 4)()
    assert L.sb_gemv_batched_resolve(arr, 4, out) == 0
    # binary32, 16-byte rows: 256-column blocks, 32 rows a pass, 256 KiB tiles
    assert (out[0].group, out[0].rows_per_tile, out[0].split) == (0, 256, 4)
    assert (out[1].group, out[1].rows_per_tile, out[1].split) == (0, 96, 1)      # binary64: 128 columns, 70 rows
    assert out[2].group in (4, 8, 16, 32, 64) and out[2].split == 1
    assert (out[3].group, out[3].rows_per_tile, out[3].split) == (0, 100, 10)    # rows of 3001 floats: unaligned
    assert all((out[k].m, out[k].n, out[k].layout, out[k].op) == (arr[k].m, arr[k].n, arr[k].layout, arr[k].op)
               for k in range(4))
    img = ctypes.c_size_t(0)
    total = L.sb_gemv_batched_table_bytes(arr, 4, ctypes.byref(img))
    buf = (ctypes.c_ubyte * img.value)()
    assert L.sb_gemv_batched_encode(arr, 4, ctypes.c_void_p(1 << 44), buf, img.value) == 0
    want = [  # stored rows, stored columns, block or chunk width, output tiles, aligned, column form
        (1000, 3000, 256, 12, 1, 1), (70, 3000, 128, 24, 1, 1), (20000, 500, None, None, 1, 0),
        (1000, 3001, 64, 47, 0, 1)]
    ntiles = 0
    for k, (rows, cols, kc, rt, al, form) in enumerate(want):
        rec = 64 + 144 * k
        dtype, G, RT, S = struct.unpack_from("<iiii", buf, rec)
        m, n, lda, KC, tile0, rtiles = struct.unpack_from("<qqqqqq", buf, rec + 16)
        aligned, colform = struct.unpack_from("<ii", buf, rec + 128)
        assert (m, n, aligned, colform) == (rows, cols, al, form)
        assert (RT, S) == (out[k].rows_per_tile, out[k].split)
        if form:
            assert (KC, rtiles) == (kc, rt)
        else:
            assert rtiles == -(-rows // RT)
        ntiles += rtiles * S
    assert struct.unpack_from("<q", buf, 8)[0] == ntiles
    # partial sums of the split column axpys: S x (output columns) each
    assert total - img.value >= 4 * 3000 * 4 + 10 * 3001 * 4
    # second-stage items: the outputs of each split problem once, 1024 at a time
    nfinish, finish_off = struct.unpack_from("<iq", buf, 52)
    covered = {}
    for j in range(nfinish):
        prob, cnt, first = struct.unpack_from("<iiq", buf, finish_off + 16 * j)
        assert 1 <= cnt <= 1024 and first % 1024 == 0
        covered.setdefault(prob, []).append((first, cnt))
    assert sorted(covered) == [0, 3]                      # the problems with split > 1
    for prob, out_len in ((0, 3000), (3, 3001)):
        spans = sorted(covered[prob])
        assert spans[0][0] == 0 and sum(c for _, c in spans) == out_len
        assert all(a + c == b for (a, c), (b, _) in zip(spans, spans[1:]))


def test_batched_descriptor_mirrors_agree():
    """The serving loop's numpy descriptor and the ctypes one have the C
    struct's layout (80 bytes, checked by a static assertion in the library)."""
    import paper_2108_02025_amd as sb
    from paper_2108_02025_amd.serve import GEMV_DESC
    assert ctypes.sizeof(sb.sb_gemv_desc) == GEMV_DESC.itemsize == 80
    for name, *_ in sb.sb_gemv_desc._fields_:
        assert getattr(sb.sb_gemv_desc, name).offset == GEMV_DESC.fields[name][1], name


def test_batched_layout_validation(L):
    import paper_2108_02025_amd as sb
    bad = [
        (_desc(sb, 1, 10, 10, A_, C_, layout=2), -1),                          # bad layout
        (_desc(sb, 1, 10, 10, A_, C_, op=5), -1),                              # bad op
        (_desc(sb, 1, 10, 20, A_, C_, layout=1, lda=5), -1),                   # column-major lda < m
        (_desc(sb, 1, 10, 10, A_, C_, op=1, group=8), -1),                     # group on a column axpy
        (_desc(sb, 1, 1000, 10, A_, C_, op=1, rows_per_tile=100, split=3), -1),  # chunking disagrees
        (_desc(sb, 2, 10, 10, A_, C_, scales=X_, op=1), -4),                   # codes: row-major N only
        (_desc(sb, 3, 10, 10, A_, C_, scales=X_, layout=1), -4),
    ]
    for d, st in bad:
        arr = (sb.sb_gemv_desc * 1)(d)
        assert L.sb_gemv_batched_table_bytes(arr, 1, None) == (1 << 64) - 1
        assert L.sb_gemv_batched_resolve(arr, 1, (sb.sb_gemv_desc * 1)()) == st
    # a column axpy's output has n entries: 10 x 100 row-major T writes 400 bytes
    two = (sb.sb_gemv_desc * 2)(_desc(sb, 1, 10, 100, A_, C_, op=1), _desc(sb, 1, 10, 10, A_, C_ + 200))
    assert L.sb_gemv_batched_resolve(two, 2, (sb.sb_gemv_desc * 2)()) == -1
    assert b"overlap" in L.sb_last_error(None)
    ok = (sb.sb_gemv_desc * 2)(_desc(sb, 1, 10, 100, A_, C_, op=1), _desc(sb, 1, 10, 10, A_, C_ + 400))
    assert L.sb_gemv_batched_resolve(ok, 2, (sb.sb_gemv_desc * 2)()) == 0
