"""Host logic of the batched path (no GPU): item validation, workspace size,
the tile lists of every pass (each unit of work covered exactly once, under
every schedule) and the tuning-table reader."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1304_2062_amd", "libse2n.so")


class Item(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("N", ctypes.c_int), ("n_steps", ctypes.c_int), ("scheme", ctypes.c_int),
                ("proj", ctypes.c_int), ("reserved", ctypes.c_int), ("T", ctypes.c_double),
                ("beta", ctypes.c_double), ("sigma", ctypes.c_double), ("f", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("rmap_out", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class Tune(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_int), ("order", ctypes.c_int), ("row_groups", ctypes.c_int),
                ("reserved", ctypes.c_int)]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is not built (run python -m paper_1304_2062_amd.build)")
    L = ctypes.CDLL(LIB)
    L.se2n_last_error.restype = ctypes.c_char_p
    L.se2n_batch_workspace_bytes.restype = ctypes.c_size_t
    return L


def items_of(specs, sigmas=None):
    """specs: (M, N, proj) triples; pointers stay NULL (host-only calls)."""
    arr = (Item * len(specs))()
    for k, (M, N, proj) in enumerate(specs):
        sigma = 2.0 if sigmas is None else sigmas[k]
        arr[k] = Item(M, N, 100, 0, proj, 0, 1.0, 1.0, sigma, None, None, None, None)
    return arr


SPECS = [(16, 4, 0), (24, 6, 1), (128, 16, 0), (192, 24, 0), (384, 30, 1), (512, 32, 0), (768, 8, 0),
         (1024, 64, 0), (72, 10, 0)]
# Gaussian widths: 6 at M >= 128 and 1 at M = 768 take the FFT route of the
# orientation step, the others the stencil (6 at M = 24 keeps the whole circle)
SIGMAS = [2.0, 6.0, 6.0, 2.0, 6.0, 2.0, 1.0, 2.0, 2.0]


def stencil_radius(lib, M, sigma):
    g = (ctypes.c_float * 65)()
    r = ctypes.c_int(-1)
    assert lib.se2n_orient_stencil_taps(M, ctypes.c_double(sigma), g, g, ctypes.byref(r)) == 0
    return r.value


def geometry(M):
    """Rows / columns per tile of the FP32 kernels (4096 complex values per workgroup)."""
    H = M // 2
    rows = 8
    while rows * 2 * H <= 4096 and M % (rows * 2) == 0 and rows * 2 <= M:
        rows *= 2
    cols = max(4096 // M, 1)
    ocols = max(4096 // (2 * M), 1)
    return rows, cols, ocols


def paired_cols(M):
    _, cols, _ = geometry(M)
    return cols & ~1 if cols >= 2 else 2


def solve_classes(N):
    """Classes per solve tile: the largest power of two <= 16 whose staged
    propagators fit in 72 KB of LDS, S floats per class (the two packed
    blocks, the second at an odd offset, S = 2 mod 4)."""
    eh = (N // 2) * (N // 2 + 1) // 2
    need = (eh | 1) + eh
    S = need + (6 - need % 4) % 4
    c = 16
    while c > 1 and S * c * 4 > 72 * 1024:
        c //= 2
    return c


def tiles(lib, arr, pass_, tune=None):
    n = ctypes.c_int(0)
    tp = None if tune is None else ctypes.byref(Tune(*tune, 0))
    assert lib.se2n_batch_tiles(arr, len(arr), tp, pass_, None, 0, ctypes.byref(n)) == 0, lib.se2n_last_error()
    buf = (ctypes.c_int * (4 * max(n.value, 1)))()
    assert lib.se2n_batch_tiles(arr, len(arr), tp, pass_, buf, n.value, ctypes.byref(n)) == 0
    return [tuple(buf[4 * k:4 * k + 4]) for k in range(n.value)]


def groups_of(N, proj, row_groups):
    if proj == 1:
        return 1
    g = min(row_groups, N)
    spg = -(-N // g)
    return -(-N // spg)


TUNES = [(2, 0, 1), (0, 1, 1), (1, 0, 2), (4, 1, 4), (2, 0, 64)]


@pytest.mark.parametrize("tune", TUNES)
def test_row_tiles_cover_every_row_block_and_slice_once(lib, tune):
    arr = items_of(SPECS, SIGMAS)
    for pass_ in (0, 2, 3, 6):
        seen = {}
        for (i, rb, sb, se) in tiles(lib, arr, pass_, tune):
            for s in range(sb, se):
                key = (i, rb, s)
                assert key not in seen, (pass_, key)
                seen[key] = 1
        for i, (M, N, proj) in enumerate(SPECS):
            rows, _, _ = geometry(M)
            ns = {0: 1, 2: 2}.get(pass_, N)
            want = {(i, rb, s) for rb in range(M // rows) for s in range(ns)}
            if pass_ in (0, 2) and stencil_radius(lib, M, SIGMAS[i]) > 0:
                want = set()  # orientation by the stencil (pass 9)
            got = {k for k in seen if k[0] == i}
            assert got == want, (pass_, M, N)
            if pass_ in (3, 6):
                per_item = [t for t in tiles(lib, arr, pass_, tune) if t[0] == i]
                assert len(per_item) == (M // rows) * groups_of(N, proj, tune[2])


@pytest.mark.parametrize("tune", TUNES)
def test_column_tiles_partition_every_column_run(lib, tune):
    arr = items_of(SPECS, SIGMAS)
    col = tiles(lib, arr, 4, tune)
    ocol = tiles(lib, arr, 1, tune)
    for i, (M, N, _) in enumerate(SPECS):
        _, cols, ocols = geometry(M)
        K = M // 2 + 1
        starts = sorted(t[1] for t in col if t[0] == i)
        assert starts == list(range(0, N * K, cols))
        ostarts = sorted(t[1] for t in ocol if t[0] == i)
        assert ostarts == ([] if stencil_radius(lib, M, SIGMAS[i]) > 0 else list(range(0, K, ocols)))


@pytest.mark.parametrize("tune", TUNES)
def test_stencil_tiles_cover_every_128_by_32_tile_of_stencil_items(lib, tune):
    """Pass 9 holds exactly the items without FFT-route orientation passes, one
    tile per 128 x 32 block of bins, with the item's compiled radius."""
    arr = items_of(SPECS, SIGMAS)
    st = tiles(lib, arr, 9, tune)
    routes = 0
    for i, (M, N, _) in enumerate(SPECS):
        rad = stencil_radius(lib, M, SIGMAS[i])
        mine = sorted(t[1:] for t in st if t[0] == i)
        nt = -(-M // 128) * -(-M // 32)
        if rad > 0:
            assert mine == [(tt, rad, 0) for tt in range(nt)]
            routes |= 1
        else:
            assert mine == []
            assert any(t[0] == i for t in tiles(lib, arr, 0, tune))
            routes |= 2
    assert routes == 3  # both routes occur in this batch


@pytest.mark.parametrize("tune", TUNES)
def test_paired_inverse_column_tiles_cover_every_pair_once(lib, tune):
    """Pass 8: per slice the pairs (k, M/2-k), k = 0 .. M/4, in blocks of
    pcols/2 pairs; tile = slice * blocks + block."""
    arr = items_of(SPECS)
    pc = tiles(lib, arr, 8, tune)
    for i, (M, N, _) in enumerate(SPECS):
        P = paired_cols(M) // 2
        blocks = -(-(M // 4 + 1) // P)
        got = sorted(t[1] for t in pc if t[0] == i)
        assert got == list(range(N * blocks))
        pairs = sorted({(tt // blocks, k) for tt in got
                        for k in range((tt % blocks) * P, min((tt % blocks + 1) * P, M // 4 + 1))})
        assert pairs == [(r, k) for r in range(N) for k in range(M // 4 + 1)]


@pytest.mark.parametrize("tune", TUNES)
def test_solve_tiles_cover_every_frequency_class_once(lib, tune):
    arr = items_of(SPECS)
    sol = tiles(lib, arr, 5, tune)
    for i, (M, N, _) in enumerate(SPECS):
        Q = M // 4 + 1
        c = solve_classes(N)
        got = sorted((t[1], t[2]) for t in sol if t[0] == i)
        assert got == [(lx, ly) for lx in range(Q) for ly in range(0, Q, c)]
        assert all(t[3] == N for t in sol if t[0] == i)


@pytest.mark.parametrize("tune", TUNES)
def test_clear_tiles_exist_exactly_for_max_items_with_slice_groups(lib, tune):
    arr = items_of(SPECS)
    enc = tiles(lib, arr, 7, tune)
    for i, (M, N, proj) in enumerate(SPECS):
        mine = sorted((t[1], t[2]) for t in enc if t[0] == i)
        if proj == 0 and groups_of(N, proj, tune[2]) > 1:
            pos = 0
            for start, cnt in mine:
                assert start == pos and 0 < cnt <= 8192
                pos += cnt
            assert pos == M * M
        else:
            assert mine == []


def test_orders_are_permutations_and_largest_first_puts_big_images_first(lib):
    arr = items_of(SPECS)
    for pass_ in range(10):
        a = tiles(lib, arr, pass_, (2, 0, 2))
        b = tiles(lib, arr, pass_, (2, 1, 2))
        assert sorted(a) == sorted(b)
        items_b = [t[0] for t in b]
        assert items_b == sorted(items_b)  # image-major order
    lift = tiles(lib, arr, 3, (2, 0, 1))
    # cost per tile is slices x rows x H log H: the M = 1024, N = 64 image leads
    assert lift[0][0] == SPECS.index((1024, 64, 0))


def test_workspace_bytes_is_the_sum_of_per_item_buffers(lib):
    arr = items_of(SPECS)
    b = lib.se2n_batch_workspace_bytes(arr, len(arr))

    def a256(x):
        return (x + 255) // 256 * 256
    # sides 512, 768 and 1024 hold a second, row-blocked spectrum for their inverse passes
    want = sum((2 if M in (512, 768, 1024) else 1) * a256(N * (M // 2 + 1) * M * 8) + a256(M * M * 4) + a256(M * M)
               for M, N, _ in SPECS)
    assert b == want


@pytest.mark.parametrize("spec,what", [
    ((2048, 16, 0), "M"), ((100, 16, 0), "M"), ((12, 4, 0), "M"), ((64, 15, 0), "N"), ((64, 2, 0), "N"),
    ((64, 66, 0), "N"), ((64, 16, 2), "projection"),
])
def test_bad_items_are_rejected_on_the_host(lib, spec, what):
    arr = items_of([SPECS[0], spec])
    assert lib.se2n_batch_workspace_bytes(arr, 2) == 0
    assert what in lib.se2n_last_error().decode()
    n = ctypes.c_int(0)
    assert lib.se2n_batch_tiles(arr, 2, None, 0, None, 0, ctypes.byref(n)) == -1


def test_bad_counts_tunes_and_passes(lib):
    arr = items_of(SPECS[:2])
    n = ctypes.c_int(0)
    assert lib.se2n_batch_workspace_bytes(arr, 0) == 0
    assert lib.se2n_batch_workspace_bytes(None, 1) == 0
    assert lib.se2n_batch_tiles(arr, 2, None, 10, None, 0, ctypes.byref(n)) == -1
    assert lib.se2n_batch_tiles(arr, 2, ctypes.byref(Tune(17, 0, 1, 0)), 0, None, 0, ctypes.byref(n)) == -1
    assert lib.se2n_batch_tiles(arr, 2, ctypes.byref(Tune(1, 2, 1, 0)), 0, None, 0, ctypes.byref(n)) == -1
    assert lib.se2n_batch_tiles(arr, 2, ctypes.byref(Tune(1, 0, 0, 0)), 0, None, 0, ctypes.byref(n)) == -1
    # the pointers of f, mask, out are checked before anything is enqueued
    assert lib.se2n_inpaint_batched(arr, 2, ctypes.c_void_p(1), None) == -1
    assert "non-NULL" in lib.se2n_last_error().decode()


def test_tuning_table_reader_skips_unparsable_lines(lib, tmp_path):
    p = tmp_path / "tune.jsonl"
    p.write_text('{"arch": "gfx950", "signature": "00ff", "wg_per_cu": 4, "order": 1, "row_groups": 2}\n'
                 'not json at all\n'
                 '{"arch": "gfx950", "signature": "0100", "wg_per_cu": 99, "order": 0, "row_groups": 1}\n')
    assert lib.se2n_batch_load_tune_table(str(p).encode()) == 0
    assert lib.se2n_batch_load_tune_table(str(tmp_path / "missing.jsonl").encode()) == -4
    assert lib.se2n_batch_load_tune_table(None) == -1
