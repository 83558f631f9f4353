"""Host-side checks of the batched entry points: workspace size and every
argument error, with fake device pointers.  Each call below fails validation
(or has count == 0), so nothing is ever enqueued."""
import ctypes

from paper_1605_00561_amd import dwt2
from test_abi_host import FAKE, _al, header_define

MiB = 1 << 20


def images(*entries):
    return dwt2.make_images(list(entries)), len(entries)


def img(wav="cdf53", lev=1, w=64, h=64, src=FAKE, sp=None, dst=FAKE + 64 * MiB, dp=None):
    return (wav, lev, w, h, src, sp if sp is not None else w, dst, dp if dp is not None else w)


def ws_bytes(arr, n, **opt):
    st, b = dwt2.dwt2_batch_workspace_bytes(arr, n, dwt2.make_options(**opt))
    assert st == dwt2.OK
    return b


def both(arr, n, ws=FAKE + 1024 * MiB, nws=1 << 40, opt=None):
    return [f(arr, n, 0, opt, ws, nws, None)
            for f in (dwt2.dwt2_forward_batch, dwt2.dwt2_inverse_batch)]


def test_batch_max_matches_header():
    assert header_define("DWT2_BATCH_MAX") == dwt2.BATCH_MAX


def test_workspace_bytes_is_table_plus_each_images_ll_buffers():
    a, n = images(img("cdf97", 3, 1000, 700), img("cdf53", 1, 64, 64),
                  img("cdf53", 6, 999, 333, src=FAKE + 8 * MiB, dst=FAKE + 16 * MiB))
    per = [dwt2.dwt2_workspace_bytes(w, l, x, y, None)[1]
           for (w, l, x, y) in [("cdf97", 3, 1000, 700), ("cdf53", 1, 64, 64),
                                ("cdf53", 6, 999, 333)]]
    lmax = 6
    rows_table = _al(((n + 3) // 4 * 4) * lmax)  # one byte per image and level, rows of 4k bytes
    # tile-image index: two bytes per tile, every level at the wavelet's shortest height
    bound = 0
    for (wav, lev, w, h) in [("cdf97", 3, 1000, 700), ("cdf53", 1, 64, 64), ("cdf53", 6, 999, 333)]:
        for _ in range(lev):
            bound += tiles(wav, min(dwt2.TILE_ROWS[wav]), w, h)
            w, h = (w + 1) // 2, (h + 1) // 2
    assert ws_bytes(a, n) == _al(64 * n) + _al(4 * lmax * (n + 1)) + rows_table + _al(2 * bound) + sum(per)
    assert ws_bytes(a, 0) == 0
    # arithmetic and norm do not change the layout
    assert ws_bytes(a, n, arithmetic="fp64", norm="paper") == ws_bytes(a, n)


def test_count_and_array_errors():
    a, n = images(img())
    lib = dwt2.library()
    b = ctypes.c_size_t()
    assert lib.dwt2_batch_workspace_bytes(a, -1, None, ctypes.byref(b)) == dwt2.E_ARG
    assert lib.dwt2_batch_workspace_bytes(a, dwt2.BATCH_MAX + 1, None, ctypes.byref(b)) == \
        dwt2.E_ARG
    assert lib.dwt2_batch_workspace_bytes(None, 1, None, ctypes.byref(b)) == dwt2.E_ARG
    assert lib.dwt2_batch_workspace_bytes(a, 1, None, None) == dwt2.E_ARG
    assert both(a, -1) == [dwt2.E_ARG] * 2
    assert both(None, 2) == [dwt2.E_ARG] * 2
    # count == 0 is a no-op (returns before any launch)
    assert both(None, 0) == [dwt2.OK] * 2


def test_per_image_errors_name_the_same_status_as_single_calls():
    cases = [
        (img(lev=0), dwt2.E_ARG),
        (img(w=0), dwt2.E_ARG),
        (img(src=0), dwt2.E_ARG),
        (img(dst=0), dwt2.E_ARG),
        (img(sp=63), dwt2.E_ARG),
        (img(dp=10), dwt2.E_ARG),
        (img(sp=2 ** 62), dwt2.E_ARG),              # span beyond 2^60 elements
        (img(src=FAKE + 2), dwt2.E_ARG),
        (img(w=1), dwt2.E_SIZE),
        (img(lev=7, w=64, h=64), dwt2.E_SIZE),
        (img(lev=32), dwt2.E_SIZE),
        (img(wav=7), dwt2.E_UNSUPPORTED),
    ]
    good = img(src=FAKE + 512 * MiB, dst=FAKE + 640 * MiB)
    for bad, status in cases:
        if bad[0] == 7:
            arr = (dwt2.Image * 2)()
            arr[0] = dwt2.Image(*[dwt2.WAVELETS[good[0]]] + list(good[1:]))
            arr[1] = dwt2.Image(7, *bad[1:])
        else:
            arr, _ = images(good, bad)
        assert both(arr, 2) == [status] * 2, (bad, status)
        st, _ = dwt2.dwt2_batch_workspace_bytes(arr, 2, None)
        assert st == status


def test_options_errors():
    a, n = images(img())
    for opt, status in [(dict(scheme="sweldens"), dwt2.E_UNSUPPORTED),
                        (dict(scheme="rowcol"), dwt2.E_UNSUPPORTED),
                        (dict(scheme="monolithic*-tile"), dwt2.E_UNSUPPORTED),
                        # batches run at their own tile height; tile_rows must be 0
                        (dict(tile_rows=3), dwt2.E_UNSUPPORTED),
                        (dict(tile_rows=4), dwt2.E_UNSUPPORTED),
                        (dict(lds_buffers=1), dwt2.E_UNSUPPORTED)]:
        assert both(a, n, opt=dwt2.make_options(**opt)) == [status] * 2
    o = dwt2.make_options()
    o.reserved[0] = 1
    assert both(a, n, opt=o) == [dwt2.E_ARG] * 2
    o = dwt2.make_options()
    o.norm = 9
    assert both(a, n, opt=o) == [dwt2.E_UNSUPPORTED] * 2
    assert [f(a, n, 1, None, FAKE + 1024 * MiB, 1 << 40, None)
            for f in (dwt2.dwt2_forward_batch, dwt2.dwt2_inverse_batch)] == \
        [dwt2.E_UNSUPPORTED] * 2


def test_workspace_errors():
    a, n = images(img(lev=3), img(lev=2, src=FAKE + 8 * MiB, dst=FAKE + 16 * MiB))
    need = ws_bytes(a, n)
    assert both(a, n, ws=None) == [dwt2.E_WORKSPACE] * 2
    assert both(a, n, nws=need - 1) == [dwt2.E_WORKSPACE] * 2
    assert both(a, n, ws=FAKE + 1024 * MiB + 4) == [dwt2.E_ARG] * 2


def test_alias_errors():
    base = FAKE
    span = 64 * 64 * 4
    # one image's dst over another's src, over another's dst, over its own src
    for second in [img(src=base + 100 * MiB, dst=base + span // 2),
                   img(src=base + 100 * MiB, dst=base + 64 * MiB + 4 * 64),
                   img(src=base + 200 * MiB, dst=base + 200 * MiB + span - 4)]:
        a, n = images(img(src=base, dst=base + 64 * MiB), second)
        assert both(a, n) == [dwt2.E_ALIAS] * 2, second
    # the workspace over an image
    a, n = images(img(src=base, dst=base + 64 * MiB))
    assert both(a, n, ws=base + 64 * MiB - 256) == [dwt2.E_ALIAS] * 2
    # pitched spans: the byte range runs from the first to the last element
    a, n = images(img(w=64, h=64, sp=1024, src=base, dst=base + 64 * MiB),
                  img(src=base + 256 * MiB, dst=base + 63 * 1024 * 4))
    assert both(a, n) == [dwt2.E_ALIAS] * 2


# The batched 5/3 tile: 64 x 12 quadruples (3 rows per wavefront) including
# a halo of one quadruple per side.
TILE_QW, TILE_QH = 64, 12


def test_tile_total_overflow_is_an_argument_error():
    # 2^19 x 2^19 is the largest accepted image (2^38 pixels); a few dozen of
    # them hold more than 2^31 tiles in level 0, which a level launch cannot
    # index.
    side = 2 ** 19
    tiles = -(-(side // 2) // (TILE_QW - 2)) * -(-(side // 2) // (TILE_QH - 2))
    n_ok = (2 ** 31 - 8) // tiles
    assert n_ok * tiles <= 2 ** 31 - 8 < (n_ok + 1) * tiles
    for n, status in [(n_ok, dwt2.OK), (n_ok + 1, dwt2.E_ARG)]:
        a, _ = images(*[img("cdf53", 1, side, side)] * n)
        st, _ = dwt2.dwt2_batch_workspace_bytes(a, n, None)
        assert st == status
    a, _ = images(img("cdf53", 1, side, side + 1))
    assert dwt2.dwt2_batch_workspace_bytes(a, 1, None)[0] == dwt2.E_SIZE


# --- tile heights of batched calls (host-side plan; nothing is launched) -----
TALLEST = {w: max(r) for w, r in dwt2.TILE_ROWS.items()}


def tiles(wav, rows, w, h):
    hq = {"cdf53": 1, "cdf97": 2, "dd137": 3}[wav]
    ix, iy = 64 - 2 * hq, 4 * rows - 2 * hq
    return -(-((w + 1) // 2) // ix) * -(-((h + 1) // 2) // iy)


# Fill thresholds (tiles) of the single-image height rule, per wavelet.
FILL = {"cdf53": 256, "cdf97": 512, "dd137": 1536}


def model_rows(entries, level, tuned=None, fp64=False):
    """The rule of dwt2_batch_tile_rows, written out: tuned sizes keep their
    height; the others step down together from the tallest height until the
    launch has as many tiles as the largest fill threshold of their
    wavelets."""
    tuned = tuned or {}
    live = []
    for (wav, lev, w, h, *_ ) in entries:
        if lev <= level:
            live.append(None)
            continue
        for _ in range(level):
            w, h = (w + 1) // 2, (h + 1) // 2
        live.append((wav, w, h))
    if fp64:
        return [0 if e is None else dwt2.TILE_ROWS_FP64[e[0]] for e in live]

    def height(wav, step):
        hs = dwt2.TILE_ROWS[wav]
        return hs[max(0, len(hs) - 1 - step)]

    def pick(step):
        return [0 if e is None else tuned.get(e, height(e[0], step)) for e in live]

    fill = max([FILL[e[0]] for e in live if e and e not in tuned], default=0)
    for step in range(3):
        rows = pick(step)
        if sum(tiles(e[0], r, e[1], e[2]) for e, r in zip(live, rows) if e) >= fill:
            return rows
    return pick(2)


def test_batch_tile_rows_follow_the_launch_fill_rule():
    import numpy as np
    rng = np.random.default_rng(40)
    dwt2.dwt2_tune_reset()
    for trial in range(60):
        n = int(rng.integers(1, 12))
        entries = []
        for i in range(n):
            w, h = int(rng.integers(2, 3000)), int(rng.integers(2, 3000))
            wav = ("cdf53", "cdf97", "dd137")[int(rng.integers(0, 3))]
            lev, ww, hh = 0, w, h
            while lev < 6 and ww >= 2 and hh >= 2:
                lev, ww, hh = lev + 1, (ww + 1) // 2, (hh + 1) // 2
            entries.append(img(wav, int(rng.integers(1, lev + 1)), w, h,
                               src=FAKE + (2 * i) * 64 * MiB, dst=FAKE + (2 * i + 1) * 64 * MiB))
        a, _ = images(*entries)
        for level in range(7):
            for inverse in (0, 1):
                st, rows = dwt2.dwt2_batch_tile_rows(inverse, a, n, level)
                assert st == dwt2.OK
                assert rows == model_rows(entries, level), (trial, level, entries)
        st, rows = dwt2.dwt2_batch_tile_rows(0, a, n, 0, dwt2.make_options(arithmetic="fp64"))
        assert st == dwt2.OK and rows == model_rows(entries, 0, fp64=True)


def test_batch_tile_rows_take_tuned_heights():
    entries = [img("cdf97", 3, 2000, 1500), img("cdf53", 2, 800, 600, src=FAKE + 128 * MiB,
                                                  dst=FAKE + 192 * MiB)]
    a, n = images(*entries)
    try:
        dwt2.dwt2_tune_reset()
        st, rows = dwt2.dwt2_batch_tile_rows(0, a, n, 0)
        assert st == dwt2.OK and rows == [TALLEST["cdf97"], TALLEST["cdf53"]]
        # a forward entry for the 9/7 image's level 1 (1000 x 750) and an
        # inverse one for the 5/3 image's level 1 (400 x 300)
        assert dwt2.dwt2_tune_import("1 0 1000 750 2 1\n0 1 400 300 2 1\n") == dwt2.OK
        fwd = {("cdf97", 1000, 750): 2}
        inv = {("cdf53", 400, 300): 2}
        assert dwt2.dwt2_batch_tile_rows(0, a, n, 1)[1] == model_rows(entries, 1, fwd) == [2, 3]
        # the inverse launch of level 1 is short of work-groups: the untuned
        # 9/7 image steps down, the tuned 5/3 image keeps its height
        assert dwt2.dwt2_batch_tile_rows(1, a, n, 1)[1] == model_rows(entries, 1, inv) == [3, 2]
        assert dwt2.dwt2_batch_tile_rows(1, a, n, 0)[1] == model_rows(entries, 0, inv)
        assert dwt2.dwt2_batch_tile_rows(0, a, n, 2)[1][1] == 0  # the 5/3 image has 2 levels
        # FP64 lifting has one height per wavelet, tuned or not
        st, rows = dwt2.dwt2_batch_tile_rows(0, a, n, 1, dwt2.make_options(arithmetic="fp64"))
        assert rows == [dwt2.TILE_ROWS_FP64["cdf97"], dwt2.TILE_ROWS_FP64["cdf53"]]
    finally:
        dwt2.dwt2_tune_reset()
    assert dwt2.dwt2_batch_tile_rows(0, a, n, -1)[0] == dwt2.E_ARG
    assert dwt2.dwt2_batch_tile_rows(0, a, n, 0, dwt2.make_options(tile_rows=3))[0] == \
        dwt2.E_UNSUPPORTED
