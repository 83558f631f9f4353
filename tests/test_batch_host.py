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
    assert ws_bytes(a, n) == _al(64 * n) + _al(4 * lmax * (n + 1)) + sum(per)
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
