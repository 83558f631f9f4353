"""GPU tests of the fused kernel's tile heights, tile orders and of
dwt2_autotune (through the C ABI).

Every built height and both tile orders must give bitwise the coefficients
(and samples) of the automatic choice, in both directions, for all wavelets,
at sizes that span several centring cells and end in ragged tiles; the
automatic choice is held to the oracle by the parity tests, and again here
on the same inputs.  dwt2_autotune must leave in dst exactly what the plain
call gives and record only built heights and valid orders.
"""
import numpy as np
import pytest

import oracle
from paper_1605_00561_amd import workloads as wl
from test_gpu_parity import check, dev, empty_dev, exact_expected, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import dwt2  # noqa: E402

WAVELETS = ["cdf53", "cdf97", "dd137"]
# (width, height, levels, pitch): several 18..30-row cells per level, odd
# sizes, a pitched buffer, a tall narrow image.
CASES = [(300, 500, 3, None), (1030, 770, 2, 1040), (77, 45, 3, None), (129, 1201, 4, None),
         (2, 2, 1, None), (5, 7, 2, None)]


@pytest.fixture(autouse=True)
def empty_table():
    dwt2.dwt2_tune_reset()
    yield
    dwt2.dwt2_tune_reset()


@pytest.mark.parametrize("norm", ["unit_dc", "paper"])
@pytest.mark.parametrize("wav", WAVELETS)
def test_every_height_gives_the_same_bits(wav, norm):
    rng = np.random.default_rng(400)
    for (w, h, lev, pitch) in CASES:
        x = rng.integers(0, 256, size=(h, w)).astype(np.float32)
        xd = to_dev(x, pitch)
        base = dwt2.forward(xd, wav, lev, norm, out=empty_dev(h, w, pitch))
        back = dwt2.inverse(base, wav, lev, norm, out=empty_dev(h, w, pitch))
        what = f"{wav} {norm} {w}x{h} L{lev}"
        for rows in dwt2.TILE_ROWS[wav]:
            for nb in (1, 2):  # single- and double-buffered LDS planes
                for order in ("runs", "bands"):
                    y = dwt2.forward(xd, wav, lev, norm, out=empty_dev(h, w, pitch), tile_rows=rows,
                                     lds_buffers=nb, tile_order=order)
                    z = dwt2.inverse(base, wav, lev, norm, out=empty_dev(h, w, pitch),
                                     tile_rows=rows, lds_buffers=nb, tile_order=order)
                    torch.cuda.synchronize()
                    assert torch.equal(y, base), f"forward {what} rows {rows} buffers {nb} {order}"
                    assert torch.equal(z, back), f"inverse {what} rows {rows} buffers {nb} {order}"
        y0 = dwt2.forward(xd, wav, lev, norm, out=empty_dev(h, w, pitch), arithmetic="fp64")
        z0 = dwt2.inverse(y0, wav, lev, norm, out=empty_dev(h, w, pitch), arithmetic="fp64")
        for order in ("runs", "bands"):  # FP64 lifting, both orders and bufferings
            for nb in (1, 2):
                y = dwt2.forward(xd, wav, lev, norm, out=empty_dev(h, w, pitch), arithmetic="fp64",
                                 tile_order=order, lds_buffers=nb)
                z = dwt2.inverse(y0, wav, lev, norm, out=empty_dev(h, w, pitch), arithmetic="fp64",
                                 tile_order=order, lds_buffers=nb)
                torch.cuda.synchronize()
                assert torch.equal(y, y0), f"fp64 forward {what} {order} buffers {nb}"
                assert torch.equal(z, z0), f"fp64 inverse {what} {order} buffers {nb}"
        if norm == "unit_dc":
            got = to_host(base)
            check(got, oracle.forward(x.astype(np.float64), wav, lev, norm),
                  exact_expected(wav, lev, norm), "fwd " + what)
            check(to_host(back), oracle.inverse(got, wav, lev, norm),
                  exact_expected(wav, lev, norm), "inv " + what)


def test_every_height_at_8192():
    """The headline level (8192^2, 9/7) at every height and in both tile
    orders: identical bits."""
    x = to_dev(wl.workload_image("cdf97_8192_l1"))
    base = dwt2.forward(x, "cdf97", 1)
    back = dwt2.inverse(base, "cdf97", 1)
    for rows in dwt2.TILE_ROWS["cdf97"]:
        for nb in (1, 2):
            for order in ("runs", "bands"):
                assert torch.equal(dwt2.forward(x, "cdf97", 1, tile_rows=rows, lds_buffers=nb,
                                                tile_order=order), base)
                assert torch.equal(dwt2.inverse(base, "cdf97", 1, tile_rows=rows, lds_buffers=nb,
                                                tile_order=order), back)


@pytest.mark.parametrize("wav", ["cdf53", "cdf97"])
def test_both_orders_at_16384(wav):
    """16384^2, where the rule picks the band order: the run order gives the
    same bits in both directions."""
    x = to_dev(wl.workload_image(f"{wav}_16384_l5"))
    assert dwt2.tile_order(wav, 16384, 16384) == "bands"
    base = dwt2.forward(x, wav, 1)
    assert torch.equal(dwt2.forward(x, wav, 1, tile_order="runs"), base)
    back = dwt2.inverse(base, wav, 1)
    assert torch.equal(dwt2.inverse(base, wav, 1, tile_order="runs"), back)
    del base, back
    torch.cuda.empty_cache()


def test_band_order_with_fewer_tile_columns_than_xcds():
    """Levels 1 to 7 tile columns wide leave some XCDs without a band; every
    tile is still computed once (bits equal to the run order, NaN-filled
    outputs would show a skipped tile)."""
    rng = np.random.default_rng(402)
    for w in (2, 60, 130, 250, 500, 800, 1000):
        for wav in WAVELETS:
            x = to_dev(rng.integers(0, 256, size=(97, w)).astype(np.float32))
            a = dwt2.forward(x, wav, 1, tile_order="runs", out=empty_dev(97, w))
            b = dwt2.forward(x, wav, 1, tile_order="bands", out=empty_dev(97, w))
            torch.cuda.synchronize()
            assert torch.equal(a, b), (w, wav)
            assert bool(torch.isfinite(b).all()), (w, wav)


@pytest.mark.parametrize("wav", WAVELETS)
def test_autotune_leaves_the_plain_result_and_records_built_heights(wav):
    rng = np.random.default_rng(401)
    w, h, lev = 1500, 900, 4
    x = to_dev(rng.integers(0, 256, size=(h, w)).astype(np.float32))
    want = dwt2.forward(x, wav, lev)
    got = dwt2.autotune(x, wav, lev, repeats=3, out=empty_dev(h, w))
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    want_inv = dwt2.inverse(want, wav, lev)
    got_inv = dwt2.autotune(want, wav, lev, inverse=True, repeats=3, out=empty_dev(h, w))
    torch.cuda.synchronize()
    assert torch.equal(got_inv, want_inv)
    st, text = dwt2.dwt2_tune_export()
    assert st == dwt2.OK
    entries = [tuple(map(int, line.split())) for line in text.splitlines()]
    sizes, (cw, ch) = [], (w, h)
    for _ in range(lev):
        sizes.append((cw, ch))
        cw, ch = (cw + 1) // 2, (ch + 1) // 2
    wid = dwt2.WAVELETS[wav]
    assert sorted(e[:4] for e in entries) == sorted((wid, d, a, b) for d in (0, 1) for (a, b) in sizes)
    for (_, d, a, b, rows, order) in entries:
        assert rows in dwt2.TILE_ROWS[wav]
        assert order in (dwt2.ORDER_RUNS, dwt2.ORDER_BANDS)
        assert dwt2.tile_rows(wav, a, b, inverse=bool(d)) == rows
        assert dwt2.tile_order(wav, a, b, inverse=bool(d)) == ("runs", "bands")[order - 1]
    # calls now run at the tuned heights and still give the same bits
    assert torch.equal(dwt2.forward(x, wav, lev), want)
    assert torch.equal(dwt2.inverse(want, wav, lev), want_inv)
