"""Seeded random sweep of single-image calls against the FP64 oracle.

Each case draws a wavelet, a scheme, the arithmetic, a tile height, LDS
buffering and tile order (fused kernel), the normalisation, a size (biased towards tile
boundaries: multiples of the fused tile's output width and height, plus or
minus one), the level count, row pitches at or above the width, and a base
offset of one element (so that rows are not 8-byte aligned and the kernels
take their scalar-access path).  Inputs are integers in [0, 255] or real
values in the same range.  Forward and inverse are checked as in
test_gpu_parity.py; the drawing is host-only and tested on the CPU.
"""
import numpy as np
import pytest

import oracle
from paper_1605_00561_amd import dwt2

SEED = 2024
N_CASES = 64
OTHER_SCHEMES = ["monolithic*-tile", "sweldens", "iwahashi", "rowcol", "monolithic",
                 "explosive", "explosive*", "iwahashi*", "polyphase*"]
HQ = {"cdf53": 1, "cdf97": 2, "dd137": 3}


def _levels_possible(w, h):
    n = 0
    while w >= 2 and h >= 2:
        n += 1
        w, h = (w + 1) // 2, (h + 1) // 2
    return n


def _side(rng, wav, rows, axis):
    """A side in [2, 900]: half the time one pixel off a multiple of the
    fused tile's output extent in pixels along that axis."""
    if rng.random() < 0.5:
        return int(rng.integers(2, 901))
    quads = 64 - 2 * HQ[wav] if axis == 0 else 4 * rows - 2 * HQ[wav]
    k = int(rng.integers(1, max(2, 900 // (2 * quads))))
    return max(2, 2 * quads * k + int(rng.integers(-1, 2)))


def draw_cases(seed=SEED, n=N_CASES):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(n):
        wav = ["cdf53", "cdf97", "dd137"][i % 3]
        fused = wav == "dd137" or rng.random() < 0.7
        scheme = "monolithic*" if fused else str(rng.choice(OTHER_SCHEMES))
        arith = "fp64" if fused and rng.random() < 0.25 else "auto"
        rows, lds = 0, 0
        order = ("auto", "runs", "bands")[(i // 3) % 3] if fused else "auto"
        if fused and arith != "fp64":
            choices = (0,) + dwt2.TILE_ROWS[wav]       # cycled, so that each is reached
            rows = choices[(i // 3) % len(choices)]
            lds = (i // 3) % 3
        eff_rows = rows or dwt2.TILE_ROWS[wav][-1]
        w, h = _side(rng, wav, eff_rows, 0), _side(rng, wav, eff_rows, 1)
        # PAPER scaling doubles LL per level; past three levels its FP32 ulp
        # nears the absolute bar (the normalisation relation covers it).
        norm = str(rng.choice(("unit_dc", "paper")))
        cap = 3 if norm == "paper" else 6
        levels = int(rng.integers(1, min(_levels_possible(w, h), cap) + 1))
        pad = int(rng.choice((0, 0, 1, 3, 64)))
        cases.append(dict(
            wav=wav, scheme=scheme, arith=arith, rows=rows, lds=lds, order=order, w=w, h=h,
            levels=levels,
            norm=norm, src_pitch=w + pad,
            dst_pitch=w + int(rng.choice((0, 1, 64))), offset=int(rng.random() < 0.3),
            real=bool(rng.random() < 0.3), seed=seed * 1000 + i))
    return cases


CASES = draw_cases()


def case_id(c):
    return (f"{c['wav']}-{c['scheme']}-{c['arith']}-r{c['rows']}-b{c['lds']}-{c['order']}"
            f"-{c['w']}x{c['h']}"
            f"-L{c['levels']}-{c['norm']}-p{c['src_pitch']}.{c['dst_pitch']}-o{c['offset']}"
            f"-{'real' if c['real'] else 'int'}")


def test_draw_covers_every_option():
    """CPU: the sweep reaches every wavelet, scheme, arithmetic, height,
    buffering, pitch and offset kind, and every case is a valid call."""
    seen = {k: set() for k in ("wav", "scheme", "arith", "lds", "order", "offset", "real", "norm")}
    heights = set()
    padded = False
    for c in CASES:
        for k in seen:
            seen[k].add(c[k])
        heights.add((c["wav"], c["rows"]))
        padded |= c["src_pitch"] > c["w"] and c["dst_pitch"] > c["w"]
        assert c["w"] >= 2 and c["h"] >= 2 and 1 <= c["levels"] <= _levels_possible(c["w"], c["h"])
        assert c["levels"] <= (3 if c["norm"] == "paper" else 6)
        assert c["src_pitch"] >= c["w"] and c["dst_pitch"] >= c["w"]
        if c["scheme"] != "monolithic*":
            assert c["wav"] != "dd137" and c["arith"] == "auto" and c["rows"] == 0 and c["lds"] == 0
            assert c["order"] == "auto"
        if c["arith"] == "fp64":
            assert c["rows"] == 0 and c["lds"] == 0
    assert seen["wav"] == {"cdf53", "cdf97", "dd137"}
    assert seen["arith"] == {"auto", "fp64"}
    assert seen["lds"] == {0, 1, 2} and seen["offset"] == {0, 1} and seen["real"] == {False, True}
    assert seen["norm"] == {"unit_dc", "paper"}
    assert seen["order"] == {"auto", "runs", "bands"}
    assert len(seen["scheme"]) >= 6
    for wav, rows in dwt2.TILE_ROWS.items():
        assert {(wav, r) for r in rows} <= heights, wav
    assert padded
    assert len({case_id(c) for c in CASES}) == len(CASES)


@pytest.mark.gpu
@pytest.mark.parametrize("case", CASES, ids=[case_id(c) for c in CASES])
def test_sweep_case(case):
    torch = pytest.importorskip("torch")
    from test_gpu_parity import check, dev, exact_expected

    c = case
    w, h = c["w"], c["h"]
    rng = np.random.default_rng(c["seed"])
    if c["real"]:
        x = rng.uniform(0.0, 255.0, size=(h, w)).astype(np.float32)
    else:
        x = rng.integers(0, 256, size=(h, w)).astype(np.float32)

    def placed(a, pitch, off):
        buf = torch.full((off + (h - 1) * pitch + w,), float("nan"), dtype=torch.float32,
                         device=dev())
        view = torch.as_strided(buf, (h, w), (pitch, 1), off)
        if a is not None:
            view.copy_(torch.from_numpy(a))
        return view

    kw = dict(norm=c["norm"], scheme=c["scheme"], arithmetic=c["arith"], tile_rows=c["rows"],
              lds_buffers=c["lds"], tile_order=c["order"])
    xd = placed(x, c["src_pitch"], c["offset"])
    y = dwt2.forward(xd, c["wav"], c["levels"], out=placed(None, c["dst_pitch"], c["offset"]), **kw)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    exact = exact_expected(c["wav"], c["levels"], c["norm"]) and not c["real"]
    ref = oracle.forward(x.astype(np.float64), c["wav"], c["levels"], c["norm"])
    check(got, ref, exact, "fwd " + case_id(c))
    z = dwt2.inverse(y, c["wav"], c["levels"], out=placed(None, c["src_pitch"], c["offset"]), **kw)
    torch.cuda.synchronize()
    check(z.cpu().numpy().astype(np.float64), oracle.inverse(got, c["wav"], c["levels"], c["norm"]),
          exact, "inv " + case_id(c))
