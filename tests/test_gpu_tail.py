"""GPU tests of the fused multi-level tail (dwt2_options.fuse_tail, through
the C ABI): the levels from 128 x 128 pixels down run in one work-group with
their LL bands in LDS, and must give bitwise the coefficients (and samples)
of the per-level launches, for all wavelets and normalisations, images that
start at or above the tail size, pitched and misaligned buffers, and levels
down to 2 x 2; one case is also held to the oracle directly."""
import numpy as np
import pytest

import oracle
from test_gpu_parity import check, dev, empty_dev, exact_expected, max_levels, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import dwt2  # noqa: E402

WAVELETS = ["cdf53", "cdf97", "dd137"]
# (width, height, levels, pitch): the tail from level 0 (both sides <= 128),
# from a deeper level, tall and wide images, and every level down to 2 x 2.
CASES = [(128, 128, 3, None), (100, 60, 4, None), (37, 22, 3, None), (300, 500, 6, None),
         (1030, 770, 7, 1040), (40, 1000, 5, None), (3000, 70, 7, None), (129, 128, 5, None),
         (6, 5, 2, None)]


def tail_start(w, h, lev):
    """First level the library fuses into the tail (lev when none): the first
    level whose input has both sides <= 128, if at least two levels remain."""
    for k in range(lev - 1):
        if w <= 128 and h <= 128:
            return k
        w, h = (w + 1) // 2, (h + 1) // 2
    return lev


def test_every_case_reaches_the_tail():
    for (w, h, lev, _) in CASES:
        lev = min(lev, max_levels(w, h, 30))
        assert tail_start(w, h, lev) <= lev - 2, (w, h, lev)
    assert tail_start(40, 1000, 5) == 3  # tall: level 3's input is 5 x 125
    assert tail_start(64, 3000, 6) == 6  # level 4 (4 x 188) is too tall, level 5 is the last


def placed(a, h, w, pitch, offset):
    """A (h, w) device view with the given row pitch, one element past an
    8-byte boundary when offset is 1; NaN around it."""
    pitch = pitch or w
    buf = torch.full((offset + (h - 1) * pitch + w,), float("nan"), dtype=torch.float32, device=dev())
    v = torch.as_strided(buf, (h, w), (pitch, 1), offset)
    if a is not None:
        v.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)))
    return v


@pytest.mark.parametrize("norm", ["unit_dc", "paper"])
@pytest.mark.parametrize("wav", WAVELETS)
def test_tail_equals_per_level_launches(wav, norm):
    rng = np.random.default_rng(500)
    for (w, h, lev, pitch) in CASES:
        lev = min(lev, max_levels(w, h, 30))
        for offset in (0, 1):
            x = rng.integers(0, 256, size=(h, w)).astype(np.float32)
            xd = placed(x, h, w, pitch, offset)
            want = dwt2.forward(xd, wav, lev, norm, out=placed(None, h, w, pitch, offset))
            got = dwt2.forward(xd, wav, lev, norm, out=placed(None, h, w, pitch, offset), fuse_tail=1)
            back = dwt2.inverse(want, wav, lev, norm, out=placed(None, h, w, pitch, offset))
            back_t = dwt2.inverse(want, wav, lev, norm, out=placed(None, h, w, pitch, offset),
                                  fuse_tail=1)
            torch.cuda.synchronize()
            what = f"{wav} {norm} {w}x{h} L{lev} pitch {pitch} offset {offset}"
            assert torch.equal(got, want), "forward " + what
            assert torch.equal(back_t, back), "inverse " + what


def test_tail_against_the_oracle():
    rng = np.random.default_rng(501)
    for wav in WAVELETS:
        w, h = 120, 90
        lev = max_levels(w, h, 30)
        x = rng.integers(0, 256, size=(h, w)).astype(np.float32)
        y = dwt2.forward(to_dev(x), wav, lev, out=empty_dev(h, w), fuse_tail=1)
        got = to_host(y)
        check(got, oracle.forward(x.astype(np.float64), wav, lev), exact_expected(wav, lev, "unit_dc"),
              f"fwd {wav} {w}x{h} L{lev}")
        z = dwt2.inverse(y, wav, lev, out=empty_dev(h, w), fuse_tail=1)
        check(to_host(z), oracle.inverse(got, wav, lev), exact_expected(wav, lev, "unit_dc"),
              f"inv {wav} {w}x{h} L{lev}")
