"""GPU parity at the size limits (through the C ABI).

* 65536 x 32768 (2^31 pixels, 8 GiB per FP32 buffer): element and byte
  offsets pass 2^31 and 2^32.  The oracle checks windows: crops whose
  coefficients (one level, CDF 9/7) do not depend on pixels outside them,
  except within a margin at crop edges that are not image edges, which is
  left out.  Corner crops share the image's own borders, so the mirrored
  extension is checked there too.  The inverse is checked the same way on
  the GPU's own coefficients.
* extreme aspect ratios: 2^20 x 2, 2 x 2^20 and odd neighbours, compared
  whole.
"""
import numpy as np
import pytest

import oracle
from test_gpu_parity import check, dev, empty_dev, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import dwt2  # noqa: E402

MARGIN = 8  # quadruples dropped at a crop edge that is not an image edge (one 9/7 level reaches 2)


def window_bounds(q0, qn, QN):
    lo = 0 if q0 == 0 else MARGIN
    hi = qn if q0 + qn == QN else qn - MARGIN
    return lo, hi


@pytest.mark.parametrize("wav", ["cdf97", "cdf53"])
def test_2_pow_31_pixels_windows(wav):
    W, H = 65536, 32768
    QW, QH = W // 2, H // 2
    free, _ = torch.cuda.mem_get_info()
    if free < 3 * 4 * W * H + (1 << 30):
        pytest.skip("needs 25 GiB of free device memory")
    g = torch.Generator(device=dev()).manual_seed(500)
    x = torch.empty((H, W), dtype=torch.float32, device=dev()).random_(0, 256, generator=g)
    y = dwt2.forward(x, wav, 1)
    z = dwt2.inverse(y, wav, 1)
    torch.cuda.synchronize()
    # (first quadruple row, first quadruple column) of 128 x 256-quadruple windows
    qh, qw = 128, 256
    starts = [(0, 0), (0, QW - qw), (QH - qh, 0), (QH - qh, QW - qw), (QH // 2 - 61, QW // 2 - 97),
              (1000, 20000), (QH - qh - 3, 7)]
    for (i0, j0) in starts:
        what = f"{wav} window at quadruple ({i0}, {j0})"
        crop = x[2 * i0:2 * (i0 + qh), 2 * j0:2 * (j0 + qw)].cpu().numpy().astype(np.float64)
        ref = oracle.forward(crop, wav, 1)
        (ilo, ihi), (jlo, jhi) = window_bounds(i0, qh, QH), window_bounds(j0, qw, QW)
        coef = np.zeros((2 * qh, 2 * qw))
        for sr in (0, 1):
            for sc in (0, 1):
                blk = y[sr * QH + i0:sr * QH + i0 + qh, sc * QW + j0:sc * QW + j0 + qw]
                blk = blk.cpu().numpy().astype(np.float64)
                coef[sr * qh:(sr + 1) * qh, sc * qw:(sc + 1) * qw] = blk
                exp = ref[sr * qh + ilo:sr * qh + ihi, sc * qw + jlo:sc * qw + jhi]
                check(blk[ilo:ihi, jlo:jhi], exp, False, f"fwd subband {sr}{sc} {what}")
        # inverse: the window's coefficients, reassembled in Mallat order
        rec = oracle.inverse(coef, wav, 1)
        got = z[2 * i0:2 * (i0 + qh), 2 * j0:2 * (j0 + qw)].cpu().numpy().astype(np.float64)
        check(got[2 * ilo:2 * ihi, 2 * jlo:2 * jhi], rec[2 * ilo:2 * ihi, 2 * jlo:2 * jhi], False,
              f"inv {what}")
    del x, y, z
    torch.cuda.empty_cache()


@pytest.mark.parametrize("shape", [(2, 1 << 20), (3, (1 << 20) + 1), (1 << 20, 2),
                                   ((1 << 20) + 1, 3), (5, 300001)])
def test_extreme_aspect_ratios(shape):
    h, w = shape
    rng = np.random.default_rng(501)
    x = rng.integers(0, 256, size=(h, w)).astype(np.float32)
    lev = 1 if min(h, w) < 4 else 2
    for wav in ("cdf53", "cdf97", "dd137"):
        xd = to_dev(x)
        y = dwt2.forward(xd, wav, lev, out=empty_dev(h, w))
        got = to_host(y)
        check(got, oracle.forward(x.astype(np.float64), wav, lev), wav == "cdf53" and lev == 1,
              f"fwd {wav} {w}x{h} L{lev}")
        z = dwt2.inverse(y, wav, lev, out=empty_dev(h, w))
        check(to_host(z), oracle.inverse(got, wav, lev), wav == "cdf53" and lev == 1,
              f"inv {wav} {w}x{h} L{lev}")
