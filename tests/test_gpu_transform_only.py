"""GPU tests of dwt2_transform_only (through the C ABI), the measurement mode
of the paper's transform-only experiments: every scheme, wavelet, height,
buffering and order launches and completes on ragged and degenerate sizes,
never writes its sink (the checksum never matches its key), and leaves the
device usable for a transform that still matches the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
from test_gpu_parity import check, dev, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import dwt2  # noqa: E402

SCHEMES = ["monolithic*", "monolithic*-tile", "sweldens", "iwahashi", "monolithic", "explosive",
           "explosive*", "iwahashi*", "polyphase*"]
SIZES = [(2, 2), (3, 7), (130, 67), (1030, 770), (64, 3000)]


def run(inverse, wav, w, h, opt, sink):
    st = dwt2.library().dwt2_transform_only(inverse, dwt2.WAVELETS[wav], w, h, ctypes.byref(opt),
                                            sink.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == dwt2.OK, (inverse, wav, w, h, st)


def test_every_kernel_runs_and_stores_nothing():
    sink = torch.full((4,), 12.5, dtype=torch.float32, device=dev())
    for wav in ("cdf53", "cdf97"):
        for scheme in SCHEMES:
            for (w, h) in SIZES:
                for inverse in (0, 1):
                    run(inverse, wav, w, h, dwt2.make_options(scheme=scheme), sink)
    for wav in ("cdf53", "cdf97", "dd137"):
        for rows in dwt2.TILE_ROWS[wav]:
            for nb in (1, 2):
                for order in ("runs", "bands"):
                    for (w, h) in SIZES:
                        for inverse in (0, 1):
                            opt = dwt2.make_options(tile_rows=rows, lds_buffers=nb, tile_order=order)
                            run(inverse, wav, w, h, opt, sink)
    torch.cuda.synchronize()
    assert sink.tolist() == [12.5] * 4
    # the device still computes transforms correctly afterwards
    x = np.random.default_rng(700).integers(0, 256, size=(300, 517)).astype(np.float32)
    y = dwt2.forward(to_dev(x), "cdf97", 3)
    check(to_host(y), oracle.forward(x.astype(np.float64), "cdf97", 3), False, "after transform-only")


def test_full_size_launches():
    """The 8192^2 level the benchmark's transform-only table times."""
    sink = torch.full((1,), -3.0, dtype=torch.float32, device=dev())
    for wav in ("cdf53", "cdf97", "dd137"):
        for inverse in (0, 1):
            run(inverse, wav, 8192, 8192, dwt2.make_options(), sink)
    for scheme in SCHEMES[1:]:
        run(0, "cdf97", 8192, 8192, dwt2.make_options(scheme=scheme), sink)
    torch.cuda.synchronize()
    assert float(sink[0]) == -3.0
