"""GPU test of dwt2_transform_noalloc (through the C ABI): the allocation-free
call, whose workspace is the library's static device array, gives exactly
the bits of dwt2_forward / dwt2_inverse with a caller workspace, on two calls
in a row with the second on a smaller image (the array keeps the first call's
contents), and rejects a workspace need beyond the array's size."""
import ctypes

import numpy as np
import pytest

import oracle
from test_gpu_parity import check, dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import dwt2  # noqa: E402


def noalloc(inverse, wav, lev, x, y, opt=None):
    h, w = x.shape
    return dwt2.dwt2_transform_noalloc(inverse, wav, lev, w, h, x.data_ptr(), x.stride(0),
                                       y.data_ptr(), y.stride(0), dwt2.EXT_WHOLE_SYMMETRIC, opt,
                                       torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("wav,scheme", [("cdf97", "auto"), ("cdf53", "auto"), ("dd137", "auto"),
                                        ("cdf97", "rowcol")])
def test_noalloc_equals_the_workspace_call_twice_in_a_row(wav, scheme):
    rng = np.random.default_rng(800)
    opt = dwt2.make_options(scheme=scheme)
    for (h, w, lev) in [(1800, 2500, 5), (301, 203, 3)]:  # the second call is smaller
        print(f"noalloc {wav} {scheme} {w}x{h} L{lev}", flush=True)
        img = rng.integers(0, 256, size=(h, w)).astype(np.float32)
        x = torch.from_numpy(img).to(dev())
        want_y = dwt2.forward(x, wav, lev, scheme=scheme)
        want_z = dwt2.inverse(want_y, wav, lev, scheme=scheme)
        y = torch.full_like(x, float("nan"))
        z = torch.full_like(x, float("nan"))
        assert noalloc(0, wav, lev, x, y, opt) == dwt2.OK
        assert noalloc(1, wav, lev, y, z, opt) == dwt2.OK
        torch.cuda.synchronize()
        assert torch.equal(y, want_y), f"forward {wav} {w}x{h} L{lev}"
        assert torch.equal(z, want_z), f"inverse {wav} {w}x{h} L{lev}"
        if scheme == "auto" and w < 1000:
            check(to_host(y), oracle.forward(img.astype(np.float64), wav, lev), False,
                  f"oracle {wav} {w}x{h} L{lev}")


def test_noalloc_rejects_a_workspace_beyond_the_array():
    w, h, lev = 8192, 8192, 3  # LL buffers of 64 MiB + 16 MiB
    st, need = dwt2.dwt2_workspace_bytes("cdf97", lev, w, h)
    assert st == dwt2.OK and need > dwt2.NOALLOC_SCRATCH_BYTES
    x = torch.zeros((h, w), device=dev())
    y = torch.zeros_like(x)
    assert noalloc(0, "cdf97", lev, x, y) == dwt2.E_WORKSPACE
    # one level needs no workspace: any size runs
    assert noalloc(0, "cdf97", 1, x, y) == dwt2.OK
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0
