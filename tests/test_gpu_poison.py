"""GPU correctness aids (through the C ABI):

* LDS poisoning: the test-only build libdwt2_poison.so fills every
  work-group's LDS with NaN before its first LDS access.  If a kernel read a
  cell it had not written since it started, a NaN (or another value) would
  reach its outputs; every kernel with LDS (the fused kernel at every height,
  buffering and order, FP32 and FP64, the multi-level tail, the batched
  launches and every tile-harness scheme) must give the normal library's bits.
* Fault injection: a launch failed on purpose from the host
  (dwt2_debug_fail_launches) makes the call return DWT2_E_HIP before anything
  runs, and the next call works.
"""
import ctypes

import numpy as np
import pytest

from test_gpu_parity import dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import build, dwt2  # noqa: E402


@pytest.fixture(scope="module")
def poison():
    lib = ctypes.CDLL(build.POISON_LIB)
    ref = dwt2.library()
    for name in dwt2.EXPORTS:
        f, g = getattr(lib, name), getattr(ref, name)
        f.argtypes, f.restype = g.argtypes, g.restype
    return lib


def call(lib, inverse, x, y, wav, lev, opt):
    h, w = x.shape
    nbytes = ctypes.c_size_t()
    assert lib.dwt2_workspace_bytes(dwt2.WAVELETS[wav], lev, w, h, ctypes.byref(opt),
                                    ctypes.byref(nbytes)) == dwt2.OK
    ws = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=dev())
    f = lib.dwt2_inverse if inverse else lib.dwt2_forward
    st = f(dwt2.WAVELETS[wav], lev, w, h, x.data_ptr(), x.stride(0), y.data_ptr(), y.stride(0), 0,
           ctypes.byref(opt), ws.data_ptr(), nbytes.value, torch.cuda.current_stream().cuda_stream)
    assert st == dwt2.OK
    torch.cuda.synchronize()
    return y


CASES = [(300, 203, 3), (1030, 770, 2), (64, 700, 4), (7, 5, 2)]


def both(poison, x, wav, lev, **kw):
    opt = dwt2.make_options(**kw)
    want = call(dwt2.library(), 0, x, torch.empty_like(x), wav, lev, opt)
    got = call(poison, 0, x, torch.full_like(x, 7.0), wav, lev, opt)
    assert torch.equal(got, want), ("forward", wav, lev, kw)
    back = call(dwt2.library(), 1, want, torch.empty_like(x), wav, lev, opt)
    got_b = call(poison, 1, want, torch.full_like(x, 7.0), wav, lev, opt)
    assert torch.equal(got_b, back), ("inverse", wav, lev, kw)


def images(seed):
    rng = np.random.default_rng(seed)
    return [(torch.from_numpy(rng.integers(0, 256, size=(h, w)).astype(np.float32)).to(dev()), lev)
            for (w, h, lev) in CASES]


def test_fused_kernels_read_only_what_they_wrote(poison):
    for x, lev in images(900):
        for wav in ("cdf53", "cdf97", "dd137"):
            for rows in dwt2.TILE_ROWS[wav]:
                for nb in (1, 2):
                    for order in ("runs", "bands"):
                        both(poison, x, wav, lev, tile_rows=rows, lds_buffers=nb, tile_order=order)
            both(poison, x, wav, lev, arithmetic="fp64")
            both(poison, x, wav, lev, arithmetic="fp64", lds_buffers=1)
            both(poison, x, wav, lev, fuse_tail=1)


def test_tile_harness_kernels_read_only_what_they_wrote(poison):
    for x, lev in images(901):
        for wav in ("cdf53", "cdf97"):
            for scheme in ("monolithic*-tile", "sweldens", "iwahashi", "monolithic", "explosive",
                           "explosive*", "iwahashi*", "polyphase*", "rowcol"):
                both(poison, x, wav, lev, scheme=scheme)


def test_batched_kernels_read_only_what_they_wrote(poison):
    xs = [x for x, _ in images(902)]
    wavs = ["cdf53", "cdf97", "dd137", "cdf97"]
    levs = [3, 2, 4, 2]
    for inverse in (0, 1):
        ys = [torch.empty_like(x) for x in xs]
        zs = [torch.full_like(x, 7.0) for x in xs]
        ents = [(wav, lev, x.shape[1], x.shape[0], x.data_ptr(), x.stride(0), y.data_ptr(), y.stride(0))
                for x, y, wav, lev in zip(xs, ys, wavs, levs)]
        entp = [(wav, lev, x.shape[1], x.shape[0], x.data_ptr(), x.stride(0), z.data_ptr(), z.stride(0))
                for x, z, wav, lev in zip(xs, zs, wavs, levs)]
        for lib, e, outs in ((dwt2.library(), ents, ys), (poison, entp, zs)):
            arr = dwt2.make_images(e)
            n = ctypes.c_size_t()
            assert lib.dwt2_batch_workspace_bytes(arr, len(e), None, ctypes.byref(n)) == dwt2.OK
            ws = torch.empty(n.value, dtype=torch.uint8, device=dev())
            f = lib.dwt2_inverse_batch if inverse else lib.dwt2_forward_batch
            assert f(arr, len(e), 0, None, ws.data_ptr(), n.value,
                     torch.cuda.current_stream().cuda_stream) == dwt2.OK
            torch.cuda.synchronize()
        for i in range(len(xs)):
            assert torch.equal(zs[i], ys[i]), (inverse, i)


def test_injected_launch_failure_runs_nothing_and_the_next_call_works():
    x = torch.from_numpy(np.random.default_rng(903).integers(0, 256, size=(500, 600))
                         .astype(np.float32)).to(dev())
    y = torch.full_like(x, float("nan"))
    try:
        assert dwt2.dwt2_debug_fail_launches(1) == dwt2.OK
        with pytest.raises(dwt2.Dwt2Error) as e:
            dwt2.forward(x, "cdf97", 4, out=y)
        assert e.value.status == dwt2.E_HIP and dwt2.dwt2_last_hip_error() == 9
    finally:
        dwt2.dwt2_debug_fail_launches(0)
    torch.cuda.synchronize()
    assert bool(torch.isnan(y).all())  # nothing ran
    want = dwt2.forward(x, "cdf97", 4)
    dwt2.forward(x, "cdf97", 4, out=y)
    torch.cuda.synchronize()
    assert torch.equal(y, want)
