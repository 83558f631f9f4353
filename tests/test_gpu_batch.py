"""GPU tests of the batched entry points (dwt2_forward_batch /
dwt2_inverse_batch, through the C ABI).

A batched call must give every image exactly the bits of the single-image
call with the same arguments (same tile kernel, same per-tile arithmetic), so
the main check is bitwise equality with dwt2_forward / dwt2_inverse, which the
parity tests pin to the oracle; the oracle is also run directly on the small
images of each batch, to the parity bar.
"""
import numpy as np
import pytest

import oracle
from paper_1605_00561_amd import workloads as wl
from test_gpu_parity import check, dev, empty_dev, exact_expected, paper_ratio, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import dwt2  # noqa: E402

# (width, height, wavelet, levels, pitch or None): odd sizes, 2x2, deep pyramids,
# pitched buffers, both wavelets.
MIXED = [(2, 2, "cdf53", 1, None), (3, 5, "cdf97", 2, None), (37, 22, "cdf97", 3, 41),
         (129, 64, "cdf53", 4, None), (300, 500, "cdf97", 5, 333), (1030, 770, "cdf53", 3, None),
         (520, 131, "cdf97", 1, None), (64, 3000, "cdf53", 6, 80), (1000, 999, "cdf97", 7, None),
         (258, 130, "cdf53", 2, None), (77, 45, "dd137", 3, None), (513, 260, "dd137", 4, 520)]


def mixed_inputs(seed=200):
    rng = np.random.default_rng(seed)
    xs, hs = [], []
    for (w, h, wav, lev, pitch) in MIXED:
        x = rng.integers(0, 256, size=(h, w)).astype(np.float32)
        hs.append(x)
        xs.append(to_dev(x, pitch))
    return xs, hs


def outs_like(xs):
    return [empty_dev(x.shape[0], x.shape[1], x.stride(0) if x.stride(0) != x.shape[1] else None)
            for x in xs]


def single(x, wav, lev, norm, arith, inverse=False):
    f = dwt2.inverse if inverse else dwt2.forward
    return f(x, wav, lev, norm, "auto", out=torch.empty_like(x), arithmetic=arith)


@pytest.mark.parametrize("arith", ["fp32", "fp64"])
@pytest.mark.parametrize("norm", ["unit_dc", "paper"])
def test_mixed_batch_equals_single_calls(norm, arith):
    xs, hosts = mixed_inputs()
    # the last image shares image 4's source with another wavelet and depth
    xs.append(xs[4])
    hosts.append(hosts[4])
    cfg = [(w, l) for (_, _, w, l, _) in MIXED] + [("cdf53", 4)]
    wavs, levs = [c[0] for c in cfg], [c[1] for c in cfg]
    ys = dwt2.forward_batch(xs, wavs, levs, norm, arith, outs=outs_like(xs))
    zs = dwt2.inverse_batch(ys, wavs, levs, norm, arith, outs=outs_like(xs))
    torch.cuda.synchronize()
    for i, (x, y, z, wav, lev) in enumerate(zip(xs, ys, zs, wavs, levs)):
        what = f"image {i} {x.shape[1]}x{x.shape[0]} {wav} L{lev} {norm} {arith}"
        assert torch.equal(y, single(x, wav, lev, norm, arith)), "forward " + what
        assert torch.equal(z, single(y, wav, lev, norm, arith, inverse=True)), "inverse " + what
        if arith == "fp32":
            got = to_host(y)
            ref = oracle.forward(hosts[i].astype(np.float64), wav, lev, "unit_dc")
            # PAPER's LL doubles per level (2^7 x 255 at level 7, where one FP32
            # ulp already exceeds 1e-3): compare it in UNIT_DC scale, dividing
            # each subband by its exact power-of-two factor.
            scale = paper_ratio(x.shape[1], x.shape[0], lev) if norm == "paper" else 1.0
            check(got / scale, ref, exact_expected(wav, lev, norm), "fwd " + what)
            check(to_host(z), oracle.inverse(got, wav, lev, norm), exact_expected(wav, lev, norm),
                  "inv " + what)


def test_workspace_reuse_with_a_smaller_batch():
    """The image table of a previous, larger call must not leak into the next."""
    xs, _ = mixed_inputs(201)
    wavs, levs = [m[2] for m in MIXED], [m[3] for m in MIXED]
    big = dwt2.Batch(xs, outs_like(xs), wavs, levs)
    big()
    sub = [1, 5, 8]
    small = dwt2.Batch([xs[i] for i in sub], outs_like([xs[i] for i in sub]),
                       [wavs[i] for i in sub], [levs[i] for i in sub], workspace=big.workspace)
    for rep in range(2):
        small()
        torch.cuda.synchronize()
        for j, i in enumerate(sub):
            assert torch.equal(small.outputs[j], single(xs[i], wavs[i], levs[i], "unit_dc", "auto"))
            assert torch.equal(big.outputs[i], single(xs[i], wavs[i], levs[i], "unit_dc", "auto"))


def test_graph_replay_matches_eager():
    """A batched call captured in a HIP graph: each replay, with the inputs
    changed by eager work in between, equals an eager call on the same inputs."""
    xs, _ = mixed_inputs(202)
    wavs, levs = [m[2] for m in MIXED], [m[3] for m in MIXED]
    graphed = dwt2.Batch(xs, outs_like(xs), wavs, levs)
    eager = dwt2.Batch(xs, outs_like(xs), wavs, levs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        graphed()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graphed()
    gen = torch.Generator(device=dev()).manual_seed(7)
    for rep in range(4):
        for x in xs:
            x.copy_(torch.randint(0, 256, x.shape, generator=gen, device=dev()).float())
        torch.cuda.synchronize()
        g.replay()
        eager()
        torch.cuda.synchronize()
        for i in range(len(xs)):
            assert torch.equal(graphed.outputs[i], eager.outputs[i]), f"replay {rep} image {i}"


def test_full_batch_of_512_uneven_images():
    """The 512-image batch (even sizes 256..4096, levels 3..6, both wavelets)
    in the configuration the benchmark times: every image equals its
    single-image call, forward and inverse; three images are checked against
    the oracle outright."""
    specs = wl.batch_specs()
    xs = []
    for i, (w, h, wav, lev) in enumerate(specs):
        xs.append(torch.from_numpy(wl.batch_image(i, w, h)).to(dev()).float())
    wavs, levs = [s[2] for s in specs], [s[3] for s in specs]
    ys = dwt2.forward_batch(xs, wavs, levs)
    zs = dwt2.inverse_batch(ys, wavs, levs)
    torch.cuda.synchronize()
    for i, (w, h, wav, lev) in enumerate(specs):
        assert torch.equal(ys[i], single(xs[i], wav, lev, "unit_dc", "auto")), f"forward image {i}"
        assert torch.equal(zs[i], single(ys[i], wav, lev, "unit_dc", "auto", inverse=True)), \
            f"inverse image {i}"
    by_size = sorted(range(len(specs)), key=lambda i: specs[i][0] * specs[i][1])
    for i in by_size[:2] + by_size[-1:]:
        w, h, wav, lev = specs[i]
        got = to_host(ys[i])
        ref = oracle.forward(wl.batch_image(i, w, h).astype(np.float64), wav, lev, "unit_dc")
        check(got, ref, False, f"fwd batch image {i} {w}x{h} {wav} L{lev}")
        check(to_host(zs[i]), oracle.inverse(got, wav, lev, "unit_dc"), False,
              f"inv batch image {i}")


def test_batch_at_tuned_and_stepped_down_heights():
    """Images whose level sizes have tuned heights (every built height is
    used by some image level) and small batches whose launches step down to
    shorter tiles: every image still equals its single-image call bit for
    bit, and the small ones the oracle."""
    xs, hosts = mixed_inputs(203)
    wavs, levs = [m[2] for m in MIXED], [m[3] for m in MIXED]
    lines = []
    for (w, h, wav, lev, _) in MIXED:
        heights = dwt2.TILE_ROWS[wav]
        for k in range(lev):
            for inv in (0, 1):
                lines.append(f"{dwt2.WAVELETS[wav]} {inv} {w} {h} {heights[(k + inv) % len(heights)]} 1")
            w, h = (w + 1) // 2, (h + 1) // 2
    try:
        dwt2.dwt2_tune_reset()
        assert dwt2.dwt2_tune_import("\n".join(lines) + "\n") == dwt2.OK
        a = dwt2.make_images([(wav, lev, x.shape[1], x.shape[0], x.data_ptr(), x.stride(0),
                               x.data_ptr() + 4, x.stride(0))
                              for x, wav, lev in zip(xs, wavs, levs)])
        used = set()
        for k in range(max(levs)):
            st, rows = dwt2.dwt2_batch_tile_rows(0, a, len(xs), k)
            assert st == dwt2.OK
            used |= {(wavs[i], r) for i, r in enumerate(rows) if r}
        assert used == {(w, r) for w in set(wavs) for r in dwt2.TILE_ROWS[w]}
        ys = dwt2.forward_batch(xs, wavs, levs, outs=outs_like(xs))
        zs = dwt2.inverse_batch(ys, wavs, levs, outs=outs_like(xs))
        torch.cuda.synchronize()
    finally:
        dwt2.dwt2_tune_reset()
    for i, (x, y, z, wav, lev) in enumerate(zip(xs, ys, zs, wavs, levs)):
        what = f"image {i} {x.shape[1]}x{x.shape[0]} {wav} L{lev}"
        assert torch.equal(y, single(x, wav, lev, "unit_dc", "auto")), "forward " + what
        assert torch.equal(z, single(y, wav, lev, "unit_dc", "auto", inverse=True)), "inverse " + what
        got = to_host(y)
        check(got, oracle.forward(hosts[i].astype(np.float64), wav, lev), exact_expected(wav, lev, "unit_dc"),
              "fwd " + what)
    # two small images: every level launch is short of work-groups
    for sub in ([0, 2], [3, 11]):
        st, rows = dwt2.dwt2_batch_tile_rows(0, dwt2.make_images(
            [(wavs[i], levs[i], xs[i].shape[1], xs[i].shape[0], 1 << 40, xs[i].stride(0),
              1 << 41, xs[i].stride(0)) for i in sub]), len(sub), 0)
        assert rows == [min(dwt2.TILE_ROWS[wavs[i]]) for i in sub]
        ys = dwt2.forward_batch([xs[i] for i in sub], [wavs[i] for i in sub], [levs[i] for i in sub])
        torch.cuda.synchronize()
        for j, i in enumerate(sub):
            assert torch.equal(ys[j], single(xs[i], wavs[i], levs[i], "unit_dc", "auto")), f"small {i}"


def test_large_levels_single_calls_equal_batch():
    """Single-image levels of 2^26 pixels and more run with six work-groups per
    CU (LDS reserved per work-group); batched launches never do.  The
    reservation changes where work-groups run, not what they compute: at a
    ragged size just above the threshold both give the same bits, forward and
    inverse, and the smallest image of the batch (whose levels are below the
    threshold) stays pinned to the oracle."""
    rng = np.random.default_rng(210)
    w, h = 8203, 8193  # 67.2 M pixels >= 2^26; odd sides, ragged last tiles
    assert w * h >= 1 << 26
    x = rng.integers(0, 256, size=(h, w)).astype(np.float32)
    small = rng.integers(0, 256, size=(300, 517)).astype(np.float32)
    xs = [to_dev(x), to_dev(small)]
    for wav in ("cdf97", "cdf53"):
        wavs, levs = [wav, wav], [2, 2]
        ys = dwt2.forward_batch(xs, wavs, levs, outs=outs_like(xs))
        zs = dwt2.inverse_batch(ys, wavs, levs, outs=outs_like(xs))
        y1 = single(xs[0], wav, 2, "unit_dc", "auto")
        z1 = single(ys[0], wav, 2, "unit_dc", "auto", inverse=True)
        assert torch.equal(ys[0], y1), wav
        assert torch.equal(zs[0], z1), wav
        check(to_host(ys[1]), oracle.forward(small.astype(np.float64), wav, 2), False, f"small {wav}")
    del xs, ys, zs, y1, z1
    torch.cuda.empty_cache()
