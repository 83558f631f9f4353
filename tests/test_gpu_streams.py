"""GPU tests of how the single-image entry points behave under HIP graphs,
several streams and several host threads (through the C ABI).

The library enqueues only kernel launches (no memsets, copies or
allocations) on the caller's stream, so a call can be captured in a graph
and replayed, and calls on different streams or threads on disjoint buffers
must give exactly the bits of the same calls made one at a time.
"""
import threading

import numpy as np
import pytest

from test_gpu_parity import dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import dwt2  # noqa: E402


def image(seed, h, w):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.integers(0, 256, size=(h, w)).astype(np.float32)).to(dev())


@pytest.mark.parametrize("wav", ["cdf53", "cdf97", "dd137"])
def test_multilevel_call_replays_from_a_graph(wav):
    h, w, lev = 700, 1030, 4
    x = image(600, h, w)
    y, z = torch.empty_like(x), torch.empty_like(x)
    st, nbytes = dwt2.dwt2_workspace_bytes(wav, lev, w, h)
    assert st == dwt2.OK
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        dwt2.forward(x, wav, lev, out=y, workspace=ws)
        dwt2.inverse(y, wav, lev, out=z, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dwt2.forward(x, wav, lev, out=y, workspace=ws)
        dwt2.inverse(y, wav, lev, out=z, workspace=ws)
    gen = torch.Generator(device=dev()).manual_seed(601)
    for rep in range(4):
        x.copy_(torch.randint(0, 256, x.shape, generator=gen, device=dev()).float())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want_y = dwt2.forward(x, wav, lev)
        want_z = dwt2.inverse(want_y, wav, lev)
        torch.cuda.synchronize()
        assert torch.equal(y, want_y), f"replay {rep} forward"
        assert torch.equal(z, want_z), f"replay {rep} inverse"


def test_two_streams_at_once():
    shapes = [(2048, 2048, "cdf97", 3), (1500, 900, "cdf53", 4)]
    xs = [image(610 + i, h, w) for i, (h, w, _, _) in enumerate(shapes)]
    want = [dwt2.forward(x, wav, lev) for x, (_, _, wav, lev) in zip(xs, shapes)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty_like(x) for x in xs]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        for i, (x, (_, _, wav, lev)) in enumerate(zip(xs, shapes)):
            with torch.cuda.stream(streams[i]):
                outs[i].fill_(float("nan"))
                dwt2.forward(x, wav, lev, out=outs[i])
        torch.cuda.synchronize()
        for i in range(2):
            assert torch.equal(outs[i], want[i]), f"rep {rep} stream {i}"


def test_host_threads_share_the_library():
    jobs = [(image(620 + i, 300 + 37 * i, 500 - 29 * i), ("cdf53", "cdf97", "dd137")[i % 3], 1 + i % 4)
            for i in range(8)]
    want = [dwt2.inverse(dwt2.forward(x, wav, lev), wav, lev) for x, wav, lev in jobs]
    torch.cuda.synchronize()
    got = [None] * len(jobs)
    errors = []

    def work(i):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                x, wav, lev = jobs[i]
                for _ in range(5):
                    got[i] = dwt2.inverse(dwt2.forward(x, wav, lev), wav, lev)
            s.synchronize()
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for i in range(len(jobs)):
        assert torch.equal(got[i], want[i]), f"job {i}"


@pytest.mark.parametrize("batched", [False, True])
def test_stream_argument_keeps_buffers_until_its_work_ran(batched):
    """forward(..., stream=side) allocates its output and workspace for the
    side stream: a tensor of the same size allocated and filled on the
    current stream right after the call, while the side stream is still busy,
    must not land on the workspace the queued kernels read."""
    import oracle
    h, w, lev = 1200, 1500, 3
    x = image(630, h, w)
    st, nbytes = dwt2.dwt2_workspace_bytes("cdf97", lev, w, h)
    assert st == dwt2.OK and nbytes > 0
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(20_000_000)  # hold the side stream (bounded spin)
    if batched:
        y = dwt2.forward_batch([x], ["cdf97"], [lev], stream=side)[0]
    else:
        y = dwt2.forward(x, "cdf97", lev, stream=side)
    junk = [torch.full((nbytes // 4 + 1,), float("nan"), device=dev()) for _ in range(4)]
    junk += [torch.full((h, w), float("nan"), device=dev()) for _ in range(2)]
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    ref = oracle.forward(x.cpu().numpy().astype(np.float64), "cdf97", lev)
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() <= 1e-3
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-6
    del junk
