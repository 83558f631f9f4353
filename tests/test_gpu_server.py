"""GPU tests of the serving loop (dwt2_server_*, through the C ABI): every
request's result matches the FP64 oracle (forward requests on integer images,
inverse requests on oracle-forward coefficients, as the serving workload
feeds them) and equals, bit for bit, the single-image call's result, whether
it ran alone, in a mix submitted from two threads, behind a dependency,
through a full arena or footprint cap, or under a replayed arrival
schedule."""
import threading

import numpy as np
import pytest

import oracle
from test_gpu_parity import check, dev, exact_expected, max_levels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1605_00561_amd import dwt2  # noqa: E402

MiB = 1 << 20


def request_input(rng, w, h, wav, lev, inverse):
    """A forward request's integer image, or an inverse request's FP32
    coefficients: the oracle's forward transform of such an image."""
    img = rng.integers(0, 256, size=(h, w)).astype(np.float32)
    if inverse:
        img = oracle.forward(img.astype(np.float64), wav, lev).astype(np.float32)
    return torch.from_numpy(img).to(dev())


def random_requests(n, seed, lo=16, hi=1500):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        w = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        h = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        wav = ("cdf53", "cdf97", "dd137")[int(rng.integers(0, 3))]
        lev = int(rng.integers(1, max_levels(w, h, 6) + 1))
        inverse = bool(rng.random() < 0.5)
        x = request_input(rng, w, h, wav, lev, inverse)
        y = torch.full_like(x, float("nan"))
        out.append((x, y, wav, lev, inverse))
    return out


def expected(x, wav, lev, inverse):
    f = dwt2.inverse if inverse else dwt2.forward
    return f(x, wav, lev, out=torch.empty_like(x))


def check_oracle(x, y, wav, lev, inv, what):
    """The served result against the FP64 oracle on the same FP32 input: the
    stated bar (max-abs <= 1e-3, rel-L2 <= 1e-6), bit-exact where 5/3 on
    integer input is exactly representable."""
    src = x.cpu().numpy().astype(np.float64)
    got = y.cpu().numpy().astype(np.float64)
    if inv:
        check(got, oracle.inverse(src, wav, lev), False, what)
    else:
        check(got, oracle.forward(src, wav, lev), exact_expected(wav, lev, "unit_dc"), what)


def check_all(reqs):
    torch.cuda.synchronize()
    for i, (x, y, wav, lev, inv) in enumerate(reqs):
        what = f"request {i}: {x.shape[1]}x{x.shape[0]} {wav} L{lev} {'inv' if inv else 'fwd'}"
        assert torch.equal(y, expected(x, wav, lev, inv)), what
        check_oracle(x, y, wav, lev, inv, what)


def test_mix_from_two_threads_equals_single_calls():
    reqs = random_requests(60, 300)
    with dwt2.Server(64 * MiB, max_batch=16) as srv:
        tickets = [None, None]

        def worker(k):
            tickets[k] = [srv.submit(*r) for r in reqs[k::2]]

        th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for k in range(2):
            for t in tickets[k]:
                c = srv.wait(t)
                assert c.status == dwt2.OK and c.latency_us >= c.queue_us >= 0.0
    check_all(reqs)


def test_dependent_requests_run_in_order():
    """forward A -> B, then inverse B -> C, then forward C -> D: each consumes
    the previous output, so they must not share a batch."""
    rng = np.random.default_rng(301)
    with dwt2.Server(64 * MiB) as srv:
        for (w, h, wav, lev) in [(300, 200, "cdf97", 3), (77, 1025, "cdf53", 4)]:
            a = torch.from_numpy(rng.integers(0, 256, size=(h, w)).astype(np.float32)).to(dev())
            b, c, d = (torch.full_like(a, float("nan")) for _ in range(3))
            ts = [srv.submit(a, b, wav, lev), srv.submit(b, c, wav, lev, inverse=True),
                  srv.submit(c, d, wav, lev)]
            for t in ts:
                srv.wait(t)
            torch.cuda.synchronize()
            eb = expected(a, wav, lev, False)
            ec = expected(eb, wav, lev, True)
            assert torch.equal(b, eb) and torch.equal(c, ec)
            assert torch.equal(d, expected(ec, wav, lev, False))
            what = f"{w}x{h} {wav} L{lev}"
            check_oracle(a, b, wav, lev, False, "fwd " + what)
            check_oracle(b, c, wav, lev, True, "inv " + what)
            check(c.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64), False,
                  "round trip " + what)


def test_full_arena_admits_requests_one_at_a_time():
    w, h, wav, lev = 1024, 768, "cdf97", 4
    img = dwt2.make_images([(wav, lev, w, h, 1 << 40, w, 1 << 41, w)])
    st, one = dwt2.dwt2_batch_workspace_bytes(img, 1, None)
    assert st == dwt2.OK
    rng = np.random.default_rng(302)
    reqs = []
    for i in range(12):
        x = request_input(rng, w, h, wav, lev, bool(i % 2))
        reqs.append((x, torch.full_like(x, float("nan")), wav, lev, bool(i % 2)))
    with dwt2.Server(one + 256, max_inflight=3) as srv:
        ts = [srv.submit(*r) for r in reqs]
        for t in ts:
            assert srv.wait(t).status == dwt2.OK
    check_all(reqs)


def test_footprint_cap_admits_requests_within_it():
    """A footprint cap that holds two of these requests (input + output + LL
    buffers) but not three: later requests wait for earlier ones to retire,
    and each still gets its result.  A request over the cap alone is refused.
    (Which requests share the device is checked on the CPU against a model of
    the rule, in test_server_plan.)"""
    w, h, wav, lev = 1024, 768, "cdf53", 3
    st, ll = dwt2.dwt2_workspace_bytes(wav, lev, w, h)
    assert st == dwt2.OK
    one = 2 * 4 * w * h + ll
    cap_mib = (2 * one + MiB - 1) // MiB
    assert cap_mib * MiB < 3 * one
    rng = np.random.default_rng(304)
    reqs = []
    for i in range(10):
        x = request_input(rng, w, h, wav, lev, bool(i % 3 == 0))
        reqs.append((x, torch.full_like(x, float("nan")), wav, lev, bool(i % 3 == 0)))
    with dwt2.Server(64 * MiB, max_inflight=4, max_footprint_mib=cap_mib) as srv:
        big = torch.zeros((2048, 2048), device=dev())
        with pytest.raises(dwt2.Dwt2Error) as e:  # 32 MiB of input + output alone
            srv.submit(big, torch.zeros_like(big), "cdf53", 1)
        assert e.value.status == dwt2.E_WORKSPACE
        ts = [srv.submit(*r) for r in reqs]
        for t in ts:
            assert srv.wait(t).status == dwt2.OK
    check_all(reqs)


def test_replay_schedule():
    reqs = random_requests(40, 303, hi=700)
    arrivals = np.cumsum(np.full(len(reqs), 150.0)) - 150.0
    with dwt2.Server(64 * MiB, max_batch=8) as srv:
        done = srv.replay(reqs, arrivals)
    assert all(c.status == dwt2.OK for c in done)
    assert all(c.latency_us >= c.queue_us >= 0.0 for c in done)
    check_all(reqs)


def test_submit_and_wait_errors():
    with dwt2.Server(4 * MiB) as srv:
        x = torch.zeros((64, 64), device=dev())
        y = torch.zeros_like(x)
        with pytest.raises(dwt2.Dwt2Error) as e:
            srv.submit(x, y, "cdf53", 7)  # 64 -> 1 before level 7
        assert e.value.status == dwt2.E_SIZE
        inside = srv.arena[:64 * 64 * 4].view(torch.float32).view(64, 64)
        with pytest.raises(dwt2.Dwt2Error) as e:
            srv.submit(inside, y, "cdf53", 1)
        assert e.value.status == dwt2.E_ALIAS
        big = torch.zeros((2048, 2048), device=dev())
        with pytest.raises(dwt2.Dwt2Error) as e:
            srv.submit(big, torch.zeros_like(big), "cdf97", 3)  # LL buffers of 4 MiB + 1 MiB
        assert e.value.status == dwt2.E_WORKSPACE
        with pytest.raises(dwt2.Dwt2Error) as e:
            srv.submit(x, x, "cdf53", 1)
        assert e.value.status == dwt2.E_ALIAS
        st, _ = dwt2.dwt2_server_wait(srv.handle, 12345)
        assert st == dwt2.E_STATE
        t = srv.submit(x, y, "cdf53", 2)
        assert srv.wait(t).status == dwt2.OK
        st, _ = dwt2.dwt2_server_wait(srv.handle, t)
        assert st == dwt2.E_STATE
