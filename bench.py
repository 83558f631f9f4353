"""Benchmark of the 2-D lifting DWT on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = the forward and the inverse transform (one level, CDF 9/7) of one
8192 x 8192 FP32 image (smooth cosine gradient + Gaussian noise, seeded),
with inputs resident in HBM, by the fused Monolithic* kernel.  Untimed steps
run for --device-warmup seconds (the device's clocks ramp over the first ~100
launches), then W warm-up steps, then K timed steps.  Prints ONE JSON line:

  value        Gpixel/s over the timed steps (2 x 8192^2 pixels per step)
  roofline     the fused forward kernel against the HBM roofline: algorithmic
               bytes (4 B read + 4 B written per pixel) / its mean duration,
               timed with HIP events on the launch stream
  schemes      per-scheme forward / inverse Gpixel/s and % of 8 TB/s: the fused
               register-blocked Monolithic*, and in the LDS tile harness
               Monolithic* and Monolithic (2 barriers per pair), separable
               Sweldens (4), Iwahashi, Iwahashi*, Explosive, Explosive* (3) and
               Polyphase* (1), plus the row-column separable two-pass kernels
  transform_only  the paper's transform-only mode (no image input or output)
               per scheme at 8192^2: 5/3 and 9/7 in every scheme, DD 13/7 in
               the fused kernel
  c1_512       the 512^2 5/3 one-level workload, row-column and fused
               (cache-resident, launch-bound)
  pyramid      per-level and five-level times of the 16384^2 9/7 pyramid
  pyramid_cdf53  the same for the 16384^2 5/3 pyramid
  batch        512 uneven images: batched call, HIP-graph replay, and one
               call per image (images/s, p99, fraction of 8 TB/s)
  serve        the serving loop under a Poisson request stream at 0.8 x its
               saturated rate: images/s, p50 / p99 latency
  cpu_baseline the FP64 CPU oracle on the host cores, forward + inverse of the
               same image (all cores), and on one thread (a crop of it)
GPU times are medians, with the minimum beside them where a table has one.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BYTES_PER_PX = 8.0             # algorithmic: 4 B read + 4 B written per pixel per level
WORKLOAD = "cdf97_8192_l1"
NSETS = 3                      # rotating buffer sets (each 3 x 256 MiB) defeat the 256 MB MALL
DEVICE_WARMUP_S = 0.5          # untimed steps before the W warm-up steps (clock ramp)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scheme-reps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget for the oracle baseline")
    ap.add_argument("--device-warmup", type=float, default=DEVICE_WARMUP_S,
                    help="seconds of untimed steps before the W warm-up steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-schemes", action="store_true")
    ap.add_argument("--no-pyramid", action="store_true",
                    help="skip the per-level table of the 16384^2 five-level workload")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 512-image batched workload")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving-loop request stream")
    ap.add_argument("--no-tiles", action="store_true",
                    help="skip the tile-height table (every built height per wavelet and size)")
    ap.add_argument("--no-transform-only", action="store_true",
                    help="skip the transform-only table (no image I/O, every scheme)")
    ap.add_argument("--no-c1", action="store_true",
                    help="skip the 512^2 5/3 one-level table")
    ap.add_argument("--no-copy", action="store_true",
                    help="skip the device-to-device copy (the bandwidth and counter reference)")
    return ap.parse_args()


def source_digest(paths) -> str:
    """SHA-256 of C/C++/HIP sources with comments removed and whitespace
    collapsed: it changes with the code, not with its comments."""
    import hashlib
    import re
    h = hashlib.sha256()
    for p in paths:
        text = open(os.path.join(ROOT, p)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def traffic_from_profiles(tag: str, kernel: str):
    """HBM bytes per launch of the dominant kernel from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None when it is
    absent, was taken on different kernel code or of another kernel."""
    path = os.path.join(ROOT, "profiles", f"{tag}_hbm_counters.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if source_digest(rec["sources"]) != rec["sources_digest"] or rec["kernel"] != kernel:
            return None
        return int(round(rec["bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


class HipTimer:
    """Timing events of the HIP runtime in this process (the one torch loaded),
    created with hipEventDisableSystemFence: a timing-only event then records
    without the system-scope cache writeback and invalidation that a default
    event adds around the work it brackets (HIP documents the flag for exactly
    this use), so the interval is the kernels' own time."""

    DISABLE_SYSTEM_FENCE = 0x20000000

    def __init__(self, n):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = []
        for _ in range(n):
            e = ctypes.c_void_p()
            if self.hip.hipEventCreateWithFlags(ctypes.byref(e), self.DISABLE_SYSTEM_FENCE) != 0:
                raise RuntimeError("hipEventCreateWithFlags failed")
            self.ev.append(e)

    def record(self, i, stream_handle):
        if self.hip.hipEventRecord(self.ev[i], stream_handle) != 0:
            raise RuntimeError("hipEventRecord failed")

    def ms(self, i, j):
        out = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(out), self.ev[i], self.ev[j]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return out.value

    def close(self):
        for e in self.ev:
            self.hip.hipEventDestroy(e)
        self.ev = []


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the transform runs on one GPU per process; --gpus {args.gpus} is not "
              "supported (several GPUs would each take whole images or row bands)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1605_00561_amd import dwt2, workloads

    dev = torch.device("cuda:0")
    spec = workloads.WORKLOADS[WORKLOAD]
    W, H, wav, lev = spec["width"], spec["height"], spec["wavelet"], spec["levels"]
    img = workloads.workload_image(WORKLOAD)
    xs = [torch.from_numpy(img).to(dev) for _ in range(NSETS)]
    ys = [torch.empty_like(xs[0]) for _ in range(NSETS)]
    zs = [torch.empty_like(xs[0]) for _ in range(NSETS)]
    stream = torch.cuda.current_stream()
    npx = W * H

    # The timed step calls the C ABI directly with arguments marshalled once, so
    # that the host enqueues faster than the GPU drains (the torch conveniences
    # cost tens of microseconds per call, enough to leave the GPU idle between
    # the two ~100 us kernels and to inflate the event times).
    lib = dwt2.library()
    opt = dwt2.make_options(scheme="monolithic*")
    st, nws = dwt2.dwt2_workspace_bytes(wav, lev, W, H, opt)
    assert st == dwt2.OK and nws == 0  # one level needs no workspace
    hs = stream.cuda_stream
    wcode = dwt2.WAVELETS[wav]
    fargs = [(wcode, lev, W, H, xs[k].data_ptr(), xs[k].stride(0), ys[k].data_ptr(), ys[k].stride(0),
              dwt2.EXT_WHOLE_SYMMETRIC, ctypes.byref(opt), None, 0, hs) for k in range(NSETS)]
    iargs = [(wcode, lev, W, H, ys[k].data_ptr(), ys[k].stride(0), zs[k].data_ptr(), zs[k].stride(0),
              dwt2.EXT_WHOLE_SYMMETRIC, ctypes.byref(opt), None, 0, hs) for k in range(NSETS)]
    status = []

    # Events 2i and 2i + 1 bracket step i's forward, 2i + 1 and 2i + 2 its
    # inverse: a step's closing event is the next step's opening one.
    timer = HipTimer(2 * args.steps + 1)

    def step(i, timed=False):
        k = i % NSETS
        if timed and i == 0:
            timer.record(0, hs)
        status.append(lib.dwt2_forward(*fargs[k]))
        if timed:
            timer.record(2 * i + 1, hs)
        status.append(lib.dwt2_inverse(*iargs[k]))
        if timed:
            timer.record(2 * i + 2, hs)

    # Device warm-up: the kernels run ~10% slower over the first ~100 launches
    # of a process (measured), so untimed steps run for at least
    # --device-warmup seconds (default DEVICE_WARMUP_S) before the requested
    # warm-up steps.
    t_w = time.perf_counter()
    n_dev_warm = 0
    while time.perf_counter() - t_w < args.device_warmup:
        for i in range(8):
            step(i)
        torch.cuda.synchronize()
        n_dev_warm += 8
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i, timed=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if any(st != dwt2.OK for st in status):
        raise dwt2.Dwt2Error(next(st for st in status if st != dwt2.OK), "timed step")
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    fwd_ms = [timer.ms(2 * i, 2 * i + 1) for i in range(args.steps)]
    inv_ms = [timer.ms(2 * i + 1, 2 * i + 2) for i in range(args.steps)]
    timer.close()
    value = 2 * npx / (ms_per_step * 1e-3) / 1e9

    fwd_mean = statistics.fmean(fwd_ms)
    achieved = BYTES_PER_PX * npx / (fwd_mean * 1e-3) / 1e9
    kernel = f"k_fused_forward<{wcode}, {dwt2.tile_rows(wav, W, H)}, float, 2>"
    traffic = traffic_from_profiles("fused_forward_cdf97_8192", kernel)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": kernel,
                "algorithmic_bytes_per_launch": int(BYTES_PER_PX * npx),
                "mean_launch_us": round(fwd_mean * 1e3, 2),
                "inverse_mean_launch_us": round(statistics.fmean(inv_ms) * 1e3, 2)}

    # Sanity: the timed output round-trips the input.
    torch.cuda.synchronize()
    rt_err = float((zs[(args.steps - 1) % NSETS] - xs[0]).abs().max())

    out = {
        "metric": "Gpixel/s (2-D DWT, one level, forward + inverse)",
        "value": round(value, 2), "unit": "Gpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cdf97_8192x8192_l1_fwd+inv", "wavelet": wav, "width": W,
                   "height": H, "levels": lev, "scheme": "monolithic*",
                   "tile_rows": {"forward": dwt2.tile_rows(wav, W, H),
                                 "inverse": dwt2.tile_rows(wav, W, H, inverse=True)},
                   "tile_order": {"forward": dwt2.tile_order(wav, W, H),
                                  "inverse": dwt2.tile_order(wav, W, H, inverse=True)},
                   "image": "cosine gradient (period 512) + N(0, 8^2), clipped to [0, 255]",
                   "buffer_sets": NSETS},
        "device_warmup_steps": n_dev_warm,
        "device": device_info(torch, lib),
        "roofline": roofline,
        "round_trip_max_abs": rt_err,
    }

    if not args.no_schemes:
        out["schemes"] = scheme_table(dwt2, torch, xs, ys, zs, wav, lev, npx, args.scheme_reps)
    if not args.no_tiles:
        out["tiles"] = tile_table(dwt2, torch, xs[0], ys[0], zs[0], args.scheme_reps)
    if not args.no_transform_only:
        out["transform_only"] = transform_only_table(dwt2, torch, dev)
    if not args.no_c1:
        out["c1_512"] = c1_table(dwt2, torch, workloads, dev)
    if not args.no_pyramid:
        del xs, ys, zs
        torch.cuda.empty_cache()
        out["pyramid"] = pyramid_table(dwt2, torch, workloads, args.scheme_reps)
        torch.cuda.empty_cache()
        out["pyramid_cdf53"] = pyramid_table(dwt2, torch, workloads, args.scheme_reps,
                                             name="cdf53_16384_l5")
    if not args.no_batch:
        torch.cuda.empty_cache()
        out["batch"] = batch_table(dwt2, torch, workloads, args.scheme_reps)
        torch.cuda.empty_cache()
    if not args.no_serve:
        out["serve"] = serve_table(dwt2, torch, workloads)
        torch.cuda.empty_cache()
    if not args.no_copy:
        out["copy_GBs"] = copy_bandwidth(torch, dev)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(img, wav, lev, args.cpu_seconds)

    print(json.dumps(out), flush=True)


# hipDeviceAttribute_t values of ROCm 7's hip_runtime_api.h.
HIP_ATTR_CLOCK_RATE, HIP_ATTR_MEMORY_BUS_WIDTH, HIP_ATTR_MEMORY_CLOCK_RATE = 5, 59, 60


def device_info(torch, lib):
    """The device, its peak clocks and the software versions of the run."""
    props = torch.cuda.get_device_properties(0)
    info = {"name": props.name, "arch": props.gcnArchName, "compute_units": props.multi_processor_count,
            "memory_GiB": round(props.total_memory / 2**30, 1), "torch": torch.__version__,
            "torch_hip": torch.version.hip}
    try:
        info["rocm"] = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        info["rocm"] = None
    get = lib.hipDeviceGetAttribute  # resolved in the HIP runtime the library links
    get.argtypes, get.restype = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int], ctypes.c_int
    for key, attr, scale in (("peak_engine_clock_MHz", HIP_ATTR_CLOCK_RATE, 1e-3),
                             ("peak_memory_clock_MHz", HIP_ATTR_MEMORY_CLOCK_RATE, 1e-3),
                             ("memory_bus_bits", HIP_ATTR_MEMORY_BUS_WIDTH, 1)):
        v = ctypes.c_int(0)
        info[key] = round(v.value * scale) if get(ctypes.byref(v), attr, 0) == 0 else None
    rv = ctypes.c_int(0)
    lib.hipRuntimeGetVersion.argtypes = [ctypes.POINTER(ctypes.c_int)]
    info["hip_runtime"] = rv.value if lib.hipRuntimeGetVersion(ctypes.byref(rv)) == 0 else None
    return info


def tile_table(dwt2, torch, x, y, z, reps, sizes=(8192, 2048, 512)):
    """Forward / inverse device time (us, HIP-graph timed) of one fused level
    at every built tile height, on n x n crops of the workload image, with the
    height the selection rule picks; then dwt2_autotune's pick for the full
    8192^2 9/7 level (the table is emptied again afterwards)."""
    out = {}
    for wav in ("cdf97", "cdf53", "dd137"):
        for n in sizes:
            xc = x[:n, :n].contiguous()
            yc, zc = torch.empty_like(xc), torch.empty_like(xc)
            row = {"rule": [dwt2.tile_rows(wav, n, n), dwt2.tile_rows(wav, n, n, inverse=True)]}
            for r in dwt2.TILE_ROWS[wav]:
                tf = _graph_us(torch, lambda: dwt2.forward(xc, wav, 1, out=yc, tile_rows=r), reps=reps)
                ti = _graph_us(torch, lambda: dwt2.inverse(yc, wav, 1, out=zc, tile_rows=r), reps=reps)
                row[f"rows{r}_us"] = [round(tf, 2), round(ti, 2)]
            out[f"{wav}@{n}"] = row
    dwt2.dwt2_tune_reset()
    n = x.shape[0]
    dwt2.autotune(x, "cdf97", 1, repeats=20, out=y)
    dwt2.autotune(y, "cdf97", 1, inverse=True, repeats=20, out=z)
    out[f"autotuned_cdf97@{n}"] = [[dwt2.tile_rows("cdf97", n, n), dwt2.tile_order("cdf97", n, n)],
                                   [dwt2.tile_rows("cdf97", n, n, inverse=True),
                                    dwt2.tile_order("cdf97", n, n, inverse=True)]]
    dwt2.dwt2_tune_reset()
    return out


def scheme_table(dwt2, torch, xs, ys, zs, wav, lev, npx, reps):
    """Device time of one level per scheme (HIP-graph timed, as _graph_us)."""
    table = {}
    for name in ("monolithic*", "monolithic*:fp64", "monolithic*:1buf", "monolithic*:fp64:1buf",
                 "monolithic*:fp64:2buf",
                 "monolithic*-tile",
                 "monolithic", "sweldens",
                 "iwahashi", "iwahashi*", "explosive", "explosive*", "polyphase*", "rowcol",
                 "monolithic*@cdf53", "sweldens@cdf53", "monolithic*@dd137"):
        name_w, _, wname = name.partition("@")
        scheme, _, variant = name_w.partition(":")
        arith = "fp64" if "fp64" in variant.split(":") else "auto"
        parts = variant.split(":")
        nb = 1 if "1buf" in parts else 2 if "2buf" in parts else 0
        wav_ = wname or wav
        ws = None
        st, nbytes = dwt2.dwt2_workspace_bytes(wav_, lev, xs[0].shape[1], xs[0].shape[0],
                                               dwt2.make_options(scheme=scheme))
        if nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=xs[0].device)
        res = {}
        for direction in ("forward", "inverse"):
            f = dwt2.forward if direction == "forward" else dwt2.inverse
            src, dst = (xs[0], ys[0]) if direction == "forward" else (ys[0], zs[0])
            us, us_min = _graph_stats(torch, lambda: f(src, wav_, lev, scheme=scheme, out=dst, workspace=ws,
                                                       arithmetic=arith, lds_buffers=nb), reps=reps)
            gbs = BYTES_PER_PX * npx / (us * 1e-6) / 1e9
            res[direction] = {"us": round(us, 2), "min_us": round(us_min, 2),
                              "Gpixel_s": round(npx / (us * 1e-6) / 1e9, 1),
                              "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        table[name] = res
    return table


TRANSFORM_ONLY_SCHEMES = ("monolithic*", "monolithic*-tile", "monolithic", "explosive*", "explosive",
                          "iwahashi*", "sweldens", "iwahashi", "polyphase*")


def transform_only_table(dwt2, torch, dev, n=8192):
    """The paper's transform-only mode (Sec. 6, Experiments 1 and 2): one
    level of an n x n image per scheme with no image input or output
    (dwt2_transform_only), device time per launch from a HIP graph (median
    and min), for the degree-1 wavelets (5/3 and 9/7) and, in the fused
    kernel, the degree-3 DD 13/7."""
    lib = dwt2.library()
    sink = torch.zeros(1, dtype=torch.float32, device=dev)
    out = {"size": [n, n], "unit": "us per launch / Gpixel/s"}
    for wav in ("cdf53", "cdf97", "dd137"):
        row = {}
        for scheme in TRANSFORM_ONLY_SCHEMES if wav != "dd137" else ("monolithic*",):
            opt = dwt2.make_options(scheme=scheme)
            res = {}
            for inverse in (0, 1):
                def call():
                    st = lib.dwt2_transform_only(inverse, dwt2.WAVELETS[wav], n, n, ctypes.byref(opt),
                                                 sink.data_ptr(), torch.cuda.current_stream().cuda_stream)
                    if st != dwt2.OK:
                        raise dwt2.Dwt2Error(st, "dwt2_transform_only")
                med, mn = _graph_stats(torch, call)
                d = "inverse" if inverse else "forward"
                res[d + "_us"] = round(med, 2)
                res[d + "_min_us"] = round(mn, 2)
                res[d + "_Gpixel_s"] = round(n * n / med / 1e3, 1)
            row[scheme] = res
        if wav != "dd137":
            row["monolithic*_vs_sweldens"] = round(row["sweldens"]["forward_us"] /
                                                   row["monolithic*"]["forward_us"], 3)
            row["monolithic*-tile_vs_sweldens"] = round(row["sweldens"]["forward_us"] /
                                                        row["monolithic*-tile"]["forward_us"], 3)
        out[wav] = row
    torch.cuda.synchronize()
    assert float(sink[0]) == 0.0  # never written
    return out


def c1_table(dwt2, torch, workloads, dev):
    """The 512^2 CDF 5/3 one-level workload (uniform 0-255 integers, seed 0),
    plain separable row-column lifting and the fused kernel: device time per
    call from a HIP graph (median and min).  2 MiB in and out stay in the
    caches, so the launch latency bounds it and the HBM fraction does not
    apply."""
    name = "cdf53_512_l1"
    spec = workloads.WORKLOADS[name]
    W, H = spec["width"], spec["height"]
    x = torch.from_numpy(workloads.workload_image(name)).to(dev)
    out = {"workload": f"{name} ({W}x{H}, cdf53, 1 level, uniform 0-255 integers, seed 0)",
           "bound": "launch latency (cache-resident)"}
    for scheme in ("rowcol", "monolithic*"):
        st, nbytes = dwt2.dwt2_workspace_bytes("cdf53", 1, W, H, dwt2.make_options(scheme=scheme))
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        y, z = torch.empty_like(x), torch.empty_like(x)
        tf, tf_min = _graph_stats(torch, lambda: dwt2.forward(x, "cdf53", 1, scheme=scheme, out=y,
                                                              workspace=ws))
        ti, ti_min = _graph_stats(torch, lambda: dwt2.inverse(y, "cdf53", 1, scheme=scheme, out=z,
                                                              workspace=ws))
        torch.cuda.synchronize()
        out[scheme] = {"forward_us": round(tf, 2), "forward_min_us": round(tf_min, 2),
                       "inverse_us": round(ti, 2), "inverse_min_us": round(ti_min, 2),
                       "forward_Gpixel_s": round(W * H / tf / 1e3, 1),
                       "inverse_Gpixel_s": round(W * H / ti / 1e3, 1),
                       "round_trip_max_abs": float((z - x).abs().max())}
    return out


def _median_us(torch, fn, reps):
    stream = torch.cuda.current_stream()
    fn(0)
    ev = []
    for i in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(i)
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    return statistics.median(a.elapsed_time(b) for a, b in ev) * 1e3


def _graph_us(torch, fn, n=20, reps=5, warm_s=0.03):
    """Median device time per call of fn (see _graph_stats)."""
    return _graph_stats(torch, fn, n, reps, warm_s)[0]


def _graph_stats(torch, fn, n=20, reps=5, warm_s=0.03):
    """Device time per call of fn, from a HIP graph of n back-to-back calls
    (host launch overhead excluded; what remains is the kernels and the gaps
    between graph nodes): (median, min) over reps replays, after untimed
    replays for at least warm_s seconds (kernels launched right after the idle
    gap of a graph capture were measured ~3 % slower)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(n):
            fn()
    stream = torch.cuda.current_stream()
    t_warm = time.perf_counter()
    while True:
        g.replay()
        torch.cuda.synchronize()
        if time.perf_counter() - t_warm >= warm_s:
            break
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3 / n)
    return statistics.median(ts), min(ts)


def pyramid_table(dwt2, torch, workloads, reps, name="cdf97_16384_l5"):
    """Per-level forward and inverse of the fused kernel on a 16384^2
    five-level workload: each level's input size timed as a one-level call on
    the LL band the previous level produced (device time per call from a HIP
    graph of back-to-back calls: median and min) in the tile order the rule
    picks and in the other one, plus the whole five-level call."""
    spec = workloads.WORKLOADS[name]
    W, H, wav, lev = spec["width"], spec["height"], spec["wavelet"], spec["levels"]
    dev = torch.device("cuda:0")
    x = torch.from_numpy(workloads.workload_image(name)).to(dev)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    levels = []
    cur = x
    w, h = W, H
    for k in range(lev):
        src = cur.contiguous()
        dst = torch.empty_like(src)
        back = torch.empty_like(src)
        tf, tf_min = _graph_stats(torch, lambda: dwt2.forward(src, wav, 1, out=dst))
        ti, ti_min = _graph_stats(torch, lambda: dwt2.inverse(dst, wav, 1, out=back))
        order = [dwt2.tile_order(wav, w, h), dwt2.tile_order(wav, w, h, inverse=True)]
        other = ["bands" if o == "runs" else "runs" for o in order]
        of = _graph_us(torch, lambda: dwt2.forward(src, wav, 1, out=dst, tile_order=other[0]))
        oi = _graph_us(torch, lambda: dwt2.inverse(dst, wav, 1, out=back, tile_order=other[1]))
        npx = w * h
        levels.append({"level": k + 1, "width": w, "height": h, "tile_order": order,
                       "forward_us": round(tf, 2), "inverse_us": round(ti, 2),
                       "forward_min_us": round(tf_min, 2), "inverse_min_us": round(ti_min, 2),
                       "other_order_us": [round(of, 2), round(oi, 2)],
                       "forward_Gpixel_s": round(npx / tf / 1e3, 1),
                       "inverse_Gpixel_s": round(npx / ti / 1e3, 1),
                       "forward_hbm_frac": round(BYTES_PER_PX * npx / tf / 1e3 / HBM_PEAK_GBS, 4),
                       "inverse_hbm_frac": round(BYTES_PER_PX * npx / ti / 1e3 / HBM_PEAK_GBS, 4)})
        w, h = (w + 1) // 2, (h + 1) // 2
        cur = dst[:h, :w]
    st, nbytes = dwt2.dwt2_workspace_bytes(wav, lev, W, H)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    # Device time per five-level call, from a HIP graph as the levels above
    # (a single eager call also counts the binding's host work before its
    # first launch, tens of microseconds).
    tf, tf_min = _graph_stats(torch, lambda: dwt2.forward(x, wav, lev, out=y, workspace=ws), n=10)
    ti, ti_min = _graph_stats(torch, lambda: dwt2.inverse(y, wav, lev, out=z, workspace=ws), n=10)
    te = _median_us(torch, lambda i: dwt2.forward(x, wav, lev, out=y, workspace=ws), reps)
    total_px = sum(l["width"] * l["height"] for l in levels)
    return {"workload": f"{name} ({W}x{H}, {wav}, {lev} levels, fused kernel)", "levels": levels,
            "five_level_forward_us": round(tf, 1), "five_level_inverse_us": round(ti, 1),
            "five_level_forward_min_us": round(tf_min, 1), "five_level_inverse_min_us": round(ti_min, 1),
            "sum_of_levels_forward_us": round(sum(l["forward_us"] for l in levels), 1),
            "sum_of_levels_inverse_us": round(sum(l["inverse_us"] for l in levels), 1),
            "five_level_forward_eager_us": round(te, 1),
            "five_level_forward_Gpixel_s": round(total_px / tf / 1e3, 1),
            "five_level_inverse_Gpixel_s": round(total_px / ti / 1e3, 1)}


def _times_us(torch, fn, reps):
    stream = torch.cuda.current_stream()
    fn()
    ev = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    return sorted(a.elapsed_time(b) * 1e3 for a, b in ev)


def batch_table(dwt2, torch, workloads, reps):
    """512 uneven images (even sizes 256..4096, 5/3 or 9/7, 3..6 levels):
    one batched call (one fused launch per level index over all images, plus
    the image-table copy kernels), the same call replayed from a HIP graph, and
    one single-image call per image (one launch per image per level)."""
    dev = torch.device("cuda:0")
    specs = workloads.batch_specs()
    xs = [torch.from_numpy(workloads.batch_image(i, w, h)).to(dev).float()
          for i, (w, h, _, _) in enumerate(specs)]
    ys = [torch.empty_like(x) for x in xs]
    zs = [torch.empty_like(x) for x in xs]
    wavs, levs = [s[2] for s in specs], [s[3] for s in specs]
    fwd = dwt2.Batch(xs, ys, wavs, levs)
    inv = dwt2.Batch(ys, zs, wavs, levs, inverse=True)
    px0 = sum(w * h for (w, h, _, _) in specs)
    px_all = 0
    for (w, h, _, lev) in specs:
        for _ in range(lev):
            px_all += w * h
            w, h = (w + 1) // 2, (h + 1) // 2
    n = len(specs)

    def row(times):
        med = statistics.median(times)
        return {"median_us": round(med, 1), "min_us": round(times[0], 1),
                "p99_us": round(times[min(len(times) - 1, int(0.99 * len(times)))], 1),
                "images_per_s": round(n / med * 1e6, 1),
                "Gpixel_s": round(px0 / med / 1e3, 1),
                "hbm_frac": round(BYTES_PER_PX * px_all / med / 1e3 / HBM_PEAK_GBS, 4)}

    out = {"workload": f"{n} images, even sides uniform in [256, 4096], cdf53/cdf97, "
                       f"3-6 levels (seed 3)",
           "level0_pixels": px0, "all_level_pixels": px_all,
           "algorithmic_bytes": int(BYTES_PER_PX * px_all)}
    out["batched_forward"] = row(_times_us(torch, fwd, reps))
    out["batched_inverse"] = row(_times_us(torch, inv, reps))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fwd()
        inv()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    gf, gi = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(gf):
        fwd()
    with torch.cuda.graph(gi):
        inv()
    out["graph_forward"] = row(_times_us(torch, gf.replay, reps))
    out["graph_inverse"] = row(_times_us(torch, gi.replay, reps))

    # one call per image through the C ABI, arguments marshalled beforehand
    stream = torch.cuda.current_stream().cuda_stream
    calls = []
    for x, y, z, wav, lev in zip(xs, ys, zs, wavs, levs):
        h, w = x.shape
        st, nb = dwt2.dwt2_workspace_bytes(wav, lev, w, h)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        calls.append((wav, lev, w, h, x, y, z, ws, nb))

    lib = dwt2.library()
    args = {inverse: [(dwt2.WAVELETS[wav], lev, w, h, (y if inverse else x).data_ptr(), w,
                       (z if inverse else y).data_ptr(), w, dwt2.EXT_WHOLE_SYMMETRIC, None,
                       ws.data_ptr(), nb, stream)
                      for (wav, lev, w, h, x, y, z, ws, nb) in calls] for inverse in (False, True)}

    def loop(inverse):
        f = lib.dwt2_inverse if inverse else lib.dwt2_forward
        status = [f(*a) for a in args[inverse]]
        if any(st != dwt2.OK for st in status):
            raise dwt2.Dwt2Error(next(st for st in status if st != dwt2.OK), "per-image call")

    out["per_image_forward"] = row(_times_us(torch, lambda: loop(False), reps))
    out["per_image_inverse"] = row(_times_us(torch, lambda: loop(True), reps))
    lmax = max(levs)
    rows_words = lmax * ((n + 3) // 4 * 4) // 4  # the tile-height table, one byte per image and level
    out["launches_per_direction"] = {
        # record, tile-start and tile-height copies, the tile-image index, the levels
        "batched": -(-16 * n // 768) - (-lmax * (n + 1) // 768) - (-rows_words // 768) + 1 + lmax,
        "per_image": sum(levs)}
    torch.cuda.synchronize()
    rt = max(float((z - x).abs().max()) for x, z in zip(xs, zs))
    out["round_trip_max_abs"] = rt
    return out


def serve_table(dwt2, torch, workloads, n_requests=11000, warm=1000, n_slots=512):
    """Serving loop under a Poisson request stream (forward or inverse, sides
    log-uniform in [64, 8192], 1-6 levels).  Requests cycle over n_slots
    distinct (input, output) buffer pairs.  First the saturated rate (all
    requests arriving at once), then 0.8 x that rate; latency is submission to
    observed completion, over the requests after the first `warm`."""
    import numpy as np
    dev = torch.device("cuda:0")
    specs = workloads.serve_specs(n_slots)
    slots = []
    for i, (inverse, w, h, wav, lev) in enumerate(specs):
        x = torch.from_numpy(workloads.batch_image(i, w, h, seed=4)).to(dev).float()
        if inverse:  # coefficients of the image as input
            x = dwt2.forward(x, wav, lev)
        slots.append((x, torch.empty_like(x), wav, lev, inverse))
    reqs = [slots[i % n_slots] for i in range(n_requests)]
    mean_px = sum(s[0].numel() for s in slots) / n_slots
    out = {"workload": f"{n_requests} requests over {n_slots} buffer slots: fwd/inv p=1/2, sides "
                       f"log-uniform [64, 8192], cdf53/cdf97, 1-6 levels (seed 4)",
           "mean_pixels_per_request": round(mean_px)}
    with dwt2.Server(4 << 30, max_batch=256, max_inflight=2) as srv:
        srv.replay(reqs[:warm], [0.0] * warm)
        # the request arrays are marshalled before the timed replays
        prep = srv.prepare(reqs, [0.0] * n_requests)
        t0 = time.perf_counter()
        done = srv.run(prep)
        sat = n_requests / (time.perf_counter() - t0)
        assert all(done[i].status == dwt2.OK for i in range(n_requests))
        rate = 0.8 * sat
        prep = srv.prepare(reqs, workloads.poisson_arrivals(n_requests, rate))
        t0 = time.perf_counter()
        done = srv.run(prep)
        elapsed = time.perf_counter() - t0
        done = [done[i] for i in range(n_requests)]
    assert all(c.status == dwt2.OK for c in done)
    single = _single_call_rate(dwt2, torch, reqs[:2000])
    lat = np.sort(np.array([c.latency_us for c in done[warm:]]))
    q = np.array([c.queue_us for c in done[warm:]])
    out.update({"saturated_images_per_s": round(sat, 1),
                "saturated_Gpixel_s": round(sat * mean_px / 1e9, 2),
                "offered_rate_per_s": round(rate, 1),
                "achieved_images_per_s": round(n_requests / elapsed, 1),
                "p50_latency_us": round(float(np.percentile(lat, 50)), 1),
                "p99_latency_us": round(float(np.percentile(lat, 99)), 1),
                "mean_queue_us": round(float(q.mean()), 1),
                "one_call_per_request_images_per_s": round(single, 1),
                "saturated_vs_one_call_per_request": round(sat / single, 2)})
    return out


def _single_call_rate(dwt2, torch, reqs):
    """Requests per second when each request is its own dwt2_forward /
    dwt2_inverse call (C ABI, arguments marshalled beforehand, one stream,
    each call with its own workspace), timed from the first call to the
    stream's completion."""
    lib = dwt2.library()
    stream = torch.cuda.current_stream()
    spaces, calls = {}, []  # one workspace per buffer slot: its calls run in stream order
    for (x, y, wav, lev, inverse) in reqs:
        h, w = x.shape
        st, nbytes = dwt2.dwt2_workspace_bytes(wav, lev, w, h)
        ws = spaces.setdefault(x.data_ptr(), torch.empty(max(nbytes, 1), dtype=torch.uint8,
                                                         device=x.device))
        f = lib.dwt2_inverse if inverse else lib.dwt2_forward
        calls.append((f, (dwt2.WAVELETS[wav], lev, w, h, x.data_ptr(), x.stride(0), y.data_ptr(),
                          y.stride(0), dwt2.EXT_WHOLE_SYMMETRIC, None, ws.data_ptr(), nbytes,
                          stream.cuda_stream)))
    for f, a in calls[:100]:  # warm
        f(*a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = [f(*a) for f, a in calls]
    torch.cuda.synchronize()
    rate = len(calls) / (time.perf_counter() - t0)
    assert all(st == dwt2.OK for st in status)
    return rate


def copy_bandwidth(torch, dev):
    n = 64 << 20  # 256 MiB of floats
    a = torch.empty(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    return round(2 * 4 * n / t / 1e9, 1)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, x, wav, lev, budget_s):
    """(Gpixel/s, reps, seconds) of forward + inverse of x: median of per-rep
    rates over about budget_s seconds after one warm-up."""
    y = oracle.forward(x, wav, lev)
    oracle.inverse(y, wav, lev)
    rates, t_all = [], time.perf_counter()
    while True:
        t0 = time.perf_counter()
        y = oracle.forward(x, wav, lev)
        oracle.inverse(y, wav, lev)
        rates.append(2 * x.size / (time.perf_counter() - t0) / 1e9)
        if time.perf_counter() - t_all >= budget_s and len(rates) >= 3:
            break
    return statistics.median(rates), len(rates), time.perf_counter() - t_all


def cpu_baseline(img, wav, lev, budget_s):
    """The FP64 C oracle on the host: all cores (OpenMP) on the full image,
    and one thread on a 2048 x 2048 crop of it (the rate per pixel does not
    depend on the size at these sizes; the crop keeps the run short)."""
    import numpy as np

    import oracle

    x = img.astype(np.float64)
    threads = oracle.num_threads()
    affinity = len(os.sched_getaffinity(0))
    rate, reps, t = _oracle_rate(oracle, x, wav, lev, 0.7 * budget_s)
    crop = np.ascontiguousarray(x[:2048, :2048])
    oracle.set_num_threads(1)
    try:
        rate1, reps1, t1 = _oracle_rate(oracle, crop, wav, lev, 0.3 * budget_s)
    finally:
        oracle.set_num_threads(threads)
    return {"value": round(rate, 4), "unit": "Gpixel/s", "cores": threads,
            "kind": "oracle",
            "sample": f"full {x.shape[1]}x{x.shape[0]} image, forward+inverse, median of {reps} reps "
                      f"after 1 warm-up ({t:.1f} s), FP64 C with OpenMP on {threads} threads",
            "single_thread": {"value": round(rate1, 5), "unit": "Gpixel/s", "cores": 1,
                              "sample": f"2048x2048 crop, forward+inverse, median of {reps1} reps "
                                        f"after 1 warm-up ({t1:.1f} s)"},
            "cpu_model": _cpu_model(), "affinity_cpus": affinity}


if __name__ == "__main__":
    main()
