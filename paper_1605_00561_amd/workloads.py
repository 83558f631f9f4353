"""Seeded synthetic inputs for the DWT workloads.

This module holds no wavelet arithmetic: it only draws pixels.  Both the GPU
path's tests/benchmarks and the oracle checks take their inputs from here.

Workloads (all pixels are FP32 values in [0, 255]; the paper's images are
unspecified, so these synthetic images stand in for them):

* ``uniform_u8``      integers uniform in [0, 255] cast to float.
* ``cosine_noise``    127.5 + 63.75 (cos(2 pi x / 512) + cos(2 pi y / 512))
                      + N(0, 8^2), clipped to [0, 255]  (smooth gradient + noise).
* ``rect_noise``      uniform integer noise, then 512 axis-aligned rectangles of
                      constant integer value painted in order; each rectangle's
                      top-left corner is uniform in the image and its sides are
                      uniform in [8, 2048], clipped to the image.
* ``batch_specs``     512 (w, h, wavelet, levels) tuples, w and h uniform over
                      the even integers in [256, 4096], wavelet 5/3 or 9/7 with
                      probability 1/2, levels uniform in {3, 4, 5, 6}.
* ``batch_image``     the pixels of image i of a batch: integers uniform in
                      [0, 255], drawn from the seed sequence (seed, i).
* ``serve_specs``     a request stream: direction forward or inverse with
                      probability 1/2, width and height independent and
                      log-uniform in [64, 8192] (rounded, odd sizes allowed),
                      wavelet 5/3 or 9/7 with probability 1/2, levels uniform
                      in 1..6; ``poisson_arrivals`` gives exponential gaps.
"""
from __future__ import annotations

import numpy as np

# Named workloads: (generator, width, height, seed, wavelet, levels).
WORKLOADS = {
    "cdf53_512_l1": dict(kind="uniform_u8", width=512, height=512, seed=0,
                         wavelet="cdf53", levels=1),
    "cdf97_8192_l1": dict(kind="cosine_noise", width=8192, height=8192, seed=1,
                          wavelet="cdf97", levels=1),
    "cdf53_16384_l5": dict(kind="rect_noise", width=16384, height=16384, seed=2,
                           wavelet="cdf53", levels=5),
    "cdf97_16384_l5": dict(kind="rect_noise", width=16384, height=16384, seed=2,
                           wavelet="cdf97", levels=5),
}


def uniform_u8(width: int, height: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=(height, width), dtype=np.int32).astype(np.float32)


def cosine_noise(width: int, height: int, seed: int, period: float = 512.0,
                 sigma: float = 8.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = np.arange(width, dtype=np.float64)
    y = np.arange(height, dtype=np.float64)
    cx = np.cos(2.0 * np.pi * x / period)
    cy = np.cos(2.0 * np.pi * y / period)
    img = np.empty((height, width), dtype=np.float32)
    # Row blocks keep the FP64 temporaries small for large images.
    step = max(1, (1 << 22) // max(1, width))
    for r0 in range(0, height, step):
        r1 = min(height, r0 + step)
        block = 127.5 + 63.75 * (cx[None, :] + cy[r0:r1, None])
        block += rng.normal(0.0, sigma, size=block.shape)
        img[r0:r1] = np.clip(block, 0.0, 255.0)
    return img


def rect_noise(width: int, height: int, seed: int, n_rect: int = 512,
               side_min: int = 8, side_max: int = 2048) -> np.ndarray:
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(height, width), dtype=np.int32).astype(np.float32)
    for _ in range(n_rect):
        x0 = int(rng.integers(0, width))
        y0 = int(rng.integers(0, height))
        w = int(rng.integers(side_min, side_max + 1))
        h = int(rng.integers(side_min, side_max + 1))
        v = float(rng.integers(0, 256))
        img[y0:min(height, y0 + h), x0:min(width, x0 + w)] = v
    return img


GENERATORS = {"uniform_u8": uniform_u8, "cosine_noise": cosine_noise, "rect_noise": rect_noise}


def make_image(kind: str, width: int, height: int, seed: int) -> np.ndarray:
    """(height, width) float32 image of the named kind."""
    return GENERATORS[kind](width, height, seed)


def workload_image(name: str) -> np.ndarray:
    spec = WORKLOADS[name]
    return make_image(spec["kind"], spec["width"], spec["height"], spec["seed"])


def batch_specs(n: int = 512, seed: int = 3):
    """[(width, height, wavelet, levels)] of a batch of uneven images."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        w = 2 * int(rng.integers(128, 2049))
        h = 2 * int(rng.integers(128, 2049))
        wav = "cdf53" if rng.random() < 0.5 else "cdf97"
        lev = int(rng.integers(3, 7))
        out.append((w, h, wav, lev))
    return out


def batch_image(i: int, width: int, height: int, seed: int = 3) -> np.ndarray:
    """Pixels of image i of a batch (uint8 values, returned as uint8 to keep
    host memory small; cast to FP32 on the device)."""
    rng = np.random.default_rng([seed, i])
    return rng.integers(0, 256, size=(height, width), dtype=np.uint8)


def serve_specs(n: int, seed: int = 4):
    """[(inverse, width, height, wavelet, levels)] of a request stream."""
    rng = np.random.default_rng(seed)
    out = []
    lo, hi = np.log(64.0), np.log(8192.0)
    for _ in range(n):
        inverse = bool(rng.random() < 0.5)
        w = int(round(float(np.exp(rng.uniform(lo, hi)))))
        h = int(round(float(np.exp(rng.uniform(lo, hi)))))
        wav = "cdf53" if rng.random() < 0.5 else "cdf97"
        lev = int(rng.integers(1, 7))
        out.append((inverse, w, h, wav, lev))
    return out


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 5) -> np.ndarray:
    """Arrival times in microseconds of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1e6 / rate_per_s, size=n)
    return np.cumsum(gaps) - gaps[0]
