"""Brute-force 2-D DWT by convolution with the analysis filters (test-only).

This is the paper's Convolution scheme (Sec. 2): four 2-D FIR filters with the
subsampling built in, evaluated directly on the whole-sample symmetric
extension of the image.  The filter taps are derived here independently of any
lifting factorisation:

* CDF 5/3 (Le Gall): low-pass (-1/8, 1/4, 3/4, 1/4, -1/8) centred on x[2n],
  high-pass (-1/2, 1, -1/2) centred on x[2n+1]; DC gain 1 (unit-DC scale).
* CDF 9/7 (4 vanishing moments each): with y = sin^2(w/2) and
  1 + 4y + 10y^2 + 20y^3 = (1 - y/y_r) q(y), the analysis low-pass is
  sqrt(2) cos^4(w/2) q(y) (9 taps) and the analysis high-pass is the 7-tap
  synthesis low-pass sqrt(2) cos^4(w/2) (1 - y/y_r) modulated by (-1)^k,
  centred on x[2n+1].  These are in the paper's scale (DC gain sqrt(2)).

* DD 13/7 ((4,4) Deslauriers-Dubuc): the 7-tap high-pass is x[2n+1] minus the
  cubic Lagrange interpolation of x[2n-2], x[2n], x[2n+2], x[2n+4] at 2n+1,
  with the weights computed here from the Lagrange formula; the 13-tap
  low-pass adds to x[2n] the paper's update U(z) = 9/32 (1 + z) -
  1/32 (z^-1 + z^2) (Sec. 5) of that high-pass, i.e. 9/32 (H[n-1] + H[n]) -
  1/32 (H[n-2] + H[n+1]).  DC gain 1 (unit-DC scale).

The paper's normalisation scales L by zeta and H by 1/zeta per axis, which
for every wavelet here gives a low-pass DC gain of sqrt(2); the unit-DC scale
divides the low-pass by sqrt(2) and multiplies the high-pass by sqrt(2).
"""
from __future__ import annotations

import numpy as np

SQRT2 = np.sqrt(2.0)


def _lconv(a: dict, b: dict) -> dict:
    out = {}
    for i, x in a.items():
        for j, y in b.items():
            out[i + j] = out.get(i + j, 0.0) + x * y
    return out


def _ladd(a: dict, b: dict) -> dict:
    out = dict(a)
    for j, y in b.items():
        out[j] = out.get(j, 0.0) + y
    return out


def _lscale(a: dict, s: float) -> dict:
    return {k: v * s for k, v in a.items()}


def daubechies_real_root() -> float:
    roots = np.roots([20.0, 10.0, 4.0, 1.0])  # 20y^3 + 10y^2 + 4y + 1
    real = [r.real for r in roots if abs(r.imag) < 1e-12]
    assert len(real) == 1
    y = real[0]
    # one Newton step in FP64 to polish
    f = 1 + 4 * y + 10 * y * y + 20 * y ** 3
    df = 4 + 20 * y + 60 * y * y
    return y - f / df


def cdf97_taps_paper_scale():
    """(low, high) as {offset: tap}; low centred on x[2n], high on x[2n+1]."""
    yr = daubechies_real_root()
    cos2 = {-1: 0.25, 0: 0.5, 1: 0.25}
    ypol = {-1: -0.25, 0: 0.5, 1: -0.25}
    one = {0: 1.0}
    cos4 = _lconv(cos2, cos2)
    lin = _ladd(one, _lscale(ypol, -1.0 / yr))
    # q(y) = (1 + 4y + 10y^2 + 20y^3) / (1 - y/y_r) = q0 + q1 y + q2 y^2
    q0 = 1.0
    q1 = 4.0 + q0 / yr
    q2 = 10.0 + q1 / yr
    q = _ladd(_ladd(_lscale(one, q0), _lscale(ypol, q1)), _lscale(_lconv(ypol, ypol), q2))
    low = _lscale(_lconv(cos4, q), SQRT2)
    syn = _lscale(_lconv(cos4, lin), SQRT2)
    high = {k: ((-1) ** abs(k)) * v for k, v in syn.items()}
    return low, high


def cdf53_taps_unit_dc():
    low = {-2: -1 / 8, -1: 1 / 4, 0: 3 / 4, 1: 1 / 4, 2: -1 / 8}
    high = {-1: -1 / 2, 0: 1.0, 1: -1 / 2}
    return low, high


def lagrange_weights(nodes, t):
    """Weights of the Lagrange interpolation through `nodes`, evaluated at t."""
    out = []
    for i, a in enumerate(nodes):
        w = 1.0
        for j, b in enumerate(nodes):
            if j != i:
                w *= (t - b) / (a - b)
        out.append(w)
    return out


def dd137_taps_unit_dc():
    nodes = [-3, -1, 1, 3]  # even neighbours, relative to the odd sample
    high = {0: 1.0}
    for t, w in zip(nodes, lagrange_weights(nodes, 0.0)):
        high[t] = -w
    low = {0: 1.0}
    for m, cu in ((-1, 9 / 32), (0, 9 / 32), (-2, -1 / 32), (1, -1 / 32)):
        centre = 2 * m + 1  # H[n+m] sits at x[2(n+m)+1]
        for k, v in high.items():
            low[centre + k] = low.get(centre + k, 0.0) + cu * v
    return low, high


def analysis_taps(wavelet: str, norm: str):
    if wavelet in ("cdf53", "dd137"):
        low, high = cdf53_taps_unit_dc() if wavelet == "cdf53" else dd137_taps_unit_dc()
        if norm == "paper":
            low, high = _lscale(low, SQRT2), _lscale(high, 1 / SQRT2)
    elif wavelet == "cdf97":
        low, high = cdf97_taps_paper_scale()
        if norm == "unit_dc":
            low, high = _lscale(low, 1 / SQRT2), _lscale(high, SQRT2)
    else:
        raise KeyError(wavelet)
    return ({k: v for k, v in low.items() if v != 0.0},
            {k: v for k, v in high.items() if v != 0.0})


def mirror(j, n):
    """Whole-sample symmetric extension index, period 2(n-1)."""
    p = 2 * (n - 1)
    j = np.mod(j, p)
    return np.where(j >= n, p - j, j)


def level_bruteforce(x: np.ndarray, low: dict, high: dict):
    """(LL, HL, LH, HH) of one level: direct 2-D sums over the extended image."""
    h, w = x.shape
    hl, wl = (h + 1) // 2, (w + 1) // 2
    hh, wh = h // 2, w // 2
    rl = 2 * np.arange(hl)          # rows of low-pass outputs
    rh = 2 * np.arange(hh) + 1      # rows of high-pass outputs
    cl = 2 * np.arange(wl)
    ch = 2 * np.arange(wh) + 1

    def band(rows, vfilt, cols, hfilt):
        out = np.zeros((len(rows), len(cols)))
        for i, fv in vfilt.items():
            ri = mirror(rows + i, h)
            for j, fh in hfilt.items():
                cj = mirror(cols + j, w)
                out += fv * fh * x[np.ix_(ri, cj)]
        return out

    LL = band(rl, low, cl, low)
    HL = band(rl, low, ch, high)     # horizontal high, vertical low
    LH = band(rh, high, cl, low)     # horizontal low, vertical high
    HH = band(rh, high, ch, high)
    return LL, HL, LH, HH


def forward_bruteforce(x, wavelet="cdf53", levels=1, norm="unit_dc"):
    low, high = analysis_taps(wavelet, norm)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    cur = x
    for _ in range(levels):
        h, w = cur.shape
        hl, wl = (h + 1) // 2, (w + 1) // 2
        LL, HL, LH, HH = level_bruteforce(cur, low, high)
        out[:hl, wl:w] = HL
        out[hl:h, :wl] = LH
        out[hl:h, wl:w] = HH
        out[:hl, :wl] = LL
        cur = LL
    return out


def forward_1d_bruteforce(x, wavelet="cdf53", norm="unit_dc"):
    low, high = analysis_taps(wavelet, norm)
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    nl, nh = (n + 1) // 2, n // 2
    L = np.zeros(nl)
    H = np.zeros(nh)
    for k, t in low.items():
        L += t * x[mirror(2 * np.arange(nl) + k, n)]
    for k, t in high.items():
        H += t * x[mirror(2 * np.arange(nh) + 1 + k, n)]
    return np.concatenate([L, H])
