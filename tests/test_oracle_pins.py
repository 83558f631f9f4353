"""Pins of the FP64 oracle against things other than itself (CPU only).

* brute-force 2-D convolution with analysis taps derived independently of any
  lifting factorisation (bruteforce.py), on every size 2..12 x 2..12 and on
  random sizes, one to three levels;
* the CDF 9/7 lifting constants re-derived from the Daubechies polynomial;
* the CDF 5/3 and DD 13/7 operators printed in Sec. 5;
* DD 13/7: the high-pass annihilates cubics, the low-pass has no second
  moment (the property its update was built for);
* perfect reconstruction, linearity, constant / ramp / cubic images;
* the exact power-of-two relation between the two normalisations;
* error statuses.
"""
import itertools

import numpy as np
import pytest

import bruteforce as bf
import oracle

WAVS = ["cdf53", "cdf97", "dd137"]
NORMS = ["unit_dc", "paper"]


def max_levels(w, h, cap=3):
    n = 0
    while n < cap and w >= 2 and h >= 2:
        n += 1
        w, h = (w + 1) // 2, (h + 1) // 2
    return n


SMALL = list(itertools.product(range(2, 13), range(2, 13)))


@pytest.mark.parametrize("wav", WAVS)
@pytest.mark.parametrize("norm", NORMS)
def test_bruteforce_convolution_small_sizes(wav, norm):
    rng = np.random.default_rng(11)
    for w, h in SMALL:
        x = rng.integers(0, 256, size=(h, w)).astype(np.float64)
        for lev in range(1, max_levels(w, h) + 1):
            got = oracle.forward(x, wav, lev, norm)
            ref = bf.forward_bruteforce(x, wav, lev, norm)
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10,
                                       err_msg=f"{wav} {norm} {w}x{h} L{lev}")


@pytest.mark.parametrize("wav", WAVS)
def test_bruteforce_convolution_random_sizes(wav):
    rng = np.random.default_rng(12)
    for _ in range(12):
        w, h = (int(v) for v in rng.integers(13, 90, size=2))
        x = rng.normal(100, 60, size=(h, w))
        lev = int(rng.integers(1, max_levels(w, h) + 1))
        norm = NORMS[int(rng.integers(0, 2))]
        got = oracle.forward(x, wav, lev, norm)
        ref = bf.forward_bruteforce(x, wav, lev, norm)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9,
                                   err_msg=f"{wav} {norm} {w}x{h} L{lev}")


@pytest.mark.parametrize("wav", WAVS)
@pytest.mark.parametrize("norm", NORMS)
def test_bruteforce_1d(wav, norm):
    rng = np.random.default_rng(13)
    for n in list(range(2, 40)) + [97, 128, 255]:
        x = rng.normal(0, 50, size=n)
        np.testing.assert_allclose(oracle.forward_1d(x, wav, norm),
                                   bf.forward_1d_bruteforce(x, wav, norm), rtol=0, atol=1e-11)


def test_cdf53_operators_as_printed():
    # Sec. 5: P(z) = -1/2 (1 + z^-1), U(z) = 1/4 (1 + z), zeta = sqrt(2).
    pairs, zeta = oracle.lifting_constants("cdf53")
    assert pairs == [(-0.5, 0.25)]
    assert zeta == np.sqrt(2.0)


def test_cdf97_constants_rederived():
    """Derive alpha..delta and zeta from the polynomial taps (bruteforce.py) in
    closed form and compare with the oracle's values.

    With L = x[2n] and H = x[2n+1], the unscaled high-pass after
    predict(alpha), update(beta), predict(gamma) has taps, from the centre out,
    1 + 2 beta gamma, alpha + gamma (1 + 3 alpha beta), beta gamma,
    alpha beta gamma; the outermost low-pass tap is alpha beta gamma delta.
    The paper-scale high-pass is that times 1/zeta, the low-pass times zeta."""
    low, high = bf.cdf97_taps_paper_scale()
    g0, g1, g2, g3 = high[0], high[1], high[2], high[3]
    alpha = g3 / g2
    s = g0 - 2 * g2                 # = 1/zeta
    bg = g2 / s
    gamma = g1 / s - alpha - 3 * alpha * bg
    beta = bg / gamma
    zeta = 1 / s
    delta = low[4] / (zeta * alpha * beta * gamma)
    pairs, z_or = oracle.lifting_constants("cdf97")
    np.testing.assert_allclose([pairs[0][0], pairs[0][1], pairs[1][0], pairs[1][1], z_or],
                               [alpha, beta, gamma, delta, zeta], rtol=1e-13)
    # Both normalisations give the low-pass a DC gain of sqrt(2) per axis at
    # the paper's scale, i.e. zeta * K = sqrt(2) with K the unscaled DC gain.
    s_lo, s_hi = oracle.scales("cdf97", "unit_dc")
    assert s_lo * s_hi == pytest.approx(1.0, rel=1e-15)
    assert zeta / s_lo == pytest.approx(np.sqrt(2.0), rel=1e-14)


def test_taps_are_biorthogonal_pair():
    """Independent check of the 9/7 taps themselves: low-pass sums to sqrt(2),
    high-pass has four vanishing moments."""
    low, high = bf.cdf97_taps_paper_scale()
    assert sum(low.values()) == pytest.approx(np.sqrt(2.0), rel=1e-14)
    for p in range(4):
        assert abs(sum(v * k ** p for k, v in high.items())) < 1e-12


@pytest.mark.parametrize("wav", WAVS)
@pytest.mark.parametrize("norm", NORMS)
def test_perfect_reconstruction(wav, norm):
    rng = np.random.default_rng(14)
    for w, h in [(2, 2), (2, 7), (3, 3), (5, 4), (37, 22), (64, 64), (129, 66), (255, 31)]:
        x = rng.integers(0, 256, size=(h, w)).astype(np.float64)
        for lev in range(1, max_levels(w, h, cap=6) + 1):
            y = oracle.forward(x, wav, lev, norm)
            np.testing.assert_allclose(oracle.inverse(y, wav, lev, norm), x, rtol=0, atol=1e-10)


@pytest.mark.parametrize("wav", WAVS)
def test_linearity(wav):
    rng = np.random.default_rng(15)
    a, b = rng.normal(size=(23, 31)), rng.normal(size=(23, 31))
    lhs = oracle.forward(2.5 * a - 0.75 * b, wav, 3)
    rhs = 2.5 * oracle.forward(a, wav, 3) - 0.75 * oracle.forward(b, wav, 3)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12)


@pytest.mark.parametrize("wav", WAVS)
@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("shape", [(2, 2), (7, 5), (32, 48), (33, 17)])
def test_constant_image(wav, norm, shape):
    h, w = shape
    c = 93.0
    lev = max_levels(w, h, cap=4)
    y = oracle.forward(np.full((h, w), c), wav, lev, norm)
    wl, hl = w, h
    for _ in range(lev):
        wl, hl = (wl + 1) // 2, (hl + 1) // 2
    gain = 1.0 if norm == "unit_dc" else 2.0 ** lev
    ll = y[:hl, :wl]
    np.testing.assert_allclose(ll, c * gain, rtol=1e-14)
    det = y.copy()
    det[:hl, :wl] = 0
    tol = 0.0 if wav == "cdf53" else 1e-11 * c
    assert np.abs(det).max() <= tol


@pytest.mark.parametrize("w", [8, 9, 16, 17])
@pytest.mark.parametrize("h", [6, 7, 12])
def test_linear_ramp_cdf53(w, h):
    """5/3 kills linear functions except where the mirror breaks linearity at the
    far edge: the last HL column iff W is even, the last LH row iff H is even."""
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    x = 3.0 + 1.5 * xx - 2.25 * yy
    out = oracle.forward(x, "cdf53", 1)
    hl, wl = (h + 1) // 2, (w + 1) // 2
    HL, LH, HH = out[:hl, wl:], out[hl:, :wl], out[hl:, wl:]
    assert np.all(HH == 0)
    assert np.all(HL[:, :-1] == 0)
    assert np.all(LH[:-1, :] == 0)
    assert np.all(HL[:, -1] != 0) == (w % 2 == 0) and np.all(HL[:, -1] == 0) == (w % 2 == 1)
    assert np.all(LH[-1, :] != 0) == (h % 2 == 0) and np.all(LH[-1, :] == 0) == (h % 2 == 1)


@pytest.mark.parametrize("n", [21, 24, 33])
def test_cubic_cdf97(n):
    """9/7 high-pass has four vanishing moments: H[k] = 0 wherever the 7-tap
    support [2k-2, 2k+4] lies inside the signal (1 <= k <= (n-5)/2)."""
    t = np.arange(n, dtype=np.float64)
    x = 0.5 - 0.3 * t + 0.02 * t ** 2 - 0.001 * t ** 3
    y = oracle.forward_1d(x, "cdf97")
    H = y[(n + 1) // 2:]
    kmax = (n - 5) // 2
    assert np.abs(H[1:kmax + 1]).max() < 1e-12
    assert abs(H[0]) > 1e-6 and abs(H[-1]) > 1e-6
    # 2-D: f = cubic(x) + cubic(y): HL zero on interior columns, LH on interior rows.
    img = x[None, :n] + x[:n, None]
    out = oracle.forward(img, "cdf97", 1)
    hl = wl = (n + 1) // 2
    HL, LH, HH = out[:hl, wl:], out[hl:, :wl], out[hl:, wl:]
    assert np.abs(HL[:, 1:kmax + 1]).max() < 1e-11
    assert np.abs(LH[1:kmax + 1, :]).max() < 1e-11
    assert np.abs(HH[1:kmax + 1, 1:kmax + 1]).max() < 1e-11


def test_dd137_operators_as_printed():
    """Sec. 5: P(z) = 1/16 (z + z^-2) - 9/16 (1 + z^-1), U(z) = 9/32 (1 + z) -
    1/32 (z^-1 + z^2): in the L = x[2n] phase the predict adds -9/16 of L[n],
    L[n+1] and 1/16 of L[n-1], L[n+2]; the update 9/32 of H[n-1], H[n] and
    -1/32 of H[n-2], H[n+1].  Read back from 1-D impulse responses."""
    n = 64
    # H[k] response to a unit even sample x[2m] = L[m]: predict taps
    x = np.zeros(n)
    x[30] = 1.0  # L[15]
    H = oracle.forward_1d(x, "dd137")[n // 2:]
    np.testing.assert_allclose(H[12:18], [0, 1 / 16, -9 / 16, -9 / 16, 1 / 16, 0], rtol=0, atol=1e-15)
    # L[k] response to a unit odd sample x[2m+1] = H[m] (which the predict
    # leaves unchanged): update taps
    x = np.zeros(n)
    x[31] = 1.0  # H[15]
    L = oracle.forward_1d(x, "dd137")[:n // 2]
    np.testing.assert_allclose(L[12:20], [0, 0, -1 / 32, 9 / 32, 9 / 32, -1 / 32, 0, 0], rtol=0,
                               atol=1e-15)


@pytest.mark.parametrize("n", [24, 33, 40])
def test_dd137_highpass_annihilates_cubics(n):
    """Deslauriers-Dubuc 4-point interpolation is exact for cubics, so H[k] = 0
    wherever the 7-tap support [2k-2, 2k+4] lies inside the signal."""
    t = np.arange(n, dtype=np.float64)
    x = 2.0 + 0.7 * t - 0.05 * t ** 2 + 0.003 * t ** 3
    H = oracle.forward_1d(x, "dd137")[(n + 1) // 2:]
    kmax = (n - 5) // 2
    assert np.abs(H[1:kmax + 1]).max() < 1e-10
    assert abs(H[0]) > 1e-6


def test_dd137_lowpass_moments():
    """The low-pass impulse response (13 taps) sums to 1 and has zero first,
    second and third moments about its centre."""
    n = 64
    ell = {}
    for k in range(-8, 9):
        x = np.zeros(n)
        x[32 + k] = 1.0
        ell[k] = oracle.forward_1d(x, "dd137")[16]  # L[16] sits at x[32]
    support = [k for k, v in ell.items() if abs(v) > 1e-15]
    assert min(support) == -6 and max(support) == 6
    assert sum(ell.values()) == pytest.approx(1.0, abs=1e-15)
    for m in (1, 2, 3):
        assert abs(sum(v * k ** m for k, v in ell.items())) < 1e-13
    assert abs(sum(v * k ** 4 for k, v in ell.items())) > 1.0


@pytest.mark.parametrize("wav", WAVS)
def test_normalisation_relation(wav):
    """PAPER = UNIT_DC x 2^(k-1) x {2 for LL, 1 for HL/LH, 1/2 for HH} at level k."""
    rng = np.random.default_rng(16)
    w, h, lev = 45, 38, 4
    x = rng.integers(0, 256, size=(h, w)).astype(np.float64)
    u = oracle.forward(x, wav, lev, "unit_dc")
    p = oracle.forward(x, wav, lev, "paper")
    ratio = np.ones_like(u)
    wk, hk = w, h
    for k in range(1, lev + 1):
        wl, hl = (wk + 1) // 2, (hk + 1) // 2
        f = 2.0 ** (k - 1)
        ratio[:hl, wl:wk] = f
        ratio[hl:hk, :wl] = f
        ratio[hl:hk, wl:wk] = f / 2
        ratio[:hl, :wl] = 2 * f
        wk, hk = wl, hl
    np.testing.assert_allclose(p, u * ratio, rtol=1e-14, atol=1e-12)


def test_transpose_symmetry():
    """Transposing the image swaps HL and LH (the separable transform is
    symmetric in the two axes)."""
    rng = np.random.default_rng(17)
    x = rng.normal(size=(20, 14))
    a = oracle.forward(x, "cdf97", 1)
    b = oracle.forward(x.T, "cdf97", 1)
    np.testing.assert_allclose(a.T, b, atol=1e-12)


def test_integer_input_5_3_is_dyadic():
    """With integer input, one 5/3 level yields multiples of 1/64 (each 1-D pass
    has denominators up to 8: predict -1/2, update 1/4 of halves) of small
    magnitude, which is what makes an FP32 result bit-exact."""
    rng = np.random.default_rng(18)
    x = rng.integers(0, 256, size=(30, 26)).astype(np.float64)
    y = oracle.forward(x, "cdf53", 1)
    assert np.all(y * 64 == np.round(y * 64))
    assert np.abs(y).max() < 2 ** 11


def test_error_statuses():
    x = np.zeros((4, 4))
    with pytest.raises(oracle.OracleError) as e:
        oracle.forward(np.zeros((1, 5)), "cdf53", 1)
    assert e.value.status == oracle.E_SIZE
    with pytest.raises(oracle.OracleError) as e:
        oracle.forward(x, "cdf53", 3)          # 4 -> 2 -> 1: third level too small
    assert e.value.status == oracle.E_SIZE
    with pytest.raises(oracle.OracleError) as e:
        oracle.forward(x, "cdf53", 0)
    assert e.value.status == oracle.E_ARG
    st = oracle.lib().oracle_dwt2_forward(7, 0, 1, 4, 4, oracle._dp(x), oracle._dp(x.copy()))
    assert st == oracle.E_UNSUPPORTED
    st = oracle.lib().oracle_dwt2_forward(0, 5, 1, 4, 4, oracle._dp(x), oracle._dp(x.copy()))
    assert st == oracle.E_UNSUPPORTED
