"""FP64 CPU oracle for the 2-D lifting DWT (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (``libdwt2.so`` and
``paper_1605_00561_amd``) never imports it, and the two share no code.

The arithmetic lives in ``dwt2_oracle.c`` (plain C, FP64, OpenMP): separable
1-D lifting with whole-sample symmetric extension applied to rows then columns,
per level, which the paper states every one of its 2-D schemes reproduces
exactly (Conclusions; Sec. 3, the check S_U T_P = N_{P,U}).  This module only
marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dwt2_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_dwt2.so")

CDF53, CDF97, DD137 = 0, 1, 2
NORM_UNIT_DC, NORM_PAPER = 0, 1
WAVELETS = {"cdf53": CDF53, "cdf97": CDF97, "dd137": DD137, CDF53: CDF53, CDF97: CDF97,
            DD137: DD137}
NORMS = {"unit_dc": NORM_UNIT_DC, "paper": NORM_PAPER,
         NORM_UNIT_DC: NORM_UNIT_DC, NORM_PAPER: NORM_PAPER}

# Status codes of the C functions.
OK, E_ARG, E_SIZE, E_UNSUPPORTED, E_NOMEM = 0, -1, -2, -3, -7


def compile_library(force: bool = False) -> str:
    """Compile dwt2_oracle.c into liboracle_dwt2.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = compile_library()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        L.oracle_dwt2_forward.argtypes = [i, i, i, i, i, dp, dp]
        L.oracle_dwt2_inverse.argtypes = [i, i, i, i, i, dp, dp]
        L.oracle_dwt1_forward.argtypes = [i, i, i, dp, dp]
        L.oracle_dwt1_inverse.argtypes = [i, i, i, dp, dp]
        L.oracle_lifting_constants.argtypes = [i, ctypes.POINTER(i), dp, dp]
        L.oracle_scales.argtypes = [i, i, dp, dp]
        L.oracle_num_threads.argtypes = []
        L.oracle_set_num_threads.argtypes = [i]
        for f in (L.oracle_dwt2_forward, L.oracle_dwt2_inverse, L.oracle_dwt1_forward,
                  L.oracle_dwt1_inverse, L.oracle_lifting_constants, L.oracle_scales,
                  L.oracle_num_threads, L.oracle_set_num_threads):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(st: int, what: str):
    if st != OK:
        raise OracleError(st, what)


def forward(img, wavelet="cdf53", levels=1, norm="unit_dc") -> np.ndarray:
    """Multi-level 2-D forward DWT of a (H, W) array; returns the FP64 Mallat layout."""
    src = np.ascontiguousarray(img, dtype=np.float64)
    if src.ndim != 2:
        raise ValueError("expected a 2-D array")
    h, w = src.shape
    dst = np.empty_like(src)
    _check(lib().oracle_dwt2_forward(WAVELETS[wavelet], NORMS[norm], levels, w, h,
                                     _dp(src), _dp(dst)), "oracle_dwt2_forward")
    return dst


def inverse(coef, wavelet="cdf53", levels=1, norm="unit_dc") -> np.ndarray:
    """Multi-level 2-D inverse DWT of a (H, W) Mallat-layout array; returns FP64 pixels."""
    src = np.ascontiguousarray(coef, dtype=np.float64)
    if src.ndim != 2:
        raise ValueError("expected a 2-D array")
    h, w = src.shape
    dst = np.empty_like(src)
    _check(lib().oracle_dwt2_inverse(WAVELETS[wavelet], NORMS[norm], levels, w, h,
                                     _dp(src), _dp(dst)), "oracle_dwt2_inverse")
    return dst


def forward_1d(x, wavelet="cdf53", norm="unit_dc") -> np.ndarray:
    """1-D forward DWT of a vector; returns [L | H]."""
    src = np.ascontiguousarray(x, dtype=np.float64)
    dst = np.empty_like(src)
    _check(lib().oracle_dwt1_forward(WAVELETS[wavelet], NORMS[norm], src.size,
                                     _dp(src), _dp(dst)), "oracle_dwt1_forward")
    return dst


def inverse_1d(y, wavelet="cdf53", norm="unit_dc") -> np.ndarray:
    src = np.ascontiguousarray(y, dtype=np.float64)
    dst = np.empty_like(src)
    _check(lib().oracle_dwt1_inverse(WAVELETS[wavelet], NORMS[norm], src.size,
                                     _dp(src), _dp(dst)), "oracle_dwt1_inverse")
    return dst


def lifting_constants(wavelet="cdf97"):
    """(list of (predict, update) pairs, zeta) as the oracle holds them."""
    n = ctypes.c_int()
    coef = np.zeros(4)
    zeta = np.zeros(1)
    _check(lib().oracle_lifting_constants(WAVELETS[wavelet], ctypes.byref(n), _dp(coef),
                                          _dp(zeta)), "oracle_lifting_constants")
    return [(coef[2 * k], coef[2 * k + 1]) for k in range(n.value)], float(zeta[0])


def scales(wavelet="cdf53", norm="unit_dc"):
    """(s_lo, s_hi): per-1-D-pass scale factors of L and H."""
    lo = np.zeros(1)
    hi = np.zeros(1)
    _check(lib().oracle_scales(WAVELETS[wavelet], NORMS[norm], _dp(lo), _dp(hi)),
           "oracle_scales")
    return float(lo[0]), float(hi[0])


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> int:
    return int(lib().oracle_set_num_threads(int(n)))


def level_shapes(width: int, height: int, levels: int):
    """[(w_k, h_k)] of the block each level transforms."""
    out = []
    w, h = width, height
    for _ in range(levels):
        out.append((w, h))
        w, h = (w + 1) // 2, (h + 1) // 2
    return out
