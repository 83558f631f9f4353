"""The barrier counts of the built kernels equal the paper's Table 1 (CPU only).

Each kernel source is compiled to gfx950 assembly with the library's own
flags, and the `s_barrier` instructions of every kernel are counted.  A tile
kernel runs one lifting scheme on one tile, so its static count is the number
of memory barriers Table 1 lists for that scheme and wavelet (transcribed in
tests/golden/).  The fused Monolithic* kernels inline the tile body twice (the
vector path for interior tiles and the scalar path for edge tiles), so their
count is twice Table 1's.  The row-column kernels share nothing across
threads and have none.
"""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

from paper_1605_00561_amd import build, dwt2
from scheme_model import read_table1

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE1 = read_table1(os.path.join(ROOT, "tests", "golden", "table1_barriers_operations.txt"))
WAVELET_IDS = {0: "cdf53", 1: "cdf97", 2: "dd137"}
SCHEME_IDS = {2: "sweldens", 3: "iwahashi", 5: "monolithic*", 6: "monolithic", 7: "explosive",
              8: "explosive*", 9: "iwahashi*", 10: "polyphase*"}


def _barriers(source, tmpdir):
    out = os.path.join(tmpdir, source + ".s")
    cmd = [build.HIPCC, *build.CFLAGS, "--cuda-device-only", "-S",
           os.path.join(build.CSRC, source), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    text = open(out).read()
    parts = re.split(r"^\s*\.type\s+(\S+),@function\s*$", text, flags=re.M)
    counts = {}
    for name, body in zip(parts[1::2], parts[2::2]):
        body = body.split("; Kernel info:")[0]
        dem = subprocess.run(["c++filt", name], capture_output=True, text=True).stdout.strip()
        counts[dem] = len(re.findall(r"^\s*s_barrier\b", body, re.M))
    return counts


@pytest.fixture(scope="module")
def counts(tmp_path_factory):
    if shutil.which(build.HIPCC) is None and not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    tmp = str(tmp_path_factory.mktemp("isa"))
    with cf.ThreadPoolExecutor(3) as ex:
        parts = list(ex.map(lambda s: _barriers(s, tmp),
                            ["tile_kernels.hip", "fused_kernels.hip", "rowcol_kernels.hip"]))
    merged = {}
    for p in parts:
        merged.update(p)
    return merged


def _find(counts, pattern):
    hits = [v for k, v in counts.items() if re.search(pattern, k)]
    assert len(hits) == 1, (pattern, [k for k in counts if re.search(pattern, k)])
    return hits[0]


@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_tile_kernels_have_table1_barriers(counts, direction):
    for wid in (0, 1):
        for sid, scheme in SCHEME_IDS.items():
            n = _find(counts, rf"k_tile_{direction}<{wid}, {sid}>")
            assert n == TABLE1[(WAVELET_IDS[wid], scheme)][0], (direction, WAVELET_IDS[wid], scheme)


@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_fused_kernels_have_two_barriers_per_pair(counts, direction):
    """Every built tile height, FP32 and FP64, double-buffered: Table 1's count
    (the height only widens each step).  Single-buffered: one more barrier
    per spatial step, except before the first publication."""
    for wid, wav in WAVELET_IDS.items():
        table1 = TABLE1[(wav, "monolithic*")][0]
        built = [(r, "float", 2) for r in dwt2.TILE_ROWS[wav]] + \
                [(r, "float", 1) for r in dwt2.TILE_ROWS[wav]] + \
                [(dwt2.TILE_ROWS_FP64[wav], "double", 2), (dwt2.TILE_ROWS_FP64[wav], "double", 1)]
        for rows, t, nb in built:
            n = _find(counts, rf"k_fused_{direction}<{wid}, {rows}, {t}, {nb}>")
            per_body = table1 if nb == 2 else 2 * table1 - 1
            assert n == 2 * per_body, (direction, wav, rows, t, nb)
        kernels = [k for k in counts if re.search(rf"k_fused_{direction}<{wid}, ", k)]
        assert len(kernels) == len(built), kernels


def test_rowcol_kernels_have_no_barriers(counts):
    for k, v in counts.items():
        if "k_rows_" in k or "k_cols_" in k:
            assert v == 0, k


@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_fused_tail_kernels_add_one_barrier_per_level(counts, direction):
    """The fused multi-level tail inlines the double-buffered tile body twice
    (Table 1's count each) plus the one barrier between levels."""
    for wid, wav in WAVELET_IDS.items():
        table1 = TABLE1[(wav, "monolithic*")][0]
        n = _find(counts, rf"k_fused_tail_{direction}<{wid}>")
        assert n == 2 * table1 + 1, (direction, wav, n)


@pytest.mark.parametrize("inverse", [False, True])
def test_transform_only_kernels_keep_the_barriers(counts, inverse):
    """The transform-only kernels lift one tile body with every barrier of
    their scheme: Table 1's count (fused, single-buffered: one more per
    spatial step after the first)."""
    inv = "true" if inverse else "false"
    for wid, wav in WAVELET_IDS.items():
        table1 = TABLE1[(wav, "monolithic*")][0]
        for rows in dwt2.TILE_ROWS[wav]:
            for nb in (1, 2):
                n = _find(counts, rf"k_fused_none<{wid}, {rows}, {nb}, {inv}>")
                assert n == (table1 if nb == 2 else 2 * table1 - 1), (wav, rows, nb, inverse)
    for wid in (0, 1):
        for sid, scheme in SCHEME_IDS.items():
            n = _find(counts, rf"k_tile_none<{wid}, {sid}, {inv}>")
            assert n == TABLE1[(WAVELET_IDS[wid], scheme)][0], (WAVELET_IDS[wid], scheme, inverse)


def _alu_ops(source, tmpdir):
    """Per kernel: (FMA, MUL, ADD/SUB) FP32 vector instruction counts."""
    out = os.path.join(tmpdir, source + ".ops.s")
    cmd = [build.HIPCC, *build.CFLAGS, "--cuda-device-only", "-S",
           os.path.join(build.CSRC, source), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    text = open(out).read()
    parts = re.split(r"^\s*\.type\s+(\S+),@function\s*$", text, flags=re.M)
    ops = {}
    for name, body in zip(parts[1::2], parts[2::2]):
        if "none" not in name:
            continue
        body = body.split("; Kernel info:")[0]
        dem = subprocess.run(["c++filt", name], capture_output=True, text=True).stdout.strip()
        ops[dem] = tuple(len(re.findall(rf"^\s*v_({pat})_f32", body, re.M))
                         for pat in ("fma|fmac|fmamk|fmaak", "mul", "add|sub|subrev"))
    return ops


def test_transform_only_kernels_keep_every_operation(tmp_path):
    """No lifting arithmetic is dropped in the transform-only kernels: the
    fused Monolithic* kernel's FMAs per lane are Table 1's operations per
    quadruple times its rows per wavefront, and the tile harness's FP32
    operations per quadruple row (less the checksum's four adds) are Table
    1's for the schemes whose steps it writes with one operation per tap
    (Monolithic*, Sweldens, Iwahashi, Polyphase*; the squared coefficient of a
    diagonal tap is formed once per kernel)."""
    if shutil.which(build.HIPCC) is None and not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    fused = _alu_ops("fused_kernels.hip", str(tmp_path))
    for wid, wav in ((0, "cdf53"), (1, "cdf97")):
        table1 = TABLE1[(wav, "monolithic*")][1]
        for rows in dwt2.TILE_ROWS[wav]:
            for nb in (1, 2):
                for inv in ("false", "true"):
                    fma = [v for k, v in fused.items()
                           if re.search(rf"k_fused_none<{wid}, {rows}, {nb}, {inv}>", k)][0][0]
                    assert fma == table1 * rows, (wav, rows, nb, inv, fma)
    tile = _alu_ops("tile_kernels.hip", str(tmp_path))
    rows_per_lane = 7  # 28 quadruple rows over 4 wavefronts
    for wid, wav in ((0, "cdf53"), (1, "cdf97")):
        for sid, scheme in ((5, "monolithic*"), (2, "sweldens"), (3, "iwahashi"), (10, "polyphase*")):
            for inv in ("false", "true"):
                fma, mul, add = [v for k, v in tile.items()
                                 if re.search(rf"k_tile_none<{wid}, {sid}, {inv}>", k)][0]
                per_row = (fma + mul + add - 4 * rows_per_lane) // rows_per_lane
                assert per_row == TABLE1[(wav, scheme)][1], (wav, scheme, inv, fma, mul, add)
