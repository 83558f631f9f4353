"""C-ABI checks that need no GPU: the library loads, exports every function
include/dwt2.h declares, and rejects bad arguments on the host before any
launch.  No call here is valid, so nothing is ever enqueued."""
import ctypes
import os
import re

import pytest

from paper_1605_00561_amd import dwt2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwt2.h")
FAKE = 0x7F0000000000  # never dereferenced: every call below fails validation


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dwt2_\w+)\s*\(", text)))


def header_define(name):
    m = re.search(rf"#define\s+{name}\s+\(?(-?\d+)\)?", open(HEADER).read())
    return int(m.group(1))


def test_exports_every_declared_function():
    names = header_functions()
    assert set(names) == set(dwt2.EXPORTS)
    lib = ctypes.CDLL(dwt2.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_status_codes_match_header():
    assert dwt2.dwt2_version() == header_define("DWT2_VERSION")
    for name, val in [("DWT2_OK", dwt2.OK), ("DWT2_E_ARG", dwt2.E_ARG),
                      ("DWT2_E_SIZE", dwt2.E_SIZE), ("DWT2_E_UNSUPPORTED", dwt2.E_UNSUPPORTED),
                      ("DWT2_E_WORKSPACE", dwt2.E_WORKSPACE), ("DWT2_E_ALIAS", dwt2.E_ALIAS),
                      ("DWT2_E_HIP", dwt2.E_HIP), ("DWT2_E_STATE", dwt2.E_STATE)]:
        assert header_define(name) == val
        assert dwt2.dwt2_status_string(val) != "unknown status"
    assert dwt2.dwt2_status_string(12345) == "unknown status"
    assert dwt2.dwt2_last_hip_error() == 0


def _ws(wav, lev, w, h, scheme="auto"):
    st, n = dwt2.dwt2_workspace_bytes(wav, lev, w, h, dwt2.make_options(scheme=scheme))
    assert st == dwt2.OK
    return n


def _al(n):
    return (n + 255) // 256 * 256


def _p(w):
    """Row pitch of a workspace LL buffer: the width rounded up to 64 floats."""
    return (w + 63) // 64 * 64


def test_workspace_bytes():
    assert _ws("cdf53", 1, 512, 512) == 0
    assert _ws("cdf97", 1, 8192, 8192) == 0
    assert _ws("cdf97", 2, 100, 60) == _al(4 * _p(50) * 30)
    assert _ws("cdf53", 5, 101, 61) == _al(4 * _p(51) * 31) + _al(4 * _p(26) * 16)
    assert _ws("cdf53", 3, 8192, 8192) == 4 * 4096 * 4096 + 4 * 2048 * 2048
    assert _ws("cdf53", 1, 100, 60, "rowcol") == _al(4 * 100 * 60)
    assert _ws("cdf97", 3, 100, 60, "rowcol") == \
        _al(4 * _p(50) * 30) + _al(4 * _p(25) * 15) + _al(4 * 6000)
    st, _ = dwt2.dwt2_workspace_bytes("cdf53", 1, 1, 8, None)
    assert st == dwt2.E_SIZE
    n = ctypes.c_size_t()
    assert dwt2.library().dwt2_workspace_bytes(0, 1, 8, 8, None, None) == dwt2.E_ARG
    assert dwt2.library().dwt2_workspace_bytes(5, 1, 8, 8, None, ctypes.byref(n)) == \
        dwt2.E_UNSUPPORTED


def _fwd(**kw):
    a = dict(wavelet=0, levels=1, width=16, height=16, src=FAKE, src_pitch=16,
             dst=FAKE + (1 << 24), dst_pitch=16, ext=0, opt=None, workspace=None,
             workspace_bytes=0, stream=None)
    a.update(kw)
    lib = dwt2.library()
    res = []
    for f in (lib.dwt2_forward, lib.dwt2_inverse):
        res.append(f(a["wavelet"], a["levels"], a["width"], a["height"], a["src"], a["src_pitch"],
                     a["dst"], a["dst_pitch"], a["ext"],
                     ctypes.byref(a["opt"]) if a["opt"] is not None else None,
                     a["workspace"], a["workspace_bytes"], a["stream"]))
    assert res[0] == res[1]
    return res[0]


def test_argument_errors():
    assert _fwd(src=None) == dwt2.E_ARG
    assert _fwd(dst=None) == dwt2.E_ARG
    assert _fwd(width=0) == dwt2.E_ARG
    assert _fwd(height=-3) == dwt2.E_ARG
    assert _fwd(levels=0) == dwt2.E_ARG
    assert _fwd(src_pitch=15) == dwt2.E_ARG
    assert _fwd(dst_pitch=8) == dwt2.E_ARG
    assert _fwd(src=FAKE + 2) == dwt2.E_ARG  # not 4-byte aligned
    o = dwt2.make_options()
    o.reserved[0] = 1
    assert _fwd(opt=o) == dwt2.E_ARG


def test_pitch_whose_span_passes_2_60_elements_is_rejected():
    """(height - 1) * pitch + width is capped at 2^60 elements, so byte
    offsets and address ranges cannot wrap."""
    limit = (2 ** 60 - 16) // 15        # largest pitch for 16 rows of 16
    assert _fwd(src_pitch=limit + 1) == dwt2.E_ARG
    assert _fwd(dst_pitch=limit + 1) == dwt2.E_ARG
    assert _fwd(src_pitch=2 ** 62) == dwt2.E_ARG


def test_size_errors():
    assert _fwd(width=1, src_pitch=1, dst_pitch=1) == dwt2.E_SIZE
    assert _fwd(height=1) == dwt2.E_SIZE
    assert _fwd(levels=5) == dwt2.E_SIZE        # 16 -> 8 -> 4 -> 2 -> 1
    assert _fwd(levels=40) == dwt2.E_SIZE
    big = 2 ** 19  # at most 2^38 pixels
    assert _fwd(width=big, height=big + 1, src_pitch=big, dst_pitch=big) == dwt2.E_SIZE
    assert dwt2.dwt2_workspace_bytes("cdf53", 2, big, big, None) == \
        (dwt2.OK, _al(4 * (big // 2) ** 2))


def test_unsupported():
    for bad in (3, -1, 99):  # one past the last wavelet id, and garbage
        assert _fwd(wavelet=bad) == dwt2.E_UNSUPPORTED
    # DD 13/7 runs in the fused kernel only
    for scheme in ("monolithic*-tile", "sweldens", "iwahashi", "rowcol", "monolithic", "explosive",
                   "explosive*", "iwahashi*", "polyphase*"):
        assert _fwd(wavelet=2, opt=dwt2.make_options(scheme=scheme)) == dwt2.E_UNSUPPORTED
    assert _fwd(ext=1) == dwt2.E_UNSUPPORTED
    o = dwt2.make_options()
    o.norm = 2
    assert _fwd(opt=o) == dwt2.E_UNSUPPORTED
    for bad in (11, -1, 1 << 20):  # one past the last scheme id, and garbage
        o = dwt2.make_options()
        o.scheme = bad
        assert _fwd(opt=o) == dwt2.E_UNSUPPORTED
    o = dwt2.make_options()
    o.arithmetic = 3
    assert _fwd(opt=o) == dwt2.E_UNSUPPORTED
    for scheme in ("monolithic*-tile", "sweldens", "iwahashi", "rowcol", "monolithic", "explosive",
                   "explosive*", "iwahashi*", "polyphase*"):
        assert _fwd(opt=dwt2.make_options(scheme=scheme, arithmetic="fp64")) == dwt2.E_UNSUPPORTED


def test_scheme_ids_match_header():
    text = open(HEADER).read()
    ids = dict(re.findall(r"DWT2_SCHEME_(\w+) = (\d+)", text))
    names = {"AUTO": "auto", "MONOLITHIC_STAR": "monolithic*", "SWELDENS": "sweldens",
             "IWAHASHI": "iwahashi", "ROWCOL": "rowcol", "MONOLITHIC_STAR_TILE": "monolithic*-tile",
             "MONOLITHIC": "monolithic", "EXPLOSIVE": "explosive", "EXPLOSIVE_STAR": "explosive*",
             "IWAHASHI_STAR": "iwahashi*", "POLYPHASE_STAR": "polyphase*"}
    assert set(ids) == set(names)
    for k, v in ids.items():
        assert dwt2.SCHEMES[names[k]] == int(v), k
    assert max(int(v) for v in ids.values()) == 10


def test_workspace_and_alias_errors():
    assert _fwd(levels=2) == dwt2.E_WORKSPACE           # needs a workspace
    assert _fwd(levels=2, workspace=FAKE + (2 << 24), workspace_bytes=16) == dwt2.E_WORKSPACE
    assert _fwd(levels=2, workspace=FAKE + (2 << 24) + 4, workspace_bytes=4096) == dwt2.E_ARG
    assert _fwd(dst=FAKE) == dwt2.E_ALIAS                # dst == src
    assert _fwd(dst=FAKE + 4 * 16 * 15) == dwt2.E_ALIAS  # last row of src overlaps dst
    assert _fwd(levels=2, workspace=FAKE + (1 << 24), workspace_bytes=4096) == dwt2.E_ALIAS


def test_torch_wrappers_reject_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        dwt2.forward(torch.zeros(8, 8))
    with pytest.raises(TypeError):
        dwt2.inverse(torch.zeros(8, 8, dtype=torch.float64))


def test_single_hip_runtime_when_binding_is_imported_first():
    """Importing the binding before torch must not leave two HIP runtimes mapped
    (torch's bundled libamdhip64 and the system one): with two, every launch of
    one fails in the other's context."""
    import subprocess
    import sys
    code = ("import paper_1605_00561_amd.dwt2, torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_transform_only_argument_errors():
    """dwt2_transform_only validates on the host like dwt2_forward (nothing
    below is launched)."""
    def call(inverse=0, wav="cdf97", w=64, h=64, opt=None, sink=FAKE):
        return dwt2.dwt2_transform_only(inverse, wav, w, h, opt, sink, None)
    assert call(sink=None) == dwt2.E_ARG
    assert call(sink=FAKE + 2) == dwt2.E_ARG
    assert call(w=0) == dwt2.E_ARG and call(h=-1) == dwt2.E_ARG
    assert call(w=1) == dwt2.E_SIZE and call(h=1) == dwt2.E_SIZE
    assert call(w=1 << 20, h=1 << 20) == dwt2.E_SIZE
    assert call(opt=dwt2.make_options(arithmetic="fp64")) == dwt2.E_UNSUPPORTED
    assert call(opt=dwt2.make_options(scheme="rowcol")) == dwt2.E_UNSUPPORTED
    assert call(opt=dwt2.make_options(fuse_tail=1)) == dwt2.E_UNSUPPORTED
    assert call(opt=dwt2.make_options(tile_rows=5)) == dwt2.E_UNSUPPORTED
    assert call(wav="dd137", opt=dwt2.make_options(scheme="sweldens")) == dwt2.E_UNSUPPORTED
    o = dwt2.make_options()
    o.reserved[0] = 1
    assert call(opt=o) == dwt2.E_ARG
    assert dwt2.library().dwt2_transform_only(0, 7, 64, 64, None, FAKE, None) == dwt2.E_UNSUPPORTED


def test_noalloc_argument_errors():
    """dwt2_transform_noalloc validates everything but the workspace (its own
    static array) on the host first, and refuses a workspace need beyond the
    array before touching the device."""
    def call(wav="cdf97", lev=2, w=64, h=64, src=FAKE, sp=64, dst=FAKE + (1 << 26), dp=64, opt=None,
             inverse=0):
        return dwt2.dwt2_transform_noalloc(inverse, wav, lev, w, h, src, sp, dst, dp, 0, opt, None)
    for inverse in (0, 1):
        assert call(src=None, inverse=inverse) == dwt2.E_ARG
        assert call(sp=10, inverse=inverse) == dwt2.E_ARG
        assert call(lev=0, inverse=inverse) == dwt2.E_ARG
        assert call(lev=8, inverse=inverse) == dwt2.E_SIZE
        assert call(dst=FAKE + 4, inverse=inverse) == dwt2.E_ALIAS
        bad = dwt2.make_options()
        bad.scheme = 99
        assert call(opt=bad, inverse=inverse) == dwt2.E_UNSUPPORTED
        big = dict(w=8192, h=8192, sp=8192, dp=8192, dst=FAKE + (1 << 30), lev=3)
        assert call(inverse=inverse, **big) == dwt2.E_WORKSPACE  # 64 + 16 MiB of LL buffers
        assert call(inverse=inverse, opt=dwt2.make_options(scheme="rowcol"), w=4096, h=4096, sp=4096,
                    dp=4096, dst=FAKE + (1 << 30)) == dwt2.E_WORKSPACE  # + 64 MiB intermediate
    assert header_define("DWT2_NOALLOC_SCRATCH_BYTES") == dwt2.NOALLOC_SCRATCH_BYTES
    assert dwt2.dwt2_workspace_bytes("cdf97", 3, 8192, 8192)[1] > dwt2.NOALLOC_SCRATCH_BYTES
    assert dwt2.dwt2_workspace_bytes("cdf97", 2, 8192, 8192)[1] == dwt2.NOALLOC_SCRATCH_BYTES


def test_fault_injection_reaches_every_launching_entry_point():
    """dwt2_debug_fail_launches makes the calling thread's next launches fail
    with hipErrorInvalidConfiguration without launching, so each entry point's
    DWT2_E_HIP path and dwt2_last_hip_error() are exercised on the host.  Every
    call below fails at its first launch; nothing reaches the device."""
    import threading
    INVALID_CONFIGURATION = 9  # hipErrorInvalidConfiguration
    lib = dwt2.library()
    assert dwt2.dwt2_debug_fail_launches(-1) == dwt2.E_ARG
    src, dst, ws = FAKE, FAKE + (1 << 26), FAKE + (1 << 28)
    calls = [
        lambda: dwt2.dwt2_forward("cdf97", 1, 64, 64, src, 64, dst, 64, 0, None, None, 0, None),
        lambda: dwt2.dwt2_inverse("cdf53", 3, 64, 64, src, 64, dst, 64, 0, None, ws, 1 << 20, None),
        lambda: dwt2.dwt2_forward("cdf53", 2, 64, 64, src, 64, dst, 64, 0,
                                  dwt2.make_options(scheme="rowcol"), ws, 1 << 20, None),
        lambda: dwt2.dwt2_forward("cdf97", 1, 64, 64, src, 64, dst, 64, 0,
                                  dwt2.make_options(scheme="sweldens"), None, 0, None),
        lambda: dwt2.dwt2_forward("dd137", 3, 100, 100, src, 100, dst, 100, 0,
                                  dwt2.make_options(fuse_tail=1), ws, 1 << 20, None),
        lambda: dwt2.dwt2_forward_batch(dwt2.make_images([("cdf97", 2, 64, 64, src, 64, dst, 64)]), 1,
                                        0, None, ws, 1 << 20, None),
        lambda: dwt2.dwt2_inverse_batch(dwt2.make_images([("cdf53", 1, 64, 64, src, 64, dst, 64)]), 1,
                                        0, None, ws, 1 << 20, None),
        lambda: dwt2.dwt2_transform_only(1, "cdf97", 64, 64, None, src, None),
        lambda: dwt2.dwt2_transform_noalloc(0, "cdf53", 1, 64, 64, src, 64, dst, 64, 0, None, None),
    ]
    try:
        assert dwt2.dwt2_debug_fail_launches(len(calls) + 2) == dwt2.OK
        for i, call in enumerate(calls):
            assert call() == dwt2.E_HIP, i
            assert dwt2.dwt2_last_hip_error() == INVALID_CONFIGURATION, i
        # the count is per thread: another thread's own count does not touch this one's
        seen = []

        def other():
            dwt2.dwt2_debug_fail_launches(1)
            seen.append((calls[0](), dwt2.dwt2_last_hip_error()))
        t = threading.Thread(target=other)
        t.start()
        t.join()
        assert seen == [(dwt2.E_HIP, INVALID_CONFIGURATION)]
        for i in range(2):  # this thread's last two injected failures
            assert calls[3]() == dwt2.E_HIP
    finally:
        dwt2.dwt2_debug_fail_launches(0)
    assert lib.dwt2_debug_fail_launches(0) == dwt2.OK
