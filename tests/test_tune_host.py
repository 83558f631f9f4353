"""Host-side checks of the fused kernel's tile heights and the autotuning table
(no GPU): option validation, the per-level selection rule, and the table's
text import / export.  Every transform call here fails validation, so
nothing is enqueued."""
import ctypes
import threading

import pytest

from paper_1605_00561_amd import dwt2

FAKE = 0x7F0000000000  # never dereferenced
HALO = {"cdf53": 1, "cdf97": 2, "dd137": 3}  # quadruples of halo per tile side


@pytest.fixture(autouse=True)
def empty_table():
    assert dwt2.dwt2_tune_reset() == dwt2.OK
    yield
    assert dwt2.dwt2_tune_reset() == dwt2.OK


def _fwd(opt, levels=1, **kw):
    a = dict(wavelet=0, width=16, height=16, src=FAKE, dst=FAKE + (1 << 24))
    a.update(kw)
    lib = dwt2.library()
    res = [f(a["wavelet"], levels, a["width"], a["height"], a["src"], a["width"], a["dst"],
             a["width"], 0, ctypes.byref(opt), None, 0, None)
           for f in (lib.dwt2_forward, lib.dwt2_inverse)]
    assert res[0] == res[1]
    return res[0]


def test_unbuilt_heights_are_rejected():
    for wav, rows in dwt2.TILE_ROWS.items():
        for r in range(-1, 12):
            if r == 0 or r in rows:
                continue
            opt = dwt2.make_options(tile_rows=r)
            assert _fwd(opt, wavelet=dwt2.WAVELETS[wav]) == dwt2.E_UNSUPPORTED, (wav, r)
    # FP64 is built at one height per wavelet
    for wav, rows in dwt2.TILE_ROWS.items():
        for r in rows:
            if r != dwt2.TILE_ROWS_FP64[wav]:
                opt = dwt2.make_options(arithmetic="fp64", tile_rows=r)
                assert _fwd(opt, wavelet=dwt2.WAVELETS[wav]) == dwt2.E_UNSUPPORTED, (wav, r)
    # a height selects the fused kernel: other schemes reject it
    for scheme in ("sweldens", "rowcol", "monolithic*-tile", "polyphase*"):
        assert _fwd(dwt2.make_options(scheme=scheme, tile_rows=3)) == dwt2.E_UNSUPPORTED


def test_lds_buffering_option_is_validated():
    for bad in (-1, 3, 7):
        assert _fwd(dwt2.make_options(lds_buffers=bad)) == dwt2.E_UNSUPPORTED
    # accepted (the aliased buffers then fail the call before any launch)
    assert _fwd(dwt2.make_options(arithmetic="fp64", lds_buffers=1), dst=FAKE) == dwt2.E_ALIAS
    for scheme in ("sweldens", "rowcol", "monolithic*-tile", "explosive*"):
        assert _fwd(dwt2.make_options(scheme=scheme, lds_buffers=1)) == dwt2.E_UNSUPPORTED
        assert _fwd(dwt2.make_options(scheme=scheme, lds_buffers=2)) == dwt2.E_UNSUPPORTED
    o = dwt2.make_options(lds_buffers=1)
    o.reserved[0] = 1
    assert _fwd(o) == dwt2.E_ARG


def tiles(wav, rows, w, h):
    hq = HALO[wav]
    qw, qh = (w + 1) // 2, (h + 1) // 2
    return -(-qw // (64 - 2 * hq)) * -(-qh // (4 * rows - 2 * hq))


FILL = {"cdf53": 256, "cdf97": 512, "dd137": 1536}


def expected_rule(wav, w, h):
    ok = [r for r in dwt2.TILE_ROWS[wav] if tiles(wav, r, w, h) >= FILL[wav]]
    return max(ok) if ok else min(dwt2.TILE_ROWS[wav])


SIZES = [(2, 2), (17, 3), (512, 512), (1024, 1024), (2048, 2048), (4096, 4096), (8192, 8192),
         (16384, 16384), (8192, 64), (64, 8192), (3000, 1000), (1 << 19, 1 << 19)]


def test_selection_rule():
    for wav in dwt2.TILE_ROWS:
        for (w, h) in SIZES:
            for inverse in (False, True):
                assert dwt2.tile_rows(wav, w, h, inverse) == expected_rule(wav, w, h), (wav, w, h)
    # the measured choices the rule encodes
    assert dwt2.tile_rows("cdf97", 512, 512) == 2
    assert dwt2.tile_rows("cdf97", 2048, 2048) == 4
    assert dwt2.tile_rows("cdf97", 8192, 8192) == 4
    assert dwt2.tile_rows("cdf53", 8192, 8192) == 3
    assert dwt2.tile_rows("cdf53", 1024, 1024) == 3
    assert dwt2.tile_rows("cdf53", 512, 512) == 2
    assert dwt2.tile_rows("cdf97", 1024, 1024) == 3
    assert dwt2.tile_rows("cdf97", 1920, 1080) == 4
    assert dwt2.tile_rows("dd137", 1024, 1024) == 3
    assert dwt2.tile_rows("dd137", 2048, 2048) == 3
    assert dwt2.tile_rows("dd137", 4096, 4096) == 6


def test_forced_and_fp64_heights():
    for wav, rows in dwt2.TILE_ROWS.items():
        for r in rows:
            assert dwt2.tile_rows(wav, 8192, 8192, rows=r) == r
        assert dwt2.tile_rows(wav, 300, 200, arithmetic="fp64") == dwt2.TILE_ROWS_FP64[wav]


def test_tile_rows_errors():
    st, _ = dwt2.dwt2_tile_rows(0, "cdf53", 1, 8)
    assert st == dwt2.E_SIZE
    st, _ = dwt2.dwt2_tile_rows(0, "cdf53", 0, 8)
    assert st == dwt2.E_ARG
    st, _ = dwt2.dwt2_tile_rows(0, "cdf53", 1 << 20, 1 << 19)
    assert st == dwt2.E_SIZE
    st, _ = dwt2.dwt2_tile_rows(0, "cdf53", 64, 64, dwt2.make_options(scheme="sweldens"))
    assert st == dwt2.E_UNSUPPORTED
    assert dwt2.library().dwt2_tile_rows(0, 0, 64, 64, None, None) == dwt2.E_ARG
    assert dwt2.library().dwt2_tile_rows(0, 7, 64, 64, None, ctypes.byref(ctypes.c_int())) == \
        dwt2.E_UNSUPPORTED


def test_table_entries_override_the_rule_for_their_key_only():
    assert dwt2.dwt2_tune_import("1 0 8192 8192 2\n2 1 300 200 6\n") == dwt2.OK
    assert dwt2.tile_rows("cdf97", 8192, 8192) == 2
    assert dwt2.tile_rows("cdf97", 8192, 8192, inverse=True) == 4   # other direction: rule
    assert dwt2.tile_rows("cdf97", 8192, 8190) == 4                 # other size: rule
    assert dwt2.tile_rows("cdf53", 8192, 8192) == expected_rule("cdf53", 8192, 8192)
    assert dwt2.tile_rows("dd137", 300, 200, inverse=True) == 6
    assert dwt2.tile_rows("cdf97", 8192, 8192, rows=3) == 3         # an explicit height wins
    assert dwt2.tile_rows("cdf97", 8192, 8192, arithmetic="fp64") == 4
    assert dwt2.dwt2_tune_reset() == dwt2.OK
    assert dwt2.tile_rows("cdf97", 8192, 8192) == 4


def test_export_import_round_trip():
    text = "0 0 40 30 3\n1 1 100 60 3\n1 0 100 60 2\n2 0 5000 7 6\n"
    assert dwt2.dwt2_tune_import(text) == dwt2.OK
    st, out = dwt2.dwt2_tune_export()
    assert st == dwt2.OK
    # key order; entries imported without a tile order export order 0
    assert out == "0 0 40 30 3 0\n1 0 100 60 2 0\n1 1 100 60 3 0\n2 0 5000 7 6 0\n"
    # replacing an entry keeps one line per key
    assert dwt2.dwt2_tune_import("1 0 100 60 4 2") == dwt2.OK  # no final newline needed
    st, out2 = dwt2.dwt2_tune_export()
    assert out2 == out.replace("1 0 100 60 2 0", "1 0 100 60 4 2")
    assert dwt2.dwt2_tune_reset() == dwt2.OK
    assert dwt2.dwt2_tune_import(out2) == dwt2.OK
    assert dwt2.dwt2_tune_export() == (dwt2.OK, out2)
    assert dwt2.dwt2_tune_import("") == dwt2.OK


def test_export_buffer_too_small():
    assert dwt2.dwt2_tune_import("1 0 8192 8192 4\n") == dwt2.OK
    n = ctypes.c_size_t()
    lib = dwt2.library()
    assert lib.dwt2_tune_export(None, 0, ctypes.byref(n)) == dwt2.E_SIZE
    assert n.value == len("1 0 8192 8192 4 0\n")
    buf = ctypes.create_string_buffer(b"x" * 8, n.value)
    assert lib.dwt2_tune_export(buf, n.value, ctypes.byref(n)) == dwt2.E_SIZE  # no room for NUL
    assert buf.raw[0] == 0
    buf = ctypes.create_string_buffer(n.value + 1)
    assert lib.dwt2_tune_export(buf, n.value + 1, ctypes.byref(n)) == dwt2.OK
    assert buf.value == b"1 0 8192 8192 4 0\n"
    assert lib.dwt2_tune_export(None, 4, ctypes.byref(n)) == dwt2.E_ARG
    assert lib.dwt2_tune_export(buf, 4, None) == dwt2.E_ARG


@pytest.mark.parametrize("bad", [
    "1 0 8192 8192\n", "1 0 8192 8192 4 5\n", "1  0 8192 8192 4\n", " 1 0 8192 8192 4\n",
    "1 0 8192 8192 4 \n", "1 0 8192 8192 5\n", "3 0 64 64 2\n", "1 2 64 64 2\n",
    "1 0 1 64 2\n", "1 0 64 1 2\n", "1 0 -64 64 2\n", "1 0 64 64 +2\n", "1 0 64 64 2\r\n",
    "1 0 99999999999 64 2\n", "x\n", "\n", "0 0 64 64 4\n", "2 0 64 64 4\n", "1 0 64 64 7\n",
    "1 0 64 64 2\n\n", "1 0 64 64 2 3\n", "1 0 64 64 2 1 1\n", "1 0 64 64 2 -1\n",
    "1 0 64 64 2 1 \n"])
def test_import_rejects_malformed_text_atomically(bad):
    assert dwt2.dwt2_tune_import("1 1 64 64 3\n") == dwt2.OK
    before = dwt2.dwt2_tune_export()
    assert dwt2.dwt2_tune_import("0 0 64 64 3\n" + bad) == dwt2.E_ARG
    assert dwt2.dwt2_tune_export() == before


def test_import_capacity():
    lines = "".join(f"1 0 {64 + i} 64 2\n" for i in range(4096))
    assert dwt2.dwt2_tune_import(lines) == dwt2.OK
    assert dwt2.dwt2_tune_import("1 0 64 64 3\n") == dwt2.OK          # replaces: no growth
    assert dwt2.dwt2_tune_import("1 0 5000 64 3\n") == dwt2.E_SIZE    # a 4097th key
    assert dwt2.dwt2_tune_export()[1].count("\n") == 4096
    assert dwt2.library().dwt2_tune_import(None) == dwt2.E_ARG


def test_concurrent_table_use():
    errors = []

    def worker(k):
        try:
            for i in range(200):
                assert dwt2.dwt2_tune_import(f"1 {k % 2} {100 + i} {64 + k} 3\n") == dwt2.OK
                assert dwt2.tile_rows("cdf97", 100 + i, 64 + k, inverse=bool(k % 2)) == 3
                assert dwt2.dwt2_tune_export()[0] == dwt2.OK
        except AssertionError as e:  # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors
    assert dwt2.dwt2_tune_export()[1].count("\n") == 800


def test_autotune_argument_errors():
    lib = dwt2.library()

    def tune(opt=None, repeats=5, levels=1, inverse=0):
        return lib.dwt2_autotune(inverse, 1, levels, 16, 16, FAKE, 16, FAKE + (1 << 24), 16, 0,
                                 ctypes.byref(opt) if opt is not None else None, None, 0, repeats,
                                 None)
    for inverse in (0, 1):
        assert tune(repeats=0, inverse=inverse) == dwt2.E_ARG
        assert tune(repeats=1001, inverse=inverse) == dwt2.E_ARG
        assert tune(dwt2.make_options(scheme="sweldens"), inverse=inverse) == dwt2.E_UNSUPPORTED
        assert tune(dwt2.make_options(arithmetic="fp64"), inverse=inverse) == dwt2.E_UNSUPPORTED
        assert tune(dwt2.make_options(tile_rows=4), inverse=inverse) == dwt2.E_UNSUPPORTED
        assert tune(dwt2.make_options(lds_buffers=1), inverse=inverse) == dwt2.E_UNSUPPORTED
        assert tune(levels=2, inverse=inverse) == dwt2.E_WORKSPACE
        assert lib.dwt2_autotune(inverse, 1, 1, 16, 16, FAKE, 16, FAKE, 16, 0, None, None, 0, 5,
                                 None) == dwt2.E_ALIAS
    assert dwt2.dwt2_tune_export() == (dwt2.OK, "")


def test_tuning_file_round_trip_and_architecture_check(tmp_path):
    import json
    assert dwt2.dwt2_tune_import("1 0 8192 8192 3\n2 1 300 200 6\n") == dwt2.OK
    path = str(tmp_path / "tuning.json")
    dwt2.save_tuning(path, arch="gfx950")
    d = json.load(open(path))
    assert d["arch"] == "gfx950"
    assert {(e["wavelet"], e["inverse"], e["width"], e["height"], e["rows"], e["order"])
            for e in d["entries"]} == {(1, 0, 8192, 8192, 3, 0), (2, 1, 300, 200, 6, 0)}
    assert dwt2.dwt2_tune_reset() == dwt2.OK
    assert dwt2.load_tuning(path, arch="gfx950") == 2
    assert dwt2.tile_rows("cdf97", 8192, 8192) == 3
    assert dwt2.tile_rows("dd137", 300, 200, inverse=True) == 6
    with pytest.raises(ValueError):
        dwt2.load_tuning(path, arch="gfx942")
    d["entries"].append({"wavelet": 1, "inverse": 0, "width": 64, "height": 64, "rows": 9})
    json.dump(d, open(path, "w"))
    with pytest.raises(dwt2.Dwt2Error):  # a height that is not built: the table stays as it was
        dwt2.load_tuning(path, arch="gfx950")
    assert dwt2.tile_rows("cdf97", 64, 64) == dwt2.tile_rows("cdf97", 64, 64, rows=2)


# --- tile order -----------------------------------------------------------------

def test_tile_order_option_validation():
    """dst == src makes every call an error after option parsing (DWT2_E_ALIAS
    means the options were accepted); nothing is launched."""
    for order in ("runs", "bands"):
        assert _fwd(dwt2.make_options(tile_order=order), dst=FAKE) == dwt2.E_ALIAS
        for scheme in ("sweldens", "rowcol", "polyphase*"):
            assert _fwd(dwt2.make_options(scheme=scheme, tile_order=order), dst=FAKE) == \
                dwt2.E_UNSUPPORTED
        assert _fwd(dwt2.make_options(arithmetic="fp64", tile_order=order), dst=FAKE) == dwt2.E_ALIAS
    for bad in (3, -1, 7):
        assert _fwd(dwt2.make_options(tile_order=bad), dst=FAKE) == dwt2.E_UNSUPPORTED


def test_tile_order_rule():
    """Bands from 5 x 2^25 pixels on when the level is at least 2048 pixels wide."""
    for wav in ("cdf53", "cdf97", "dd137"):
        for inverse in (False, True):
            assert dwt2.tile_order(wav, 8192, 8192, inverse=inverse) == "runs"
            assert dwt2.tile_order(wav, 10240, 10240, inverse=inverse) == "runs"
            assert dwt2.tile_order(wav, 12288, 12288, inverse=inverse) == "runs"
            assert dwt2.tile_order(wav, 16384, 10240, inverse=inverse) == "bands"  # exactly 5 x 2^25
            assert dwt2.tile_order(wav, 16384, 10239, inverse=inverse) == "runs"
            assert dwt2.tile_order(wav, 13312, 13312, inverse=inverse) == "bands"
            assert dwt2.tile_order(wav, 16384, 16384, inverse=inverse) == "bands"
            assert dwt2.tile_order(wav, 2048, 81920, inverse=inverse) == "bands"
            assert dwt2.tile_order(wav, 2047, 82000, inverse=inverse) == "runs"   # too narrow
            assert dwt2.tile_order(wav, 16384, 16384, arithmetic="fp64") == "bands"
    assert dwt2.tile_order("cdf97", 16384, 16384, order="runs") == "runs"      # explicit wins
    assert dwt2.tile_order("cdf97", 64, 64, order="bands") == "bands"
    st, _ = dwt2.dwt2_tile_order(0, "cdf97", 64, 64, dwt2.make_options(scheme="rowcol"))
    assert st == dwt2.E_UNSUPPORTED
    st, _ = dwt2.dwt2_tile_order(0, "cdf97", 1, 64)
    assert st == dwt2.E_SIZE
    assert dwt2.library().dwt2_tile_order(0, 1, 64, 64, None, None) == dwt2.E_ARG


def test_tuned_order_overrides_the_rule_for_its_key_only():
    assert dwt2.dwt2_tune_import("1 0 8192 8192 4 2\n1 1 16384 16384 3 1\n0 0 16384 16384 3\n") \
        == dwt2.OK
    assert dwt2.tile_order("cdf97", 8192, 8192) == "bands"
    assert dwt2.tile_rows("cdf97", 8192, 8192) == 4
    assert dwt2.tile_order("cdf97", 8192, 8192, inverse=True) == "runs"          # rule
    assert dwt2.tile_order("cdf97", 16384, 16384, inverse=True) == "runs"
    assert dwt2.tile_order("cdf53", 16384, 16384) == "bands"                     # order 0: rule
    assert dwt2.tile_rows("cdf53", 16384, 16384) == 3
    assert dwt2.tile_order("cdf97", 8192, 8192, order="runs") == "runs"          # explicit wins
    assert dwt2.tile_order("cdf97", 8192, 8192, arithmetic="fp64") == "runs"     # FP32 entries only
    assert dwt2.dwt2_tune_reset() == dwt2.OK
    assert dwt2.tile_order("cdf97", 8192, 8192) == "runs"


def test_autotune_and_batches_reject_an_explicit_order():
    lib = dwt2.library()
    for order in (1, 2):
        o = dwt2.make_options(tile_order=order)
        assert lib.dwt2_autotune(0, 1, 1, 16, 16, FAKE, 16, FAKE + (1 << 24), 16, 0,
                                 ctypes.byref(o), None, 0, 5, None) == dwt2.E_UNSUPPORTED
        arr = (dwt2.Image * 1)(dwt2.Image(1, 1, 64, 64, FAKE, 64, FAKE + (1 << 24), 64))
        st, _ = dwt2.dwt2_batch_workspace_bytes(arr, 1, o)
        assert st == dwt2.E_UNSUPPORTED


def test_tuning_file_keeps_the_order(tmp_path):
    import json
    assert dwt2.dwt2_tune_import("1 0 16384 16384 4 1\n0 1 8192 8192 3 2\n") == dwt2.OK
    path = str(tmp_path / "tuning.json")
    dwt2.save_tuning(path, arch="gfx950")
    assert dwt2.dwt2_tune_reset() == dwt2.OK
    assert dwt2.load_tuning(path, arch="gfx950") == 2
    assert dwt2.tile_order("cdf97", 16384, 16384) == "runs"
    assert dwt2.tile_order("cdf53", 8192, 8192, inverse=True) == "bands"
    # a file written before orders were recorded still loads (the rule decides)
    d = json.load(open(path))
    for e in d["entries"]:
        del e["order"]
    json.dump(d, open(path, "w"))
    assert dwt2.dwt2_tune_reset() == dwt2.OK
    assert dwt2.load_tuning(path, arch="gfx950") == 2
    assert dwt2.tile_order("cdf97", 16384, 16384) == "bands"
    assert dwt2.tile_rows("cdf97", 16384, 16384) == 4


# --- fused multi-level tail -----------------------------------------------------

def test_fuse_tail_option_validation():
    """dst == src makes every call an error after option parsing (DWT2_E_ALIAS
    means the options were accepted); nothing is launched."""
    assert _fwd(dwt2.make_options(fuse_tail=1), dst=FAKE) == dwt2.E_ALIAS
    assert _fwd(dwt2.make_options(fuse_tail=1, tile_rows=2, tile_order="bands"), dst=FAKE) == \
        dwt2.E_ALIAS
    for bad in (2, -1):
        assert _fwd(dwt2.make_options(fuse_tail=bad), dst=FAKE) == dwt2.E_UNSUPPORTED
    assert _fwd(dwt2.make_options(fuse_tail=1, arithmetic="fp64"), dst=FAKE) == dwt2.E_UNSUPPORTED
    for scheme in ("sweldens", "rowcol", "explosive*"):
        assert _fwd(dwt2.make_options(scheme=scheme, fuse_tail=1), dst=FAKE) == dwt2.E_UNSUPPORTED
    o = dwt2.make_options(fuse_tail=1)
    lib = dwt2.library()
    assert lib.dwt2_autotune(0, 1, 1, 16, 16, FAKE, 16, FAKE + (1 << 24), 16, 0, ctypes.byref(o),
                             None, 0, 5, None) == dwt2.E_UNSUPPORTED
    arr = (dwt2.Image * 1)(dwt2.Image(1, 1, 64, 64, FAKE, 64, FAKE + (1 << 24), 64))
    st, _ = dwt2.dwt2_batch_workspace_bytes(arr, 1, o)
    assert st == dwt2.E_UNSUPPORTED
