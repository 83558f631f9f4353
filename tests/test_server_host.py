"""Host-side checks of the serving-loop entry points: every argument error of
dwt2_server_create and the null-handle errors of the others.  No call here
creates a server that could launch work (no request is ever submitted)."""
import ctypes

from paper_1605_00561_amd import dwt2
from test_abi_host import FAKE

ARENA = FAKE + (1 << 30)


def create(opt=None, cfg=None, arena=ARENA, nbytes=1 << 30, out=True):
    h = ctypes.c_void_p()
    st = dwt2.library().dwt2_server_create(
        ctypes.byref(opt) if opt is not None else None,
        ctypes.byref(cfg) if cfg is not None else None, arena, nbytes, None,
        ctypes.byref(h) if out else None)
    if st == dwt2.OK:  # only where a GPU is present: a server with no requests
        dwt2.dwt2_server_destroy(h)
    return st


def test_create_argument_errors():
    assert create(out=False) == dwt2.E_ARG
    o = dwt2.make_options()
    o.reserved[0] = 1
    assert create(opt=o) == dwt2.E_ARG
    for scheme in ("sweldens", "iwahashi", "rowcol", "monolithic*-tile"):
        assert create(opt=dwt2.make_options(scheme=scheme)) == dwt2.E_UNSUPPORTED
    assert create(opt=dwt2.make_options(tile_rows=3)) == dwt2.E_UNSUPPORTED
    assert create(opt=dwt2.make_options(lds_buffers=1)) == dwt2.E_UNSUPPORTED
    assert create(opt=dwt2.make_options(tile_order="bands")) == dwt2.E_UNSUPPORTED
    assert create(opt=dwt2.make_options(fuse_tail=1)) == dwt2.E_UNSUPPORTED
    o = dwt2.make_options()
    o.norm = 5
    assert create(opt=o) == dwt2.E_UNSUPPORTED
    o = dwt2.make_options()
    o.arithmetic = 3
    assert create(opt=o) == dwt2.E_UNSUPPORTED
    for field, val in [("max_batch", -1), ("max_batch", dwt2.BATCH_MAX + 1), ("max_inflight", -1),
                       ("max_footprint_mib", -1)]:
        c = dwt2.ServerConfig()
        setattr(c, field, val)
        assert create(cfg=c) == dwt2.E_ARG, field
    c = dwt2.ServerConfig()
    c.reserved[4] = 2
    assert create(cfg=c) == dwt2.E_ARG
    assert create(arena=None) == dwt2.E_WORKSPACE
    assert create(nbytes=255) == dwt2.E_WORKSPACE
    assert create(arena=ARENA + 128) == dwt2.E_ARG


def test_create_with_valid_arguments_needs_a_device():
    # Without a GPU the device query fails; with one, a server is created and
    # destroyed at once (nothing is submitted).
    assert create() in (dwt2.OK, dwt2.E_HIP)


def test_null_handles():
    lib = dwt2.library()
    t = ctypes.c_ulonglong()
    r = dwt2.Request()
    c = dwt2.Completion()
    assert lib.dwt2_server_submit(None, ctypes.byref(r), ctypes.byref(t)) == dwt2.E_ARG
    assert lib.dwt2_server_wait(None, 1, ctypes.byref(c)) == dwt2.E_ARG
    assert lib.dwt2_server_replay(None, None, None, 0, None) == dwt2.E_ARG
    assert lib.dwt2_server_destroy(None) == dwt2.E_ARG
