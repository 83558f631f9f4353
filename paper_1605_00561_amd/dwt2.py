"""Python binding of libdwt2 (the C ABI in include/dwt2.h).

The functions named like the C entry points (``dwt2_forward`` ...) only
marshal arguments.  ``forward`` / ``inverse`` are conveniences on top of them
that allocate the output and workspace with torch on the input's device and
enqueue on torch's current stream.  Every transform step runs in the HIP
kernels of libdwt2.so; there is no CPU fallback: importing this module
without a built library raises.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdwt2.so")

OK, E_ARG, E_SIZE, E_UNSUPPORTED, E_WORKSPACE, E_ALIAS, E_HIP, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
CDF53, CDF97, DD137 = 0, 1, 2
EXT_WHOLE_SYMMETRIC = 0
NORM_UNIT_DC, NORM_PAPER = 0, 1
SCHEME_AUTO, SCHEME_MONOLITHIC_STAR, SCHEME_SWELDENS, SCHEME_IWAHASHI, SCHEME_ROWCOL = 0, 1, 2, 3, 4
SCHEME_MONOLITHIC_STAR_TILE = 5
SCHEME_MONOLITHIC, SCHEME_EXPLOSIVE, SCHEME_EXPLOSIVE_STAR = 6, 7, 8
SCHEME_IWAHASHI_STAR, SCHEME_POLYPHASE_STAR = 9, 10

WAVELETS = {"cdf53": CDF53, "cdf97": CDF97, "dd137": DD137, CDF53: CDF53, CDF97: CDF97,
            DD137: DD137}
NORMS = {"unit_dc": NORM_UNIT_DC, "paper": NORM_PAPER, NORM_UNIT_DC: NORM_UNIT_DC,
         NORM_PAPER: NORM_PAPER}
SCHEMES = {"auto": SCHEME_AUTO, "monolithic*": SCHEME_MONOLITHIC_STAR,
           "monolithic*-tile": SCHEME_MONOLITHIC_STAR_TILE, "sweldens": SCHEME_SWELDENS,
           "iwahashi": SCHEME_IWAHASHI, "rowcol": SCHEME_ROWCOL, "monolithic": SCHEME_MONOLITHIC,
           "explosive": SCHEME_EXPLOSIVE, "explosive*": SCHEME_EXPLOSIVE_STAR,
           "iwahashi*": SCHEME_IWAHASHI_STAR, "polyphase*": SCHEME_POLYPHASE_STAR}
SCHEMES.update({v: v for v in list(SCHEMES.values())})

EXPORTS = ["dwt2_forward", "dwt2_inverse", "dwt2_workspace_bytes", "dwt2_status_string",
           "dwt2_last_hip_error", "dwt2_version", "dwt2_batch_workspace_bytes",
           "dwt2_forward_batch", "dwt2_inverse_batch", "dwt2_server_create", "dwt2_server_submit",
           "dwt2_server_wait", "dwt2_server_replay", "dwt2_server_destroy", "dwt2_autotune",
           "dwt2_tile_rows", "dwt2_tile_order", "dwt2_tune_export", "dwt2_tune_import",
           "dwt2_tune_reset", "dwt2_batch_tile_rows", "dwt2_transform_only",
           "dwt2_transform_noalloc", "dwt2_debug_fail_launches"]
BATCH_MAX = 65536
# Tile heights the fused kernel is built for (FP32 lifting; FP64: one each).
TILE_ROWS = {"cdf53": (2, 3), "cdf97": (2, 3, 4), "dd137": (3, 6)}
TILE_ROWS_FP64 = {"cdf53": 3, "cdf97": 4, "dd137": 6}
# Tile orders of the fused kernel (how the XCDs share a level's tiles).
ORDER_AUTO, ORDER_RUNS, ORDER_BANDS = 0, 1, 2
ORDERS = {"auto": ORDER_AUTO, "runs": ORDER_RUNS, "bands": ORDER_BANDS,
          ORDER_AUTO: ORDER_AUTO, ORDER_RUNS: ORDER_RUNS, ORDER_BANDS: ORDER_BANDS}


ARITH_AUTO, ARITH_FP32, ARITH_FP64 = 0, 1, 2
ARITHS = {"auto": ARITH_AUTO, "fp32": ARITH_FP32, "fp64": ARITH_FP64,
          ARITH_AUTO: ARITH_AUTO, ARITH_FP32: ARITH_FP32, ARITH_FP64: ARITH_FP64}


class Options(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_int), ("scheme", ctypes.c_int), ("arithmetic", ctypes.c_int),
                ("tile_rows", ctypes.c_int), ("lds_buffers", ctypes.c_int),
                ("tile_order", ctypes.c_int), ("fuse_tail", ctypes.c_int),
                ("reserved", ctypes.c_int * 1)]


class Image(ctypes.Structure):
    """struct dwt2_image: one image of a batched call."""
    _fields_ = [("wavelet", ctypes.c_int), ("levels", ctypes.c_int), ("width", ctypes.c_int),
                ("height", ctypes.c_int), ("src", ctypes.c_void_p), ("src_pitch", ctypes.c_ssize_t),
                ("dst", ctypes.c_void_p), ("dst_pitch", ctypes.c_ssize_t)]


class Request(ctypes.Structure):
    """struct dwt2_request: one request to a server."""
    _fields_ = [("inverse", ctypes.c_int), ("wavelet", ctypes.c_int), ("levels", ctypes.c_int),
                ("width", ctypes.c_int), ("height", ctypes.c_int), ("src", ctypes.c_void_p),
                ("src_pitch", ctypes.c_ssize_t), ("dst", ctypes.c_void_p),
                ("dst_pitch", ctypes.c_ssize_t)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int), ("max_inflight", ctypes.c_int),
                ("max_footprint_mib", ctypes.c_int), ("reserved", ctypes.c_int * 5)]


class Completion(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("queue_us", ctypes.c_double),
                ("latency_us", ctypes.c_double)]


class Dwt2Error(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = f"{what}: {dwt2_status_string(status)} (status {status})"
        if status == E_HIP:
            msg += f", hipError {dwt2_last_hip_error()}"
        super().__init__(msg)
        self.status = status


def _load() -> ctypes.CDLL:
    # One HIP runtime per process.  torch bundles its own libamdhip64 with the
    # same soname (libamdhip64.so.7) as the system one libdwt2.so links to.  If
    # torch is loaded first, libdwt2.so binds to torch's copy; if libdwt2.so
    # came first, torch's NEEDED entry (libamdhip64.so) would not match and a
    # second runtime would be loaded, and the two fail each other's calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1605_00561_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i, pd = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_ssize_t
    L.dwt2_forward.argtypes = [i, i, i, i, vp, pd, vp, pd, i, ctypes.POINTER(Options), vp, sz, vp]
    L.dwt2_inverse.argtypes = L.dwt2_forward.argtypes
    L.dwt2_forward.restype = L.dwt2_inverse.restype = i
    L.dwt2_workspace_bytes.argtypes = [i, i, i, i, ctypes.POINTER(Options), ctypes.POINTER(sz)]
    L.dwt2_workspace_bytes.restype = i
    ip = ctypes.POINTER(Image)
    L.dwt2_batch_workspace_bytes.argtypes = [ip, i, ctypes.POINTER(Options), ctypes.POINTER(sz)]
    L.dwt2_forward_batch.argtypes = [ip, i, i, ctypes.POINTER(Options), vp, sz, vp]
    L.dwt2_inverse_batch.argtypes = L.dwt2_forward_batch.argtypes
    L.dwt2_batch_workspace_bytes.restype = i
    L.dwt2_forward_batch.restype = L.dwt2_inverse_batch.restype = i
    L.dwt2_batch_tile_rows.argtypes = [i, ip, i, ctypes.POINTER(Options), i, ctypes.POINTER(i)]
    L.dwt2_batch_tile_rows.restype = i
    L.dwt2_transform_only.argtypes = [i, i, i, i, ctypes.POINTER(Options), vp, vp]
    L.dwt2_transform_only.restype = i
    L.dwt2_transform_noalloc.argtypes = [i, i, i, i, i, vp, pd, vp, pd, i, ctypes.POINTER(Options), vp]
    L.dwt2_transform_noalloc.restype = i
    sp = ctypes.c_void_p  # dwt2_server *
    u64 = ctypes.c_ulonglong
    L.dwt2_server_create.argtypes = [ctypes.POINTER(Options), ctypes.POINTER(ServerConfig), vp, sz,
                                     vp, ctypes.POINTER(sp)]
    L.dwt2_server_submit.argtypes = [sp, ctypes.POINTER(Request), ctypes.POINTER(u64)]
    L.dwt2_server_wait.argtypes = [sp, u64, ctypes.POINTER(Completion)]
    L.dwt2_server_replay.argtypes = [sp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_double),
                                     i, ctypes.POINTER(Completion)]
    L.dwt2_server_destroy.argtypes = [sp]
    for f in ("create", "submit", "wait", "replay", "destroy"):
        getattr(L, "dwt2_server_" + f).restype = i
    L.dwt2_status_string.argtypes = [i]
    L.dwt2_status_string.restype = ctypes.c_char_p
    L.dwt2_last_hip_error.argtypes = []
    L.dwt2_last_hip_error.restype = i
    L.dwt2_version.argtypes = []
    L.dwt2_version.restype = i
    L.dwt2_debug_fail_launches.argtypes = [i]
    L.dwt2_debug_fail_launches.restype = i
    L.dwt2_autotune.argtypes = [i, i, i, i, i, vp, pd, vp, pd, i, ctypes.POINTER(Options), vp, sz,
                                i, vp]
    L.dwt2_tile_rows.argtypes = [i, i, i, i, ctypes.POINTER(Options), ctypes.POINTER(i)]
    L.dwt2_tile_order.argtypes = [i, i, i, i, ctypes.POINTER(Options), ctypes.POINTER(i)]
    L.dwt2_tune_export.argtypes = [ctypes.c_char_p, sz, ctypes.POINTER(sz)]
    L.dwt2_tune_import.argtypes = [ctypes.c_char_p]
    L.dwt2_tune_reset.argtypes = []
    for f in ("autotune", "tile_rows", "tile_order", "tune_export", "tune_import", "tune_reset"):
        getattr(L, "dwt2_" + f).restype = i
    return L


_lib = _load()


def library() -> ctypes.CDLL:
    return _lib


def make_options(norm="unit_dc", scheme="auto", arithmetic="auto", tile_rows=0,
                 lds_buffers=0, tile_order="auto", fuse_tail=0) -> Options:
    o = Options()
    o.norm = NORMS[norm]
    o.scheme = SCHEMES[scheme]
    o.arithmetic = ARITHS[arithmetic]
    o.tile_rows = int(tile_rows)
    o.lds_buffers = int(lds_buffers)
    o.tile_order = ORDERS[tile_order] if tile_order in ORDERS else int(tile_order)
    o.fuse_tail = int(fuse_tail)
    return o


# --- C-ABI mirrors ------------------------------------------------------------
def dwt2_version() -> int:
    return _lib.dwt2_version()


def dwt2_status_string(status: int) -> str:
    return _lib.dwt2_status_string(int(status)).decode()


def dwt2_last_hip_error() -> int:
    return _lib.dwt2_last_hip_error()


def dwt2_debug_fail_launches(count: int) -> int:
    return _lib.dwt2_debug_fail_launches(int(count))


def dwt2_workspace_bytes(wavelet, levels, width, height, opt: Options | None = None):
    """(status, bytes)."""
    n = ctypes.c_size_t(0)
    st = _lib.dwt2_workspace_bytes(WAVELETS[wavelet], levels, width, height,
                                   ctypes.byref(opt) if opt is not None else None, ctypes.byref(n))
    return st, n.value


def dwt2_forward(wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext,
                 opt: Options | None, workspace, workspace_bytes, stream) -> int:
    return _lib.dwt2_forward(WAVELETS[wavelet], levels, width, height, src, src_pitch, dst,
                             dst_pitch, ext, ctypes.byref(opt) if opt is not None else None,
                             workspace, workspace_bytes, stream)


def dwt2_inverse(wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext,
                 opt: Options | None, workspace, workspace_bytes, stream) -> int:
    return _lib.dwt2_inverse(WAVELETS[wavelet], levels, width, height, src, src_pitch, dst,
                             dst_pitch, ext, ctypes.byref(opt) if opt is not None else None,
                             workspace, workspace_bytes, stream)


NOALLOC_SCRATCH_BYTES = 64 << 20


def dwt2_transform_noalloc(inverse, wavelet, levels, width, height, src, src_pitch, dst, dst_pitch,
                           ext, opt: Options | None, stream) -> int:
    return _lib.dwt2_transform_noalloc(int(bool(inverse)), WAVELETS[wavelet], levels, width, height,
                                       src, src_pitch, dst, dst_pitch, ext,
                                       ctypes.byref(opt) if opt is not None else None, stream)


def dwt2_transform_only(inverse, wavelet, width, height, opt: Options | None, sink, stream) -> int:
    return _lib.dwt2_transform_only(int(bool(inverse)), WAVELETS[wavelet], width, height,
                                    ctypes.byref(opt) if opt is not None else None, sink, stream)


def dwt2_autotune(inverse, wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext,
                  opt: Options | None, workspace, workspace_bytes, repeats, stream) -> int:
    return _lib.dwt2_autotune(int(bool(inverse)), WAVELETS[wavelet], levels, width, height, src,
                              src_pitch, dst, dst_pitch, ext,
                              ctypes.byref(opt) if opt is not None else None, workspace,
                              workspace_bytes, repeats, stream)


def dwt2_tile_rows(inverse, wavelet, width, height, opt: Options | None = None):
    """(status, rows)."""
    r = ctypes.c_int(0)
    st = _lib.dwt2_tile_rows(int(bool(inverse)), WAVELETS[wavelet], width, height,
                             ctypes.byref(opt) if opt is not None else None, ctypes.byref(r))
    return st, r.value


def dwt2_tile_order(inverse, wavelet, width, height, opt: Options | None = None):
    """(status, order)."""
    r = ctypes.c_int(0)
    st = _lib.dwt2_tile_order(int(bool(inverse)), WAVELETS[wavelet], width, height,
                              ctypes.byref(opt) if opt is not None else None, ctypes.byref(r))
    return st, r.value


def dwt2_tune_export():
    """(status, text)."""
    n = ctypes.c_size_t(0)
    st = _lib.dwt2_tune_export(None, 0, ctypes.byref(n))
    if st not in (OK, E_SIZE):
        return st, ""
    while True:  # the table may grow between the two calls
        buf = ctypes.create_string_buffer(n.value + 1)
        st = _lib.dwt2_tune_export(buf, len(buf), ctypes.byref(n))
        if st != E_SIZE:
            return st, buf.value.decode() if st == OK else ""


def dwt2_tune_import(text: str) -> int:
    return _lib.dwt2_tune_import(text.encode())


def dwt2_tune_reset() -> int:
    return _lib.dwt2_tune_reset()


def make_images(entries) -> ctypes.Array:
    """A dwt2_image array from (wavelet, levels, width, height, src, src_pitch,
    dst, dst_pitch) tuples."""
    arr = (Image * max(len(entries), 1))()
    for k, (wav, lev, w, h, src, sp, dst, dp) in enumerate(entries):
        arr[k] = Image(WAVELETS[wav], lev, w, h, src, sp, dst, dp)
    return arr


def dwt2_batch_workspace_bytes(images, count, opt: Options | None = None):
    """(status, bytes)."""
    n = ctypes.c_size_t(0)
    st = _lib.dwt2_batch_workspace_bytes(images, count,
                                         ctypes.byref(opt) if opt is not None else None,
                                         ctypes.byref(n))
    return st, n.value


def dwt2_batch_tile_rows(inverse, images, count, level, opt: Options | None = None):
    """(status, [rows per image]) of level `level` of a batched call."""
    rows = (ctypes.c_int * max(count, 1))()
    st = _lib.dwt2_batch_tile_rows(int(bool(inverse)), images, count,
                                   ctypes.byref(opt) if opt is not None else None, level, rows)
    return st, list(rows)[:count]


def dwt2_forward_batch(images, count, ext, opt: Options | None, workspace, workspace_bytes,
                       stream) -> int:
    return _lib.dwt2_forward_batch(images, count, ext,
                                   ctypes.byref(opt) if opt is not None else None, workspace,
                                   workspace_bytes, stream)


def dwt2_inverse_batch(images, count, ext, opt: Options | None, workspace, workspace_bytes,
                       stream) -> int:
    return _lib.dwt2_inverse_batch(images, count, ext,
                                   ctypes.byref(opt) if opt is not None else None, workspace,
                                   workspace_bytes, stream)


def dwt2_server_create(opt: Options | None, cfg: ServerConfig | None, arena, arena_bytes, stream):
    """(status, handle)."""
    h = ctypes.c_void_p()
    st = _lib.dwt2_server_create(ctypes.byref(opt) if opt is not None else None,
                                 ctypes.byref(cfg) if cfg is not None else None, arena,
                                 arena_bytes, stream, ctypes.byref(h))
    return st, h


def dwt2_server_submit(server, request: Request):
    """(status, ticket)."""
    t = ctypes.c_ulonglong(0)
    st = _lib.dwt2_server_submit(server, ctypes.byref(request) if request is not None else None,
                                 ctypes.byref(t))
    return st, t.value


def dwt2_server_wait(server, ticket):
    """(status, Completion)."""
    c = Completion()
    st = _lib.dwt2_server_wait(server, ticket, ctypes.byref(c))
    return st, c


def dwt2_server_replay(server, requests, arrival_us, count, done) -> int:
    return _lib.dwt2_server_replay(server, requests, arrival_us, count, done)


def dwt2_server_destroy(server) -> int:
    return _lib.dwt2_server_destroy(server)


# --- torch conveniences -------------------------------------------------------
def _check_image(t):
    import torch
    if not isinstance(t, torch.Tensor) or t.dim() != 2 or t.dtype != torch.float32:
        raise TypeError("expected a 2-D float32 torch tensor")
    if not t.is_cuda:
        raise TypeError("expected a device tensor (libdwt2 runs on the GPU only)")
    if t.stride(1) != 1:
        raise ValueError("rows must be contiguous (stride(1) == 1)")


def _workspace(wavelet, levels, w, h, opt, device, workspace):
    import torch
    st, nbytes = dwt2_workspace_bytes(wavelet, levels, w, h, opt)
    if st != OK:
        raise Dwt2Error(st, "dwt2_workspace_bytes")
    if nbytes == 0:
        return None, 0
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
    return workspace, workspace.numel() * workspace.element_size()


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _on_stream(stream):
    """Context in which torch allocates for work enqueued on `stream`: the
    caching allocator then keeps those blocks until that stream's work has
    passed them, instead of handing them to the current stream's next
    allocation while the kernels still read or write them."""
    import contextlib
    import torch
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _transform(name, call, x, wavelet, levels, norm, scheme, out, workspace, arithmetic,
               tile_rows, lds_buffers=0, tile_order="auto", fuse_tail=0, stream=None):
    """Allocate out / workspace as needed (on `stream`'s pool) and run
    call(opt, ws, ws_bytes) -> status, a closure over the C entry point with
    the tensors' pointers."""
    import torch
    _check_image(x)
    h, w = x.shape
    opt = make_options(norm, scheme, arithmetic, tile_rows, lds_buffers, tile_order, fuse_tail)
    with _on_stream(stream):
        if out is None:
            out = torch.empty((h, w), dtype=torch.float32, device=x.device)
        _check_image(out)
        ws, nws = _workspace(wavelet, levels, w, h, opt, x.device, workspace)
    st = call(out, opt, ws.data_ptr() if ws is not None else None, nws)
    if st != OK:
        raise Dwt2Error(st, name)
    return out


def forward(img, wavelet="cdf53", levels=1, norm="unit_dc", scheme="auto", out=None,
            workspace=None, stream=None, arithmetic="auto", tile_rows=0, lds_buffers=0,
            tile_order="auto", fuse_tail=0):
    """Forward DWT of a (H, W) float32 device tensor; returns the Mallat layout."""
    def call(y, opt, ws, nws):
        return dwt2_forward(wavelet, levels, img.shape[1], img.shape[0], img.data_ptr(),
                            img.stride(0), y.data_ptr(), y.stride(0), EXT_WHOLE_SYMMETRIC, opt, ws,
                            nws, _stream_handle(stream))
    return _transform("dwt2_forward", call, img, wavelet, levels, norm, scheme, out, workspace,
                      arithmetic, tile_rows, lds_buffers, tile_order, fuse_tail, stream)


def inverse(coef, wavelet="cdf53", levels=1, norm="unit_dc", scheme="auto", out=None,
            workspace=None, stream=None, arithmetic="auto", tile_rows=0, lds_buffers=0,
            tile_order="auto", fuse_tail=0):
    """Inverse DWT of a (H, W) Mallat-layout float32 device tensor; returns the image."""
    def call(y, opt, ws, nws):
        return dwt2_inverse(wavelet, levels, coef.shape[1], coef.shape[0], coef.data_ptr(),
                            coef.stride(0), y.data_ptr(), y.stride(0), EXT_WHOLE_SYMMETRIC, opt, ws,
                            nws, _stream_handle(stream))
    return _transform("dwt2_inverse", call, coef, wavelet, levels, norm, scheme, out, workspace,
                      arithmetic, tile_rows, lds_buffers, tile_order, fuse_tail, stream)


def autotune(x, wavelet="cdf53", levels=1, inverse=False, norm="unit_dc", repeats=20, out=None,
             workspace=None, stream=None):
    """dwt2_autotune: the forward (or inverse) transform of x, as forward() (or
    inverse()) computes it, timing every built tile height in both tile orders
    at every level and recording the fastest in the process-wide table.
    Blocks until done."""
    def call(y, opt, ws, nws):
        return dwt2_autotune(inverse, wavelet, levels, x.shape[1], x.shape[0], x.data_ptr(),
                             x.stride(0), y.data_ptr(), y.stride(0), EXT_WHOLE_SYMMETRIC, opt, ws,
                             nws, repeats, _stream_handle(stream))
    return _transform("dwt2_autotune", call, x, wavelet, levels, norm, "auto", out, workspace,
                      "auto", 0, stream=stream)


def tile_rows(wavelet, width, height, inverse=False, norm="unit_dc", arithmetic="auto",
              rows=0) -> int:
    """Tile height a call with these options uses for one width x height level."""
    st, r = dwt2_tile_rows(inverse, wavelet, width, height,
                           make_options(norm, "auto", arithmetic, rows))
    if st != OK:
        raise Dwt2Error(st, "dwt2_tile_rows")
    return r


def tile_order(wavelet, width, height, inverse=False, norm="unit_dc", arithmetic="auto",
               order="auto") -> str:
    """Tile order ("runs" or "bands") a call with these options uses for one
    width x height level."""
    st, r = dwt2_tile_order(inverse, wavelet, width, height,
                            make_options(norm, "auto", arithmetic, tile_order=order))
    if st != OK:
        raise Dwt2Error(st, "dwt2_tile_order")
    return {ORDER_RUNS: "runs", ORDER_BANDS: "bands"}[r]


def save_tuning(path, arch=None):
    """Write the tuned table to a JSON file, tagged with the GPU architecture
    (that of device 0 unless given)."""
    import json
    st, text = dwt2_tune_export()
    if st != OK:
        raise Dwt2Error(st, "dwt2_tune_export")
    if arch is None:
        import torch
        arch = torch.cuda.get_device_properties(0).gcnArchName
    entries = [dict(zip(("wavelet", "inverse", "width", "height", "rows", "order"),
                        map(int, l.split())))
               for l in text.splitlines()]
    with open(path, "w") as f:
        json.dump({"arch": arch, "entries": entries}, f, indent=1)


def load_tuning(path, arch=None) -> int:
    """Add the entries of a save_tuning file to the table; a file tuned on
    another architecture is refused (ValueError).  Returns the entry count."""
    import json
    with open(path) as f:
        d = json.load(f)
    if arch is None:
        import torch
        arch = torch.cuda.get_device_properties(0).gcnArchName
    if d.get("arch") != arch:
        raise ValueError(f"tuning for {d.get('arch')!r}, this device is {arch!r}")
    text = "".join(f"{e['wavelet']} {e['inverse']} {e['width']} {e['height']} {e['rows']}"
                   f" {e.get('order', 0)}\n" for e in d["entries"])
    st = dwt2_tune_import(text)
    if st != OK:
        raise Dwt2Error(st, "dwt2_tune_import")
    return len(d["entries"])


class Batch:
    """A fixed set of images for repeated batched calls (the image table is
    built once on the host; each call still copies it to the device, as the
    C entry point does).  ``inputs`` and ``outputs`` are lists of (H, W)
    float32 device tensors; ``wavelets`` and ``levels`` have one entry per
    image."""

    def __init__(self, inputs, outputs, wavelets, levels, norm="unit_dc", arithmetic="auto",
                 inverse=False, workspace=None):
        import torch
        if not (len(inputs) == len(outputs) == len(wavelets) == len(levels)):
            raise ValueError("inputs, outputs, wavelets and levels differ in length")
        entries = []
        for x, y, wav, lev in zip(inputs, outputs, wavelets, levels):
            _check_image(x)
            _check_image(y)
            if x.shape != y.shape:
                raise ValueError("input and output shapes differ")
            h, w = x.shape
            entries.append((wav, int(lev), w, h, x.data_ptr(), x.stride(0), y.data_ptr(),
                            y.stride(0)))
        self.inputs, self.outputs = list(inputs), list(outputs)
        self.count = len(entries)
        self.images = make_images(entries)
        self.opt = make_options(norm, "auto", arithmetic)
        self.inverse = inverse
        st, nbytes = dwt2_batch_workspace_bytes(self.images, self.count, self.opt)
        if st != OK:
            raise Dwt2Error(st, "dwt2_batch_workspace_bytes")
        device = inputs[0].device if inputs else torch.device("cuda")
        if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
            workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        self.workspace = workspace
        self.workspace_bytes = workspace.numel() * workspace.element_size()

    def __call__(self, stream=None):
        import torch
        fn = dwt2_inverse_batch if self.inverse else dwt2_forward_batch
        st = fn(self.images, self.count, EXT_WHOLE_SYMMETRIC, self.opt,
                self.workspace.data_ptr(), self.workspace_bytes, _stream_handle(stream))
        if st != OK:
            raise Dwt2Error(st, fn.__name__)
        if stream is not None and stream != torch.cuda.current_stream(self.workspace.device):
            # the workspace came from another stream's pool: keep its block
            # from reuse until this stream's work has passed it
            self.workspace.record_stream(stream)
        return self.outputs


def forward_batch(images, wavelets, levels, norm="unit_dc", arithmetic="auto", outs=None,
                  stream=None):
    """Forward DWT of a list of (H, W) float32 device tensors in one batched
    call; returns their Mallat layouts."""
    import torch
    with _on_stream(stream):
        if outs is None:
            outs = [torch.empty_like(x) for x in images]
        batch = Batch(images, outs, wavelets, levels, norm, arithmetic)
    return batch(stream)


def inverse_batch(coefs, wavelets, levels, norm="unit_dc", arithmetic="auto", outs=None,
                  stream=None):
    """Inverse DWT of a list of Mallat-layout device tensors in one batched call."""
    import torch
    with _on_stream(stream):
        if outs is None:
            outs = [torch.empty_like(x) for x in coefs]
        batch = Batch(coefs, outs, wavelets, levels, norm, arithmetic, inverse=True)
    return batch(stream)


class Server:
    """Serving loop over an arena of `arena_bytes` device bytes (allocated here
    with torch).  Requests are (src, dst) device tensors; the server keeps a
    reference to both until the request is waited for.  max_footprint_mib
    caps the device memory (inputs, outputs and LL buffers) of the requests
    in flight (0: no cap beyond the arena)."""

    def __init__(self, arena_bytes, norm="unit_dc", arithmetic="auto", max_batch=0,
                 max_inflight=0, stream=None, device=None, max_footprint_mib=0):
        import torch
        device = device if device is not None else torch.device("cuda")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = ServerConfig()
        cfg.max_batch, cfg.max_inflight = max_batch, max_inflight
        cfg.max_footprint_mib = int(max_footprint_mib)
        st, self.handle = dwt2_server_create(make_options(norm, "auto", arithmetic), cfg,
                                             self.arena.data_ptr(), int(arena_bytes),
                                             self.stream.cuda_stream)
        if st != OK:
            raise Dwt2Error(st, "dwt2_server_create")
        self._held = {}

    @staticmethod
    def request(src, dst, wavelet, levels, inverse=False) -> Request:
        _check_image(src)
        _check_image(dst)
        if src.shape != dst.shape:
            raise ValueError("src and dst shapes differ")
        h, w = src.shape
        return Request(int(bool(inverse)), WAVELETS[wavelet], int(levels), w, h, src.data_ptr(),
                       src.stride(0), dst.data_ptr(), dst.stride(0))

    def submit(self, src, dst, wavelet, levels, inverse=False) -> int:
        st, t = dwt2_server_submit(self.handle, self.request(src, dst, wavelet, levels, inverse))
        if st != OK:
            raise Dwt2Error(st, "dwt2_server_submit")
        self._held[t] = (src, dst)
        return t

    def wait(self, ticket) -> Completion:
        st, c = dwt2_server_wait(self.handle, ticket)
        self._held.pop(ticket, None)
        if st != OK:
            raise Dwt2Error(st, "dwt2_server_wait")
        return c

    def replay(self, requests, arrival_us):
        """requests: [(src, dst, wavelet, levels, inverse)]; returns the
        Completion of each, submitted at arrival_us[i] microseconds."""
        done = self.run(self.prepare(requests, arrival_us))
        return [done[i] for i in range(len(requests))]

    def prepare(self, requests, arrival_us):
        """Marshal a replay once (the C arrays of requests and arrival times);
        run() then costs only the C call."""
        n = len(requests)
        arr = (Request * max(n, 1))(*[self.request(*r) for r in requests])
        t = (ctypes.c_double * max(n, 1))(*[float(a) for a in arrival_us])
        return n, arr, t, list(requests)  # the tensors stay referenced

    def run(self, prepared):
        """dwt2_server_replay of a prepare()d replay; returns the C array of
        Completions (indexable)."""
        n, arr, t, _ = prepared
        done = (Completion * max(n, 1))()
        st = dwt2_server_replay(self.handle, arr, t, n, done)
        if st != OK:
            raise Dwt2Error(st, "dwt2_server_replay")
        return done

    def close(self):
        if self.handle:
            dwt2_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
