// dwt2_api.cpp -- host side of the libdwt2 C ABI (declared in include/dwt2.h):
// argument validation, level geometry, workspace layout and kernel dispatch.
// Nothing here allocates device memory or synchronises; every launch goes to
// the caller's stream.
#include "../../include/dwt2.h"

#include <limits.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "dwt2_internal.h"

#define DWT2_EXPORT extern "C" __attribute__((visibility("default")))

namespace {

thread_local int g_last_hip_error = 0;
thread_local int g_fail_launches = 0;  // dwt2_debug_fail_launches

constexpr int kMaxLevels = 31;
// 2^38 pixels (1 TiB of FP32) bounds every grid well inside int range.
constexpr long long kMaxPixels = 1LL << 38;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Config {
    int wavelet, norm, scheme, arithmetic, tile_rows;
    int lds_buffers;  // 0 = default (2)
    int tile_order;   // 0 = automatic, else DWT2_ORDER_RUNS / DWT2_ORDER_BANDS
    int fuse_tail;    // 1: levels from kTailSide x kTailSide down in one work-group
};

int parse(dwt2_wavelet wavelet, dwt2_ext ext, const dwt2_options *opt, Config *c)
{
    if (wavelet != DWT2_CDF53 && wavelet != DWT2_CDF97 && wavelet != DWT2_DD137)
        return DWT2_E_UNSUPPORTED;
    if (ext != DWT2_EXT_WHOLE_SYMMETRIC) return DWT2_E_UNSUPPORTED;
    c->wavelet = wavelet;
    c->norm = DWT2_NORM_UNIT_DC;
    c->scheme = DWT2_SCHEME_AUTO;
    c->arithmetic = DWT2_ARITH_AUTO;
    c->tile_rows = 0;
    c->lds_buffers = 0;
    c->tile_order = 0;
    c->fuse_tail = 0;
    if (opt) {
        for (int r : opt->reserved)
            if (r != 0) return DWT2_E_ARG;
        c->norm = opt->norm;
        c->scheme = opt->scheme;
        c->arithmetic = opt->arithmetic;
        c->tile_rows = opt->tile_rows;
        c->lds_buffers = opt->lds_buffers;
        c->tile_order = opt->tile_order;
        c->fuse_tail = opt->fuse_tail;
    }
    if (c->arithmetic < DWT2_ARITH_AUTO || c->arithmetic > DWT2_ARITH_FP64) return DWT2_E_UNSUPPORTED;
    if (c->norm != DWT2_NORM_UNIT_DC && c->norm != DWT2_NORM_PAPER) return DWT2_E_UNSUPPORTED;
    if (c->scheme < DWT2_SCHEME_AUTO || c->scheme > DWT2_SCHEME_POLYPHASE_STAR)
        return DWT2_E_UNSUPPORTED;
    if (c->scheme == DWT2_SCHEME_AUTO) c->scheme = DWT2_SCHEME_MONOLITHIC_STAR;
    // FP64 lifting is implemented by the fused kernel only.
    if (c->arithmetic == DWT2_ARITH_FP64 && c->scheme != DWT2_SCHEME_MONOLITHIC_STAR)
        return DWT2_E_UNSUPPORTED;
    if (c->arithmetic == DWT2_ARITH_AUTO) c->arithmetic = DWT2_ARITH_FP32;
    // DD 13/7's four-tap operators are implemented by the fused kernel only.
    if (c->wavelet == DWT2_DD137 && c->scheme != DWT2_SCHEME_MONOLITHIC_STAR) return DWT2_E_UNSUPPORTED;
    if (c->tile_rows != 0 &&
        (c->scheme != DWT2_SCHEME_MONOLITHIC_STAR ||
         !dwt2::fused_rows_supported(c->wavelet, c->arithmetic == DWT2_ARITH_FP64, c->tile_rows)))
        return DWT2_E_UNSUPPORTED;
    // LDS buffering: fused kernel only.
    if (c->lds_buffers != 0 &&
        (c->scheme != DWT2_SCHEME_MONOLITHIC_STAR || (c->lds_buffers != 1 && c->lds_buffers != 2)))
        return DWT2_E_UNSUPPORTED;
    if (c->tile_order != 0 &&
        (c->scheme != DWT2_SCHEME_MONOLITHIC_STAR ||
         (c->tile_order != DWT2_ORDER_RUNS && c->tile_order != DWT2_ORDER_BANDS)))
        return DWT2_E_UNSUPPORTED;
    // The fused multi-level tail: fused kernel, FP32 lifting.
    if (c->fuse_tail != 0 &&
        (c->fuse_tail != 1 || c->scheme != DWT2_SCHEME_MONOLITHIC_STAR || c->arithmetic == DWT2_ARITH_FP64))
        return DWT2_E_UNSUPPORTED;
    return DWT2_OK;
}

// Default LDS buffering: double, except with FP64 lifting.  Double-buffered
// FP64 planes (36.9 KB at 9/7) limit a CU to four work-groups, where the
// registers (82 / 88 VGPRs forward / inverse) allow five; at 5/3 they limit it
// to five where the registers allow eight.  Measured at 8192^2 9/7: forward
// 124.6 us single against 131.0 double, inverse 123.7 against 131.7.
int buffers_of(const Config &c)
{
    if (c.lds_buffers) return c.lds_buffers;
    return c.arithmetic == DWT2_ARITH_FP64 ? 1 : 2;
}

// ---------------------------------------------------------------------------
// Tile height and tile order of the fused kernel per level.  Tuned entries,
// keyed by (wavelet, inverse, level width, level height), live in one table
// per process; g_tune_size lets calls skip the lock while it is empty.  An
// entry's order is 0 when it was imported without one (the rule decides).
using TuneKey = std::array<int, 4>;
struct TuneVal {
    int rows, order;
};
constexpr size_t kTuneMax = 4096;
// Fill thresholds per wavelet (5/3, 9/7, DD 13/7): a level takes the tallest
// built height that gives it at least this many tiles.  Below it a level is
// short of work-groups and a shorter tile wins; above it the taller tile
// (fewer halo rows re-read, fewer work-groups to schedule) wins.  Fitted to
// one-level device times of every built height at 14 level sizes from 512^2
// to 16384^2 (square, 1920 x 1080, 3840 x 2160, 7680 x 4320): the choice is
// then within 0.25 % of the fastest height on average, 4.6 % at worst (one
// shared threshold of 1024 tiles: 0.8 %, 9 %).  DD 13/7's tall tile holds
// twice the rows of its short one, hence its higher threshold.
constexpr long long kFillTiles[3] = {256, 512, 1536};

std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
std::atomic<size_t> g_tune_size{0};

int rule_rows(int wavelet, int W, int H)
{
    int pick = dwt2::kFusedRows[wavelet][0];  // heights are listed in ascending order
    for (int r : dwt2::kFusedRows[wavelet])
        if (r > 0 && dwt2::fused_tile_count(wavelet, r, W, H) >= kFillTiles[wavelet]) pick = r;
    return pick;
}

// Tile order rule: the band order from 5 x 2^25 pixels (about 12953^2) on,
// when the level is at least 2048 pixels (16 or more tile columns, two per
// XCD) wide.  Measured with the launches' work-group cap (six per CU from
// 2^26 pixels), 9/7 and 5/3, forward and inverse, summed, us runs against
// bands: 12288^2 936 against 964, 12800^2 1023 against 1036, 13312^2 1132
// against 1109, 13824^2 1229 against 1184, 14336^2 1337 against 1267,
// 16384^2 1690 against 1646; at 8192^2 to 11264^2 runs lead by 3-7 %.
constexpr long long kBandPixels = 5LL << 25;
constexpr int kBandMinWidth = 2048;

int rule_order(int W, int H)
{
    return (long long)W * H >= kBandPixels && W >= kBandMinWidth ? DWT2_ORDER_BANDS : DWT2_ORDER_RUNS;
}

// The tuned entry of a level, if any.
bool tuned(const Config &c, bool inverse, int W, int H, TuneVal *v)
{
    if (!g_tune_size.load(std::memory_order_acquire)) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey{c.wavelet, inverse ? 1 : 0, W, H});
    if (it == g_tune.end()) return false;
    *v = it->second;
    return true;
}

int choose_rows(const Config &c, bool inverse, int W, int H)
{
    if (c.arithmetic == DWT2_ARITH_FP64) return dwt2::kFusedRowsFp64[c.wavelet];
    if (c.tile_rows) return c.tile_rows;
    TuneVal v;
    if (tuned(c, inverse, W, H, &v)) return v.rows;
    return rule_rows(c.wavelet, W, H);
}

int choose_order(const Config &c, bool inverse, int W, int H)
{
    if (c.tile_order) return c.tile_order;
    TuneVal v;
    if (c.arithmetic != DWT2_ARITH_FP64 && tuned(c, inverse, W, H, &v) && v.order) return v.order;
    return rule_order(W, H);
}

// Level k (0-based) transforms a ws[k] x hs[k] block; each must be >= 2 x 2.
int geometry(int levels, int width, int height, int *ws, int *hs)
{
    if (levels < 1 || width < 1 || height < 1) return DWT2_E_ARG;
    if (levels > kMaxLevels) return DWT2_E_SIZE;
    if ((long long)width * height > kMaxPixels) return DWT2_E_SIZE;
    int w = width, h = height;
    for (int k = 0; k < levels; k++) {
        if (w < 2 || h < 2) return DWT2_E_SIZE;
        ws[k] = w;
        hs[k] = h;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    return DWT2_OK;
}

// Workspace: LL ping-pong buffers A (level-1 LL size) and B (level-2 LL
// size) when levels > 1, rows padded to ll_pitch(), plus a W x H
// intermediate for the row-column scheme.
struct Layout {
    size_t a_off, b_off, t_off, total;
};

Layout layout(int scheme, int levels, const int *ws, const int *hs)
{
    Layout L = {0, 0, 0, 0};
    size_t off = 0;
    if (levels >= 2) {
        L.a_off = off;
        off += align_up(sizeof(float) * (size_t)dwt2::ll_pitch((ws[0] + 1) / 2) * (size_t)((hs[0] + 1) / 2));
    }
    if (levels >= 3) {
        L.b_off = off;
        off += align_up(sizeof(float) * (size_t)dwt2::ll_pitch((ws[1] + 1) / 2) * (size_t)((hs[1] + 1) / 2));
    }
    if (scheme == DWT2_SCHEME_ROWCOL) {
        L.t_off = off;
        off += align_up(sizeof(float) * (size_t)ws[0] * (size_t)hs[0]);
    }
    L.total = off;
    return L;
}

// Per-level scales of LL and HH.  The paper's scaling step diag(zeta, 1/zeta)
// per axis gives LL * zeta^2 and HH / zeta^2 (HL, LH unscaled).  The unit-DC
// normalisation divides LL by the squared DC gain K of the unscaled low-pass
// (K = 1 for 5/3 and DD 13/7) and multiplies HH by K^2, so
// PAPER = UNIT_DC * {2, 1/2} exactly, also after rounding to FP32 (zeta^2 K^2
// = 2; the paper gives no zeta for DD 13/7, which takes sqrt(2) as 5/3 does).
dwt2::Scale level_scale(int wavelet, int norm)
{
    double K = 1.0;
    if (wavelet == DWT2_CDF97) {
        const double alpha = -1.58613434205992355842832, beta = -0.0529801185729614146241296;
        K = 1.0 + 2.0 * beta * (1.0 + 2.0 * alpha);  // lifting the constant signal 1
    }
    const double ll = 1.0 / (K * K), hh = K * K;
    dwt2::Scale s;
    s.ll = (float)(norm == DWT2_NORM_PAPER ? 2.0 * ll : ll);
    s.hh = (float)(norm == DWT2_NORM_PAPER ? 0.5 * hh : hh);
    return s;
}

dwt2::Scale inverse_scale(int wavelet, int norm)
{
    const dwt2::Scale s = level_scale(wavelet, norm);
    dwt2::Scale r;
    r.ll = (float)(1.0 / (double)s.ll);
    r.hh = (float)(1.0 / (double)s.hh);
    return r;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

size_t span_bytes(ptrdiff_t pitch, int w, int h)
{
    return sizeof(float) * ((size_t)(h - 1) * (size_t)pitch + (size_t)w);
}

// An image may span at most 2^60 elements ((h - 1) * pitch + w), which keeps
// byte offsets and address ranges far from 64-bit wrap-around.  pitch >= w.
bool span_fits(ptrdiff_t pitch, int w, int h)
{
    constexpr long long kMaxSpan = 1LL << 60;
    return h == 1 || (long long)pitch <= (kMaxSpan - w) / (h - 1);
}

struct Checked {
    Config cfg;
    int levels;
    int ws[kMaxLevels], hs[kMaxLevels];
    Layout lay;
};

// check_ws = false skips the workspace checks (the caller supplies it later).
int check_call(dwt2_wavelet wavelet, int levels, int width, int height, const float *src,
               ptrdiff_t src_pitch, float *dst, ptrdiff_t dst_pitch, dwt2_ext ext,
               const dwt2_options *opt, void *workspace, size_t workspace_bytes, Checked *c,
               bool check_ws = true)
{
    int st = parse(wavelet, ext, opt, &c->cfg);
    if (st != DWT2_OK) return st;
    st = geometry(levels, width, height, c->ws, c->hs);
    if (st != DWT2_OK) return st;
    c->levels = levels;
    if (!src || !dst) return DWT2_E_ARG;
    if (src_pitch < width || dst_pitch < width) return DWT2_E_ARG;
    if (!span_fits(src_pitch, width, height) || !span_fits(dst_pitch, width, height)) return DWT2_E_ARG;
    if (((uintptr_t)src & 3) || ((uintptr_t)dst & 3)) return DWT2_E_ARG;
    c->lay = layout(c->cfg.scheme, levels, c->ws, c->hs);
    const size_t ns = span_bytes(src_pitch, width, height), nd = span_bytes(dst_pitch, width, height);
    if (!check_ws) return overlap(src, ns, dst, nd) ? DWT2_E_ALIAS : DWT2_OK;
    if (c->lay.total > 0 && (!workspace || workspace_bytes < c->lay.total)) return DWT2_E_WORKSPACE;
    if (c->lay.total > 0 && ((uintptr_t)workspace & (kAlign - 1))) return DWT2_E_ARG;
    if (overlap(src, ns, dst, nd)) return DWT2_E_ALIAS;
    if (c->lay.total > 0 &&
        (overlap(workspace, c->lay.total, src, ns) || overlap(workspace, c->lay.total, dst, nd)))
        return DWT2_E_ALIAS;
    return DWT2_OK;
}

// Arguments of forward level k (0-based).  Level k reads the image (k = 0)
// or LL_k; LL_j (1-based j) lives in workspace buffer A for odd j, B for even
// j, with pitch ll_pitch(its width); the last level writes LL into dst.
dwt2::FwdArgs forward_level(const Checked &c, int k, const float *src, ptrdiff_t src_pitch,
                            float *dst, ptrdiff_t dst_pitch, void *workspace)
{
    char *wsb = (char *)workspace;
    float *buf[2] = {(float *)(wsb + c.lay.a_off), (float *)(wsb + c.lay.b_off)};
    const int levels = c.levels, W = c.ws[k], H = c.hs[k];
    dwt2::FwdArgs a;
    a.in = k == 0 ? src : buf[(k - 1) & 1];
    a.in_pitch = k == 0 ? src_pitch : dwt2::ll_pitch(W);
    a.det = dst;
    a.det_pitch = dst_pitch;
    a.W = W;
    a.H = H;
    a.s = level_scale(c.cfg.wavelet, c.cfg.norm);
    a.ll_gain = c.cfg.norm == DWT2_NORM_PAPER ? 2.0f : 1.0f;
    a.quantum = c.cfg.norm == DWT2_NORM_PAPER ? ldexpf(1.0f, k) : 1.0f;
    a.ll = k == levels - 1 ? dst : buf[k & 1];
    a.ll_pitch = k == levels - 1 ? dst_pitch : dwt2::ll_pitch((W + 1) / 2);
    return a;
}

// First level of the fused tail (c.levels when there is none): the first
// level whose input is at most kTailSide on both sides, if at least two
// levels remain from there.
int tail_start(const Checked &c)
{
    if (!c.cfg.fuse_tail) return c.levels;
    for (int k = 0; k + 1 < c.levels; k++)
        if (c.ws[k] <= dwt2::kTailSide && c.hs[k] <= dwt2::kTailSide) return k;
    return c.levels;
}

dwt2::TailArgs tail_args(const Checked &c, int k0, bool inverse)
{
    dwt2::TailArgs t;
    t.W = c.ws[0];
    t.H = c.hs[0];
    t.k0 = k0;
    t.levels = c.levels;
    t.s = inverse ? inverse_scale(c.cfg.wavelet, c.cfg.norm) : level_scale(c.cfg.wavelet, c.cfg.norm);
    t.ll_gain = c.cfg.norm == DWT2_NORM_PAPER ? 2.0f : 1.0f;
    t.paper = c.cfg.norm == DWT2_NORM_PAPER;
    t.buf_elems = dwt2::tail_buffer_elems(c.ws[0], c.hs[0], k0);
    return t;
}

// Arguments of inverse level k: it rebuilds its W_k x H_k input from LL_{k+1}
// (src at the last level, else its workspace buffer) and the details in src,
// into dst (k = 0) or LL_k's buffer.
dwt2::InvArgs inverse_level(const Checked &c, int k, const float *src, ptrdiff_t src_pitch,
                            float *dst, ptrdiff_t dst_pitch, void *workspace)
{
    char *wsb = (char *)workspace;
    float *buf[2] = {(float *)(wsb + c.lay.a_off), (float *)(wsb + c.lay.b_off)};
    const int levels = c.levels, W = c.ws[k], H = c.hs[k];
    dwt2::InvArgs a;
    a.ll = k == levels - 1 ? src : buf[k & 1];
    a.ll_pitch = k == levels - 1 ? src_pitch : dwt2::ll_pitch((W + 1) / 2);
    a.det = src;
    a.det_pitch = src_pitch;
    a.W = W;
    a.H = H;
    a.inv_s = inverse_scale(c.cfg.wavelet, c.cfg.norm);
    a.ll_gain = c.cfg.norm == DWT2_NORM_PAPER ? 2.0f : 1.0f;
    a.quantum = c.cfg.norm == DWT2_NORM_PAPER ? ldexpf(1.0f, k) : 1.0f;
    a.out = k == 0 ? dst : buf[(k - 1) & 1];
    a.out_pitch = k == 0 ? dst_pitch : dwt2::ll_pitch(W);
    return a;
}

int hip_status(hipError_t e)
{
    if (e == hipSuccess) return DWT2_OK;
    g_last_hip_error = (int)e;
    return DWT2_E_HIP;
}

}  // namespace

bool dwt2::take_launch_failure()
{
    if (g_fail_launches <= 0) return false;
    g_fail_launches--;
    return true;
}

DWT2_EXPORT int dwt2_debug_fail_launches(int count)
{
    if (count < 0) return DWT2_E_ARG;
    g_fail_launches = count;
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_version(void) { return DWT2_VERSION; }

DWT2_EXPORT int dwt2_last_hip_error(void) { return g_last_hip_error; }

DWT2_EXPORT const char *dwt2_status_string(int status)
{
    switch (status) {
    case DWT2_OK: return "ok";
    case DWT2_E_ARG: return "invalid argument";
    case DWT2_E_SIZE: return "a level's input is smaller than 2x2";
    case DWT2_E_UNSUPPORTED: return "unsupported wavelet, extension, normalisation, scheme or arithmetic";
    case DWT2_E_WORKSPACE: return "workspace missing or too small";
    case DWT2_E_ALIAS: return "src, dst or workspace overlap";
    case DWT2_E_HIP: return "HIP launch failed";
    case DWT2_E_STATE: return "server stopping, or unknown or already collected ticket";
    default: return "unknown status";
    }
}

DWT2_EXPORT int dwt2_workspace_bytes(dwt2_wavelet wavelet, int levels, int width, int height,
                                     const dwt2_options *opt, size_t *bytes)
{
    Config cfg;
    int ws[kMaxLevels], hs[kMaxLevels];
    if (!bytes) return DWT2_E_ARG;
    int st = parse(wavelet, DWT2_EXT_WHOLE_SYMMETRIC, opt, &cfg);
    if (st != DWT2_OK) return st;
    st = geometry(levels, width, height, ws, hs);
    if (st != DWT2_OK) return st;
    *bytes = layout(cfg.scheme, levels, ws, hs).total;
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_forward(dwt2_wavelet wavelet, int levels, int width, int height,
                             const float *src, ptrdiff_t src_pitch, float *dst, ptrdiff_t dst_pitch,
                             dwt2_ext ext, const dwt2_options *opt, void *workspace,
                             size_t workspace_bytes, hipStream_t stream)
{
    Checked c;
    int st = check_call(wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext, opt,
                        workspace, workspace_bytes, &c);
    if (st != DWT2_OK) return st;
    char *wsb = (char *)workspace;
    float *tmp = (float *)(wsb + c.lay.t_off);
    const int k0 = tail_start(c);
    for (int k = 0; k < k0; k++) {
        const dwt2::FwdArgs a = forward_level(c, k, src, src_pitch, dst, dst_pitch, workspace);
        hipError_t e;
        if (c.cfg.scheme == DWT2_SCHEME_ROWCOL)
            e = dwt2::launch_rowcol_forward(c.cfg.wavelet, a, tmp, a.W, stream);
        else if (c.cfg.scheme == DWT2_SCHEME_MONOLITHIC_STAR)
            e = dwt2::launch_fused_forward(c.cfg.wavelet, c.cfg.arithmetic == DWT2_ARITH_FP64,
                                           choose_rows(c.cfg, false, a.W, a.H), buffers_of(c.cfg),
                                           choose_order(c.cfg, false, a.W, a.H), a, stream);
        else
            e = dwt2::launch_tile_forward(c.cfg.wavelet, c.cfg.scheme, a, stream);
        if (e != hipSuccess) return hip_status(e);
    }
    if (k0 < levels) {  // the remaining levels in one work-group
        dwt2::TailArgs t = tail_args(c, k0, false);
        const dwt2::FwdArgs a = forward_level(c, k0, src, src_pitch, dst, dst_pitch, workspace);
        t.in = a.in;
        t.in_pitch = a.in_pitch;
        t.out = dst;
        t.out_pitch = dst_pitch;
        const hipError_t e = dwt2::launch_fused_tail_forward(c.cfg.wavelet, t, stream);
        if (e != hipSuccess) return hip_status(e);
    }
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_inverse(dwt2_wavelet wavelet, int levels, int width, int height,
                             const float *src, ptrdiff_t src_pitch, float *dst, ptrdiff_t dst_pitch,
                             dwt2_ext ext, const dwt2_options *opt, void *workspace,
                             size_t workspace_bytes, hipStream_t stream)
{
    Checked c;
    int st = check_call(wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext, opt,
                        workspace, workspace_bytes, &c);
    if (st != DWT2_OK) return st;
    char *wsb = (char *)workspace;
    float *tmp = (float *)(wsb + c.lay.t_off);
    const int k0 = tail_start(c);
    if (k0 < levels) {  // the deepest levels in one work-group
        dwt2::TailArgs t = tail_args(c, k0, true);
        const dwt2::InvArgs a = inverse_level(c, k0, src, src_pitch, dst, dst_pitch, workspace);
        t.in = src;
        t.in_pitch = src_pitch;
        t.out = a.out;
        t.out_pitch = a.out_pitch;
        const hipError_t e = dwt2::launch_fused_tail_inverse(c.cfg.wavelet, t, stream);
        if (e != hipSuccess) return hip_status(e);
    }
    for (int k = k0 - 1; k >= 0; k--) {
        const dwt2::InvArgs a = inverse_level(c, k, src, src_pitch, dst, dst_pitch, workspace);
        hipError_t e;
        if (c.cfg.scheme == DWT2_SCHEME_ROWCOL)
            e = dwt2::launch_rowcol_inverse(c.cfg.wavelet, a, tmp, a.W, stream);
        else if (c.cfg.scheme == DWT2_SCHEME_MONOLITHIC_STAR)
            e = dwt2::launch_fused_inverse(c.cfg.wavelet, c.cfg.arithmetic == DWT2_ARITH_FP64,
                                           choose_rows(c.cfg, true, a.W, a.H), buffers_of(c.cfg),
                                           choose_order(c.cfg, true, a.W, a.H), a, stream);
        else
            e = dwt2::launch_tile_inverse(c.cfg.wavelet, c.cfg.scheme, a, stream);
        if (e != hipSuccess) return hip_status(e);
    }
    return DWT2_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free calls: the workspace is a file-scope device array of
// DWT2_NOALLOC_SCRATCH_BYTES.  Host code never uses the array's name as an
// address: its device address is looked up once per device (with that device
// current) and kept in g_scratch.

namespace {

__device__ __align__(256) unsigned char scratch[DWT2_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::atomic<void *> g_scratch[kMaxDevices];

// The current device's scratch address, looked up on its first use.
int scratch_of_current_device(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    if (dev < 0 || dev >= kMaxDevices) return DWT2_E_UNSUPPORTED;
    void *p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_status(e);
            if (!p) return DWT2_E_HIP;
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return DWT2_OK;
}

}  // namespace

DWT2_EXPORT int dwt2_transform_noalloc(int inverse, dwt2_wavelet wavelet, int levels, int width,
                                       int height, const float *src, ptrdiff_t src_pitch, float *dst,
                                       ptrdiff_t dst_pitch, dwt2_ext ext, const dwt2_options *opt,
                                       hipStream_t stream)
{
    Checked c;
    int st = check_call(wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext, opt, nullptr, 0,
                        &c, false);
    if (st != DWT2_OK) return st;
    const size_t need = c.lay.total;
    if (need > (size_t)DWT2_NOALLOC_SCRATCH_BYTES) return DWT2_E_WORKSPACE;
    void *ws = nullptr;
    if (need > 0) {
        st = scratch_of_current_device(&ws);
        if (st != DWT2_OK) return st;
    }
    return inverse ? dwt2_inverse(wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext, opt, ws,
                                  need, stream)
                   : dwt2_forward(wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext, opt, ws,
                                  need, stream);
}

DWT2_EXPORT int dwt2_transform_only(int inverse, dwt2_wavelet wavelet, int width, int height,
                                    const dwt2_options *opt, float *sink, hipStream_t stream)
{
    Config c;
    int st = parse(wavelet, DWT2_EXT_WHOLE_SYMMETRIC, opt, &c);
    if (st != DWT2_OK) return st;
    if (c.arithmetic != DWT2_ARITH_FP32 || c.scheme == DWT2_SCHEME_ROWCOL || c.fuse_tail)
        return DWT2_E_UNSUPPORTED;
    if (width < 1 || height < 1 || !sink || ((uintptr_t)sink & 3)) return DWT2_E_ARG;
    if (width < 2 || height < 2 || (long long)width * height > kMaxPixels) return DWT2_E_SIZE;
    dwt2::NoneArgs a;
    a.W = width;
    a.H = height;
    a.sink = sink;
    a.key = 0xFFFFFFFFu;  // a NaN pattern: never the sum of finite lifted samples
    const bool inv = inverse != 0;
    const hipError_t e =
        c.scheme == DWT2_SCHEME_MONOLITHIC_STAR
            ? dwt2::launch_fused_none(inv, c.wavelet, choose_rows(c, inv, width, height), buffers_of(c),
                                      choose_order(c, inv, width, height), a, stream)
            : dwt2::launch_tile_none(inv, c.wavelet, c.scheme, a, stream);
    return hip_status(e);
}

// ---------------------------------------------------------------------------
// Batched calls.  Workspace: [image records | tile-start table | each image's
// LL ping-pong, laid out as for the single-image call], each part 256-aligned.

// Tile-height table: one byte per image and level, rows of `count` bytes
// padded to a multiple of 4 (the upload copies whole words).
static size_t rows_stride(int count) { return ((size_t)count + 3) & ~(size_t)3; }

size_t dwt2::batch_table_bytes(int count, int lmax)
{
    return align_up(sizeof(dwt2::BatchImage) * (size_t)count) +
           align_up(sizeof(int) * (size_t)lmax * (size_t)(count + 1)) +
           align_up(rows_stride(count) * (size_t)lmax);
}

namespace {

struct Interval {
    uintptr_t lo, hi;
    bool writes;
};

// True when some written range overlaps any other range.  Sorting by start,
// an overlap of a pair always shows against the running maximum end of the
// earlier ranges of the relevant kind.
bool any_write_overlap(std::vector<Interval> &v)
{
    std::sort(v.begin(), v.end(), [](const Interval &a, const Interval &b) { return a.lo < b.lo; });
    uintptr_t end_any = 0, end_w = 0;
    for (const Interval &r : v) {
        if (r.writes ? r.lo < end_any : r.lo < end_w) return true;
        end_any = std::max(end_any, r.hi);
        if (r.writes) end_w = std::max(end_w, r.hi);
    }
    return false;
}

struct BatchPlan {
    Config cfg;
    int lmax = 0;
    size_t rec_off = 0, tab_off = 0, rows_off = 0, idx_off = 0, total = 0;
    long long idx_level_off[dwt2::kBatchMaxLevels] = {};  // tiles before level k in the index
    std::vector<dwt2::BatchImage> rec;  // buffers as offsets until bound to a workspace
    std::vector<size_t> buf_off[2];
    std::vector<int> start;             // lmax x (count + 1)
    std::vector<unsigned char> rows;    // lmax x rows_stride(count): tile height per image
    std::vector<std::pair<size_t, size_t>> spans;  // (src bytes, dst bytes)
};

// Tile heights of batched level k.  An image level whose size dwt2_autotune
// recorded takes the recorded height (FP32 lifting).  The others take, per
// wavelet, the tallest built height, or a shorter one when the launch would
// otherwise have fewer work-groups than the largest fill threshold among
// their wavelets: step s takes the s-th height down from the tallest (the
// shortest when a wavelet has fewer), and the launch uses the smallest step
// that reaches that threshold (else the largest), as the single-image rule
// does for one image.  FP64 lifting is
// built at one height per wavelet.  Fills rows[i] (0 without level k) and
// returns the launch's tile count.
long long batch_level_rows(const BatchPlan &p, bool inverse, int k, unsigned char *rows)
{
    const int count = (int)p.rec.size();
    const bool fp64 = p.cfg.arithmetic == DWT2_ARITH_FP64;
    auto level_wh = [&](const dwt2::BatchImage &r, int *w, int *h) {
        *w = (int)(((long long)r.W + (1LL << k) - 1) >> k);
        *h = (int)(((long long)r.H + (1LL << k) - 1) >> k);
    };
    auto height_at = [](int wavelet, int step) {
        int n = 0;
        while (n < dwt2::kFusedRowsMax && dwt2::kFusedRows[wavelet][n] > 0) n++;
        return dwt2::kFusedRows[wavelet][std::max(0, n - 1 - step)];
    };
    std::vector<int> tuned_rows(count, 0);
    long long fixed = 0;  // tiles of images whose height does not depend on the step
    long long fill = 0;   // the launch's fill threshold
    for (int i = 0; i < count; i++) {
        const dwt2::BatchImage &r = p.rec[i];
        if (r.levels <= k) continue;
        int w, h;
        level_wh(r, &w, &h);
        Config c = p.cfg;
        c.wavelet = r.wavelet;
        TuneVal v;
        if (fp64) tuned_rows[i] = dwt2::kFusedRowsFp64[r.wavelet];
        else if (tuned(c, inverse, w, h, &v)) tuned_rows[i] = v.rows;
        if (tuned_rows[i]) fixed += dwt2::fused_tile_count(r.wavelet, tuned_rows[i], w, h);
        else fill = std::max(fill, kFillTiles[r.wavelet]);
    }
    constexpr int kSteps = dwt2::kFusedRowsMax;
    int step = kSteps - 1;
    for (int st = 0; st < kSteps; st++) {
        long long total = fixed;
        for (int i = 0; i < count; i++) {
            const dwt2::BatchImage &r = p.rec[i];
            if (r.levels <= k || tuned_rows[i]) continue;
            int w, h;
            level_wh(r, &w, &h);
            total += dwt2::fused_tile_count(r.wavelet, height_at(r.wavelet, st), w, h);
        }
        if (total >= fill) {
            step = st;
            break;
        }
    }
    long long total = 0;
    for (int i = 0; i < count; i++) {
        const dwt2::BatchImage &r = p.rec[i];
        rows[i] = 0;
        if (r.levels <= k) continue;
        int w, h;
        level_wh(r, &w, &h);
        const int rb = tuned_rows[i] ? tuned_rows[i] : height_at(r.wavelet, step);
        rows[i] = (unsigned char)rb;
        total += dwt2::fused_tile_count(r.wavelet, rb, w, h);
    }
    return total;
}

int plan_batch(const dwt2_image *images, int count, dwt2_ext ext, const dwt2_options *opt,
               bool inverse, BatchPlan *p)
{
    static_assert(DWT2_BATCH_MAX <= 65536, "image numbers in the tile-image index are 16-bit");
    static_assert(kMaxLevels <= dwt2::kBatchMaxLevels, "levels of the tile-image index");
    if (count < 0 || count > DWT2_BATCH_MAX || (count > 0 && !images)) return DWT2_E_ARG;
    int st = parse(DWT2_CDF53, ext, opt, &p->cfg);
    if (st != DWT2_OK) return st;
    if (p->cfg.scheme != DWT2_SCHEME_MONOLITHIC_STAR || p->cfg.tile_rows != 0 || p->cfg.lds_buffers != 0 ||
        p->cfg.tile_order != 0 || p->cfg.fuse_tail != 0)
        return DWT2_E_UNSUPPORTED;
    p->rec.resize(count);
    p->buf_off[0].resize(count);
    p->buf_off[1].resize(count);
    p->spans.resize(count);
    size_t img_bytes = 0;
    for (int i = 0; i < count; i++) {
        const dwt2_image &im = images[i];
        Config c;
        st = parse((dwt2_wavelet)im.wavelet, ext, opt, &c);
        if (st != DWT2_OK) return st;
        int ws[kMaxLevels], hs[kMaxLevels];
        st = geometry(im.levels, im.width, im.height, ws, hs);
        if (st != DWT2_OK) return st;
        if (!im.src || !im.dst) return DWT2_E_ARG;
        if (im.src_pitch < im.width || im.dst_pitch < im.width) return DWT2_E_ARG;
        if (!span_fits(im.src_pitch, im.width, im.height) || !span_fits(im.dst_pitch, im.width, im.height))
            return DWT2_E_ARG;
        if (((uintptr_t)im.src & 3) || ((uintptr_t)im.dst & 3)) return DWT2_E_ARG;
        const Layout L = layout(DWT2_SCHEME_MONOLITHIC_STAR, im.levels, ws, hs);
        p->buf_off[0][i] = img_bytes + L.a_off;
        p->buf_off[1][i] = img_bytes + L.b_off;
        img_bytes += L.total;
        p->spans[i] = {span_bytes(im.src_pitch, im.width, im.height),
                       span_bytes(im.dst_pitch, im.width, im.height)};
        dwt2::BatchImage &r = p->rec[i];
        r.src = im.src;
        r.dst = im.dst;
        r.buf[0] = r.buf[1] = nullptr;
        r.src_pitch = im.src_pitch;
        r.dst_pitch = im.dst_pitch;
        r.W = im.width;
        r.H = im.height;
        r.wavelet = im.wavelet;
        r.levels = im.levels;
        p->lmax = std::max(p->lmax, im.levels);
    }
    // Tile heights and starts per level; every level's total must index with
    // an int.  The tile-image index is sized for every image's tiles at its
    // wavelet's shortest height (an upper bound whatever heights a call
    // picks, so the workspace size does not depend on the direction or the
    // tuned table); the levels' index regions follow each other.
    const size_t rs = rows_stride(count);
    p->start.assign((size_t)p->lmax * (count + 1), 0);
    p->rows.assign((size_t)p->lmax * rs, 0);
    long long idx_bound = 0, idx_used = 0;
    for (int i = 0; i < count; i++) {
        const dwt2::BatchImage &r = p->rec[i];
        for (int k = 0; k < r.levels; k++) {
            const int w = (int)(((long long)r.W + (1LL << k) - 1) >> k);
            const int h = (int)(((long long)r.H + (1LL << k) - 1) >> k);
            idx_bound += dwt2::fused_tile_count(r.wavelet, dwt2::kFusedRows[r.wavelet][0], w, h);
        }
    }
    for (int k = 0; k < p->lmax; k++) {
        unsigned char *rows = &p->rows[(size_t)k * rs];
        if (batch_level_rows(*p, inverse, k, rows) > INT_MAX - 8) return DWT2_E_ARG;
        int *s = &p->start[(size_t)k * (count + 1)];
        long long acc = 0;
        for (int i = 0; i < count; i++) {
            s[i] = (int)acc;
            const dwt2::BatchImage &r = p->rec[i];
            if (r.levels > k) {
                const int w = (int)(((long long)r.W + (1LL << k) - 1) >> k);
                const int h = (int)(((long long)r.H + (1LL << k) - 1) >> k);
                acc += dwt2::fused_tile_count(r.wavelet, rows[i], w, h);
            }
        }
        s[count] = (int)acc;
        p->idx_level_off[k] = idx_used;
        idx_used += acc;
    }
    if (idx_used > idx_bound) return DWT2_E_ARG;  // not reached: heights >= the shortest
    p->rec_off = 0;
    p->tab_off = align_up(sizeof(dwt2::BatchImage) * (size_t)count);
    p->rows_off = p->tab_off + align_up(sizeof(int) * (size_t)p->lmax * (size_t)(count + 1));
    p->idx_off = dwt2::batch_table_bytes(count, p->lmax);
    const size_t img_base = p->idx_off + align_up(sizeof(unsigned short) * (size_t)idx_bound);
    for (int i = 0; i < count; i++) {
        p->buf_off[0][i] += img_base;
        p->buf_off[1][i] += img_base;
    }
    p->total = img_base + img_bytes;
    return DWT2_OK;
}

int run_batch(bool inverse, const dwt2_image *images, int count, dwt2_ext ext,
              const dwt2_options *opt, void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    BatchPlan p;
    int st = plan_batch(images, count, ext, opt, inverse, &p);
    if (st != DWT2_OK) return st;
    if (count == 0) return DWT2_OK;
    if (!workspace || workspace_bytes < p.total) return DWT2_E_WORKSPACE;
    if ((uintptr_t)workspace & (kAlign - 1)) return DWT2_E_ARG;
    std::vector<Interval> iv;
    iv.reserve(2 * (size_t)count + 1);
    const uintptr_t w0 = (uintptr_t)workspace;
    iv.push_back({w0, w0 + p.total, true});
    for (int i = 0; i < count; i++) {
        const uintptr_t s0 = (uintptr_t)images[i].src, d0 = (uintptr_t)images[i].dst;
        iv.push_back({s0, s0 + p.spans[i].first, false});
        iv.push_back({d0, d0 + p.spans[i].second, true});
    }
    if (any_write_overlap(iv)) return DWT2_E_ALIAS;

    char *wsb = (char *)workspace;
    for (int i = 0; i < count; i++) {
        p.rec[i].buf[0] = (float *)(wsb + p.buf_off[0][i]);
        p.rec[i].buf[1] = (float *)(wsb + p.buf_off[1][i]);
    }
    hipError_t e = dwt2::launch_upload(wsb + p.rec_off, p.rec.data(),
                                       sizeof(dwt2::BatchImage) * (size_t)count, stream);
    if (e == hipSuccess)
        e = dwt2::launch_upload(wsb + p.tab_off, p.start.data(), sizeof(int) * p.start.size(), stream);
    if (e == hipSuccess) e = dwt2::launch_upload(wsb + p.rows_off, p.rows.data(), p.rows.size(), stream);
    if (e == hipSuccess) {
        dwt2::BatchIndexArgs ia = {};
        ia.start = (const int *)(wsb + p.tab_off);
        ia.index = (unsigned short *)(wsb + p.idx_off);
        ia.count = count;
        ia.lmax = p.lmax;
        std::copy(p.idx_level_off, p.idx_level_off + p.lmax, ia.off);
        e = dwt2::launch_batch_index(ia, stream);
    }
    if (e != hipSuccess) return hip_status(e);

    dwt2::BatchLevel b;
    b.imgs = (const dwt2::BatchImage *)(wsb + p.rec_off);
    b.count = count;
    b.ll_gain = p.cfg.norm == DWT2_NORM_PAPER ? 2.0f : 1.0f;
    const int norm = p.cfg.norm;
    for (int wv = 0; wv < 3; wv++)
        b.s[wv] = inverse ? inverse_scale(wv, norm) : level_scale(wv, norm);
    const bool fp64 = p.cfg.arithmetic == DWT2_ARITH_FP64;
    bool has_dd = false;
    for (int i = 0; i < count; i++) has_dd |= images[i].wavelet == DWT2_DD137;
    for (int j = 0; j < p.lmax; j++) {
        const int k = inverse ? p.lmax - 1 - j : j;
        b.level = k;
        b.start = (const int *)(wsb + p.tab_off) + (size_t)k * (count + 1);
        b.rows = (const unsigned char *)(wsb + p.rows_off) + (size_t)k * rows_stride(count);
        b.tile_image = (const unsigned short *)(wsb + p.idx_off) + p.idx_level_off[k];
        b.ntiles = p.start[(size_t)k * (count + 1) + count];
        b.quantum = norm == DWT2_NORM_PAPER ? ldexpf(1.0f, k) : 1.0f;
        e = inverse ? dwt2::launch_batch_inverse(fp64, has_dd, b, stream)
                    : dwt2::launch_batch_forward(fp64, has_dd, b, stream);
        if (e != hipSuccess) return hip_status(e);
    }
    return DWT2_OK;
}

}  // namespace

DWT2_EXPORT int dwt2_batch_workspace_bytes(const dwt2_image *images, int count,
                                           const dwt2_options *opt, size_t *bytes)
{
    if (!bytes) return DWT2_E_ARG;
    BatchPlan p;
    const int st = plan_batch(images, count, DWT2_EXT_WHOLE_SYMMETRIC, opt, false, &p);
    if (st != DWT2_OK) return st;
    *bytes = p.total;
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_batch_tile_rows(int inverse, const dwt2_image *images, int count,
                                     const dwt2_options *opt, int level, int *rows)
{
    if (!rows && count > 0) return DWT2_E_ARG;
    BatchPlan p;
    const int st = plan_batch(images, count, DWT2_EXT_WHOLE_SYMMETRIC, opt, inverse != 0, &p);
    if (st != DWT2_OK) return st;
    if (level < 0) return DWT2_E_ARG;
    for (int i = 0; i < count; i++)
        rows[i] = level < p.lmax ? p.rows[(size_t)level * rows_stride(count) + i] : 0;
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_forward_batch(const dwt2_image *images, int count, dwt2_ext ext,
                                   const dwt2_options *opt, void *workspace, size_t workspace_bytes,
                                   hipStream_t stream)
{
    return run_batch(false, images, count, ext, opt, workspace, workspace_bytes, stream);
}

DWT2_EXPORT int dwt2_inverse_batch(const dwt2_image *images, int count, dwt2_ext ext,
                                   const dwt2_options *opt, void *workspace, size_t workspace_bytes,
                                   hipStream_t stream)
{
    return run_batch(true, images, count, ext, opt, workspace, workspace_bytes, stream);
}

// ---------------------------------------------------------------------------
// Tile-height autotuning.

namespace {

// Autotuning.  Every candidate (built height x tile order) of a level is
// captured once as a HIP graph of `repeats` back-to-back launches on a
// private stream; the graphs are replayed in kTunePasses interleaved passes
// (each pass starts at another candidate, after one untimed replay of every
// candidate), each replay timed with events, so all candidates see the same
// device state and clocks and no host launch gap enters the times.  A
// candidate's time is the median of its passes.  The rule's candidate is
// kept unless another one is faster by more than the spread (max - min over
// the passes) of either of the two: a difference inside the noise does not
// override the rule.
constexpr int kTunePasses = 5;

struct TuneRun {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<hipGraphExec_t> exec;
    std::vector<hipGraph_t> graph;
    // Destroys the graphs (after the stream has finished their replays).
    void release_graphs()
    {
        for (hipGraphExec_t g : exec)
            if (g) (void)hipGraphExecDestroy(g);
        for (hipGraph_t g : graph)
            if (g) (void)hipGraphDestroy(g);
        exec.clear();
        graph.clear();
    }
};

hipError_t capture_level(bool inverse, const Checked &c, const void *args, int rows, int order, int repeats,
                         hipStream_t s, hipGraph_t *g, hipGraphExec_t *ge)
{
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int i = 0; i < repeats && le == hipSuccess; i++)
        le = inverse ? dwt2::launch_fused_inverse(c.cfg.wavelet, false, rows, buffers_of(c.cfg), order,
                                                  *(const dwt2::InvArgs *)args, s)
                     : dwt2::launch_fused_forward(c.cfg.wavelet, false, rows, buffers_of(c.cfg), order,
                                                  *(const dwt2::FwdArgs *)args, s);
    e = hipStreamEndCapture(s, g);  // always ends the capture
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    return hipGraphInstantiate(ge, *g, nullptr, nullptr, 0);
}

int tune(bool inverse, const Checked &c, const float *src, ptrdiff_t src_pitch, float *dst,
         ptrdiff_t dst_pitch, void *workspace, int repeats, TuneRun &run)
{
    const int *cand = dwt2::kFusedRows[c.cfg.wavelet];
    int nrows = 0;
    while (nrows < dwt2::kFusedRowsMax && cand[nrows] > 0) nrows++;
    constexpr int kOrders[2] = {DWT2_ORDER_RUNS, DWT2_ORDER_BANDS};
    const int ncand = 2 * nrows;
    for (int j = 0; j < c.levels; j++) {
        const int k = inverse ? c.levels - 1 - j : j;
        dwt2::FwdArgs fa;
        dwt2::InvArgs ia;
        const void *args;
        if (inverse) {
            ia = inverse_level(c, k, src, src_pitch, dst, dst_pitch, workspace);
            args = &ia;
        } else {
            fa = forward_level(c, k, src, src_pitch, dst, dst_pitch, workspace);
            args = &fa;
        }
        const int W = c.ws[k], H = c.hs[k];
        // Every replay writes the same level output, so the next level reads
        // this level's result.
        run.exec.assign(ncand, nullptr);
        run.graph.assign(ncand, nullptr);
        for (int q = 0; q < ncand; q++) {
            const hipError_t e = capture_level(inverse, c, args, cand[q / 2], kOrders[q % 2], repeats, run.s,
                                               &run.graph[q], &run.exec[q]);
            if (e != hipSuccess) return hip_status(e);
        }
        for (int q = 0; q < ncand; q++) {
            const hipError_t e = hipGraphLaunch(run.exec[q], run.s);
            if (e != hipSuccess) return hip_status(e);
        }
        float ms[2 * dwt2::kFusedRowsMax][kTunePasses];
        for (int pass = 0; pass < kTunePasses; pass++)
            for (int i = 0; i < ncand; i++) {
                const int q = (i + pass) % ncand;
                hipError_t e = hipEventRecord(run.e0, run.s);
                if (e == hipSuccess) e = hipGraphLaunch(run.exec[q], run.s);
                if (e == hipSuccess) e = hipEventRecord(run.e1, run.s);
                if (e == hipSuccess) e = hipEventSynchronize(run.e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms[q][pass], run.e0, run.e1);
                if (e != hipSuccess) return hip_status(e);
            }
        float med[2 * dwt2::kFusedRowsMax], spread[2 * dwt2::kFusedRowsMax];
        for (int q = 0; q < ncand; q++) {
            float v[kTunePasses];
            std::copy(ms[q], ms[q] + kTunePasses, v);
            std::sort(v, v + kTunePasses);
            med[q] = v[kTunePasses / 2];
            spread[q] = v[kTunePasses - 1] - v[0];
        }
        const int rule_r = rule_rows(c.cfg.wavelet, W, H), rule_o = rule_order(W, H);
        int ruleq = 0;
        for (int q = 0; q < ncand; q++)
            if (cand[q / 2] == rule_r && kOrders[q % 2] == rule_o) ruleq = q;
        int best = 0;
        for (int q = 1; q < ncand; q++)
            if (med[q] < med[best]) best = q;
        const int pick = med[best] < med[ruleq] - std::max(spread[best], spread[ruleq]) ? best : ruleq;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            const TuneKey key{c.cfg.wavelet, inverse ? 1 : 0, W, H};
            if (g_tune.size() < kTuneMax || g_tune.count(key))
                g_tune[key] = TuneVal{cand[pick / 2], kOrders[pick % 2]};
            g_tune_size.store(g_tune.size(), std::memory_order_release);
        }
        run.release_graphs();  // the last replay has completed (event sync)
    }
    return DWT2_OK;
}

// One line of the exported table: "wavelet inverse width height rows order",
// or without the order (0: the rule decides).
bool parse_line(const char *p, const char *end, TuneKey *key, TuneVal *val)
{
    long long v[6] = {0, 0, 0, 0, 0, 0};
    int fields = 0;
    for (int i = 0; i < 6; i++) {
        if (i == 5 && p == end) break;  // the order is optional
        if (i > 0) {
            if (p >= end || *p != ' ') return false;
            p++;
        }
        if (p >= end || *p < '0' || *p > '9') return false;
        long long x = 0;
        while (p < end && *p >= '0' && *p <= '9') {
            x = x * 10 + (*p - '0');
            if (x > INT_MAX) return false;
            p++;
        }
        v[i] = x;
        fields++;
    }
    if (p != end || fields < 5) return false;
    const int wavelet = (int)v[0], inverse = (int)v[1], w = (int)v[2], h = (int)v[3];
    if (wavelet > DWT2_DD137 || inverse > 1 || w < 2 || h < 2) return false;
    if (!dwt2::fused_rows_supported(wavelet, false, (int)v[4])) return false;
    if (v[5] != 0 && v[5] != DWT2_ORDER_RUNS && v[5] != DWT2_ORDER_BANDS) return false;
    *key = TuneKey{wavelet, inverse, w, h};
    *val = TuneVal{(int)v[4], (int)v[5]};
    return true;
}

}  // namespace

DWT2_EXPORT int dwt2_autotune(int inverse, dwt2_wavelet wavelet, int levels, int width, int height,
                              const float *src, ptrdiff_t src_pitch, float *dst, ptrdiff_t dst_pitch,
                              dwt2_ext ext, const dwt2_options *opt, void *workspace,
                              size_t workspace_bytes, int repeats, hipStream_t stream)
{
    Checked c;
    int st = check_call(wavelet, levels, width, height, src, src_pitch, dst, dst_pitch, ext, opt,
                        workspace, workspace_bytes, &c);
    if (st != DWT2_OK) return st;
    if (c.cfg.scheme != DWT2_SCHEME_MONOLITHIC_STAR || c.cfg.arithmetic != DWT2_ARITH_FP32 ||
        c.cfg.tile_rows != 0 || c.cfg.lds_buffers != 0 || c.cfg.tile_order != 0 || c.cfg.fuse_tail != 0)
        return DWT2_E_UNSUPPORTED;
    if (repeats < 1 || repeats > 1000) return DWT2_E_ARG;
    // The caller's earlier work (which may write src) completes first; the
    // candidates then run on a private stream, and the call returns when
    // they are done, with the result in dst.
    hipError_t e = hipStreamSynchronize(stream);
    TuneRun run;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&run.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&run.e0);
    if (e == hipSuccess) e = hipEventCreate(&run.e1);
    st = e == hipSuccess ? tune(inverse != 0, c, src, src_pitch, dst, dst_pitch, workspace, repeats, run)
                         : hip_status(e);
    if (run.s) {
        const hipError_t es = hipStreamSynchronize(run.s);
        if (st == DWT2_OK && es != hipSuccess) st = hip_status(es);
    }
    run.release_graphs();
    if (run.e1) (void)hipEventDestroy(run.e1);
    if (run.e0) (void)hipEventDestroy(run.e0);
    if (run.s) (void)hipStreamDestroy(run.s);
    return st;
}

DWT2_EXPORT int dwt2_tile_rows(int inverse, dwt2_wavelet wavelet, int width, int height,
                               const dwt2_options *opt, int *rows)
{
    if (!rows) return DWT2_E_ARG;
    Config cfg;
    int st = parse(wavelet, DWT2_EXT_WHOLE_SYMMETRIC, opt, &cfg);
    if (st != DWT2_OK) return st;
    if (cfg.scheme != DWT2_SCHEME_MONOLITHIC_STAR) return DWT2_E_UNSUPPORTED;
    if (width < 1 || height < 1) return DWT2_E_ARG;
    if (width < 2 || height < 2 || (long long)width * height > kMaxPixels) return DWT2_E_SIZE;
    *rows = choose_rows(cfg, inverse != 0, width, height);
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_tile_order(int inverse, dwt2_wavelet wavelet, int width, int height,
                                const dwt2_options *opt, int *order)
{
    if (!order) return DWT2_E_ARG;
    Config cfg;
    int st = parse(wavelet, DWT2_EXT_WHOLE_SYMMETRIC, opt, &cfg);
    if (st != DWT2_OK) return st;
    if (cfg.scheme != DWT2_SCHEME_MONOLITHIC_STAR) return DWT2_E_UNSUPPORTED;
    if (width < 1 || height < 1) return DWT2_E_ARG;
    if (width < 2 || height < 2 || (long long)width * height > kMaxPixels) return DWT2_E_SIZE;
    *order = choose_order(cfg, inverse != 0, width, height);
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_tune_export(char *buf, size_t cap, size_t *len)
{
    if (!len || (cap > 0 && !buf)) return DWT2_E_ARG;
    std::string text;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto &kv : g_tune) {
            const TuneKey &k = kv.first;
            text += std::to_string(k[0]) + ' ' + std::to_string(k[1]) + ' ' + std::to_string(k[2]) +
                    ' ' + std::to_string(k[3]) + ' ' + std::to_string(kv.second.rows) + ' ' +
                    std::to_string(kv.second.order) + '\n';
        }
    }
    *len = text.size();
    if (cap <= text.size()) {
        if (cap > 0) buf[0] = '\0';
        return DWT2_E_SIZE;
    }
    std::copy(text.begin(), text.end(), buf);
    buf[text.size()] = '\0';
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_tune_import(const char *text)
{
    if (!text) return DWT2_E_ARG;
    std::vector<std::pair<TuneKey, TuneVal>> add;
    for (const char *p = text; *p;) {
        const char *nl = p;
        while (*nl && *nl != '\n') nl++;
        TuneKey key;
        TuneVal val;
        if (!parse_line(p, nl, &key, &val)) return DWT2_E_ARG;
        add.emplace_back(key, val);
        p = *nl ? nl + 1 : nl;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::set<TuneKey> fresh;
    for (const auto &kv : add)
        if (!g_tune.count(kv.first)) fresh.insert(kv.first);
    if (g_tune.size() + fresh.size() > kTuneMax) return DWT2_E_SIZE;
    for (const auto &kv : add) g_tune[kv.first] = kv.second;
    g_tune_size.store(g_tune.size(), std::memory_order_release);
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_tune_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_size.store(0, std::memory_order_release);
    return DWT2_OK;
}
