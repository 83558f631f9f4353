// rowcol_kernels.hip -- the row-column separable lifting baseline (Sec. 2,
// "Sweldens Scheme": row--column methods process all horizontal steps before
// all vertical ones, with the intermediate result in global memory).
//
// Forward level:  rows pass  in  -> tmp = [L | H] per row (unscaled lifting)
//                 cols pass  tmp -> LL / HL / LH / HH (Mallat), 2-D scaling
// Inverse level:  cols pass  coefficients -> tmp (rows interleaved back)
//                 rows pass  tmp -> image
// HBM traffic is 16 B per pixel per level (two reads, two writes) against the
// fused kernel's 8 B.
//
// Rows pass: one wavefront per row segment, two lifting pairs (four samples)
// per lane, neighbours exchanged with wave shuffles; K pairs of halo per side.
// Cols pass: one lane per column, streaming down a segment of rows with a
// register pipeline of K stages (each stage = one predict/update pair); the
// segment is shorter on small levels, so that they still have enough
// work-groups.
#include "dwt2_internal.h"

namespace dwt2 {
namespace {

constexpr int RT = 256;           // threads per block
constexpr int RW = 4;             // waves per block (rows pass: one row each)
constexpr int NPW = 128;          // lifting pairs per wave in the rows pass
constexpr int CSEG = 64;          // output pairs per column segment (large levels)
constexpr int CSEG_MIN = 8;       // shortest segment (small levels)
constexpr int kColBlocks = 1024;  // column work-groups a level should have (four per CU)

// Column segment length: CSEG, halved down to CSEG_MIN while the column grid
// has fewer than kColBlocks work-groups.  Each segment re-reads 2K halo
// pairs, so short segments cost reads; a small level is latency-bound
// instead (each lane streams its segment one pair after another).
int col_segment(int W, int QH)
{
    const long long gx = (W + RT - 1) / RT;
    int seg = CSEG;
    while (seg > CSEG_MIN && gx * ((QH + seg - 1) / seg) < kColBlocks) seg /= 2;
    return seg;
}

// ---------------------------------------------------------------------------
// Rows pass, forward: in (W x H) -> tmp [L | H]
// ---------------------------------------------------------------------------
template <int WAV>
__global__ __launch_bounds__(RT) void k_rows_forward(const float *in, ptrdiff_t in_pitch, float *tmp,
                                                     ptrdiff_t tmp_pitch, int W, int H)
{
    using L = Lift<WAV>;
    constexpr int K = L::K, OUTP = NPW - 2 * K;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
    const int row = blockIdx.y * RW + wv;
    if (row >= H) return;
    const int QW = (W + 1) >> 1, WH = W >> 1;
    const int n0 = blockIdx.x * OUTP - K + 2 * lane;  // first of this lane's two pairs
    const float *src = in + (ptrdiff_t)row * in_pitch;
    float L0 = src[ws_mirror(2 * n0, W)], H0 = src[ws_mirror(2 * n0 + 1, W)];
    float L1 = src[ws_mirror(2 * n0 + 2, W)], H1 = src[ws_mirror(2 * n0 + 3, W)];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const float p = L::p(k), u = L::u(k);
        const float L0n = __shfl_down(L0, 1);
        H0 = fmaf(p, L0 + L1, H0);
        H1 = fmaf(p, L1 + L0n, H1);
        const float H1p = __shfl_up(H1, 1);
        L0 = fmaf(u, H1p + H0, L0);
        L1 = fmaf(u, H0 + H1, L1);
    }
    float *dst = tmp + (ptrdiff_t)row * tmp_pitch;
    const int loc = 2 * lane;
#pragma unroll
    for (int e = 0; e < 2; e++) {
        const int n = n0 + e;
        if (loc + e < K || loc + e >= NPW - K || n >= QW) continue;
        dst[n] = e ? L1 : L0;
        if (n < WH) dst[QW + n] = e ? H1 : H0;
    }
}

// ---------------------------------------------------------------------------
// Rows pass, inverse: tmp [L | H] -> out (W x H)
// ---------------------------------------------------------------------------
template <int WAV>
__global__ __launch_bounds__(RT) void k_rows_inverse(const float *tmp, ptrdiff_t tmp_pitch, float *out,
                                                     ptrdiff_t out_pitch, int W, int H)
{
    using L = Lift<WAV>;
    constexpr int K = L::K, OUTP = NPW - 2 * K;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
    const int row = blockIdx.y * RW + wv;
    if (row >= H) return;
    const int QW = (W + 1) >> 1;
    const int n0 = blockIdx.x * OUTP - K + 2 * lane;
    const float *src = tmp + (ptrdiff_t)row * tmp_pitch;
    // L and H of a mirrored pair position: mirroring keeps sample parity.
    float L0 = src[ws_mirror(2 * n0, W) >> 1], H0 = src[QW + (ws_mirror(2 * n0 + 1, W) >> 1)];
    float L1 = src[ws_mirror(2 * n0 + 2, W) >> 1], H1 = src[QW + (ws_mirror(2 * n0 + 3, W) >> 1)];
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
        const int k = K - 1 - kk;
        const float p = L::p(k), u = L::u(k);
        const float H1p = __shfl_up(H1, 1);
        L0 = fmaf(-u, H1p + H0, L0);
        L1 = fmaf(-u, H0 + H1, L1);
        const float L0n = __shfl_down(L0, 1);
        H0 = fmaf(-p, L0 + L1, H0);
        H1 = fmaf(-p, L1 + L0n, H1);
    }
    float *dst = out + (ptrdiff_t)row * out_pitch;
    const int loc = 2 * lane;
#pragma unroll
    for (int e = 0; e < 2; e++) {
        const int n = n0 + e;
        if (loc + e < K || loc + e >= NPW - K || n >= QW) continue;
        dst[2 * n] = e ? L1 : L0;
        if (2 * n + 1 < W) dst[2 * n + 1] = e ? H1 : H0;
    }
}

// ---------------------------------------------------------------------------
// Cols pass, forward: tmp (W x H) -> Mallat subbands, with the 2-D scaling.
// Pipeline stage k keeps the pending pair (Lk, Hk) and its previous output H.
// ---------------------------------------------------------------------------
template <int WAV>
__global__ __launch_bounds__(RT) void k_cols_forward(const float *tmp, ptrdiff_t tmp_pitch, FwdArgs a, int cseg)
{
    using L = Lift<WAV>;
    constexpr int K = L::K;
    const int c = blockIdx.x * RT + threadIdx.x;
    const int W = a.W, H = a.H;
    if (c >= W) return;
    const int QW = (W + 1) >> 1, QH = (H + 1) >> 1, HH_ = H >> 1;
    const int r0 = blockIdx.y * cseg, r1 = min(r0 + cseg, QH);
    const bool lowcol = c < QW;  // column of the horizontal L half
    const float sl = lowcol ? a.s.ll : 1.0f, sh = lowcol ? 1.0f : a.s.hh;
    float *lo_base = lowcol ? a.ll : a.det;
    const ptrdiff_t lo_pitch = lowcol ? a.ll_pitch : a.det_pitch;
    const float *col = tmp + c;

    float pl[K], ph[K], php[K];
    const int n = r1 - r0 + 2 * K;
    for (int i = 0; i < n; i++) {
        const int t = r0 - K + i;
        float lin = col[(ptrdiff_t)ws_mirror(2 * t, H) * tmp_pitch];
        float hin = col[(ptrdiff_t)ws_mirror(2 * t + 1, H) * tmp_pitch];
        bool live = true;
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (!live) break;
            if (i == k) {  // prime stage k with its first input
                pl[k] = lin;
                ph[k] = hin;
                php[k] = 0.0f;
                live = false;
                break;
            }
            const float ho = fmaf(L::p(k), pl[k] + lin, ph[k]);
            const float lo = fmaf(L::u(k), php[k] + ho, pl[k]);
            php[k] = ho;
            pl[k] = lin;
            ph[k] = hin;
            lin = lo;
            hin = ho;
        }
        const int to = t - K;
        if (!live || to < r0) continue;
        lo_base[(ptrdiff_t)to * lo_pitch + c] = lin * sl;
        if (to < HH_) a.det[(ptrdiff_t)(QH + to) * a.det_pitch + c] = hin * sh;
    }
}

// ---------------------------------------------------------------------------
// Cols pass, inverse: Mallat subbands -> tmp, rows interleaved back.
// Inverse stage (one pair, last pair first), fed (L_{t+1}, H_{t+1}):
//   L'_{t+1} = L_{t+1} - u (H_t + H_{t+1})       (undo the update)
//   H'_t     = H_t - p (L'_t + L'_{t+1})          (undo the predict)
// and emits (L'_t, H'_t).  State: previous L' and the pending input H.
// ---------------------------------------------------------------------------
template <int WAV>
__global__ __launch_bounds__(RT) void k_cols_inverse(InvArgs a, float *tmp, ptrdiff_t tmp_pitch, int cseg)
{
    using L = Lift<WAV>;
    constexpr int K = L::K;
    const int c = blockIdx.x * RT + threadIdx.x;
    const int W = a.W, H = a.H;
    if (c >= W) return;
    const int QW = (W + 1) >> 1, QH = (H + 1) >> 1;
    const int r0 = blockIdx.y * cseg, r1 = min(r0 + cseg, QH);
    const bool lowcol = c < QW;
    const float sl = lowcol ? a.inv_s.ll : 1.0f, sh = lowcol ? 1.0f : a.inv_s.hh;
    const float *lo_base = lowcol ? a.ll : a.det;
    const ptrdiff_t lo_pitch = lowcol ? a.ll_pitch : a.det_pitch;
    float *col = tmp + c;

    float plp[K], ph[K];
    const int n = r1 - r0 + 2 * K;
    for (int i = 0; i < n; i++) {
        const int t = r0 - K + i;
        float lin = lo_base[(ptrdiff_t)(ws_mirror(2 * t, H) >> 1) * lo_pitch + c] * sl;
        float hin = a.det[(ptrdiff_t)(QH + (ws_mirror(2 * t + 1, H) >> 1)) * a.det_pitch + c] * sh;
        bool live = true;
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
            if (!live) break;
            const int k = K - 1 - kk;
            const float p = L::p(k), u = L::u(k);
            if (i == kk) {  // prime: the H before the first input is unknown
                plp[kk] = fmaf(-u, hin, lin);
                ph[kk] = hin;
                live = false;
                break;
            }
            const float hnew = hin;
            const float lpn = fmaf(-u, ph[kk] + hnew, lin);
            const float ho = fmaf(-p, plp[kk] + lpn, ph[kk]);
            lin = plp[kk];
            hin = ho;
            plp[kk] = lpn;
            ph[kk] = hnew;
        }
        const int to = t - K;
        if (!live || to < r0) continue;
        col[(ptrdiff_t)(2 * to) * tmp_pitch] = lin;
        if (2 * to + 1 < H) col[(ptrdiff_t)(2 * to + 1) * tmp_pitch] = hin;
    }
}

}  // namespace

hipError_t launch_rowcol_forward(int wavelet, const FwdArgs &a, float *tmp, ptrdiff_t tmp_pitch,
                                 hipStream_t s)
{
    const int K = wavelet == CDF97 ? 2 : 1;
    const int QW = (a.W + 1) / 2, QH = (a.H + 1) / 2;
    const int cseg = col_segment(a.W, QH);
    const dim3 rg((QW + NPW - 2 * K - 1) / (NPW - 2 * K), (a.H + RW - 1) / RW);
    const dim3 cg((a.W + RT - 1) / RT, (QH + cseg - 1) / cseg);
    hipError_t e = hipErrorInvalidValue;
    const float *ct = tmp;
    if (wavelet == CDF53) {
        e = launch(k_rows_forward<CDF53>, rg, dim3(RT), s, a.in, a.in_pitch, tmp, tmp_pitch, a.W, a.H);
        if (e == hipSuccess) e = launch(k_cols_forward<CDF53>, cg, dim3(RT), s, ct, tmp_pitch, a, cseg);
    } else if (wavelet == CDF97) {
        e = launch(k_rows_forward<CDF97>, rg, dim3(RT), s, a.in, a.in_pitch, tmp, tmp_pitch, a.W, a.H);
        if (e == hipSuccess) e = launch(k_cols_forward<CDF97>, cg, dim3(RT), s, ct, tmp_pitch, a, cseg);
    }
    return e;
}

hipError_t launch_rowcol_inverse(int wavelet, const InvArgs &a, float *tmp, ptrdiff_t tmp_pitch,
                                 hipStream_t s)
{
    const int K = wavelet == CDF97 ? 2 : 1;
    const int QW = (a.W + 1) / 2, QH = (a.H + 1) / 2;
    const int cseg = col_segment(a.W, QH);
    const dim3 rg((QW + NPW - 2 * K - 1) / (NPW - 2 * K), (a.H + RW - 1) / RW);
    const dim3 cg((a.W + RT - 1) / RT, (QH + cseg - 1) / cseg);
    hipError_t e = hipErrorInvalidValue;
    const float *ct = tmp;
    if (wavelet == CDF53) {
        e = launch(k_cols_inverse<CDF53>, cg, dim3(RT), s, a, tmp, tmp_pitch, cseg);
        if (e == hipSuccess)
            e = launch(k_rows_inverse<CDF53>, rg, dim3(RT), s, ct, tmp_pitch, a.out, a.out_pitch, a.W, a.H);
    } else if (wavelet == CDF97) {
        e = launch(k_cols_inverse<CDF97>, cg, dim3(RT), s, a, tmp, tmp_pitch, cseg);
        if (e == hipSuccess)
            e = launch(k_rows_inverse<CDF97>, rg, dim3(RT), s, ct, tmp_pitch, a.out, a.out_pitch, a.W, a.H);
    }
    return e;
}

}  // namespace dwt2
