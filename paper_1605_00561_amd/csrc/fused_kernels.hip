// fused_kernels.hip -- the fused Monolithic* level kernels for gfx950.
//
// Scheme (Sec. 4, "Improvements"), per lifting pair:
//   barrier | T_{P1}, then the scalar T^H_{P0}, T^V_{P0}   (spatial predict)
//   barrier | S_{U1}, then the scalar S^H_{U0}, S^V_{U0}   (spatial update)
// The inverse undoes each pair in reverse: the scalar update parts, S_{-U1}
// (barrier), the scalar predict parts, T_{-P1} (barrier).
//
// Mapping.  A work-group owns one overlapping tile of 64 x (NW * RB)
// quadruples (K quadruples of halo per side, K = lifting pairs), as in the
// paper's block-based method (Sec. 6).  Lane c of wavefront w holds the
// quadruples of column c in the tile rows w, w + NW, w + 2 NW, ... in
// registers: the rows are interleaved across the wavefronts, so at any time
// the work-group's loads and stores cover NW adjacent rows, which measured
// about 9% faster than contiguous row runs per wavefront for this access
// pattern.
//   * horizontal neighbours (c +- 1) are read from the adjacent lane with DPP
//     wave shifts, which need no barrier (a wavefront runs in lockstep);
//   * vertical neighbours (r +- 1) live in another wavefront: before each
//     spatial step every wavefront publishes the two components the step
//     reads across rows (LL, HL for the predict; LH, HH for the update) to an
//     LDS plane, and the barrier the scheme places before the step makes them
//     visible.  Two plane buffers alternate between predict and update, so
//     Monolithic* keeps its two barriers per lifting pair.
// LDS is 26 KB (FP32), so occupancy is set by registers.
//
// Borders: whole-sample symmetric extension, samples read from mirrored
// positions.  Centring: each tile subtracts the rounded mean c of its middle
// quadruple row and adds c * ll_gain back to LL (exact by linearity).
// Tiles are numbered so that each XCD (work-group id mod 8) takes a
// contiguous row-major run, so neighbouring tiles share their halo in L2.
#include <string.h>

#include "dwt2_internal.h"

namespace dwt2 {
namespace {

constexpr int TX = 64;  // quadruple columns per tile (one per lane)
constexpr int NW = 4;   // wavefronts per work-group
constexpr int RB = 4;   // quadruple rows per wavefront (tile row j * NW + w)
constexpr int TY = NW * RB;
constexpr int NTHREADS = TX * NW;

enum { LL = 0, HL = 1, LH = 2, HH = 3 };

// DPP wave shifts: wave_shl:1 gives lane i the value of lane i+1, wave_shr:1
// that of lane i-1; the end lane gets 0 (it holds a halo column).
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;
__device__ __forceinline__ float from_right(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), DPP_WAVE_SHL1, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_left(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), DPP_WAVE_SHR1, 0xf, 0xf, false));
}

__device__ __forceinline__ double from_right(double v)
{
    const int2 b = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(
        double, make_int2(__builtin_amdgcn_update_dpp(0, b.x, DPP_WAVE_SHL1, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, b.y, DPP_WAVE_SHL1, 0xf, 0xf, false)));
}
__device__ __forceinline__ double from_left(double v)
{
    const int2 b = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(
        double, make_int2(__builtin_amdgcn_update_dpp(0, b.x, DPP_WAVE_SHR1, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, b.y, DPP_WAVE_SHR1, 0xf, 0xf, false)));
}

// Fused multiply-add in the arithmetic type of the kernel.
__device__ __forceinline__ float mad(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return fma(a, b, c); }

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int xcd_tile(int ntiles)
{
    const int per = gridDim.x >> 3;  // grid is a multiple of 8
    const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    return t < ntiles ? t : -1;
}

// Row planes: [buffer][component][tile row + 1][lane]; rows -1 and TY are
// padding that only halo rows read.
template <typename T>
struct Planes {
    T v[2][2][TY + 2][TX];
};

template <typename T>
__device__ __forceinline__ T &plane(Planes<T> &s, int b, int comp, int r, int c)
{
    return s.v[b][comp][r + 1][c];
}

__device__ __forceinline__ constexpr int tile_row(int j, int w) { return j * NW + w; }

// T_{P1} on one quadruple: the neighbour part of the spatial predict, from
// pre-step neighbour values (right LL, LH; lower LL, HL; lower-right LL).
template <typename T>
__device__ __forceinline__ void predict_q(T (&q)[4], T llr, T lld, T lldr, T hld, T lhr, T p, T p2)
{
    q[HL] = mad(p, llr, q[HL]);
    q[LH] = mad(p, lld, q[LH]);
    q[HH] = mad(p2, lldr, mad(p, hld, mad(p, lhr, q[HH])));
}

// S_{U1} on one quadruple: the neighbour part of the spatial update, from
// pre-step neighbour values (left HL, HH; upper LH, HH; upper-left HH).
template <typename T>
__device__ __forceinline__ void update_q(T (&q)[4], T hll, T lhu, T hhul, T hhu, T hhl, T u, T u2)
{
    q[LL] = mad(u, hll, mad(u, lhu, mad(u2, hhul, q[LL])));
    q[HL] = mad(u, hhu, q[HL]);
    q[LH] = mad(u, hhl, q[LH]);
}

// T_{-P1} on one quadruple.
template <typename T>
__device__ __forceinline__ void unpredict_q(T (&q)[4], T llr, T lld, T lldr, T hld, T lhr, T p, T p2)
{
    q[HL] = mad(-p, llr, q[HL]);
    q[LH] = mad(-p, lld, q[LH]);
    q[HH] = mad(p2, lldr, mad(-p, hld, mad(-p, lhr, q[HH])));
}

// S_{-U1} on one quadruple.
template <typename T>
__device__ __forceinline__ void unupdate_q(T (&q)[4], T hll, T lhu, T hhul, T hhu, T hhl, T u, T u2)
{
    q[LL] = mad(-u, hll, mad(-u, lhu, mad(u2, hhul, q[LL])));
    q[HL] = mad(-u, hhu, q[HL]);
    q[LH] = mad(-u, hhl, q[LH]);
}

// Neighbour part of a predict step: the row below comes from plane buffer b
// (published before the barrier), the right neighbours by DPP.
template <bool INV, typename T>
__device__ __forceinline__ void predict_step(T (&q)[RB][4], Planes<T> &sm, int b, int w, int lane, T p)
{
    const T p2 = p * p;
#pragma unroll
    for (int j = 0; j < RB; j++) {
        const int r = tile_row(j, w);
        const T lld = plane(sm, b, 0, r + 1, lane);
        const T hld = plane(sm, b, 1, r + 1, lane);
        const T lldr = from_right(lld);
        const T llr = from_right(q[j][LL]);
        const T lhr = from_right(q[j][LH]);
        if (!INV)
            predict_q(q[j], llr, lld, lldr, hld, lhr, p, p2);
        else
            unpredict_q(q[j], llr, lld, lldr, hld, lhr, p, p2);
    }
}

// Neighbour part of an update step: the row above from plane buffer b, the
// left neighbours by DPP.
template <bool INV, typename T>
__device__ __forceinline__ void update_step(T (&q)[RB][4], Planes<T> &sm, int b, int w, int lane, T u)
{
    const T u2 = u * u;
#pragma unroll
    for (int j = 0; j < RB; j++) {
        const int r = tile_row(j, w);
        const T lhu = plane(sm, b, 0, r - 1, lane);
        const T hhu = plane(sm, b, 1, r - 1, lane);
        const T hhul = from_left(hhu);
        const T hll = from_left(q[j][HL]);
        const T hhl = from_left(q[j][HH]);
        if (!INV)
            update_q(q[j], hll, lhu, hhul, hhu, hhl, u, u2);
        else
            unupdate_q(q[j], hll, lhu, hhul, hhu, hhl, u, u2);
    }
}

// The components a step reads across rows: LL, HL for the predict (buffer
// 0), LH, HH for the update (buffer 1).
template <typename T>
__device__ __forceinline__ void publish_predict(T (&q)[RB][4], Planes<T> &sm, int w, int lane)
{
#pragma unroll
    for (int j = 0; j < RB; j++) {
        plane(sm, 0, 0, tile_row(j, w), lane) = q[j][LL];
        plane(sm, 0, 1, tile_row(j, w), lane) = q[j][HL];
    }
}
template <typename T>
__device__ __forceinline__ void publish_update(T (&q)[RB][4], Planes<T> &sm, int w, int lane)
{
#pragma unroll
    for (int j = 0; j < RB; j++) {
        plane(sm, 1, 0, tile_row(j, w), lane) = q[j][LH];
        plane(sm, 1, 1, tile_row(j, w), lane) = q[j][HH];
    }
}

template <typename T>
__device__ __forceinline__ void scalar_predict(T (&q)[RB][4], T p)
{
#pragma unroll
    for (int j = 0; j < RB; j++) {
        q[j][HL] = mad(p, q[j][LL], q[j][HL]);  // T^H_{P0}
        q[j][HH] = mad(p, q[j][LH], q[j][HH]);
        q[j][LH] = mad(p, q[j][LL], q[j][LH]);  // T^V_{P0}
        q[j][HH] = mad(p, q[j][HL], q[j][HH]);
    }
}
template <typename T>
__device__ __forceinline__ void scalar_update(T (&q)[RB][4], T u)
{
#pragma unroll
    for (int j = 0; j < RB; j++) {
        q[j][LL] = mad(u, q[j][HL], q[j][LL]);  // S^H_{U0}
        q[j][LH] = mad(u, q[j][HH], q[j][LH]);
        q[j][LL] = mad(u, q[j][LH], q[j][LL]);  // S^V_{U0}
        q[j][HL] = mad(u, q[j][HH], q[j][HL]);
    }
}
template <typename T>
__device__ __forceinline__ void scalar_unupdate(T (&q)[RB][4], T u)
{
#pragma unroll
    for (int j = 0; j < RB; j++) {
        q[j][LL] = mad(-u, q[j][LH], q[j][LL]);  // undo S^V_{U0}
        q[j][HL] = mad(-u, q[j][HH], q[j][HL]);
        q[j][LL] = mad(-u, q[j][HL], q[j][LL]);  // undo S^H_{U0}
        q[j][LH] = mad(-u, q[j][HH], q[j][LH]);
    }
}
template <typename T>
__device__ __forceinline__ void scalar_unpredict(T (&q)[RB][4], T p)
{
#pragma unroll
    for (int j = 0; j < RB; j++) {
        q[j][HH] = mad(-p, q[j][HL], q[j][HH]);  // undo T^V_{P0}
        q[j][LH] = mad(-p, q[j][LL], q[j][LH]);
        q[j][HH] = mad(-p, q[j][LH], q[j][HH]);  // undo T^H_{P0}
        q[j][HL] = mad(-p, q[j][LL], q[j][HL]);
    }
}

// Lifting constants in the arithmetic type: FP32 literals, or for FP64 the
// same values written to double precision.
template <int WAV, typename T>
struct Coef {
    __device__ static T p(int k) { return Lift<WAV>::p(k); }
    __device__ static T u(int k) { return Lift<WAV>::u(k); }
};
template <>
struct Coef<CDF97, double> {
    __device__ static double p(int k) { return k == 0 ? -1.58613434205992355842832 : 0.88291107553093329591979; }
    __device__ static double u(int k) { return k == 0 ? -0.0529801185729614146241296 : 0.443506852043971152115604; }
};

template <int WAV, typename T>
__device__ __forceinline__ void forward_tile(T (&q)[RB][4], Planes<T> &sm, int w, int lane)
{
    using C = Coef<WAV, T>;
#pragma unroll
    for (int k = 0; k < Lift<WAV>::K; k++) {
        publish_predict(q, sm, w, lane);
        __syncthreads();
        predict_step<false>(q, sm, 0, w, lane, C::p(k));
        scalar_predict(q, C::p(k));
        publish_update(q, sm, w, lane);
        __syncthreads();
        update_step<false>(q, sm, 1, w, lane, C::u(k));
        scalar_update(q, C::u(k));
    }
}

template <int WAV, typename T>
__device__ __forceinline__ void inverse_tile(T (&q)[RB][4], Planes<T> &sm, int w, int lane)
{
    using C = Coef<WAV, T>;
#pragma unroll
    for (int kk = 0; kk < Lift<WAV>::K; kk++) {
        const int k = Lift<WAV>::K - 1 - kk;
        scalar_unupdate(q, C::u(k));
        publish_update(q, sm, w, lane);
        __syncthreads();
        update_step<true>(q, sm, 1, w, lane, C::u(k));
        scalar_unpredict(q, C::p(k));
        publish_predict(q, sm, w, lane);
        __syncthreads();
        predict_step<true>(q, sm, 0, w, lane, C::p(k));
    }
}

// Plain stores: measured faster here than non-temporal ones, which slowed the
// forward's four-quadrant dword stores by a third.
__device__ __forceinline__ void store1(float *p, float v) { *p = v; }
__device__ __forceinline__ void store2(float *p, float a, float b) { *(float2 *)p = make_float2(a, b); }

// Horizontal fast path: the tile's 128 pixel columns lie inside the image and
// rows are 8-byte aligned, so each pixel-row pair is one float2 per lane.
template <int WAV, typename T, bool VEC>
__device__ __forceinline__ void fwd_body(const FwdArgs &a, Planes<T> &sm, int tc, int tr, int w, int lane)
{
    constexpr int HQ = Lift<WAV>::K;
    constexpr int IX = TX - 2 * HQ, IY = TY - 2 * HQ;
    const int W = a.W, H = a.H;
    const int QW = (W + 1) >> 1, QH = (H + 1) >> 1, WH = W >> 1, HHr = H >> 1;
    const int qc = tc * IX - HQ + lane;
    const int x0 = ws_mirror(2 * qc, W), x1 = ws_mirror(2 * qc + 1, W);
    const int qr0 = tr * IY - HQ;  // quadruple row of tile row 0

    T q[RB][4];
    auto load = [&](int qr, float &ll, float &hl, float &lh, float &hh) {
        const float *r0 = a.in + (ptrdiff_t)ws_mirror(2 * qr, H) * a.in_pitch;
        const float *r1 = a.in + (ptrdiff_t)ws_mirror(2 * qr + 1, H) * a.in_pitch;
        if constexpr (VEC) {
            const float2 e = *(const float2 *)(r0 + 2 * qc), o = *(const float2 *)(r1 + 2 * qc);
            ll = e.x; hl = e.y; lh = o.x; hh = o.y;
        } else {
            ll = r0[x0]; hl = r0[x1]; lh = r1[x0]; hh = r1[x1];
        }
    };
    float raw[RB][4];
#pragma unroll
    for (int j = 0; j < RB; j++)
        load(qr0 + tile_row(j, w), raw[j][LL], raw[j][HL], raw[j][LH], raw[j][HH]);
    float c;
    {
        float a0, a1, a2, a3;
        load(tr * IY - HQ + TY / 2, a0, a1, a2, a3);
        const float sum = wave_sum((a0 + a1) + (a2 + a3));
        c = rintf(sum * (1.0f / (4 * TX)) / a.quantum) * a.quantum;
    }
#pragma unroll
    for (int j = 0; j < RB; j++)
#pragma unroll
        for (int e = 0; e < 4; e++) q[j][e] = (T)raw[j][e] - (T)c;

    forward_tile<WAV>(q, sm, w, lane);

    if (lane < HQ || lane >= TX - HQ || qc >= QW) return;
    const float cll = c * a.ll_gain;
#pragma unroll
    for (int j = 0; j < RB; j++) {
        const int r = tile_row(j, w), qr = qr0 + r;
        if (r < HQ || r >= TY - HQ || qr >= QH) continue;
        store1(a.ll + (ptrdiff_t)qr * a.ll_pitch + qc,
                 (float)(q[j][LL] * (T)a.s.ll + (T)cll));
        float *drow = a.det + (ptrdiff_t)qr * a.det_pitch;
        if (qc < WH) store1(drow + QW + qc, (float)q[j][HL]);
        if (qr < HHr) {
            float *hrow = a.det + (ptrdiff_t)(QH + qr) * a.det_pitch;
            store1(hrow + qc, (float)q[j][LH]);
            if (qc < WH) store1(hrow + QW + qc, (float)(q[j][HH] * (T)a.s.hh));
        }
    }
}

template <int WAV, typename T, bool VEC>
__device__ __forceinline__ void inv_body(const InvArgs &a, Planes<T> &sm, int tc, int tr, int w, int lane)
{
    constexpr int HQ = Lift<WAV>::K;
    constexpr int IX = TX - 2 * HQ, IY = TY - 2 * HQ;
    const int W = a.W, H = a.H;
    const int QW = (W + 1) >> 1, QH = (H + 1) >> 1;
    const int qc = tc * IX - HQ + lane;
    const int cl = ws_mirror(2 * qc, W) >> 1, ch = ws_mirror(2 * qc + 1, W) >> 1;
    const int qr0 = tr * IY - HQ;  // quadruple row of tile row 0

    float c;
    {
        const int rm = ws_mirror(2 * (tr * IY - HQ + TY / 2), H) >> 1;
        const float sum = wave_sum(a.ll[(ptrdiff_t)rm * a.ll_pitch + cl]);
        c = rintf(sum * (1.0f / TX) / (a.ll_gain * a.quantum)) * a.quantum;
    }
    const float cll = c * a.ll_gain;

    T q[RB][4];
#pragma unroll
    for (int j = 0; j < RB; j++) {
        const int qr = qr0 + tile_row(j, w);
        const int rl = ws_mirror(2 * qr, H) >> 1, rh = ws_mirror(2 * qr + 1, H) >> 1;
        const float *lrow = a.det + (ptrdiff_t)rl * a.det_pitch;
        const float *hrow = a.det + (ptrdiff_t)(QH + rh) * a.det_pitch;
        q[j][LL] = ((T)a.ll[(ptrdiff_t)rl * a.ll_pitch + cl] - (T)cll) * (T)a.inv_s.ll;
        q[j][HL] = lrow[QW + ch];
        q[j][LH] = hrow[cl];
        q[j][HH] = (T)hrow[QW + ch] * (T)a.inv_s.hh;
    }

    inverse_tile<WAV>(q, sm, w, lane);

    if (lane < HQ || lane >= TX - HQ || qc >= QW) return;
    const int px = 2 * qc;
#pragma unroll
    for (int j = 0; j < RB; j++) {
        const int r = tile_row(j, w), qr = qr0 + r;
        if (r < HQ || r >= TY - HQ || qr >= QH) continue;
        float *o0 = a.out + (ptrdiff_t)(2 * qr) * a.out_pitch;
        const T cc = c;
        const float v0 = (float)(q[j][LL] + cc), v1 = (float)(q[j][HL] + cc);
        const float v2 = (float)(q[j][LH] + cc), v3 = (float)(q[j][HH] + cc);
        if (VEC) {
            store2(o0 + px, v0, v1);
            if (2 * qr + 1 < H) store2(o0 + a.out_pitch + px, v2, v3);
        } else {
            store1(o0 + px, v0);
            if (px + 1 < W) store1(o0 + px + 1, v1);
            if (2 * qr + 1 < H) {
                store1(o0 + a.out_pitch + px, v2);
                if (px + 1 < W) store1(o0 + a.out_pitch + px + 1, v3);
            }
        }
    }
}

template <int WAV, typename T>
__global__ __launch_bounds__(NTHREADS) void k_fused_forward(FwdArgs a, int ntx, int ntiles)
{
    constexpr int HQ = Lift<WAV>::K;
    __shared__ Planes<T> sm;
    const int tile = xcd_tile(ntiles);
    if (tile < 0) return;  // uniform over the work-group
    const int lane = threadIdx.x & (TX - 1), w = threadIdx.x / TX;
    const int tc = tile % ntx, tr = tile / ntx;
    const int px_first = 2 * (tc * (TX - 2 * HQ) - HQ);
    const bool vec = px_first >= 0 && px_first + 2 * TX <= a.W &&
                     (((uintptr_t)a.in | (uintptr_t)(a.in_pitch * 4)) & 7) == 0;
    if (vec)
        fwd_body<WAV, T, true>(a, sm, tc, tr, w, lane);
    else
        fwd_body<WAV, T, false>(a, sm, tc, tr, w, lane);
}

template <int WAV, typename T>
__global__ __launch_bounds__(NTHREADS) void k_fused_inverse(InvArgs a, int ntx, int ntiles)
{
    constexpr int HQ = Lift<WAV>::K;
    __shared__ Planes<T> sm;
    const int tile = xcd_tile(ntiles);
    if (tile < 0) return;
    const int lane = threadIdx.x & (TX - 1), w = threadIdx.x / TX;
    const int tc = tile % ntx, tr = tile / ntx;
    const int px_first = 2 * (tc * (TX - 2 * HQ) - HQ);
    const bool vec = px_first >= 0 && px_first + 2 * TX <= a.W &&
                     (((uintptr_t)a.out | (uintptr_t)(a.out_pitch * 4)) & 7) == 0;
    if (vec)
        inv_body<WAV, T, true>(a, sm, tc, tr, w, lane);
    else
        inv_body<WAV, T, false>(a, sm, tc, tr, w, lane);
}

// Batched levels.  A work-group finds its image by a search over the tile
// starts that costs one coalesced load per 64-fold narrowing (two for up to
// 4096 images), then runs the same tile body as the single-image kernel, so
// every image gets the bits the single-image call gives it.
__device__ __forceinline__ int find_image(const int *__restrict__ start, int count, int t)
{
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = count;  // start[lo] <= t, and start[hi] > t unless hi == count
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) / 64;
        const int idx = lo + lane * step;
        const bool le = idx < hi && start[idx] <= t;  // true on a prefix of the lanes
        const int m = __popcll(__ballot(le)) - 1;     // lane 0 is always true
        lo = __builtin_amdgcn_readfirstlane(lo + m * step);
        hi = min(lo + step, hi);
    }
    return lo;
}

// Level-k geometry of image `im`: size, and the pointers of the level loop.
__device__ __forceinline__ int level_size(int n, int k)
{
    return (int)(((long long)n + (1LL << k) - 1) >> k);
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_batch_forward(BatchLevel b)
{
    __shared__ Planes<T> sm;
    const int t = xcd_tile(b.ntiles);
    if (t < 0) return;
    const int i = find_image(b.start, b.count, t);
    const BatchImage &im = b.imgs[i];
    const int k = b.level, last = im.levels - 1;
    const int W = level_size(im.W, k), H = level_size(im.H, k);
    FwdArgs a;
    a.in = k == 0 ? im.src : im.buf[(k - 1) & 1];
    a.in_pitch = k == 0 ? im.src_pitch : (ptrdiff_t)W;
    a.ll = k == last ? im.dst : im.buf[k & 1];
    a.ll_pitch = k == last ? im.dst_pitch : (ptrdiff_t)((W + 1) / 2);
    a.det = im.dst;
    a.det_pitch = im.dst_pitch;
    a.W = W;
    a.H = H;
    a.s = b.s[im.wavelet == CDF97];
    a.ll_gain = b.ll_gain;
    a.quantum = b.quantum;
    const int lane = threadIdx.x & (TX - 1), w = threadIdx.x / TX;
    const int local = t - b.start[i];
    const bool aligned = (((uintptr_t)a.in | (uintptr_t)(a.in_pitch * 4)) & 7) == 0;
    if (im.wavelet == CDF97) {
        constexpr int HQ = Lift<CDF97>::K;
        const int ntx = ((W + 1) / 2 + TX - 2 * HQ - 1) / (TX - 2 * HQ);
        const int tc = local % ntx, tr = local / ntx;
        const int px_first = 2 * (tc * (TX - 2 * HQ) - HQ);
        if (aligned && px_first >= 0 && px_first + 2 * TX <= W)
            fwd_body<CDF97, T, true>(a, sm, tc, tr, w, lane);
        else
            fwd_body<CDF97, T, false>(a, sm, tc, tr, w, lane);
    } else {
        constexpr int HQ = Lift<CDF53>::K;
        const int ntx = ((W + 1) / 2 + TX - 2 * HQ - 1) / (TX - 2 * HQ);
        const int tc = local % ntx, tr = local / ntx;
        const int px_first = 2 * (tc * (TX - 2 * HQ) - HQ);
        if (aligned && px_first >= 0 && px_first + 2 * TX <= W)
            fwd_body<CDF53, T, true>(a, sm, tc, tr, w, lane);
        else
            fwd_body<CDF53, T, false>(a, sm, tc, tr, w, lane);
    }
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_batch_inverse(BatchLevel b)
{
    __shared__ Planes<T> sm;
    const int t = xcd_tile(b.ntiles);
    if (t < 0) return;
    const int i = find_image(b.start, b.count, t);
    const BatchImage &im = b.imgs[i];
    const int k = b.level, last = im.levels - 1;
    const int W = level_size(im.W, k), H = level_size(im.H, k);
    InvArgs a;
    a.ll = k == last ? im.src : im.buf[k & 1];
    a.ll_pitch = k == last ? im.src_pitch : (ptrdiff_t)((W + 1) / 2);
    a.det = im.src;
    a.det_pitch = im.src_pitch;
    a.out = k == 0 ? im.dst : im.buf[(k - 1) & 1];
    a.out_pitch = k == 0 ? im.dst_pitch : (ptrdiff_t)W;
    a.W = W;
    a.H = H;
    a.inv_s = b.s[im.wavelet == CDF97];
    a.ll_gain = b.ll_gain;
    a.quantum = b.quantum;
    const int lane = threadIdx.x & (TX - 1), w = threadIdx.x / TX;
    const int local = t - b.start[i];
    const bool aligned = (((uintptr_t)a.out | (uintptr_t)(a.out_pitch * 4)) & 7) == 0;
    if (im.wavelet == CDF97) {
        constexpr int HQ = Lift<CDF97>::K;
        const int ntx = ((W + 1) / 2 + TX - 2 * HQ - 1) / (TX - 2 * HQ);
        const int tc = local % ntx, tr = local / ntx;
        const int px_first = 2 * (tc * (TX - 2 * HQ) - HQ);
        if (aligned && px_first >= 0 && px_first + 2 * TX <= W)
            inv_body<CDF97, T, true>(a, sm, tc, tr, w, lane);
        else
            inv_body<CDF97, T, false>(a, sm, tc, tr, w, lane);
    } else {
        constexpr int HQ = Lift<CDF53>::K;
        const int ntx = ((W + 1) / 2 + TX - 2 * HQ - 1) / (TX - 2 * HQ);
        const int tc = local % ntx, tr = local / ntx;
        const int px_first = 2 * (tc * (TX - 2 * HQ) - HQ);
        if (aligned && px_first >= 0 && px_first + 2 * TX <= W)
            inv_body<CDF53, T, true>(a, sm, tc, tr, w, lane);
        else
            inv_body<CDF53, T, false>(a, sm, tc, tr, w, lane);
    }
}

// Host-to-device copy through kernel arguments (at most kUploadWords words
// per launch; kernel arguments are captured by value in a graph).
constexpr int kUploadWords = 768;
struct UploadChunk {
    uint32_t w[kUploadWords];
};

__global__ __launch_bounds__(256) void k_upload(uint32_t *dst, int n, UploadChunk c)
{
    for (int j = threadIdx.x; j < n; j += 256) dst[j] = c.w[j];
}

struct Grid {
    int ntx, ntiles, blocks;
};

Grid fused_grid(int W, int H, int HQ)
{
    const int QW = (W + 1) / 2, QH = (H + 1) / 2;
    const int ix = TX - 2 * HQ, iy = TY - 2 * HQ;
    Grid g;
    g.ntx = (QW + ix - 1) / ix;
    g.ntiles = g.ntx * ((QH + iy - 1) / iy);
    g.blocks = (g.ntiles + 7) / 8 * 8;
    return g;
}

}  // namespace

hipError_t launch_fused_forward(int wavelet, bool fp64, const FwdArgs &a, hipStream_t s)
{
    const int HQ = wavelet == CDF97 ? 2 : 1;
    const Grid g = fused_grid(a.W, a.H, HQ);
    const dim3 grid(g.blocks), block(NTHREADS);
    if (wavelet == CDF53)
        return fp64 ? launch(k_fused_forward<CDF53, double>, grid, block, s, a, g.ntx, g.ntiles)
                    : launch(k_fused_forward<CDF53, float>, grid, block, s, a, g.ntx, g.ntiles);
    if (wavelet == CDF97)
        return fp64 ? launch(k_fused_forward<CDF97, double>, grid, block, s, a, g.ntx, g.ntiles)
                    : launch(k_fused_forward<CDF97, float>, grid, block, s, a, g.ntx, g.ntiles);
    return hipErrorInvalidValue;
}

hipError_t launch_fused_inverse(int wavelet, bool fp64, const InvArgs &a, hipStream_t s)
{
    const int HQ = wavelet == CDF97 ? 2 : 1;
    const Grid g = fused_grid(a.W, a.H, HQ);
    const dim3 grid(g.blocks), block(NTHREADS);
    if (wavelet == CDF53)
        return fp64 ? launch(k_fused_inverse<CDF53, double>, grid, block, s, a, g.ntx, g.ntiles)
                    : launch(k_fused_inverse<CDF53, float>, grid, block, s, a, g.ntx, g.ntiles);
    if (wavelet == CDF97)
        return fp64 ? launch(k_fused_inverse<CDF97, double>, grid, block, s, a, g.ntx, g.ntiles)
                    : launch(k_fused_inverse<CDF97, float>, grid, block, s, a, g.ntx, g.ntiles);
    return hipErrorInvalidValue;
}

long long fused_tile_count(int wavelet, int W, int H)
{
    if (W < 2 || H < 2) return 0;
    const int HQ = wavelet == CDF97 ? 2 : 1;
    const long long QW = (W + 1LL) / 2, QH = (H + 1LL) / 2;
    const int ix = TX - 2 * HQ, iy = TY - 2 * HQ;
    return ((QW + ix - 1) / ix) * ((QH + iy - 1) / iy);
}

hipError_t launch_batch_forward(bool fp64, const BatchLevel &b, hipStream_t s)
{
    const dim3 grid((b.ntiles + 7) / 8 * 8), block(NTHREADS);
    return fp64 ? launch(k_batch_forward<double>, grid, block, s, b)
                : launch(k_batch_forward<float>, grid, block, s, b);
}

hipError_t launch_batch_inverse(bool fp64, const BatchLevel &b, hipStream_t s)
{
    const dim3 grid((b.ntiles + 7) / 8 * 8), block(NTHREADS);
    return fp64 ? launch(k_batch_inverse<double>, grid, block, s, b)
                : launch(k_batch_inverse<float>, grid, block, s, b);
}

hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t words = bytes / 4;
    for (size_t off = 0; off < words; off += kUploadWords) {
        const int n = (int)(words - off < (size_t)kUploadWords ? words - off : kUploadWords);
        UploadChunk c{};
        memcpy(c.w, (const uint32_t *)src + off, sizeof(uint32_t) * n);
        const hipError_t e = launch(k_upload, dim3(1), dim3(256), s, (uint32_t *)dst + off, n, c);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dwt2
