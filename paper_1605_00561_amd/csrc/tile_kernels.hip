// tile_kernels.hip -- block-based 2-D lifting kernels: one launch per level.
//
// Mapping (Sec. 6, "Performance"): each work-group owns one overlapping tile
// of TX x TY quadruples (including a halo of K quadruples per side, K = the
// number of lifting pairs), one thread per quadruple column and TY / 4 rows
// per thread.  A thread keeps its quadruples in registers; LDS only carries
// the components that neighbouring threads read in the next spatial step.
// Two LDS buffers alternate between consecutive steps (the paper's "double
// buffering", Table 2), so every step that reads a neighbour costs exactly
// one barrier:
//
//   Monolithic*  (Sec. 4)  T_{P1}+T^H_{P0}+T^V_{P0} | S_{U1}+S^H_{U0}+S^V_{U0}
//   (this tile form; the default fused kernel keeps its tile in registers
//   and moves horizontal neighbours by DPP)
//                          2 barriers per pair, 6 LDS cells per quadruple
//   Sweldens     (Sec. 2)  T^H_P | T^V_P | S^H_U | S^V_U
//                          4 barriers per pair, 4 LDS cells
//   Iwahashi     (Sec. 2)  T^I_P | R^I_{P,U} | S^I_U
//                          3 barriers per pair, 6 LDS cells
// and the paper's other schemes, each with Table 1's barriers: Monolithic
// (unsplit, Sec. 3), Explosive and Explosive* (Sec. 3-4), Iwahashi* and
// Polyphase* (Sec. 4); their steps are described where they are defined.
//
// Operators in the L = x[2n] phase (see dwt2_internal.h): for a component
// X at quadruple (r, c), P X = p (X + X[r][c+1]), P* X = p (X + X[r+1][c]),
// U X = u (X + X[r][c-1]), U* X = u (X + X[r-1][c]).
//
// The tile is computed on the whole-sample symmetric extension of the
// image: every halo sample is read from its mirrored position, and lifting
// steps preserve that symmetry, so interior results equal per-step index
// mirroring.  After pair k only quadruples at least k+1 from the tile edge
// are valid; the interior (TX - 2K) x (TY - 2K) quadruples are stored.
//
// FP32 conditioning: every tile subtracts a constant c (the rounded mean of
// its middle quadruple row) from all samples before lifting and adds
// c * ll_gain to LL at the end -- exact by linearity, since every stored
// quadruple depends only on samples inside the tile.  Flat regions then
// transform near zero instead of through the large 9/7 intermediates
// (1 + 2 alpha ~ -2.17 times the sample value), which cuts FP32 rounding.
// All waves compute c from the same samples in the same order, so it is
// bitwise identical across the work-group without a barrier.
//
// Work-groups are numbered so that each of the 8 XCDs (workgroup id mod 8)
// receives a contiguous run of tiles in row-major order, so the halo rows
// and columns shared by neighbouring tiles are re-read from the same L2.
#include "dwt2_internal.h"

namespace dwt2 {
namespace {

constexpr int TX = 64;  // quadruple columns per tile = wavefront size
constexpr int NWAVES = 4;
constexpr int NTHREADS = TX * NWAVES;
constexpr int TY = 28;  // quadruple rows per tile (incl. halo)
constexpr int NJ = TY / NWAVES;
constexpr int PS = TX + 2;               // padded plane row stride
constexpr int PSZ = (TY + 2) * PS;       // padded plane size (1 cell each side)

enum { LL = 0, HL = 1, LH = 2, HH = 3 };

__device__ __forceinline__ int xcd_tile(int ntiles)
{
    const int per = gridDim.x >> 3;  // grid is a multiple of 8
    const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    return t < ntiles ? t : -1;
}

// LDS access: plane `pl`, tile row r, tile column c; r in [-1, TY], c in [-1, TX].
__device__ __forceinline__ float &cell(float *lds, int pl, int r, int c)
{
    return lds[pl * PSZ + (r + 1) * PS + (c + 1)];
}

struct Quads {
    float v[NJ][4];
};

// Sum over the 64 lanes by an xor butterfly: every lane ends with the same bits.
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int C>
__device__ __forceinline__ void publish(float *lds, int pl, const Quads &q, int lane, int wv)
{
#pragma unroll
    for (int j = 0; j < NJ; j++) cell(lds, pl, j * NWAVES + wv, lane) = q.v[j][C];
}

// ---------------------------------------------------------------------------
// Monolithic* steps.  Neighbour parts read pre-step values from LDS; the
// scalar parts follow in the order T^H then T^V (S^H then S^V).  The four
// factors of each step commute (Sec. 4), so this order is exact algebra.
// ---------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ void mono_predict(float *lds, int A, Quads &q, int lane, int wv, float p)
{
    const float p2 = p * p;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float llr = cell(lds, A + 0, r, lane + 1);
        const float lld = cell(lds, A + 0, r + 1, lane);
        const float lldr = cell(lds, A + 0, r + 1, lane + 1);
        const float hld = cell(lds, A + 1, r + 1, lane);
        const float lhr = cell(lds, A + 2, r, lane + 1);
        float &ll = q.v[j][LL], &hl = q.v[j][HL], &lh = q.v[j][LH], &hh = q.v[j][HH];
        if (!INV) {
            // T_{P1}: HL += p LL[c+1]; LH += p LL[r+1]; HH += p^2 LL[r+1][c+1] + p HL[r+1] + p LH[c+1]
            hl = fmaf(p, llr, hl);
            lh = fmaf(p, lld, lh);
            hh = fmaf(p2, lldr, fmaf(p, hld, fmaf(p, lhr, hh)));
            // T^H_{P0}: HL += p LL; HH += p LH.  T^V_{P0}: LH += p LL; HH += p HL.
            hl = fmaf(p, ll, hl);
            hh = fmaf(p, lh, hh);
            lh = fmaf(p, ll, lh);
            hh = fmaf(p, hl, hh);
        } else {
            // T_{-P1} (the scalar parts were undone before the publish)
            hl = fmaf(-p, llr, hl);
            lh = fmaf(-p, lld, lh);
            hh = fmaf(p2, lldr, fmaf(-p, hld, fmaf(-p, lhr, hh)));
        }
    }
}

template <bool INV>
__device__ __forceinline__ void mono_update(float *lds, int B, Quads &q, int lane, int wv, float u)
{
    const float u2 = u * u;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float hll = cell(lds, B + 0, r, lane - 1);
        const float lhu = cell(lds, B + 1, r - 1, lane);
        const float hhul = cell(lds, B + 2, r - 1, lane - 1);
        const float hhu = cell(lds, B + 2, r - 1, lane);
        const float hhl = cell(lds, B + 2, r, lane - 1);
        float &ll = q.v[j][LL], &hl = q.v[j][HL], &lh = q.v[j][LH], &hh = q.v[j][HH];
        if (!INV) {
            // S_{U1}: LL += u HL[c-1] + u LH[r-1] + u^2 HH[r-1][c-1]; HL += u HH[r-1]; LH += u HH[c-1]
            ll = fmaf(u, hll, fmaf(u, lhu, fmaf(u2, hhul, ll)));
            hl = fmaf(u, hhu, hl);
            lh = fmaf(u, hhl, lh);
            // S^H_{U0}: LL += u HL; LH += u HH.  S^V_{U0}: LL += u LH; HL += u HH.
            ll = fmaf(u, hl, ll);
            lh = fmaf(u, hh, lh);
            ll = fmaf(u, lh, ll);
            hl = fmaf(u, hh, hl);
        } else {
            // S_{-U1}: LL += -u HL[c-1] - u LH[r-1] + u^2 HH[r-1][c-1]; HL -= u HH[r-1]; LH -= u HH[c-1]
            ll = fmaf(-u, hll, fmaf(-u, lhu, fmaf(u2, hhul, ll)));
            hl = fmaf(-u, hhu, hl);
            lh = fmaf(-u, hhl, lh);
        }
    }
}

// Inverse of the scalar parts, applied before the neighbour step.
__device__ __forceinline__ void mono_unupdate_local(Quads &q, float u)
{
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        float &ll = q.v[j][LL], &hl = q.v[j][HL], &lh = q.v[j][LH], &hh = q.v[j][HH];
        ll = fmaf(-u, lh, ll);  // undo S^V_{U0}
        hl = fmaf(-u, hh, hl);
        ll = fmaf(-u, hl, ll);  // undo S^H_{U0}
        lh = fmaf(-u, hh, lh);
    }
}

__device__ __forceinline__ void mono_unpredict_local(Quads &q, float p)
{
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        float &ll = q.v[j][LL], &hl = q.v[j][HL], &lh = q.v[j][LH], &hh = q.v[j][HH];
        hh = fmaf(-p, hl, hh);  // undo T^V_{P0}
        lh = fmaf(-p, ll, lh);
        hh = fmaf(-p, lh, hh);  // undo T^H_{P0}
        hl = fmaf(-p, ll, hl);
    }
}

// ---------------------------------------------------------------------------
// Sweldens steps (separable, one direction per step).  s = +1 forward, -1 inverse.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void swel_TH(float *lds, int A, Quads &q, int lane, int wv, float p)
{   // HL += P LL; HH += P LH       (reads LL, LH at c+1)
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        q.v[j][HL] = fmaf(p, q.v[j][LL] + cell(lds, A + 0, r, lane + 1), q.v[j][HL]);
        q.v[j][HH] = fmaf(p, q.v[j][LH] + cell(lds, A + 1, r, lane + 1), q.v[j][HH]);
    }
}
__device__ __forceinline__ void swel_TV(float *lds, int A, Quads &q, int lane, int wv, float p)
{   // LH += P* LL; HH += P* HL     (reads LL, HL at r+1)
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        q.v[j][LH] = fmaf(p, q.v[j][LL] + cell(lds, A + 0, r + 1, lane), q.v[j][LH]);
        q.v[j][HH] = fmaf(p, q.v[j][HL] + cell(lds, A + 1, r + 1, lane), q.v[j][HH]);
    }
}
__device__ __forceinline__ void swel_SH(float *lds, int A, Quads &q, int lane, int wv, float u)
{   // LL += U HL; LH += U HH       (reads HL, HH at c-1)
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        q.v[j][LL] = fmaf(u, q.v[j][HL] + cell(lds, A + 0, r, lane - 1), q.v[j][LL]);
        q.v[j][LH] = fmaf(u, q.v[j][HH] + cell(lds, A + 1, r, lane - 1), q.v[j][LH]);
    }
}
__device__ __forceinline__ void swel_SV(float *lds, int A, Quads &q, int lane, int wv, float u)
{   // LL += U* LH; HL += U* HH     (reads LH, HH at r-1)
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        q.v[j][LL] = fmaf(u, q.v[j][LH] + cell(lds, A + 0, r - 1, lane), q.v[j][LL]);
        q.v[j][HL] = fmaf(u, q.v[j][HH] + cell(lds, A + 1, r - 1, lane), q.v[j][HL]);
    }
}

// ---------------------------------------------------------------------------
// Iwahashi steps (non-separable, three per pair).  Each step reads only
// components it does not modify, so its inverse subtracts the same terms
// (the product terms flip sign with the others).  FULL: the whole operators
// P = p (1 + z), U = u (1 + z^-1) (Iwahashi); otherwise only the neighbour
// parts P1 = p z, U1 = u z^-1 (Iwahashi*, whose scalar parts run locally).
// ---------------------------------------------------------------------------
template <bool FULL, bool INV>
__device__ __forceinline__ void iwa_T(float *lds, int A, Quads &q, int lane, int wv, float p)
{   // HH += P P* LL + P* HL + P LH   (reads LL at c+1, r+1, (r+1,c+1); HL at r+1; LH at c+1)
    const float sp = INV ? -p : p;
    const float sp2 = INV ? -(p * p) : p * p;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float lldr = cell(lds, A + 0, r + 1, lane + 1);
        const float llsum = FULL ? (q.v[j][LL] + cell(lds, A + 0, r, lane + 1)) +
                                       (cell(lds, A + 0, r + 1, lane) + lldr)
                                 : lldr;
        const float hl = FULL ? q.v[j][HL] + cell(lds, A + 1, r + 1, lane) : cell(lds, A + 1, r + 1, lane);
        const float lh = FULL ? q.v[j][LH] + cell(lds, A + 2, r, lane + 1) : cell(lds, A + 2, r, lane + 1);
        float hh = q.v[j][HH];
        hh = fmaf(sp, lh, hh);
        hh = fmaf(sp, hl, hh);
        q.v[j][HH] = fmaf(sp2, llsum, hh);
    }
}
template <bool FULL, bool INV>
__device__ __forceinline__ void iwa_R(float *lds, int B, Quads &q, int lane, int wv, float p, float u)
{   // HL += P LL + U* HH; LH += P* LL + U HH   (reads LL at c+1, r+1; HH at r-1, c-1)
    const float sp = INV ? -p : p;
    const float su = INV ? -u : u;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float ll = FULL ? q.v[j][LL] : 0.0f, hh = FULL ? q.v[j][HH] : 0.0f;
        q.v[j][HL] = fmaf(su, hh + cell(lds, B + 1, r - 1, lane),
                          fmaf(sp, ll + cell(lds, B + 0, r, lane + 1), q.v[j][HL]));
        q.v[j][LH] = fmaf(su, hh + cell(lds, B + 1, r, lane - 1),
                          fmaf(sp, ll + cell(lds, B + 0, r + 1, lane), q.v[j][LH]));
    }
}
template <bool FULL, bool INV>
__device__ __forceinline__ void iwa_S(float *lds, int A, Quads &q, int lane, int wv, float u)
{   // LL += U HL + U* LH - U U* HH   (reads HL at c-1; LH at r-1; HH at c-1, r-1, (r-1,c-1))
    const float su = INV ? -u : u;
    const float su2 = INV ? (u * u) : -(u * u);
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float hhul = cell(lds, A + 2, r - 1, lane - 1);
        const float hhsum = FULL ? (q.v[j][HH] + cell(lds, A + 2, r, lane - 1)) +
                                       (cell(lds, A + 2, r - 1, lane) + hhul)
                                 : hhul;
        const float hl = FULL ? q.v[j][HL] + cell(lds, A + 0, r, lane - 1) : cell(lds, A + 0, r, lane - 1);
        const float lh = FULL ? q.v[j][LH] + cell(lds, A + 1, r - 1, lane) : cell(lds, A + 1, r - 1, lane);
        float ll = q.v[j][LL];
        ll = fmaf(su, hl, ll);
        ll = fmaf(su, lh, ll);
        q.v[j][LL] = fmaf(su2, hhsum, ll);
    }
}

// ---------------------------------------------------------------------------
// Explosive steps (Sec. 3): the predict pushes data out of LL (T^E), the
// update out of HH (S^E), and R^E joins them.  Like Iwahashi's, each step
// reads only components it leaves unchanged.  FULL as for Iwahashi
// (Explosive / Explosive*).
// ---------------------------------------------------------------------------
template <bool FULL, bool INV>
__device__ __forceinline__ void exp_T(float *lds, int A, Quads &q, int lane, int wv, float p)
{   // HL += P LL; LH += P* LL; HH -= P P* LL   (reads LL at c+1, r+1, (r+1,c+1))
    const float sp = INV ? -p : p;
    const float sp2 = INV ? p * p : -(p * p);
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float ll = FULL ? q.v[j][LL] : 0.0f;
        const float llr = cell(lds, A, r, lane + 1), lld = cell(lds, A, r + 1, lane);
        const float lldr = cell(lds, A, r + 1, lane + 1);
        q.v[j][HL] = fmaf(sp, ll + llr, q.v[j][HL]);
        q.v[j][LH] = fmaf(sp, ll + lld, q.v[j][LH]);
        q.v[j][HH] = fmaf(sp2, FULL ? (ll + llr) + (lld + lldr) : lldr, q.v[j][HH]);
    }
}
template <bool FULL, bool INV>
__device__ __forceinline__ void exp_R(float *lds, int B, Quads &q, int lane, int wv, float p, float u)
{   // LL += U HL + U* LH; HH += P* HL + P LH   (reads HL at c-1, r+1; LH at r-1, c+1)
    const float sp = INV ? -p : p;
    const float su = INV ? -u : u;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float hl = FULL ? q.v[j][HL] : 0.0f, lh = FULL ? q.v[j][LH] : 0.0f;
        q.v[j][LL] = fmaf(su, lh + cell(lds, B + 1, r - 1, lane),
                          fmaf(su, hl + cell(lds, B + 0, r, lane - 1), q.v[j][LL]));
        q.v[j][HH] = fmaf(sp, lh + cell(lds, B + 1, r, lane + 1),
                          fmaf(sp, hl + cell(lds, B + 0, r + 1, lane), q.v[j][HH]));
    }
}
template <bool FULL, bool INV>
__device__ __forceinline__ void exp_S(float *lds, int A, Quads &q, int lane, int wv, float u)
{   // LL += U U* HH; HL += U* HH; LH += U HH   (reads HH at c-1, r-1, (r-1,c-1))
    const float su = INV ? -u : u;
    const float su2 = INV ? -(u * u) : u * u;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float hh = FULL ? q.v[j][HH] : 0.0f;
        const float hhl = cell(lds, A, r, lane - 1), hhu = cell(lds, A, r - 1, lane);
        const float hhul = cell(lds, A, r - 1, lane - 1);
        q.v[j][LL] = fmaf(su2, FULL ? (hh + hhl) + (hhu + hhul) : hhul, q.v[j][LL]);
        q.v[j][HL] = fmaf(su, hh + hhu, q.v[j][HL]);
        q.v[j][LH] = fmaf(su, hh + hhl, q.v[j][LH]);
    }
}

// ---------------------------------------------------------------------------
// Unsplit Monolithic (Sec. 3): T_P = T^V_P T^H_P and S_U = S^V_U S^H_U each as
// one spatial step on pre-step values.  The inverse of T_P is T_{-P} (the two
// separable factors commute), and likewise for S_U.
// ---------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ void mono_T_full(float *lds, int A, Quads &q, int lane, int wv, float p)
{   // HL += P LL; LH += P* LL; HH += P P* LL + P* HL + P LH
    const float sp = INV ? -p : p, p2 = p * p;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float ll = q.v[j][LL], llr = cell(lds, A + 0, r, lane + 1);
        const float lld = cell(lds, A + 0, r + 1, lane), lldr = cell(lds, A + 0, r + 1, lane + 1);
        const float hl = q.v[j][HL], lh = q.v[j][LH];
        q.v[j][HH] = fmaf(p2, (ll + llr) + (lld + lldr),
                          fmaf(sp, hl + cell(lds, A + 1, r + 1, lane),
                               fmaf(sp, lh + cell(lds, A + 2, r, lane + 1), q.v[j][HH])));
        q.v[j][HL] = fmaf(sp, ll + llr, hl);
        q.v[j][LH] = fmaf(sp, ll + lld, lh);
    }
}
template <bool INV>
__device__ __forceinline__ void mono_S_full(float *lds, int B, Quads &q, int lane, int wv, float u)
{   // LL += U HL + U* LH + U U* HH; HL += U* HH; LH += U HH
    const float su = INV ? -u : u, u2 = u * u;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float hh = q.v[j][HH], hhl = cell(lds, B + 2, r, lane - 1);
        const float hhu = cell(lds, B + 2, r - 1, lane), hhul = cell(lds, B + 2, r - 1, lane - 1);
        const float hl = q.v[j][HL], lh = q.v[j][LH];
        q.v[j][LL] = fmaf(u2, (hh + hhl) + (hhu + hhul),
                          fmaf(su, hl + cell(lds, B + 0, r, lane - 1),
                               fmaf(su, lh + cell(lds, B + 1, r - 1, lane), q.v[j][LL])));
        q.v[j][HL] = fmaf(su, hh + hhu, hl);
        q.v[j][LH] = fmaf(su, hh + hhl, lh);
    }
}

// ---------------------------------------------------------------------------
// Polyphase* (Sec. 4): the neighbour parts of one whole pair as the single
// 4x4 step N_{P1,U1}, one barrier per pair.  With P1 = p z and U1 = u z^-1,
// V1 = P1 U1 + 1 = 1 + p u is a scalar.  The inverse is the single step
// N_{P1,U1}^{-1} = T_{-P1} S_{-U1} (one matrix, one barrier as well).
// ---------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ void poly_N(float *lds, int A, Quads &q, int lane, int wv, float p, float u)
{
    const float v = fmaf(p, u, 1.0f), pu = p * u, p2 = p * p, u2 = u * u;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const float llr = cell(lds, A + 0, r, lane + 1), lld = cell(lds, A + 0, r + 1, lane);
        const float lldr = cell(lds, A + 0, r + 1, lane + 1);
        const float hll = cell(lds, A + 1, r, lane - 1), hld = cell(lds, A + 1, r + 1, lane);
        const float hldl = cell(lds, A + 1, r + 1, lane - 1);
        const float lhu = cell(lds, A + 2, r - 1, lane), lhr = cell(lds, A + 2, r, lane + 1);
        const float lhur = cell(lds, A + 2, r - 1, lane + 1);
        const float hhul = cell(lds, A + 3, r - 1, lane - 1), hhu = cell(lds, A + 3, r - 1, lane);
        const float hhl = cell(lds, A + 3, r, lane - 1);
        const float ll = q.v[j][LL], hl = q.v[j][HL], lh = q.v[j][LH], hh = q.v[j][HH];
        if (!INV) {
            // LL' = V^2 LL + V u HL[c-1] + V u LH[r-1] + u^2 HH[r-1][c-1]
            q.v[j][LL] = fmaf(u2, hhul, fmaf(v * u, hll + lhu, v * v * ll));
            // HL' = V p LL[c+1] + V HL + u p LH[r-1][c+1] + u HH[r-1]
            q.v[j][HL] = fmaf(u, hhu, fmaf(pu, lhur, v * fmaf(p, llr, hl)));
            // LH' = V p LL[r+1] + p u HL[r+1][c-1] + V LH + u HH[c-1]
            q.v[j][LH] = fmaf(u, hhl, fmaf(pu, hldl, v * fmaf(p, lld, lh)));
            // HH' = p^2 LL[r+1][c+1] + p HL[r+1] + p LH[c+1] + HH
            q.v[j][HH] = fmaf(p2, lldr, fmaf(p, hld + lhr, hh));
        } else {
            // LL' = LL - u HL[c-1] - u LH[r-1] + u^2 HH[r-1][c-1]
            q.v[j][LL] = fmaf(u2, hhul, fmaf(-u, hll + lhu, ll));
            // HL' = -p LL[c+1] + V HL + p u LH[r-1][c+1] - V u HH[r-1]
            q.v[j][HL] = fmaf(-v * u, hhu, fmaf(pu, lhur, fmaf(v, hl, -p * llr)));
            // LH' = -p LL[r+1] + p u HL[r+1][c-1] + V LH - V u HH[c-1]
            q.v[j][LH] = fmaf(-v * u, hhl, fmaf(pu, hldl, fmaf(v, lh, -p * lld)));
            // HH' = p^2 LL[r+1][c+1] - V p (HL[r+1] + LH[c+1]) + V^2 HH
            q.v[j][HH] = fmaf(p2, lldr, fmaf(-v * p, hld + lhr, v * v * hh));
        }
    }
}

// Scalar parts T^H_{P0} then T^V_{P0}, and S^H_{U0} then S^V_{U0}: local to
// the quadruple, no barrier (the starred schemes run them around the
// neighbour steps).
__device__ __forceinline__ void predict_local(Quads &q, float p)
{
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        float &ll = q.v[j][LL], &hl = q.v[j][HL], &lh = q.v[j][LH], &hh = q.v[j][HH];
        hl = fmaf(p, ll, hl);  // T^H_{P0}
        hh = fmaf(p, lh, hh);
        lh = fmaf(p, ll, lh);  // T^V_{P0}
        hh = fmaf(p, hl, hh);
    }
}
__device__ __forceinline__ void update_local(Quads &q, float u)
{
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        float &ll = q.v[j][LL], &hl = q.v[j][HL], &lh = q.v[j][LH], &hh = q.v[j][HH];
        ll = fmaf(u, hl, ll);  // S^H_{U0}
        lh = fmaf(u, hh, lh);
        ll = fmaf(u, lh, ll);  // S^V_{U0}
        hl = fmaf(u, hh, hl);
    }
}

// ---------------------------------------------------------------------------
// The transform of one tile held in registers.  `step` counts spatial steps so
// that consecutive steps use alternating LDS buffers.
// ---------------------------------------------------------------------------
// LDS planes one spatial step publishes (one buffer); two buffers alternate.
template <int SCH>
constexpr int buf_planes()
{
    return SCH == SWELDENS || SCH == EXPLOSIVE || SCH == EXPLOSIVE_STAR ? 2
           : SCH == POLYPHASE_STAR                                     ? 4
                                                                       : 3;
}

template <int WAV, int SCH, bool INV>
__device__ __forceinline__ void transform_tile(float *lds, Quads &q, int lane, int wv)
{
    using L = Lift<WAV>;
    constexpr int BUF = buf_planes<SCH>();
    int step = 0;
    auto buf = [&]() { return (step++ & 1) * BUF; };
#define SYNC() __syncthreads()
    if constexpr (SCH == MONO_STAR_TILE) {
#pragma unroll
        for (int kk = 0; kk < L::K; kk++) {
            const int k = INV ? L::K - 1 - kk : kk;
            const float p = L::p(k), u = L::u(k);
            if (!INV) {
                int A = buf();
                publish<LL>(lds, A + 0, q, lane, wv);
                publish<HL>(lds, A + 1, q, lane, wv);
                publish<LH>(lds, A + 2, q, lane, wv);
                SYNC();
                mono_predict<false>(lds, A, q, lane, wv, p);
                int B = buf();
                publish<HL>(lds, B + 0, q, lane, wv);
                publish<LH>(lds, B + 1, q, lane, wv);
                publish<HH>(lds, B + 2, q, lane, wv);
                SYNC();
                mono_update<false>(lds, B, q, lane, wv, u);
            } else {
                mono_unupdate_local(q, u);
                int B = buf();
                publish<HL>(lds, B + 0, q, lane, wv);
                publish<LH>(lds, B + 1, q, lane, wv);
                publish<HH>(lds, B + 2, q, lane, wv);
                SYNC();
                mono_update<true>(lds, B, q, lane, wv, u);
                mono_unpredict_local(q, p);
                int A = buf();
                publish<LL>(lds, A + 0, q, lane, wv);
                publish<HL>(lds, A + 1, q, lane, wv);
                publish<LH>(lds, A + 2, q, lane, wv);
                SYNC();
                mono_predict<true>(lds, A, q, lane, wv, p);
            }
        }
    } else if constexpr (SCH == SWELDENS) {
#pragma unroll
        for (int kk = 0; kk < L::K; kk++) {
            const int k = INV ? L::K - 1 - kk : kk;
            const float p = L::p(k), u = L::u(k);
            int A;
            if (!INV) {
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                SYNC(); swel_TH(lds, A, q, lane, wv, p);
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
                SYNC(); swel_TV(lds, A, q, lane, wv, p);
                A = buf(); publish<HL>(lds, A, q, lane, wv); publish<HH>(lds, A + 1, q, lane, wv);
                SYNC(); swel_SH(lds, A, q, lane, wv, u);
                A = buf(); publish<LH>(lds, A, q, lane, wv); publish<HH>(lds, A + 1, q, lane, wv);
                SYNC(); swel_SV(lds, A, q, lane, wv, u);
            } else {
                A = buf(); publish<LH>(lds, A, q, lane, wv); publish<HH>(lds, A + 1, q, lane, wv);
                SYNC(); swel_SV(lds, A, q, lane, wv, -u);
                A = buf(); publish<HL>(lds, A, q, lane, wv); publish<HH>(lds, A + 1, q, lane, wv);
                SYNC(); swel_SH(lds, A, q, lane, wv, -u);
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
                SYNC(); swel_TV(lds, A, q, lane, wv, -p);
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                SYNC(); swel_TH(lds, A, q, lane, wv, -p);
            }
        }
    } else if constexpr (SCH == IWAHASHI) {
#pragma unroll
        for (int kk = 0; kk < L::K; kk++) {
            const int k = INV ? L::K - 1 - kk : kk;
            const float p = L::p(k), u = L::u(k);
            int A;
            if (!INV) {
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
                publish<LH>(lds, A + 2, q, lane, wv);
                SYNC(); iwa_T<true, false>(lds, A, q, lane, wv, p);
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HH>(lds, A + 1, q, lane, wv);
                SYNC(); iwa_R<true, false>(lds, A, q, lane, wv, p, u);
                A = buf(); publish<HL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                publish<HH>(lds, A + 2, q, lane, wv);
                SYNC(); iwa_S<true, false>(lds, A, q, lane, wv, u);
            } else {
                A = buf(); publish<HL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                publish<HH>(lds, A + 2, q, lane, wv);
                SYNC(); iwa_S<true, true>(lds, A, q, lane, wv, u);
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HH>(lds, A + 1, q, lane, wv);
                SYNC(); iwa_R<true, true>(lds, A, q, lane, wv, p, u);
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
                publish<LH>(lds, A + 2, q, lane, wv);
                SYNC(); iwa_T<true, true>(lds, A, q, lane, wv, p);
            }
        }
    } else if constexpr (SCH == IWAHASHI_STAR || SCH == EXPLOSIVE || SCH == EXPLOSIVE_STAR) {
        // Three neighbour steps per pair; the starred forms run the scalar
        // parts T^H_{P0} T^V_{P0} before them and S^H_{U0} S^V_{U0} after
        // (the neighbour steps do not commute with the scalar ones here).
        constexpr bool STAR = SCH != EXPLOSIVE, FULL = !STAR;
#pragma unroll
        for (int kk = 0; kk < L::K; kk++) {
            const int k = INV ? L::K - 1 - kk : kk;
            const float p = L::p(k), u = L::u(k);
            int A;
            if (!INV) {
                if (STAR) predict_local(q, p);
                if constexpr (SCH == IWAHASHI_STAR) {
                    A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
                    publish<LH>(lds, A + 2, q, lane, wv);
                    SYNC(); iwa_T<false, false>(lds, A, q, lane, wv, p);
                    A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HH>(lds, A + 1, q, lane, wv);
                    SYNC(); iwa_R<false, false>(lds, A, q, lane, wv, p, u);
                    A = buf(); publish<HL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                    publish<HH>(lds, A + 2, q, lane, wv);
                    SYNC(); iwa_S<false, false>(lds, A, q, lane, wv, u);
                } else {
                    A = buf(); publish<LL>(lds, A, q, lane, wv);
                    SYNC(); exp_T<FULL, false>(lds, A, q, lane, wv, p);
                    A = buf(); publish<HL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                    SYNC(); exp_R<FULL, false>(lds, A, q, lane, wv, p, u);
                    A = buf(); publish<HH>(lds, A, q, lane, wv);
                    SYNC(); exp_S<FULL, false>(lds, A, q, lane, wv, u);
                }
                if (STAR) update_local(q, u);
            } else {
                if (STAR) mono_unupdate_local(q, u);
                if constexpr (SCH == IWAHASHI_STAR) {
                    A = buf(); publish<HL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                    publish<HH>(lds, A + 2, q, lane, wv);
                    SYNC(); iwa_S<false, true>(lds, A, q, lane, wv, u);
                    A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HH>(lds, A + 1, q, lane, wv);
                    SYNC(); iwa_R<false, true>(lds, A, q, lane, wv, p, u);
                    A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
                    publish<LH>(lds, A + 2, q, lane, wv);
                    SYNC(); iwa_T<false, true>(lds, A, q, lane, wv, p);
                } else {
                    A = buf(); publish<HH>(lds, A, q, lane, wv);
                    SYNC(); exp_S<FULL, true>(lds, A, q, lane, wv, u);
                    A = buf(); publish<HL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                    SYNC(); exp_R<FULL, true>(lds, A, q, lane, wv, p, u);
                    A = buf(); publish<LL>(lds, A, q, lane, wv);
                    SYNC(); exp_T<FULL, true>(lds, A, q, lane, wv, p);
                }
                if (STAR) mono_unpredict_local(q, p);
            }
        }
    } else if constexpr (SCH == MONOLITHIC) {
#pragma unroll
        for (int kk = 0; kk < L::K; kk++) {
            const int k = INV ? L::K - 1 - kk : kk;
            const float p = L::p(k), u = L::u(k);
            int A;
            if (!INV) {
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
                publish<LH>(lds, A + 2, q, lane, wv);
                SYNC(); mono_T_full<false>(lds, A, q, lane, wv, p);
                A = buf(); publish<HL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                publish<HH>(lds, A + 2, q, lane, wv);
                SYNC(); mono_S_full<false>(lds, A, q, lane, wv, u);
            } else {
                A = buf(); publish<HL>(lds, A, q, lane, wv); publish<LH>(lds, A + 1, q, lane, wv);
                publish<HH>(lds, A + 2, q, lane, wv);
                SYNC(); mono_S_full<true>(lds, A, q, lane, wv, u);
                A = buf(); publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
                publish<LH>(lds, A + 2, q, lane, wv);
                SYNC(); mono_T_full<true>(lds, A, q, lane, wv, p);
            }
        }
    } else if constexpr (SCH == POLYPHASE_STAR) {
#pragma unroll
        for (int kk = 0; kk < L::K; kk++) {
            const int k = INV ? L::K - 1 - kk : kk;
            const float p = L::p(k), u = L::u(k);
            if (!INV) predict_local(q, p);
            else mono_unupdate_local(q, u);
            const int A = buf();
            publish<LL>(lds, A, q, lane, wv); publish<HL>(lds, A + 1, q, lane, wv);
            publish<LH>(lds, A + 2, q, lane, wv); publish<HH>(lds, A + 3, q, lane, wv);
            SYNC();
            if (!INV) {
                poly_N<false>(lds, A, q, lane, wv, p, u);
                update_local(q, u);
            } else {
                poly_N<true>(lds, A, q, lane, wv, p, u);
                mono_unpredict_local(q, p);
            }
        }
    }
#undef SYNC
}

template <int SCH>
constexpr int lds_planes() { return 2 * buf_planes<SCH>(); }

template <int WAV, int SCH>
__global__ __launch_bounds__(NTHREADS) void k_tile_forward(FwdArgs a, int ntx, int ntiles)
{
    constexpr int HQ = Lift<WAV>::K;
    constexpr int IX = TX - 2 * HQ, IY = TY - 2 * HQ;
    __shared__ float lds[lds_planes<SCH>() * PSZ];
    const int tile = xcd_tile(ntiles);
    if (tile < 0) return;
    poison_lds(lds, lds_planes<SCH>() * PSZ);
    const int lane = threadIdx.x & (TX - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / TX);  // wavefront-uniform
    const int tc = tile % ntx, tr = tile / ntx;
    const int W = a.W, H = a.H;
    const int QW = (W + 1) >> 1, QH = (H + 1) >> 1, WH = W >> 1, HH_ = H >> 1;
    const int qc = tc * IX - HQ + lane;
    const int x0 = ws_mirror(2 * qc, W), x1 = ws_mirror(2 * qc + 1, W);

    Quads q;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int qr = tr * IY - HQ + j * NWAVES + wv;
        const float *r0 = a.in + (ptrdiff_t)ws_mirror(2 * qr, H) * a.in_pitch;
        const float *r1 = a.in + (ptrdiff_t)ws_mirror(2 * qr + 1, H) * a.in_pitch;
        q.v[j][LL] = r0[x0];
        q.v[j][HL] = r0[x1];
        q.v[j][LH] = r1[x0];
        q.v[j][HH] = r1[x1];
    }
    // Tile constant: mean of the middle quadruple row (256 samples).
    float c;
    {
        const int qm = tr * IY - HQ + TY / 2;
        const float *m0 = a.in + (ptrdiff_t)ws_mirror(2 * qm, H) * a.in_pitch;
        const float *m1 = a.in + (ptrdiff_t)ws_mirror(2 * qm + 1, H) * a.in_pitch;
        const float sum = wave_sum((m0[x0] + m0[x1]) + (m1[x0] + m1[x1]));
        c = rintf(sum * (1.0f / (4 * TX)) * recip_pow2(a.quantum)) * a.quantum;
    }
#pragma unroll
    for (int j = 0; j < NJ; j++)
#pragma unroll
        for (int e = 0; e < 4; e++) q.v[j][e] -= c;

    transform_tile<WAV, SCH, false>(lds, q, lane, wv);

    if (lane < HQ || lane >= TX - HQ || qc >= QW) return;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const int qr = tr * IY - HQ + r;
        if (r < HQ || r >= TY - HQ || qr >= QH) continue;
        a.ll[(ptrdiff_t)qr * a.ll_pitch + qc] = fmaf(q.v[j][LL], a.s.ll, c * a.ll_gain);
        float *drow = a.det + (ptrdiff_t)qr * a.det_pitch;
        if (qc < WH) drow[QW + qc] = q.v[j][HL];
        if (qr < HH_) {
            float *hrow = a.det + (ptrdiff_t)(QH + qr) * a.det_pitch;
            hrow[qc] = q.v[j][LH];
            if (qc < WH) hrow[QW + qc] = q.v[j][HH] * a.s.hh;
        }
    }
}

template <int WAV, int SCH>
__global__ __launch_bounds__(NTHREADS) void k_tile_inverse(InvArgs a, int ntx, int ntiles)
{
    constexpr int HQ = Lift<WAV>::K;
    constexpr int IX = TX - 2 * HQ, IY = TY - 2 * HQ;
    __shared__ float lds[lds_planes<SCH>() * PSZ];
    const int tile = xcd_tile(ntiles);
    if (tile < 0) return;
    poison_lds(lds, lds_planes<SCH>() * PSZ);
    const int lane = threadIdx.x & (TX - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / TX);  // wavefront-uniform
    const int tc = tile % ntx, tr = tile / ntx;
    const int W = a.W, H = a.H;
    const int QW = (W + 1) >> 1, QH = (H + 1) >> 1;
    const int qc = tc * IX - HQ + lane;
    // Coefficient columns of the mirrored L and H samples (mirroring keeps parity).
    const int cl = ws_mirror(2 * qc, W) >> 1, ch = ws_mirror(2 * qc + 1, W) >> 1;

    // Tile constant in the pixel domain from the LL coefficients of the middle
    // quadruple row: LL of a constant image c is c * ll_gain.
    float c;
    {
        const int qm = tr * IY - HQ + TY / 2;
        const int rm = ws_mirror(2 * qm, H) >> 1;
        const float sum = wave_sum(a.ll[(ptrdiff_t)rm * a.ll_pitch + cl]);
        c = rintf(sum * (1.0f / TX) * recip_pow2(a.ll_gain * a.quantum)) * a.quantum;
    }
    const float cll = c * a.ll_gain;

    Quads q;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int qr = tr * IY - HQ + j * NWAVES + wv;
        const int rl = ws_mirror(2 * qr, H) >> 1, rh = ws_mirror(2 * qr + 1, H) >> 1;
        const float *lrow = a.det + (ptrdiff_t)rl * a.det_pitch;
        const float *hrow = a.det + (ptrdiff_t)(QH + rh) * a.det_pitch;
        q.v[j][LL] = (a.ll[(ptrdiff_t)rl * a.ll_pitch + cl] - cll) * a.inv_s.ll;
        q.v[j][HL] = lrow[QW + ch];
        q.v[j][LH] = hrow[cl];
        q.v[j][HH] = hrow[QW + ch] * a.inv_s.hh;
    }

    transform_tile<WAV, SCH, true>(lds, q, lane, wv);

    if (lane < HQ || lane >= TX - HQ || qc >= QW) return;
    const int px = 2 * qc;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int r = j * NWAVES + wv;
        const int qr = tr * IY - HQ + r;
        if (r < HQ || r >= TY - HQ || qr >= QH) continue;
        const int py = 2 * qr;
        float *o0 = a.out + (ptrdiff_t)py * a.out_pitch;
        o0[px] = q.v[j][LL] + c;
        if (px + 1 < W) o0[px + 1] = q.v[j][HL] + c;
        if (py + 1 < H) {
            float *o1 = o0 + a.out_pitch;
            o1[px] = q.v[j][LH] + c;
            if (px + 1 < W) o1[px + 1] = q.v[j][HH] + c;
        }
    }
}

// Transform-only tile (see NoneArgs): the scheme's transform_tile on samples
// synthesised from the quadruple coordinates, without the image loads, the
// centring and the stores.
template <int WAV, int SCH, bool INV>
__global__ __launch_bounds__(NTHREADS) void k_tile_none(NoneArgs a, int ntx, int ntiles)
{
    constexpr int HQ = Lift<WAV>::K;
    constexpr int IX = TX - 2 * HQ, IY = TY - 2 * HQ;
    __shared__ float lds[lds_planes<SCH>() * PSZ];
    const int tile = xcd_tile(ntiles);
    if (tile < 0) return;
    const int lane = threadIdx.x & (TX - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / TX);  // wavefront-uniform
    const int tc = tile % ntx, tr = tile / ntx;
    const int qc = tc * IX - HQ + lane;
    Quads q;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int qr = tr * IY - HQ + j * NWAVES + wv;
#pragma unroll
        for (int e = 0; e < 4; e++) q.v[j][e] = (float)((qc * 3 + qr * 5 + e * 7) & 255);
    }
    transform_tile<WAV, SCH, INV>(lds, q, lane, wv);
    // The checksum takes the values the level kernel would store (interior
    // rows and lanes); halo values may come from LDS cells no work-group
    // writes.
    float acc = 0.0f;
    if (lane >= HQ && lane < TX - HQ) {
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int r = j * NWAVES + wv;
            if (r >= HQ && r < TY - HQ) acc += (q.v[j][LL] + q.v[j][HL]) + (q.v[j][LH] + q.v[j][HH]);
        }
    }
    if (__float_as_uint(acc) == a.key) a.sink[0] = acc;
}

struct Grid {
    int ntx, ntiles, blocks;
};

template <int WAV>
Grid tile_grid(int W, int H)
{
    constexpr int HQ = Lift<WAV>::K;
    const int QW = (W + 1) / 2, QH = (H + 1) / 2;
    const int ix = TX - 2 * HQ, iy = TY - 2 * HQ;
    Grid g;
    g.ntx = (QW + ix - 1) / ix;
    const int nty = (QH + iy - 1) / iy;
    g.ntiles = g.ntx * nty;
    g.blocks = (g.ntiles + 7) / 8 * 8;
    return g;
}

template <int WAV, int SCH>
hipError_t fwd(const FwdArgs &a, hipStream_t s)
{
    const Grid g = tile_grid<WAV>(a.W, a.H);
    return launch(k_tile_forward<WAV, SCH>, dim3(g.blocks), dim3(NTHREADS), s, a, g.ntx, g.ntiles);
}

template <int WAV, int SCH>
hipError_t inv(const InvArgs &a, hipStream_t s)
{
    const Grid g = tile_grid<WAV>(a.W, a.H);
    return launch(k_tile_inverse<WAV, SCH>, dim3(g.blocks), dim3(NTHREADS), s, a, g.ntx, g.ntiles);
}

template <int WAV, int SCH>
hipError_t none(bool inverse, const NoneArgs &a, hipStream_t s)
{
    const Grid g = tile_grid<WAV>(a.W, a.H);
    return inverse ? launch(k_tile_none<WAV, SCH, true>, dim3(g.blocks), dim3(NTHREADS), s, a, g.ntx, g.ntiles)
                   : launch(k_tile_none<WAV, SCH, false>, dim3(g.blocks), dim3(NTHREADS), s, a, g.ntx, g.ntiles);
}

template <int WAV>
hipError_t none_scheme(bool inverse, int scheme, const NoneArgs &a, hipStream_t s)
{
    switch (scheme) {
    case MONO_STAR_TILE: return none<WAV, MONO_STAR_TILE>(inverse, a, s);
    case SWELDENS: return none<WAV, SWELDENS>(inverse, a, s);
    case IWAHASHI: return none<WAV, IWAHASHI>(inverse, a, s);
    case MONOLITHIC: return none<WAV, MONOLITHIC>(inverse, a, s);
    case EXPLOSIVE: return none<WAV, EXPLOSIVE>(inverse, a, s);
    case EXPLOSIVE_STAR: return none<WAV, EXPLOSIVE_STAR>(inverse, a, s);
    case IWAHASHI_STAR: return none<WAV, IWAHASHI_STAR>(inverse, a, s);
    case POLYPHASE_STAR: return none<WAV, POLYPHASE_STAR>(inverse, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int WAV>
hipError_t fwd_scheme(int scheme, const FwdArgs &a, hipStream_t s)
{
    switch (scheme) {
    case MONO_STAR_TILE: return fwd<WAV, MONO_STAR_TILE>(a, s);
    case SWELDENS: return fwd<WAV, SWELDENS>(a, s);
    case IWAHASHI: return fwd<WAV, IWAHASHI>(a, s);
    case MONOLITHIC: return fwd<WAV, MONOLITHIC>(a, s);
    case EXPLOSIVE: return fwd<WAV, EXPLOSIVE>(a, s);
    case EXPLOSIVE_STAR: return fwd<WAV, EXPLOSIVE_STAR>(a, s);
    case IWAHASHI_STAR: return fwd<WAV, IWAHASHI_STAR>(a, s);
    case POLYPHASE_STAR: return fwd<WAV, POLYPHASE_STAR>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int WAV>
hipError_t inv_scheme(int scheme, const InvArgs &a, hipStream_t s)
{
    switch (scheme) {
    case MONO_STAR_TILE: return inv<WAV, MONO_STAR_TILE>(a, s);
    case SWELDENS: return inv<WAV, SWELDENS>(a, s);
    case IWAHASHI: return inv<WAV, IWAHASHI>(a, s);
    case MONOLITHIC: return inv<WAV, MONOLITHIC>(a, s);
    case EXPLOSIVE: return inv<WAV, EXPLOSIVE>(a, s);
    case EXPLOSIVE_STAR: return inv<WAV, EXPLOSIVE_STAR>(a, s);
    case IWAHASHI_STAR: return inv<WAV, IWAHASHI_STAR>(a, s);
    case POLYPHASE_STAR: return inv<WAV, POLYPHASE_STAR>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_tile_forward(int wavelet, int scheme, const FwdArgs &a, hipStream_t s)
{
    if (wavelet == CDF53) return fwd_scheme<CDF53>(scheme, a, s);
    if (wavelet == CDF97) return fwd_scheme<CDF97>(scheme, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_tile_none(bool inverse, int wavelet, int scheme, const NoneArgs &a, hipStream_t s)
{
    if (a.W < 2 || a.H < 2) return hipErrorInvalidValue;
    if (wavelet == CDF53) return none_scheme<CDF53>(inverse, scheme, a, s);
    if (wavelet == CDF97) return none_scheme<CDF97>(inverse, scheme, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_tile_inverse(int wavelet, int scheme, const InvArgs &a, hipStream_t s)
{
    if (wavelet == CDF53) return inv_scheme<CDF53>(scheme, a, s);
    if (wavelet == CDF97) return inv_scheme<CDF97>(scheme, a, s);
    return hipErrorInvalidValue;
}

}  // namespace dwt2
