// dwt2_internal.h -- shared declarations of the libdwt2 kernels and host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dwt2 {

enum Wavelet : int { CDF53 = 0, CDF97 = 1, DD137 = 2 };
// Scheme ids as in dwt2.h; MONO_STAR is the fused register-blocked kernel,
// ROWCOL the two-pass kernels, all others run in the LDS tile harness.
enum Scheme : int {
    MONO_STAR = 1, SWELDENS = 2, IWAHASHI = 3, ROWCOL = 4, MONO_STAR_TILE = 5,
    MONOLITHIC = 6, EXPLOSIVE = 7, EXPLOSIVE_STAR = 8, IWAHASHI_STAR = 9, POLYPHASE_STAR = 10
};

// Lifting pairs in the L = x[2n], H = x[2n+1] phase.  The paper's operators
// (Sec. 5) P(z) = p (1 + z^-1) and U(z) = u (1 + z) become, after the index
// relabelling of H, P = p (1 + z) (predict H[n] from L[n], L[n+1]) and
// U = u (1 + z^-1) (update L[n] from H[n-1], H[n]).  The scalar part of each
// operator (Sec. 4's P0, U0) is p resp. u; the neighbour part (P1, U1) is
// p z resp. u z^-1.
//
// CDF 9/7 values (not printed in the paper): alpha..delta follow from
// factoring the 4-vanishing-moment CDF filters built on the real root of
// 1 + 4y + 10y^2 + 20y^3; K is the DC gain of the unscaled low-pass and
// zeta = sqrt(2) / K the paper's scaling factor.
template <int W>
struct Lift;

template <>
struct Lift<CDF53> {
    static constexpr int K = 1;  // lifting pairs
    __host__ __device__ static constexpr float p(int) { return -0.5f; }
    __host__ __device__ static constexpr float u(int) { return 0.25f; }
};

template <>
struct Lift<CDF97> {
    static constexpr int K = 2;
    __host__ __device__ static constexpr float p(int k)
    {
        return k == 0 ? -1.58613434205992355842832f : 0.88291107553093329591979f;
    }
    __host__ __device__ static constexpr float u(int k)
    {
        return k == 0 ? -0.0529801185729614146241296f : 0.443506852043971152115604f;
    }
};

// DD 13/7 (Sec. 5): P(z) = 1/16 (z + z^-2) - 9/16 (1 + z^-1) and
// U(z) = 9/32 (1 + z) - 1/32 (z^-1 + z^2).  In the L = x[2n] phase the
// predict reads L[n-1..n+2] and the update H[n-2..n+1]; p and u are the
// scalar parts P0, U0 (the taps at n).  The neighbour taps are listed where
// the kernels use them.
template <>
struct Lift<DD137> {
    static constexpr int K = 1;
    __host__ __device__ static constexpr float p(int) { return -0.5625f; }
    __host__ __device__ static constexpr float u(int) { return 0.28125f; }
};

// Per-level scale of LL and HH (HL and LH are unscaled in both normalisations).
struct Scale {
    float ll, hh;
};

// Row pitch (floats) of an LL buffer of width w in the library's workspace: a
// multiple of 64 floats, so every row starts on a 256-byte boundary and the
// kernels' 8-byte vector accesses apply whatever the width.
__host__ __device__ __forceinline__ ptrdiff_t ll_pitch(int w) { return ((ptrdiff_t)w + 63) & ~(ptrdiff_t)63; }

// 1 / x for a normal power of two x, exactly: the exponent field reflected
// about that of 1.  Dividing by x and multiplying by this give the same bits.
__host__ __device__ __forceinline__ float recip_pow2(float x)
{
    return __builtin_bit_cast(float, 0x7F000000u - __builtin_bit_cast(unsigned, x));
}

// Whole-sample symmetric extension: index j -> [0, n), period 2(n-1), n >= 2.
__host__ __device__ __forceinline__ int ws_mirror(int j, int n)
{
    if ((unsigned)j < (unsigned)n) return j;
    const int p = 2 * (n - 1);
    j %= p;
    if (j < 0) j += p;
    return j >= n ? p - j : j;
}

// One forward level: `in` (W x H) -> LL into `ll`, HL/LH/HH into the Mallat
// positions of `det` (HL at column ceil(W/2), LH at row ceil(H/2)).
//
// Centering (tile kernels): a tile may subtract any constant c from all the
// samples it reads and add the transform of the constant image back, which is
// c * ll_gain in LL and zero elsewhere; by linearity the result is unchanged.
// c is rounded to a multiple of `quantum` (the level input's power-of-two
// scale), so integer data stay integer and results scale exactly with it.
struct FwdArgs {
    const float *in;
    ptrdiff_t in_pitch;
    float *ll;
    ptrdiff_t ll_pitch;
    float *det;
    ptrdiff_t det_pitch;
    int W, H;
    Scale s;
    float ll_gain;  // LL of a constant image c is c * ll_gain (1 UNIT_DC, 2 PAPER)
    float quantum;  // c is a multiple of this power of two
};

// One inverse level: LL from `ll`, HL/LH/HH from `det` -> `out` (W x H).
struct InvArgs {
    const float *ll;
    ptrdiff_t ll_pitch;
    const float *det;
    ptrdiff_t det_pitch;
    float *out;
    ptrdiff_t out_pitch;
    int W, H;
    Scale inv_s;  // reciprocal scales
    float ll_gain;
    float quantum;
};

// Test hook (dwt2_debug_fail_launches): true when the calling thread's next
// launch is to fail without running; counts that launch down.
bool take_launch_failure();

// Launch `kern` with `lds` bytes of dynamic LDS and return the status of this
// launch only (hipLaunchKernel does not report errors left behind by earlier,
// unrelated HIP calls).
template <typename... Args>
inline hipError_t launch_lds(void (*kern)(Args...), dim3 grid, dim3 block, size_t lds, hipStream_t s,
                             Args... args)
{
    if (take_launch_failure()) return hipErrorInvalidConfiguration;
    void *argv[] = {(void *)&args...};
    return hipLaunchKernel((const void *)kern, grid, block, argv, lds, s);
}
template <typename... Args>
inline hipError_t launch(void (*kern)(Args...), dim3 grid, dim3 block, hipStream_t s, Args... args)
{
    return launch_lds(kern, grid, block, 0, s, args...);
}

// LDS poisoning (test builds with DWT2_POISON_LDS): every work-group fills
// its LDS with NaN before its first LDS access, so a read of a cell that the
// work-group has not written since it started shows in the results.
#ifdef DWT2_POISON_LDS
template <typename T>
__device__ __forceinline__ void poison_lds(T *lds, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = (T)__builtin_nan("");
    __syncthreads();
}
#else
template <typename T>
__device__ __forceinline__ void poison_lds(T *, int) {}
#endif

// Launchers (return the hipError_t of the launch).
hipError_t launch_tile_forward(int wavelet, int scheme, const FwdArgs &a, hipStream_t s);
hipError_t launch_tile_inverse(int wavelet, int scheme, const InvArgs &a, hipStream_t s);

// Fused Monolithic* (registers + DPP, LDS only at wavefront seams).
// A tile is 64 quadruple columns by 4 * rows quadruple rows; `rows` (rows per
// wavefront) is one of kFusedRows[wavelet] for FP32 lifting and
// kFusedRowsFp64[wavelet] for FP64 (hipErrorInvalidValue otherwise).  Every
// height gives bitwise identical coefficients: the centring constant of a
// tile is taken from a fixed cell of rows that contains the tile's outputs.
// fp64: lift in double-precision registers (samples stay FP32 in memory).
constexpr int kFusedRowsMax = 3;
constexpr int kFusedRows[3][kFusedRowsMax] = {{2, 3, 0}, {2, 3, 4}, {3, 6, 0}};
constexpr int kFusedRowsFp64[3] = {3, 4, 6};
bool fused_rows_supported(int wavelet, bool fp64, int rows);
// buffers: 2 = double-buffered LDS planes (one barrier per spatial step), 1 =
// single-buffered (two per step).  order: the order in which the
// XCDs take the tiles, kOrderRuns (each XCD a contiguous row-major run) or
// kOrderBands (each XCD a band of tile columns, all on the same rows at a
// time); it changes speed only.
constexpr int kOrderRuns = 1, kOrderBands = 2;
hipError_t launch_fused_forward(int wavelet, bool fp64, int rows, int buffers, int order,
                                const FwdArgs &a, hipStream_t s);
hipError_t launch_fused_inverse(int wavelet, bool fp64, int rows, int buffers, int order,
                                const InvArgs &a, hipStream_t s);
// Tiles of the fused kernel for one W x H level at `rows` (0 when a side is
// below 2 or the height is not built).
long long fused_tile_count(int wavelet, int rows, int W, int H);

// Multi-level tail in one work-group: levels k0 .. levels - 1 of one image
// (FP32, the wavelet's tallest built height, double-buffered planes), with
// the LL bands between them kept in LDS.  Every tile runs the per-level
// kernel's tile body, so the coefficients are bitwise those of the
// per-level launches.  Forward: `in` is level k0's input (pitch in_pitch),
// `out` the Mallat array.  Inverse: `in` is the Mallat array, `out` receives
// level k0's output.  The LDS holds the planes and two LL buffers of
// tail_buffer_elems(W, H, k0) floats each; kTailSide bounds level k0's sides
// so that this stays within 64 KiB.
constexpr int kTailSide = 128;
struct TailArgs {
    const float *in;
    ptrdiff_t in_pitch;
    float *out;
    ptrdiff_t out_pitch;
    int W, H;        // level-0 size of the image
    int k0, levels;  // the tail's first level and the image's level count
    Scale s;         // forward scales, or the inverse's reciprocals
    float ll_gain;
    int paper;       // centring quantum 2^k (PAPER) or 1
    int buf_elems;   // floats per LDS LL buffer
};
int tail_buffer_elems(int W, int H, int k0);
size_t tail_lds_bytes(int wavelet, int buf_elems);
hipError_t launch_fused_tail_forward(int wavelet, const TailArgs &t, hipStream_t s);
hipError_t launch_fused_tail_inverse(int wavelet, const TailArgs &t, hipStream_t s);

// Batched fused launches.  One record per image, in device memory; a level
// launch covers the tiles of every image that has that level.  The buffer
// roles per level are those of the single-image level loop:
//   forward level k reads `src` (k = 0) or buf[(k-1)&1] (pitch = level width)
//   and writes LL to `dst` (last level) or buf[k&1] (pitch = LL width);
//   inverse level k reads LL from `src` (last level) or buf[k&1] and writes
//   `dst` (k = 0) or buf[(k-1)&1]; details are always in the Mallat array.
struct BatchImage {
    const float *src;  // forward: image; inverse: coefficients
    float *dst;        // forward: coefficients; inverse: image
    float *buf[2];     // LL ping-pong (unused when levels == 1)
    ptrdiff_t src_pitch, dst_pitch;
    int W, H;          // level-0 size
    int wavelet, levels;
};
static_assert(sizeof(BatchImage) == 64, "BatchImage is a 64-byte record");

// One batched level.  `start` has count + 1 entries: the tiles of image i are
// [start[i], start[i+1]) (empty when the image has no level k); start[count]
// is the total.  tile_image[t] is the image of tile t (written on the device
// by k_batch_index from `start`).  rows[i] is image i's tile height at this
// level, one of the built heights of its wavelet (FP64 lifting:
// kFusedRowsFp64).
struct BatchLevel {
    const BatchImage *imgs;
    const int *start;
    const unsigned short *tile_image;
    const unsigned char *rows;
    int count, ntiles, level;
    Scale s[3];     // per wavelet: forward scales, or reciprocals for the inverse
    float ll_gain;
    float quantum;
};

// Bytes of a batched call's workspace before the tile-image index and the
// per-image LL buffers: the image records, the tile-start table and the
// tile-height table, each 256-byte aligned.
size_t batch_table_bytes(int count, int lmax);

// Tile-image index of a batched call: for each level k, the image of every
// tile of that level's launch, as 16-bit image numbers (count <= 65536), at
// offset off[k] tiles into the index.  k_batch_index fills it from the
// tile-start table, one work-group per (image, level).
constexpr int kBatchMaxLevels = 32;
struct BatchIndexArgs {
    const int *start;       // lmax x (count + 1)
    unsigned short *index;  // the index
    int count, lmax;
    long long off[kBatchMaxLevels];
};
hipError_t launch_batch_index(const BatchIndexArgs &a, hipStream_t s);

// Tallest built FP32 tile height of a wavelet (heights are listed ascending).
constexpr int tallest_rows(int wavelet)
{
    return kFusedRows[wavelet][kFusedRowsMax - 1] > 0 ? kFusedRows[wavelet][kFusedRowsMax - 1]
                                                      : kFusedRows[wavelet][kFusedRowsMax - 2];
}
// has_dd: the batch holds a DD 13/7 image (its taller tile needs more LDS).
hipError_t launch_batch_forward(bool fp64, bool has_dd, const BatchLevel &b, hipStream_t s);
hipError_t launch_batch_inverse(bool fp64, bool has_dd, const BatchLevel &b, hipStream_t s);
// Copy `bytes` (a multiple of 4) from host memory to device memory `dst` with
// kernels whose arguments carry the data: stream-ordered and capturable, and
// the host buffer may be reused as soon as the call returns.
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s);

// Transform-only launches (the measurement mode of Sec. 6 that leaves out the
// image input and output): the level's grid of tiles, each synthesising its
// samples in registers from its coordinates, lifting them exactly as the
// scheme's level kernel does (every FMA, wavefront shift, LDS access and
// barrier), and folding its results into a checksum that is stored to
// sink[0] only if its bit pattern equals `key`.  The host passes a NaN
// pattern that lifting finite samples never produces, so nothing is stored
// and no image memory is touched, while no computation can be dropped.
struct NoneArgs {
    int W, H;
    float *sink;
    unsigned key;
};
hipError_t launch_fused_none(bool inverse, int wavelet, int rows, int buffers, int order,
                             const NoneArgs &a, hipStream_t s);
hipError_t launch_tile_none(bool inverse, int wavelet, int scheme, const NoneArgs &a, hipStream_t s);

// Row-column: the intermediate `tmp` is W x H with pitch tmp_pitch.
hipError_t launch_rowcol_forward(int wavelet, const FwdArgs &a, float *tmp, ptrdiff_t tmp_pitch,
                                 hipStream_t s);
hipError_t launch_rowcol_inverse(int wavelet, const InvArgs &a, float *tmp, ptrdiff_t tmp_pitch,
                                 hipStream_t s);

}  // namespace dwt2
