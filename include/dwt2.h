/*
 * dwt2.h -- C ABI of libdwt2: 2-D forward and inverse discrete wavelet
 * transform by CDF 5/3, CDF 9/7 and Deslauriers-Dubuc 13/7 lifting on AMD
 * MI355X (gfx950).
 *
 * Method: D. Barina, M. Kula, P. Zemcik, "Parallel Wavelet Schemes for
 * Images".  One level of the 2-D transform maps each quadruple of input
 * samples (LL, HL, LH, HH) = (x[2r][2c], x[2r][2c+1], x[2r+1][2c],
 * x[2r+1][2c+1]) to the four subband coefficients at (r, c) (Sec. 2,
 * "Convolution and Polyphase Schemes": the 4x4 polyphase matrix N_{P,U}).
 * Levels are applied in sequence to the LL band (Sec. 1).  The default
 * scheme is the paper's Monolithic* (Sec. 4, "Improvements"): per lifting
 * pair one spatial predict step T_{P1} plus the scalar parts T^H_{P0},
 * T^V_{P0}, and one spatial update step S_{U1} plus S^H_{U0}, S^V_{U0},
 * separated by two barriers.  Every scheme gives the result of separable
 * lifting (Conclusions), up to FP32 rounding.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * - Samples are FP32.  Pitches are in ELEMENTS (floats), >= width, as
 *   torch.Tensor.stride(0).  Pointers are DEVICE pointers, 4-byte aligned.
 * - Phase: L = x[2n], H = x[2n+1]; a row of width W has ceil(W/2) L and
 *   floor(W/2) H samples (odd sizes allowed).
 * - Borders: whole-sample symmetric extension, period 2(N-1) (the paper
 *   does not fix a border rule; this one keeps the transform of a symmetric
 *   signal symmetric and needs no extra coefficients).
 * - Coefficient layout (Mallat): for a W x H level input, LL occupies the
 *   top-left ceil(H/2) x ceil(W/2) block, HL (horizontal high, vertical low)
 *   the top-right ceil(H/2) x floor(W/2) block, LH the bottom-left
 *   floor(H/2) x ceil(W/2) block, HH the bottom-right.  Multi-level output is
 *   recursive in the LL block.
 * - Every level's input must be at least 2 x 2: width_k = ceil(W / 2^(k-1))
 *   and height_k >= 2 for k = 1..levels, and width * height <= 2^38, else
 *   DWT2_E_SIZE.
 * - Ownership: the caller owns src, dst and workspace.  The library never
 *   allocates memory and never synchronises: work is enqueued on `stream`
 *   (0 = the null stream) and completes asynchronously; faults surface at
 *   the caller's next synchronisation.  src is read only; src and dst must
 *   not overlap (DWT2_E_ALIAS).  Calls are reentrant; calls that share a
 *   workspace or dst on different streams race.
 * - Errors are returned as status codes (no exceptions cross the ABI).
 *   Arguments are validated on the host before anything is enqueued.
 */
#ifndef DWT2_H
#define DWT2_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DWT2_VERSION 5

/*
 * The enums below have int as their underlying type in C++ as well as in C,
 * so any int a caller passes for one of them is a value of that type and is
 * answered with a status code (DWT2_E_UNSUPPORTED for unknown values).
 */
#ifdef __cplusplus
#define DWT2_ENUM(name) enum name : int
#else
#define DWT2_ENUM(name) enum name
#endif

/* Status codes. */
#define DWT2_OK 0
#define DWT2_E_ARG (-1)         /* null pointer, non-positive size, pitch < width, an image spanning
                                   more than 2^60 elements ((height - 1) * pitch + width), bad levels */
#define DWT2_E_SIZE (-2)        /* some level's input is smaller than 2 x 2 */
#define DWT2_E_UNSUPPORTED (-3) /* unknown wavelet, extension, normalisation, scheme or arithmetic */
#define DWT2_E_WORKSPACE (-4)   /* workspace missing or smaller than dwt2_workspace_bytes() */
#define DWT2_E_ALIAS (-5)       /* src and dst (or workspace) overlap */
#define DWT2_E_HIP (-6)         /* a HIP launch failed; see dwt2_last_hip_error() */
#define DWT2_E_STATE (-7)       /* server stopping, or unknown / already collected ticket */

/* Wavelets (Sec. 5, "Evaluation"). */
typedef DWT2_ENUM(dwt2_wavelet) {
    DWT2_CDF53 = 0, /* P = -1/2 (1 + z^-1), U = 1/4 (1 + z): one lifting pair */
    DWT2_CDF97 = 1, /* two lifting pairs alpha, beta, gamma, delta */
    DWT2_DD137 = 2  /* (4,4) Deslauriers-Dubuc: P = 1/16 (z + z^-2) - 9/16 (1 + z^-1),
                       U = 9/32 (1 + z) - 1/32 (z^-1 + z^2); MONOLITHIC_STAR only */
} dwt2_wavelet;

/* Boundary extension.  Only whole-sample symmetric is implemented. */
typedef DWT2_ENUM(dwt2_ext) { DWT2_EXT_WHOLE_SYMMETRIC = 0 } dwt2_ext;

/*
 * Normalisation, applied once per 2-D level to LL and HH (HL and LH have
 * scale 1 in both).  PAPER is the paper's scaling step diag(zeta, 1/zeta)
 * per axis (Sec. 2; zeta = sqrt(2) for 5/3, 1.14960439886... for 9/7):
 * LL * zeta^2, HH / zeta^2 (DD 13/7: the paper gives no zeta; sqrt(2) as for
 * 5/3).  UNIT_DC scales so that a constant image keeps its value in LL (5/3
 * and DD 13/7: no scaling; 9/7: LL / K^2, HH * K^2 with K = 1.23017410491...).
 * Per level k the two differ by exact powers of two:
 * PAPER = UNIT_DC * 2^(k-1) * {2 for LL, 1 for HL and LH, 1/2 for HH}.
 */
typedef DWT2_ENUM(dwt2_norm) { DWT2_NORM_UNIT_DC = 0, DWT2_NORM_PAPER = 1 } dwt2_norm;

/*
 * Scheme of the per-level kernel.  All give the same coefficients up to FP32
 * rounding (bit-identical for integer input with CDF 5/3).
 *   MONOLITHIC_STAR       the paper's Monolithic* steps (Sec. 4) in the fused
 *                         kernel: a tile plus halo per work-group held in
 *                         registers, horizontal neighbours by wavefront
 *                         shifts, LDS only at the seams between wavefronts,
 *                         2 barriers per lifting pair.  AUTO selects it.
 *   MONOLITHIC_STAR_TILE  the same steps in the block-based tile harness (every
 *                         neighbour exchanged through LDS, 2 barriers per pair).
 *   SWELDENS              separable steps T^H_P | T^V_P | S^H_U | S^V_U in the
 *                         tile harness, 4 barriers per pair (Sec. 2).
 *   IWAHASHI              earlier non-separable T^I_P | R^I_{P,U} | S^I_U in the
 *                         tile harness, 3 barriers per pair (Sec. 2).
 *   ROWCOL                separable row pass then column pass through memory.
 * The remaining variants of the paper, all in the tile harness:
 *   MONOLITHIC            unsplit T_P | S_U (Sec. 3), 2 barriers per pair.
 *   EXPLOSIVE             T^E_P | R^E_{P,U} | S^E_U (Sec. 3), 3 barriers.
 *   EXPLOSIVE_STAR        Explosive with the scalar parts P0, U0 split off
 *                         (Sec. 4), 3 barriers.
 *   IWAHASHI_STAR         Iwahashi with P0, U0 split off (Sec. 4), 3 barriers.
 *   POLYPHASE_STAR        scalar P0 parts, then N_{P1,U1} as one step, then
 *                         scalar U0 parts (Sec. 4): 1 barrier per pair.
 */
typedef DWT2_ENUM(dwt2_scheme) {
    DWT2_SCHEME_AUTO = 0,
    DWT2_SCHEME_MONOLITHIC_STAR = 1,
    DWT2_SCHEME_SWELDENS = 2,
    DWT2_SCHEME_IWAHASHI = 3,
    DWT2_SCHEME_ROWCOL = 4,
    DWT2_SCHEME_MONOLITHIC_STAR_TILE = 5,
    DWT2_SCHEME_MONOLITHIC = 6,
    DWT2_SCHEME_EXPLOSIVE = 7,
    DWT2_SCHEME_EXPLOSIVE_STAR = 8,
    DWT2_SCHEME_IWAHASHI_STAR = 9,
    DWT2_SCHEME_POLYPHASE_STAR = 10
} dwt2_scheme;

/*
 * Arithmetic of the lifting steps.  Samples and coefficients are FP32 in
 * memory in every case.  FP64 keeps the intermediate values of the fused
 * MONOLITHIC_STAR kernel in double precision (other schemes: FP32 only,
 * DWT2_E_UNSUPPORTED).  AUTO selects FP32.
 */
typedef DWT2_ENUM(dwt2_arith) { DWT2_ARITH_AUTO = 0, DWT2_ARITH_FP32 = 1, DWT2_ARITH_FP64 = 2 } dwt2_arith;

/*
 * Tile height of the fused MONOLITHIC_STAR kernel.  A work-group lifts one
 * overlapping tile of 64 x (4 * tile_rows) quadruples (128 x 8 * tile_rows
 * pixels) in registers, the block-based layout of Sec. 6; tall tiles re-read
 * fewer halo rows, short tiles give small levels more work-groups.  Built
 * heights (FP32 lifting): 5/3 {2, 3}, 9/7 {2, 3, 4}, DD 13/7 {3, 6};
 * FP64 lifting: 5/3 {3}, 9/7 {4}, DD 13/7 {6}.  Every height gives bitwise
 * identical coefficients (each tile takes its centring constant from a fixed
 * band of rows that contains its outputs), so the choice changes speed only.
 * 0 selects per level: the entry dwt2_autotune recorded for this wavelet,
 * direction and level size, else the tallest height that still gives at
 * least the wavelet's fill threshold of tiles (5/3: 256, 9/7: 512, DD 13/7:
 * 1536), else the shortest.  Another
 * value, or a nonzero value with another scheme or with the batched calls,
 * returns DWT2_E_UNSUPPORTED.
 */

/*
 * LDS buffering of the fused MONOLITHIC_STAR kernel (Sec. 6 and Table 2).
 * Each spatial step publishes the two components it reads across rows to
 * LDS planes.  Double buffering (2, the default) gives the predict and update
 * steps separate planes, so one barrier per step suffices: a step's planes are
 * rewritten two steps later, after the next step's barrier.  Single buffering
 * (1) overwrites one set of planes in place, adding a barrier between a step's
 * reads and the next publication (2 barriers per step, half the LDS).  Both
 * give bitwise identical results, with FP32 or FP64 lifting.  0 selects 2,
 * except with FP64 lifting, where it selects 1 (double-buffered FP64 planes
 * would leave room for fewer work-groups per compute unit).  Another value,
 * or a nonzero value with another scheme or with the batched calls returns
 * DWT2_E_UNSUPPORTED.
 */

/*
 * Tile order of the fused MONOLITHIC_STAR kernel: how the chip's eight XCDs
 * (each with its own L2) share a level's tiles.  RUNS: each XCD takes a
 * contiguous row-major run of tiles.  BANDS: each XCD takes one eighth of the
 * tile columns and sweeps them from the top down, so that all XCDs work on
 * the same rows at a time.  In both, most neighbouring tiles run on the same
 * XCD and share their halo in its L2.  Not in the paper; it changes speed
 * only, never the result.  AUTO selects per level: the entry
 * dwt2_autotune recorded, else BANDS for levels of at least 5 x 2^25
 * pixels and 2048 pixels width, else RUNS.  A nonzero value with another scheme or with
 * the batched calls returns DWT2_E_UNSUPPORTED.
 */
typedef DWT2_ENUM(dwt2_order) {
    DWT2_ORDER_AUTO = 0,
    DWT2_ORDER_RUNS = 1,
    DWT2_ORDER_BANDS = 2
} dwt2_order;

/*
 * Fused multi-level tail of the MONOLITHIC_STAR kernel (fuse_tail = 1).  The
 * levels whose input is at most 128 x 128 pixels, from the first such level
 * on (when at least two remain), run in one work-group that keeps the LL
 * bands between them in LDS: one launch instead of one per level.  The
 * coefficients are bitwise those of the per-level launches.  The tail runs
 * its tiles one after another (about 2.8 us each), while a launched level
 * runs its tiles side by side: measured slower than the per-level launches
 * for every image tried (64^2 to 1024^2), so it is off by default.
 * DWT2_E_UNSUPPORTED for fuse_tail = 1 with FP64 arithmetic or with another
 * scheme, for any value other than 0 and 1, and for a nonzero value passed
 * to the batched calls, dwt2_autotune or the server.
 */

/* Optional settings; pass NULL for defaults (UNIT_DC, AUTO, AUTO, 0, 0, AUTO, 0). */
typedef struct dwt2_options {
    int norm;        /* dwt2_norm */
    int scheme;      /* dwt2_scheme */
    int arithmetic;  /* dwt2_arith */
    int tile_rows;   /* fused-kernel tile height (above); 0 = automatic */
    int lds_buffers; /* fused-kernel LDS buffering (above); 0 = double */
    int tile_order;  /* dwt2_order (above) */
    int fuse_tail;   /* 1: fused multi-level tail (above); 0 = off */
    int reserved[1]; /* must be zero */
} dwt2_options;

/*
 * Bytes of device workspace dwt2_forward / dwt2_inverse need for these
 * arguments (0 when levels == 1 and the scheme needs none).  Writes *bytes.
 * Returns DWT2_OK or an argument/size/unsupported status.
 */
int dwt2_workspace_bytes(dwt2_wavelet wavelet, int levels, int width, int height,
                         const dwt2_options *opt, size_t *bytes);

/*
 * Forward transform: src is a width x height image (pitch src_pitch), dst
 * receives the Mallat layout of `levels` levels (pitch dst_pitch).  One level
 * is the separable 2-D decomposition into LL, HL, LH and HH of Sec. 1 and of
 * Sec. 2 ("Discrete Wavelet Transform": Mallat's pyramid, each level applied
 * to the previous LL); the default scheme computes it with the Monolithic*
 * steps of Sec. 4 ("Improvements"), the others with their sections' steps.
 * workspace: device memory of at least dwt2_workspace_bytes() bytes (may be
 * NULL when that is 0), not overlapping src or dst.
 */
int dwt2_forward(dwt2_wavelet wavelet, int levels, int width, int height,
                 const float *src, ptrdiff_t src_pitch, float *dst, ptrdiff_t dst_pitch,
                 dwt2_ext ext, const dwt2_options *opt, void *workspace,
                 size_t workspace_bytes, hipStream_t stream);

/*
 * Inverse transform: src holds the Mallat layout produced by dwt2_forward
 * with the same wavelet, levels, sizes and normalisation; dst receives the
 * width x height image.  The paper gives the forward direction only; each
 * level undoes the forward level's steps in reverse order with negated
 * lifting coefficients and reciprocal scales (every lifting step of Sec. 2,
 * "Lifting Scheme", is inverted by subtracting what it added), so the
 * Monolithic* inverse keeps the two barriers per lifting pair of Sec. 4.
 * Same argument rules as dwt2_forward.
 */
int dwt2_inverse(dwt2_wavelet wavelet, int levels, int width, int height,
                 const float *src, ptrdiff_t src_pitch, float *dst, ptrdiff_t dst_pitch,
                 dwt2_ext ext, const dwt2_options *opt, void *workspace,
                 size_t workspace_bytes, hipStream_t stream);

/*
 * Allocation-free transform, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): dwt2_forward (inverse == 0) or dwt2_inverse (inverse != 0)
 * with the same arguments except the workspace, which is a device array of
 * DWT2_NOALLOC_SCRATCH_BYTES inside the library (each device the library
 * runs on holds its own copy until the process ends).  The call allocates
 * nothing and frees nothing; on its first use on a device it looks up that
 * device's copy (a HIP symbol query, no allocation).  A call whose
 * dwt2_workspace_bytes() exceeds DWT2_NOALLOC_SCRATCH_BYTES returns
 * DWT2_E_WORKSPACE and enqueues nothing (one-level calls need no workspace,
 * so any size works; two levels up to 8192 x 8192; deeper ones up to about
 * 50 Mpixel, e.g. 7000 x 7000).  Every call on a device shares that
 * device's array: calls that overlap in time on one device (on different
 * streams, or from threads whose streams are not ordered) race on it and
 * give wrong results; calls ordered on one stream do not.  The array needs no clearing: every call
 * writes the workspace before reading it.  Statuses as dwt2_forward.
 */
#define DWT2_NOALLOC_SCRATCH_BYTES 67108864 /* 64 MiB */
int dwt2_transform_noalloc(int inverse, dwt2_wavelet wavelet, int levels, int width, int height,
                           const float *src, ptrdiff_t src_pitch, float *dst, ptrdiff_t dst_pitch,
                           dwt2_ext ext, const dwt2_options *opt, hipStream_t stream);

/*
 * Transform-only measurement (the paper's Sec. 6 mode that leaves out the
 * input and output of data, used by its Experiments 1 and 2).  Enqueues one
 * level of the forward (inverse == 0) or inverse transform of a width x height
 * image with the kernel `opt` selects (scheme, and for MONOLITHIC_STAR the
 * tile height, buffering and order, as dwt2_forward would pick them), except
 * that no image memory is read or written: every tile synthesises its samples
 * in registers from its coordinates, lifts them with all of the scheme's
 * arithmetic, wavefront shifts, LDS traffic and barriers, and keeps the
 * results.  Each work-group compares a checksum of its results with a NaN
 * pattern that finite data never produce and would store it to sink[0] on a
 * match, so the compiler keeps all the work and nothing is stored.  For
 * timing only; the result is not a transform of anything.  sink: a device
 * pointer to 4 writable bytes, 4-byte aligned.  FP32 lifting only; ROWCOL and
 * fuse_tail -> DWT2_E_UNSUPPORTED; sizes as dwt2_forward with levels = 1.
 */
int dwt2_transform_only(int inverse, dwt2_wavelet wavelet, int width, int height,
                        const dwt2_options *opt, float *sink, hipStream_t stream);

/*
 * Batched transforms
 * ------------------
 * Many independent images, each with its own wavelet, level count and size,
 * in one call.  The paper transforms one image at a time; levels of one image
 * depend on each other through LL (Sec. 1), images do not.  The library
 * launches one kernel per level index k, covering the tiles of every image
 * that has a level k, plus a few small kernels that copy the call's image
 * table into the workspace (their arguments carry the data, so the call may
 * be captured in a HIP graph; the caller's dwt2_image array may be reused as
 * soon as the call returns).  Each image gets exactly the coefficients
 * (resp. samples) that the single-image call with the same arguments gives.
 *
 * Scheme: AUTO or MONOLITHIC_STAR (others DWT2_E_UNSUPPORTED); norm and
 * arithmetic as for single images, shared by the whole batch.
 * Errors: every image is checked as by dwt2_forward (its status is returned
 * for the first failing image); count < 0 or count > DWT2_BATCH_MAX, a null
 * array with count > 0, or a total of more than 2^31 - 8 tiles in one level
 * -> DWT2_E_ARG; any overlap between one image's dst and another image's src
 * or dst, or between the workspace and any image -> DWT2_E_ALIAS (ranges are
 * the bytes from an image's first to its last element).  count == 0 enqueues
 * nothing.  Calls that share a workspace race unless ordered on one stream.
 */
#define DWT2_BATCH_MAX 65536

typedef struct dwt2_image {
    int wavelet;         /* dwt2_wavelet */
    int levels;          /* >= 1, every level's input >= 2 x 2 */
    int width, height;   /* level-0 size (forward input, inverse output) */
    const float *src;    /* forward: image; inverse: Mallat coefficients */
    ptrdiff_t src_pitch; /* elements */
    float *dst;          /* forward: Mallat coefficients; inverse: image */
    ptrdiff_t dst_pitch; /* elements */
} dwt2_image;

/* Bytes of device workspace a batched call over these images needs (0 when count == 0). */
int dwt2_batch_workspace_bytes(const dwt2_image *images, int count, const dwt2_options *opt,
                               size_t *bytes);

/* Forward transform of `count` images; workspace aligned to 256 bytes. */
int dwt2_forward_batch(const dwt2_image *images, int count, dwt2_ext ext,
                       const dwt2_options *opt, void *workspace, size_t workspace_bytes,
                       hipStream_t stream);

/* Inverse transform of `count` images (src = coefficients, dst = images). */
int dwt2_inverse_batch(const dwt2_image *images, int count, dwt2_ext ext,
                       const dwt2_options *opt, void *workspace, size_t workspace_bytes,
                       hipStream_t stream);

/*
 * Tile heights of a batched call.  Each image's level runs at the height
 * dwt2_autotune recorded for its wavelet, direction and level size (FP32
 * lifting), else at its wavelet's tallest built height; when the level
 * launch would then have fewer work-groups than the largest fill threshold
 * among the untuned images' wavelets, those images step down to shorter
 * heights together until it has, as far as the built heights go (the rule
 * of dwt2_options.tile_rows, applied to the launch instead of one image).
 * FP64 lifting runs at its one height.  Heights change speed only, never the result.  Writes
 * rows[0..count) for level `level` (0-based) of the forward (inverse == 0) or
 * inverse call with these arguments: an image's height, or 0 when it has no
 * such level.  Statuses as dwt2_batch_workspace_bytes; level < 0 or a null
 * rows with count > 0 -> DWT2_E_ARG.
 */
int dwt2_batch_tile_rows(int inverse, const dwt2_image *images, int count,
                         const dwt2_options *opt, int level, int *rows);

/*
 * Serving loop (continuous batching)
 * ----------------------------------
 * A server takes single-image requests from any number of host threads and
 * runs them through the batched transform on one stream.  A scheduler thread
 * forms each batch from the requests pending at that moment (first come,
 * first served, at most max_batch), as long as fewer than max_inflight
 * batches are enqueued and not finished; so under light load a request is
 * launched at once, and under heavy load batches grow.  Admission is by HBM
 * footprint: a batch's workspace (image table + each image's LL buffers)
 * is carved from the caller's device arena, and a request waits while the
 * arena is full; with max_footprint_mib set, a request also waits while the
 * requests in flight plus it would touch more than that many bytes of device
 * memory, counting each request's input and output spans and its LL
 * buffers.  A completion thread retires finished batches (in stream order)
 * and records each request's latency (submission to observed completion,
 * host clock).
 *
 * Ordering: requests whose buffers overlap (one writes what another reads or
 * writes) never share a batch, and batches run in submission order on the
 * stream, so a request may consume an earlier request's output.  Within a
 * batch the forward and the inverse group run concurrently: the inverse group
 * on a second stream the server creates, forked from the caller's stream
 * (after its earlier work) and joined back into it (before its later work).
 * Each request gets exactly the result of dwt2_forward / dwt2_inverse with
 * the server's options.  The arena, and every request's src and dst, are
 * owned by the caller and must stay valid until the request completes.
 */
typedef struct dwt2_server dwt2_server;

typedef struct dwt2_request {
    int inverse;         /* 0 = forward (src image -> dst coefficients), 1 = inverse */
    int wavelet;         /* dwt2_wavelet */
    int levels;
    int width, height;
    const float *src;
    ptrdiff_t src_pitch; /* elements */
    float *dst;
    ptrdiff_t dst_pitch; /* elements */
} dwt2_request;

typedef struct dwt2_server_config {
    int max_batch;         /* requests per batch, 1..DWT2_BATCH_MAX (0 = 256) */
    int max_inflight;      /* batches enqueued and not finished, >= 1 (0 = 2) */
    int max_footprint_mib; /* cap on the HBM footprint of the requests in flight, MiB
                              (0 = no cap beyond the arena) */
    int reserved[5];       /* must be zero */
} dwt2_server_config;

typedef struct dwt2_completion {
    int status;        /* DWT2_OK or the status of the failed launch */
    double queue_us;   /* submission -> batch enqueued */
    double latency_us; /* submission -> completion observed */
} dwt2_completion;

/*
 * Start a server.  opt: shared normalisation / arithmetic (scheme AUTO or
 * MONOLITHIC_STAR); cfg may be NULL.  arena: device memory (256-byte
 * aligned) for batch workspaces.  Creates threads and HIP events; no device
 * memory is allocated.  *out receives the handle.
 */
int dwt2_server_create(const dwt2_options *opt, const dwt2_server_config *cfg, void *arena,
                       size_t arena_bytes, hipStream_t stream, dwt2_server **out);

/*
 * Queue one request; returns at once.  The request is validated as by
 * dwt2_forward (status returned, nothing queued); a request whose workspace
 * alone exceeds the arena, or whose footprint alone exceeds the footprint
 * cap, gives DWT2_E_WORKSPACE, one overlapping the arena DWT2_E_ALIAS.
 * *ticket identifies it for dwt2_server_wait.
 */
int dwt2_server_submit(dwt2_server *server, const dwt2_request *request,
                       unsigned long long *ticket);

/*
 * Block until the request `ticket` has completed; fill *done (may be NULL)
 * and return its status.  Each ticket can be waited for once.
 */
int dwt2_server_wait(dwt2_server *server, unsigned long long ticket, dwt2_completion *done);

/*
 * Submit requests[i] at arrival_us[i] microseconds after the call starts
 * (non-decreasing; the calling thread spins until each arrival time), then
 * wait for all of them and fill done[i].  A load generator for measuring
 * latency under a given arrival process.  Returns DWT2_OK, or the first
 * submission error (requests before it are still waited for).
 */
int dwt2_server_replay(dwt2_server *server, const dwt2_request *requests,
                       const double *arrival_us, int count, dwt2_completion *done);

/* Finish every queued request, stop the threads and free the handle. */
int dwt2_server_destroy(dwt2_server *server);

/*
 * Tile autotuning
 * ---------------
 * Not in the paper, which fixes one work-group size per platform (Sec. 6).
 * The tile height only trades halo re-reads against work-groups in flight,
 * and the tile order only changes how the XCDs meet HBM (see dwt2_options),
 * so both are tuned by measurement, per level size.
 *
 * dwt2_autotune runs the transform that dwt2_forward (inverse == 0) or
 * dwt2_inverse (inverse != 0) runs with the same arguments and leaves the same
 * result in dst.  It first waits for the work already on `stream`, then runs
 * on a stream of its own: for each level, every built FP32 height in both
 * tile orders is captured as a HIP graph of `repeats` back-to-back launches,
 * and the graphs are replayed in five interleaved passes (each starting at
 * another candidate, after one untimed replay of each) timed with HIP events.
 * A candidate's time is the median of its passes.  The height and order the
 * rules above pick are kept unless another candidate is faster by more than
 * the spread (slowest minus fastest pass) of either, and the choice is
 * recorded for (wavelet, direction, level width, level height) in a table
 * shared by the process (entries are replaced; the table holds at most 4096
 * entries, further sizes are not recorded).  Later FP32 calls with
 * tile_rows == 0 (tile_order == AUTO) use the recorded height (order) of a
 * level of that exact size, and batched calls the recorded height.  The
 * call creates and destroys a stream, two events and the graphs; it
 * allocates no device memory of its own.
 * Argument rules are those of dwt2_forward; the scheme must be AUTO or
 * MONOLITHIC_STAR, the arithmetic AUTO or FP32, tile_rows, lds_buffers and
 * tile_order 0, else DWT2_E_UNSUPPORTED; repeats must be in [1, 1000], else
 * DWT2_E_ARG.  The call blocks until its work is done and must not be
 * called while `stream` is being captured.  The table is locked internally:
 * any thread may call any function.
 */
int dwt2_autotune(int inverse, dwt2_wavelet wavelet, int levels, int width, int height,
                  const float *src, ptrdiff_t src_pitch, float *dst, ptrdiff_t dst_pitch,
                  dwt2_ext ext, const dwt2_options *opt, void *workspace, size_t workspace_bytes,
                  int repeats, hipStream_t stream);

/*
 * Height the fused kernel uses for one width x height level of a call with
 * these options (tile_rows, the FP64 height, the table, or the rule above).
 * Writes *rows.  DWT2_E_UNSUPPORTED when the options do not select the fused
 * kernel; DWT2_E_ARG / DWT2_E_SIZE for bad sizes or a null pointer.
 */
int dwt2_tile_rows(int inverse, dwt2_wavelet wavelet, int width, int height,
                   const dwt2_options *opt, int *rows);

/*
 * Tile order (DWT2_ORDER_RUNS or DWT2_ORDER_BANDS) the fused kernel uses for
 * one width x height level of a call with these options (tile_order, the
 * table, or the rule of dwt2_options).  Writes *order.  Statuses as
 * dwt2_tile_rows.
 */
int dwt2_tile_order(int inverse, dwt2_wavelet wavelet, int width, int height,
                    const dwt2_options *opt, int *order);

/*
 * The table as text, one entry per line: "wavelet inverse width height rows
 * order" (decimal, single spaces, '\n' after each line; order 0 for an entry
 * imported without one), in ascending key order.
 * Writes up to cap bytes of it plus a terminating NUL into buf (buf may be
 * NULL when cap is 0) and the full length without the NUL into *len.
 * DWT2_E_SIZE when cap <= *len (buf then holds no partial line: buf[0] is NUL
 * if cap > 0).
 */
int dwt2_tune_export(char *buf, size_t cap, size_t *len);

/*
 * Add the entries of text in dwt2_tune_export's format to the table
 * (replacing entries of the same key); a line may omit the order (then the
 * rule picks it).  The whole text is checked first: a malformed line, an
 * unknown wavelet, a size below 2, a height that is not built for that
 * wavelet or an order other than 0, 1, 2 leaves the table unchanged and
 * returns DWT2_E_ARG; more entries than the table holds, DWT2_E_SIZE.
 */
int dwt2_tune_import(const char *text);

/* Empty the table. */
int dwt2_tune_reset(void);

/* Static text for a status code ("unknown status" for others). */
const char *dwt2_status_string(int status);

/* hipError_t of the last DWT2_E_HIP returned on the calling thread (0 if none). */
int dwt2_last_hip_error(void);

/*
 * Fault injection for tests of error handling: the next `count` kernel
 * launches the calling thread makes through the library return
 * hipErrorInvalidConfiguration without launching anything (so the call that
 * makes one returns DWT2_E_HIP, and dwt2_last_hip_error() that code); 0
 * turns it off.  Launches made by a server's own threads are not affected.
 * count < 0 -> DWT2_E_ARG.
 */
int dwt2_debug_fail_launches(int count);

/* DWT2_VERSION of the loaded library. */
int dwt2_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DWT2_H */
