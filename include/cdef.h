/*
 * cdef.h -- C ABI of the MI355X (gfx950) CDEF library, libcdef_hip.so.
 *
 * CDEF is the constrained directional enhancement filter of Midtskogen and
 * Valin, "The AV1 Constrained Directional Enhancement Filter (CDEF)".  The
 * library runs the data-parallel part of it on the GPU:
 *   - the per-8x8 direction search (Section 2, Eq. 1-5, Algorithm 1),
 *   - the constrained primary/secondary directional filter (Section 3,
 *     Eq. 6-13) over 64x64 filter blocks (Section 4),
 *   - the encoder's strength search: every 64x64 filter block filtered under
 *     every (primary, secondary) strength pair and scored by SSE against the
 *     source (Section 5, the distortion D_{b,p} with D = ||s - d||^2).
 *
 * Conventions shared by every entry point
 *   - Every buffer pointer is a DEVICE pointer (hipMalloc, or the data of a
 *     GPU tensor).  The caller owns and allocates all of them; none may
 *     alias an output of the same call.  The library keeps no per-call state.
 *   - Samples are uint16, row-major, `stride` counted in samples
 *     (stride >= plane width).  Values must be < 2^bitdepth: larger values
 *     are a contract violation (memory-safe, result unspecified).
 *   - Luma is plane 0.  With CDEF_LAYOUT_420 the chroma planes 1 and 2 are
 *     ceil(width/2) x ceil(height/2); with CDEF_LAYOUT_400 they are unused.
 *   - Per-8x8 maps (dir, var, skip) are [ceil(h/8)][ceil(w/8)] row-major
 *     over the luma plane; per-filter-block maps are [ceil(h/64)][ceil(w/64)].
 *     At 4:2:0 a 4x4 chroma block uses the direction and skip flag of its
 *     co-located 8x8 luma block, and a chroma filter block is 32x32.
 *   - Strengths are given in the 8-bit domain (Section 3.2): primary 0..15,
 *     secondary one of {0, 1, 2, 4}; luma damping D is 3..6.  For 10-bit
 *     content the library shifts strengths left by 2 and raises D by 2.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*;
 *     NULL is the null stream).  They return after enqueueing; outputs are
 *     valid once the stream has reached that point.
 *   - Errors: every argument that lives on the host is checked before
 *     anything is enqueued.  A failed check returns CDEF_E_INVAL or
 *     CDEF_E_UNSUPPORTED and writes nothing.  A failed launch returns
 *     CDEF_E_HIP.  Kernels have no data-dependent failure.
 *   - Every entry point is thread-safe.
 */
#ifndef CDEF_H
#define CDEF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CDEF_OK = 0,
  CDEF_E_INVAL = -1,       /* bad argument (null pointer, size, range, aliasing) */
  CDEF_E_UNSUPPORTED = -2, /* valid CDEF input that this library does not handle */
  CDEF_E_HIP = -3,         /* the HIP runtime reported an error */
  CDEF_E_NOMEM = -4,       /* a caller-provided workspace is too small */
  CDEF_E_TIMEOUT = -5      /* never returned by a call: names the outcome of a device-side
                              bounded wait that gave up (cdef_select_presets' result n == 0) */
} cdef_status;

/* Chroma layouts.  4:2:0 and 4:2:2 chroma planes are ceil(w/2) wide, 4:2:0
 * ones ceil(h/2) high; 4:4:4 chroma has the luma size.  Section 4: at 4:2:2
 * (subsampling differing horizontally and vertically) chroma is never
 * filtered -- the filter copies it and the searches cover luma only; at
 * 4:4:4 each 8x8 chroma block follows the co-located luma block. */
enum { CDEF_LAYOUT_400 = 0, CDEF_LAYOUT_420 = 1, CDEF_LAYOUT_422 = 2, CDEF_LAYOUT_444 = 3 };

/* One frame.  plane[1..2] may be NULL for CDEF_LAYOUT_400.  bitdepth is 8, 10
 * or 12 (Section 3.2: strengths scaled by 2^(b-8), damping raised by b-8). */
typedef struct {
  const uint16_t *plane[3];
  int64_t stride[3];
  int32_t width, height; /* luma size, >= 1 each */
  int32_t bitdepth;
  int32_t layout;
} cdef_frame;

/* Writable planes of a filtered frame; geometry is that of the input. */
typedef struct {
  uint16_t *plane[3];
  int64_t stride[3];
} cdef_frame_out;

/* The preset of one 64x64 filter block, 8-bit domain (Sections 3.2 and 4).
 * Strength ranges: pri 0..15, sec in {0, 1, 2, 4}.  Bit 7 of sec_y / sec_uv
 * is the luma / chroma skip condition bit (CDEF_SKIP_CONDITION): with it, the
 * block's skipped 8x8 blocks are filtered too, and strengths (0, 0) then mean
 * S^(p) = 19, S^(s) = 7.  A filter block whose in-frame 8x8 blocks are all
 * skipped is never filtered.  The bytes are read on the device; a value out
 * of range is a contract violation (the kernel masks pri to 4 bits and
 * treats sec > 4 as 4, and stays memory-safe). */
typedef struct {
  uint8_t pri_y, sec_y, pri_uv, sec_uv;
} cdef_strength;

#define CDEF_SKIP_CONDITION 0x80

/* Direction search, Section 2 and Algorithm 1, on the luma plane of `f`.
 *   dir[b]: the direction 0..7 that minimizes E_d^2 of Eq. (2) (ties go to
 *           the lowest d).  Direction 0 is the 45-degree line rising to the
 *           right; each step turns 22.5 degrees clockwise (2 = horizontal,
 *           6 = vertical).
 *   var[b]: the directional contrast of Algorithm 1, s_best - s_orthogonal,
 *           with s_d of Eq. (5) scaled by 840; 0 <= var <= 880,803,840.
 *   Pixels above 8 bits are reduced to 8 bits (low bits dropped) first.
 *   Blocks cut by the frame edge use their in-frame pixels only.
 * Errors: CDEF_E_INVAL for a null frame/plane/output, size < 1, stride <
 * width, unknown layout, bit depth other than 8/10/12; CDEF_E_UNSUPPORTED
 * for a side above 65536. */
cdef_status cdef_find_dir(const cdef_frame *f, uint8_t *dir, int32_t *var, void *stream);

/* Filter a frame, Sections 3 and 4: Eq. (7)-(12) with the luma primary
 * strength adjusted per 8x8 block by Eq. (13) from `var`.
 *   in, out:  same geometry; out must not overlap in.
 *   dir, var: from cdef_find_dir on `in`.
 *   skip8x8:  1 = block has no coded residual and is copied (its co-located
 *             chroma too) unless its filter block's preset has the skip
 *             condition bit; NULL means no block is skipped.
 *   damping:  luma D, 3..6; chroma uses max(D - 1, floor(log2 pri_uv)).
 *   fb:       per-filter-block presets [ceil(h/64)][ceil(w/64)].
 * A luma block whose adjusted primary strength reaches 16..19 (only the
 * (19, 7) preset can) uses damping max(D, floor(log2 S)), since D may never be
 * below floor(log2 S) (Section 3.2).
 * Out-of-frame taps are ignored (Section 3.2); every output pixel is computed
 * from unfiltered input.
 * Errors: as cdef_find_dir, plus CDEF_E_INVAL for damping outside 3..6, a null
 * dir/var/fb/out plane, or out overlapping in. */
cdef_status cdef_filter_frame(const cdef_frame *in, const cdef_frame_out *out,
                              const uint8_t *dir, const int32_t *var,
                              const uint8_t *skip8x8, int32_t damping,
                              const cdef_strength *fb, void *stream);

/* Encoder strength search, Section 5: for every 64x64 filter block b, every
 * plane and every pair (S^(p) = 0..15, S^(s) in {0,1,2,4}) the SSE between
 * the source and the reconstruction filtered with that pair (skip-condition
 * bit off: skipped 8x8 blocks stay unfiltered).  Direction search, filter
 * and SSE run fused; filtered pixels never reach memory.
 *   recon, src: same geometry; src is the uncoded frame.
 *   sse:        uint64 [nplanes][ceil(h/64)][ceil(w/64)][16][4]; the last
 *               index is S^(s) in the order 0, 1, 2, 4.  In-frame pixels only.
 *               nplanes = 3 at 4:2:0 and 4:4:4, 1 at 4:0:0 and 4:2:2.
 *   dir, var:   optional outputs of the direction search (NULL to skip).
 * Errors: as cdef_filter_frame (damping, geometry), CDEF_E_INVAL for a null
 * sse or geometry mismatch between recon and src. */
cdef_status cdef_search_strengths(const cdef_frame *recon, const cdef_frame *src,
                                  const uint8_t *skip8x8, int32_t damping, uint64_t *sse,
                                  uint8_t *dir, int32_t *var, void *stream);

/* The full encoder search of Section 5: the 16 x 4 x 2 = 128 combinations of
 * S^(p), S^(s) and the skip condition bit.  Entry (k, S^(p), S^(s)) is the SSE
 * of the filter block filtered as cdef_filter_frame would with that preset
 * (k = 1: skip condition bit set; (1, 0, 0) is the (19, 7) preset).
 *   sse: uint64 [nplanes][ceil(h/64)][ceil(w/64)][2][16][4].
 * Other arguments and errors as cdef_search_strengths. */
cdef_status cdef_search_strengths128(const cdef_frame *recon, const cdef_frame *src,
                                     const uint8_t *skip8x8, int32_t damping, uint64_t *sse,
                                     uint8_t *dir, int32_t *var, void *stream);

/* The low-complexity search of Section 5: only a subset of the presets,
 * the product of a set of S^(p) values, a set of S^(s) values and a set of
 * skip condition bits, encoded as
 *   candidates = S^(p) mask (bit S, 16 bits)
 *              | S^(s) index mask << 16 (bit i for S^(s) = 0, 1, 2, 4: 4 bits)
 *              | skip condition bit mask << 20 (bit k for the bit k: 2 bits).
 * The work shrinks with the subset: at 8 and 10 bits, strengths outside it
 * are not filtered (at 12 bits every preset is evaluated and the others are
 * only marked).
 *   sse: the 64-combination table of cdef_search_strengths when the skip
 *        mask is 1, else the 128-combination table of
 *        cdef_search_strengths128; entries of presets outside the subset hold
 *        UINT64_MAX.  Pass the same subset (cdef_candidate_mask) to
 *        cdef_select_presets.
 * Errors: as cdef_search_strengths, plus CDEF_E_INVAL for an empty mask or
 * bits above 21. */
cdef_status cdef_search_subset(const cdef_frame *recon, const cdef_frame *src,
                               const uint8_t *skip8x8, int32_t damping, uint32_t candidates,
                               uint64_t *sse, uint8_t *dir, int32_t *var, void *stream);

/* The candidate indices of a subset (bit p of mask[p / 64] for candidate p =
 * 64 * skip bit + 4 * S^(p) + index of S^(s)), as cdef_select_presets takes
 * them; 0 = every preset. */
void cdef_candidate_mask(uint32_t candidates, uint64_t mask[2]);

/* The strength search with the contrast-weighted distortion of Section 5,
 * Eq. (14), instead of the SSE: for every filter block, plane and pair,
 *   sum over filtering units of
 *   (sigma_s^2 + sigma_d^2 + C1) / (2 sqrt(sigma_s^2 sigma_d^2 + C2)) ||s - d||^2,
 * where a filtering unit is an 8x8 luma block or its co-located chroma block
 * (4x4 at 4:2:0, 8x8 at 4:4:4), sigma^2 are population variances over the unit's in-frame
 * pixels, and C1 = 6.25 * 4^(b-8), C2 = 312.5 * 16^(b-8).  The moments are
 * summed exactly in integers and the weight is evaluated in double
 * precision (relative difference to a direct double evaluation ~1e-15).
 *   dist: double [nplanes][ceil(h/64)][ceil(w/64)][16][4] (skip condition
 *         bit off: skipped units enter unfiltered).
 * Other arguments and errors as cdef_search_strengths. */
cdef_status cdef_search_weighted(const cdef_frame *recon, const cdef_frame *src,
                                 const uint8_t *skip8x8, int32_t damping, double *dist,
                                 uint8_t *dir, int32_t *var, void *stream);

/* ---- Batches ----------------------------------------------------------------
 * Many frames -- of any size, bit depth (8, 10, 12), layout and damping -- in one launch
 * over all their 64x64 filter blocks.  Each job is the strength search of
 * cdef_search_strengths, the full search of cdef_search_strengths128, the
 * weighted search of cdef_search_weighted, or the direction search + filter
 * of one frame at its own per-filter-block presets (cdef_find_dir followed by
 * cdef_filter_frame, fused).  Results are bit-identical to the per-frame
 * entry points. */
enum {
  CDEF_MODE_SEARCH = 0,
  CDEF_MODE_FILTER = 1,
  CDEF_MODE_SEARCH128 = 2,
  CDEF_MODE_SEARCH_WEIGHTED = 3
};

typedef struct {
  cdef_frame recon;          /* input frame */
  cdef_frame src;            /* searches: the source frame; filter: ignored */
  cdef_frame_out out;        /* filter: output planes (must not overlap recon); search: ignored */
  const uint8_t *skip8x8;    /* NULL = no skipped block */
  const cdef_strength *fb;   /* filter: per-filter-block strengths; search: ignored */
  uint64_t *sse;             /* searches: table as cdef_search_strengths(128); weighted: the
                                double table of cdef_search_weighted; filter: ignored */
  uint8_t *dir;              /* optional direction-search outputs (both or neither) */
  int32_t *var;
  int32_t damping;           /* luma D, 3..6 */
  int32_t mode;              /* CDEF_MODE_SEARCH, CDEF_MODE_SEARCH128, CDEF_MODE_SEARCH_WEIGHTED
                                or CDEF_MODE_FILTER */
  uint32_t candidates;       /* CDEF_MODE_SEARCH / SEARCH128: preset subset as for
                                cdef_search_subset, 0 = every preset; otherwise 0 */
  int32_t reserved;          /* 0 */
} cdef_job;

/* What cdef_batch_prepare leaves for cdef_batch_launch (host memory, owned by
 * the caller; valid while the workspace is). */
typedef struct {
  const void *table;  /* device job table inside the workspace */
  int32_t njobs;
  int32_t nitems;     /* filter blocks over all jobs */
  int32_t variant;    /* launch variant 0..CDEF_BATCH_VARIANTS-1 (see below), 0 = default */
  int32_t flags;      /* set by cdef_batch_prepare (bit 0: a job needs the extended kernels
                         -- 4:4:4 -- which run at 2 waves per SIMD
                         whatever the variant; bit 1: every job is a filter job, run by
                         the filter-only kernels, to which the variant does not apply);
                         keep */
} cdef_batch_plan;

/* Host-side checks of one job, exactly those cdef_batch_prepare applies to each
 * of its jobs; enqueues nothing.  Lets a scheduler reject a bad request alone
 * instead of failing the batch it would have joined. */
cdef_status cdef_job_validate(const cdef_job *job);

/* Launch variants a tuner may choose between (all bit-identical):
 *   0: at most 3 waves per SIMD (168 VGPRs), XCD-contiguous filter-block order
 *   1: at most 2 waves per SIMD (256 VGPRs), XCD-contiguous order
 *   2: 3 waves per SIMD, plain order
 *   3: 2 waves per SIMD, plain order
 *   4: persistent workgroups at 3 waves per SIMD: as many as fit on the
 *      device at once, each taking filter blocks from work queues (one
 *      contiguous range of filter blocks per XCD; a workgroup whose range is
 *      used up takes from the others) until none is left
 *   5: the same at 2 waves per SIMD
 * Variants 4 and 5 keep their queue counters in the batch workspace and
 * reset them as the launch ends: launches of one prepared batch in these
 * variants must not overlap (issue them on one stream, or order them). */
#define CDEF_BATCH_VARIANTS 6

/* Bytes of device workspace (and of pinned host staging, if used) for a
 * batch of njobs; 0 for njobs < 1. */
size_t cdef_batch_workspace_bytes(int32_t njobs);

/* Validate every job on the host and upload the job table to `workspace`
 * (device memory of at least cdef_batch_workspace_bytes(njobs) bytes).
 * host_staging: pinned host memory of the same size, owned by the caller;
 * the upload is then an asynchronous copy on `stream` and the caller must
 * leave the staging untouched until the stream has passed it.  With
 * host_staging NULL the call waits until the upload is done.  Either way the
 * upload is ordered on `stream` after the work already there.  Errors: CDEF_E_INVAL for a
 * bad job (its index is not reported), CDEF_E_NOMEM if the workspace is too
 * small; nothing is enqueued on error. */
cdef_status cdef_batch_prepare(const cdef_job *jobs, int32_t njobs, void *host_staging,
                               void *workspace, size_t workspace_bytes, cdef_batch_plan *plan,
                               void *stream);

/* One launch over every filter block of a prepared batch, in launch variant
 * plan->variant (CDEF_E_INVAL if out of range).  Enqueues kernels only (no
 * copies, no allocation), so it can be captured in a HIP graph and replayed
 * while the workspace and all job buffers stay valid. */
cdef_status cdef_batch_launch(const cdef_batch_plan *plan, void *stream);

/* Launch parameters of a batch, as a tuner chooses them.
 *   tile_w, tile_h: the work unit; the 64x64 filter block of Section 4 is
 *                   the only one (0 = default; anything else is
 *                   CDEF_E_UNSUPPORTED).
 *   wg_per_cu:      workgroups (of 4 waves) resident per CU, i.e. waves per
 *                   SIMD: 3 (168 VGPRs) or 2 (256 VGPRs); 0 = 3.  The
 *                   extended kernels (4:4:4) always run 2.
 *   cand_group:     strength pairs evaluated per pass over a filter block;
 *                   all 64 at once is the only grouping (0 = default).
 *   order:          0 = XCD-contiguous filter blocks, 1 = plain order.
 *   persistent:     1 = persistent workgroups on work queues (order 0 only). */
typedef struct {
  int32_t tile_w, tile_h, wg_per_cu, cand_group, order, persistent;
} cdef_tuning;

/* The launch variant (above) of a tuning.  Errors: CDEF_E_INVAL for a null
 * argument or an order/persistent value other than 0/1, CDEF_E_UNSUPPORTED
 * for a tile, grouping or occupancy the kernels do not have. */
cdef_status cdef_tuning_variant(const cdef_tuning *t, int32_t *variant);

/* cdef_batch_prepare + cdef_batch_launch in one call: validate the n jobs,
 * upload their table to `workspace` (device, at least
 * cdef_batch_workspace_bytes(n) bytes) in order on `stream`, wait for that
 * upload, and launch in the variant of `t` (NULL: variant 0; the Python
 * binding's tuner supplies a cached tuning).  The library allocates no
 * device memory; the caller owns the workspace, which must outlive the
 * launch.  Errors: those of cdef_tuning_variant and cdef_batch_prepare
 * (nothing is enqueued on error), CDEF_E_HIP from the copy or the launch.
 * The prepare/launch pair remains the form to use under HIP graph capture
 * (the copy and the wait cannot be captured). */
cdef_status cdef_search_batch(const cdef_job *jobs, int32_t n, const cdef_tuning *t,
                              void *workspace, size_t workspace_bytes, void *stream);

/* ---- Preset selection -------------------------------------------------------
 * Section 5, Eq. (15): choose the frame's presets from a strength-search SSE
 * table.  Candidates are numbered as the table's last dimensions: p =
 * S^(p) * 4 + index of S^(s) (order 0, 1, 2, 4) for the 64-combination table
 * of cdef_search_strengths, plus 64 * skip condition bit for the 128 of
 * cdef_search_strengths128.  D^luma_{b,p} is plane 0,
 * D^chroma_{b,p} the sum of planes 1 and 2 (0 for 4:0:0).  For luma and for
 * chroma a greedy sequence of 8 presets is built, each step adding the
 * candidate not yet chosen that most lowers sum_b min over the chosen set
 * (lowest p on ties).  For N = 1, 2, 4, 8 the first N are then re-optimized
 * one preset at a time, for up to refine_passes passes: a slot takes the
 * candidate, not among the other slots, that gives the smallest distortion,
 * when that is strictly smaller.  The cost of Eq. (15),
 *   J(N) = lambda * B * log2(N) + D^luma(N) + D^chroma(N),  B = fb_rows * fb_cols,
 * is evaluated in double precision in exactly that order, and the smallest N
 * of minimal J is chosen.  Each filter block gets, for luma and for chroma,
 * the slot (0..N-1) of its smallest distortion in the chosen set (lowest slot
 * on ties).  As Eq. (15) is printed, the luma and chroma slots of a block are
 * chosen independently. */
typedef struct {
  int32_t n;              /* chosen number of presets N*: 1, 2, 4 or 8 */
  int32_t reserved;
  int32_t luma[4][8];     /* candidates chosen for N = 1, 2, 4, 8; slots >= N hold -1 */
  int32_t chroma[4][8];
  uint64_t dist_luma[4];  /* sum over blocks of the minimum luma distortion, N = 1, 2, 4, 8 */
  uint64_t dist_chroma[4];
  double cost[4];         /* J(N) for N = 1, 2, 4, 8 */
} cdef_preset_result;

/* Bytes of device workspace cdef_select_presets needs (the same for every
 * table size; under 1 MiB). */
size_t cdef_select_presets_workspace_bytes(void);

/* sse:       device, uint64 [nplanes][fb_rows][fb_cols][ncand] as written by
 *            cdef_search_strengths (ncand = 64) or cdef_search_strengths128
 *            (ncand = 128).
 * cand_mask: host, two words, bit p = candidate p may be chosen (NULL: all);
 *            at least 8 of the ncand candidates must be allowed.
 * lambda:    rate multiplier, finite and >= 0.  refine_passes: 0..16.
 * result:    device pointer, written by the kernels.  result->n == 0 reports
 *            that the selection could not complete (its workgroups could not
 *            all run within a second, e.g. behind other work filling the
 *            device); the other fields are then undefined.
 * fb_luma, fb_chroma: device uint8 [fb_rows][fb_cols], the slots for N*.
 * workspace: device memory of cdef_select_presets_workspace_bytes() bytes,
 *            256-byte aligned, owned by the caller; it must not be shared by
 *            calls that may run at the same time.
 * Errors: CDEF_E_INVAL for null pointers, a short or misaligned workspace,
 * nplanes not 1 or 3, ncand not 64 or 128, fewer than 8 allowed candidates,
 * sizes < 1, a bad lambda or refine_passes;
 * CDEF_E_UNSUPPORTED for more than 2^24 filter blocks.  Three kernel launches
 * on `stream`, no allocation, no host synchronization. */
cdef_status cdef_select_presets(const uint64_t *sse, int32_t nplanes, int32_t fb_rows,
                                int32_t fb_cols, int32_t ncand, const uint64_t *cand_mask,
                                double lambda, int32_t refine_passes,
                                cdef_preset_result *result, uint8_t *fb_luma,
                                uint8_t *fb_chroma, void *workspace, size_t workspace_bytes,
                                void *stream);

/* For callers that cannot allocate device memory (code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid allocation):
 * cdef_select_presets without the workspace argument.  Results are those of
 * cdef_select_presets with the same other arguments.
 *   The workspace is a library-owned device array of
 *   CDEF_PRESET_SCRATCH_BYTES bytes, one per device, held from the first
 *   call on that device until the process ends.  It has the same size for
 *   every table (the selection's limit of 2^24 filter blocks still applies:
 *   CDEF_E_UNSUPPORTED beyond it).  Every call on one device uses the same
 *   array and starts by clearing what must start at zero, so calls that may
 *   overlap on one device -- on different streams, or from threads without
 *   ordering -- race and must be serialized by the caller (e.g. one stream).
 *   The array lives on the device of `stream` (the current device for NULL).
 * Allocates nothing: no hipMalloc/hipFree, no host synchronization.
 * Errors: as cdef_select_presets (without the workspace checks), and
 * CDEF_E_HIP if the array's device address cannot be obtained. */
#define CDEF_PRESET_SCRATCH_BYTES 20480
cdef_status cdef_select_presets_noalloc(const uint64_t *sse, int32_t nplanes, int32_t fb_rows,
                                        int32_t fb_cols, int32_t ncand,
                                        const uint64_t *cand_mask, double lambda,
                                        int32_t refine_passes, cdef_preset_result *result,
                                        uint8_t *fb_luma, uint8_t *fb_chroma, void *stream);

/* Human-readable name of a status code (static storage, never NULL). */
const char *cdef_status_str(cdef_status s);

/* ABI revision of this header; bumped on any incompatible change. */
#define CDEF_ABI_VERSION 1
int32_t cdef_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif
