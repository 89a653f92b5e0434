/*
 * cdef_oracle.h -- plain, slow, single-threaded CPU CDEF.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the product path never does.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Everything follows "The AV1 Constrained Directional Enhancement Filter
 * (CDEF)" (Midtskogen and Valin):
 *   Section 2, Eq. (1)-(5) and Algorithm 1 ... direction search
 *   Section 3, Eq. (6)-(12) ................... constrained directional filter
 *   Section 3.2, Eq. (13) ..................... strength ranges, bit depth,
 *                                               chroma damping, adjustment
 *   Section 4 ................................. 64x64 filter blocks, skip
 *   Section 5 ................................. per-filter-block SSE D_{b,p},
 *                                               Eq. (14) weighting, Eq. (15) presets
 *
 * Readings of points where the paper is silent or garbled are listed in the
 * source file next to the code that takes them.
 *
 * All sample buffers are host memory, uint16, row-major with a stride in
 * samples.  Integer arithmetic only; every result is exact.
 */
#ifndef CDEF_ORACLE_H
#define CDEF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Chroma layouts. */
enum { CDEF_ORACLE_400 = 0, CDEF_ORACLE_420 = 1, CDEF_ORACLE_422 = 2, CDEF_ORACLE_444 = 3 };

/* One frame.  nplanes = 1 (4:0:0) or 3; chroma planes are ceil(width/2) x
 * ceil(height/2) at 4:2:0, ceil(width/2) x height at 4:2:2, width x height
 * at 4:4:4.  bitdepth 8..12. */
typedef struct {
  const uint16_t *plane[3];
  int64_t stride[3];
  int32_t width, height; /* luma size */
  int32_t bitdepth;
  int32_t nplanes;
  int32_t layout;
} cdef_oracle_frame;

/* Line number k of pixel (i, j) (row i, column j, 0..7) of an 8x8 block for
 * direction d (0..7): the lost Fig. 1, read as described in the source. */
int cdef_oracle_line_number(int d, int i, int j);

/* Algorithm 1's s[d] (Eq. 5 times 840) for the bw x bh in-frame top-left
 * part of one 8x8 block (1 <= bw, bh <= 8). */
void cdef_oracle_direction_costs(const uint16_t *px, int64_t stride, int bw, int bh,
                                 int bitdepth, int64_t cost[8]);

/* Algorithm 1 on every 8x8 luma block: dir and var are [ceil(h/8)][ceil(w/8)]. */
void cdef_oracle_find_dir(const uint16_t *luma, int64_t stride, int width, int height,
                          int bitdepth, uint8_t *dir, int32_t *var);

/* Eq. (7): the constraint function f(d, S, D). */
int cdef_oracle_constrain(int diff, int strength, int damping);

/* Eq. (13): the luma primary strength after adjustment by the block's
 * directional contrast v. */
int cdef_oracle_adjust_strength(int strength, int32_t var);

/* Section 3.2: chroma damping for luma damping D and chroma primary S. */
int cdef_oracle_chroma_damping(int damping, int pri_strength);

/* Eq. (8)-(12) for one pixel of one plane.  pri/sec strengths and damping are
 * the values actually used by f (already scaled to the bit depth); w1, w2 are
 * the primary weights of the inner and outer tap (in 1/16). */
int cdef_oracle_filter_pixel(const uint16_t *p, int64_t stride, int pw, int ph, int i, int j,
                             int dir, int pri_strength, int pri_damping, int w1, int w2,
                             int sec_strength, int sec_damping);

/* Filter a whole frame (Sections 3-4).  dir/var from cdef_oracle_find_dir,
 * skip [ceil(h/8)][ceil(w/8)] (NULL = no skipped blocks), strengths
 * [ceil(h/64)][ceil(w/64)][4] = (pri_y, sec_y, pri_uv, sec_uv) in the 8-bit
 * domain, bit 7 of sec_y / sec_uv = the luma / chroma skip condition bit
 * (with strengths 0, 0 it selects the (19, 7) preset), damping = luma D
 * (3..6).  A filter block whose 8x8 blocks are all skipped is copied. */
void cdef_oracle_filter_frame(const cdef_oracle_frame *in, uint16_t *const out[3],
                              const int64_t out_stride[3], const uint8_t *dir,
                              const int32_t *var, const uint8_t *skip, int damping,
                              const uint8_t *strengths);

/* Planes that the searches cover: luma only at 4:0:0 and 4:2:2 (whose chroma
 * is never filtered), all three otherwise. */
int cdef_oracle_search_planes(const cdef_oracle_frame *f);

/* Section 5: SSE of one 64x64 filter block (fby, fbx) for every plane and
 * every (S^(p) = 0..15, S^(s) in {0,1,2,4}) pair, filtering the block in full
 * for each pair.  sse is [nplanes][16][4]. */
void cdef_oracle_search_fb(const cdef_oracle_frame *recon, const cdef_oracle_frame *src,
                           const uint8_t *dir, const int32_t *var, const uint8_t *skip,
                           int damping, int fby, int fbx, uint64_t *sse);

/* The same with nskip = 2: also the 64 presets with the skip condition bit
 * set (Section 5, 128 combinations).  sse is [nplanes][nskip][16][4]. */
void cdef_oracle_search_fb2(const cdef_oracle_frame *recon, const cdef_oracle_frame *src,
                            const uint8_t *dir, const int32_t *var, const uint8_t *skip,
                            int damping, int nskip, int fby, int fbx, uint64_t *sse);

/* The same restricted to a subset of the presets (R22): cand = S^(p) mask
 * (bits 0-15) | S^(s) index mask << 16 | skip condition bit mask << 20, or
 * 0 for all; entries outside the subset are UINT64_MAX. */
void cdef_oracle_search_fb3(const cdef_oracle_frame *recon, const cdef_oracle_frame *src,
                            const uint8_t *dir, const int32_t *var, const uint8_t *skip,
                            int damping, int nskip, uint32_t cand, int fby, int fbx,
                            uint64_t *sse);

/* Section 5, Eq. (14): the contrast-weighted distortion of filter block
 * (fby, fbx) for the 64 pairs (skip condition bit off), summed over the
 * block's filtering units (8x8 luma, 4x4 chroma at 4:2:0); C1 = 6.25 * 4^(b-8),
 * C2 = 312.5 * 16^(b-8).  dist is double [nplanes][16][4]. */
void cdef_oracle_search_fb_weighted(const cdef_oracle_frame *recon,
                                    const cdef_oracle_frame *src, const uint8_t *dir,
                                    const int32_t *var, const uint8_t *skip, int damping,
                                    int fby, int fbx, double *dist);

/* The whole-frame search: find_dir, then every filter block.
 * sse is [nplanes][ceil(h/64)][ceil(w/64)][16][4]; dir/var as find_dir. */
void cdef_oracle_search(const cdef_oracle_frame *recon, const cdef_oracle_frame *src,
                        const uint8_t *skip, int damping, uint64_t *sse,
                        uint8_t *dir, int32_t *var);

/* Section 5, Eq. (15): preset selection on an SSE table sse
 * [nplanes][nfb][ncand] (as cdef_oracle_search / search_fb2, filter blocks
 * flattened; ncand = 64 or 128).
 * Luma distortion D^l[b][p] = plane 0; chroma D^c[b][p] = planes 1 + 2 (0 for
 * nplanes = 1).  For each group a greedy sequence of 8 presets is built (each
 * step adds the candidate that most lowers sum_b min over the set, lowest
 * candidate index on ties); for N = 1, 2, 4, 8 the greedy prefix is then
 * re-optimized one preset at a time for up to refine_passes passes (a slot
 * takes the best candidate given the others, only on a strict improvement).
 * J(N) = lambda * B * log2(N) + D^l(N) + D^c(N) with B = nfb; the smallest N
 * of minimal J is chosen.  Outputs: n_chosen; sets_l/sets_c [4][8] (slot
 * entries >= N are -1); dist [2][4] (luma, chroma; N = 1, 2, 4, 8); cost[4];
 * per-block preset slots fb_l / fb_c (lowest slot on ties) for N*.
 * cand_mask: two words, bit p = candidate p may be chosen (NULL: all); at
 * least 8 candidates must be allowed. */
void cdef_oracle_select_presets(const uint64_t *sse, int nplanes, int nfb, int ncand,
                                const uint64_t *cand_mask, double lambda, int refine_passes, int32_t *n_chosen, int32_t *sets_l,
                                int32_t *sets_c, uint64_t *dist, double *cost, uint8_t *fb_l,
                                uint8_t *fb_c);

#ifdef __cplusplus
}
#endif

#endif
