/*
 * cdef_oracle.c -- plain CPU CDEF, the test oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Written from the paper's text, equation by equation, with no blocking,
 * vectorization or factorization: the encoder search below filters every
 * filter block once per strength pair and sums squared errors.
 *
 * Readings taken where the paper is silent, ambiguous or garbled (the
 * figures that would fix the geometry are lost from the available text):
 *
 *  R1  Direction labels (Fig. 1): d = 0 is the 45-degree line rising to the
 *      right, and each step of d turns the line 22.5 degrees clockwise on
 *      screen (row index grows downward), so d = 2 is horizontal, d = 4 the
 *      falling diagonal, d = 6 vertical.  The orthogonal direction is d + 4
 *      (Algorithm 1), a 45-degree turn is two steps (Section 3.1).
 *  R2  Line numbers (Fig. 1): d0 i+j, d1 i+floor(j/2), d2 i, d3 i-floor(j/2),
 *      d4 i-j, d5 j-floor(i/2), d6 j, d7 j+floor(i/2) (offset so k >= 0).
 *      This gives N_{1,0} = 2 and N_{1,4} = 8 as the text states, 90 lines
 *      in total and 34 distinct (direction, N) pairs, matching the
 *      operation count of Section 2.
 *  R3  Higher bit depths are reduced to 8 bits for the direction search by
 *      dropping the extra low bits (Section 2 says only "downscale").
 *  R4  Blocks cut by the frame edge run Algorithm 1 over their in-frame
 *      pixels only; count[d][L] is counted, so 840/count stays exact.
 *  R5  Eq. (13) when 2^10 <= v < 2^16: floor(v / 2^16) = 0 has no log, and
 *      the log term is taken as 0.
 *  R6  Eq. (7): the printed d < 0 branch is not the mirror of the d >= 0
 *      branch (ceil instead of floor), while the text says f is
 *      anti-symmetric.  The oracle uses the d >= 0 branch and
 *      f(-d) = -f(d).  f = 0 when S = 0 (log2 0 is undefined and a zero
 *      strength can pass nothing).
 *  R7  Tap positions (Figs. 4 and 5): along direction d the inner and outer
 *      taps are at (row, col) offsets
 *        d0 (-1,1) (-2,2)   d1 (0,1) (-1,2)   d2 (0,1) (0,2)   d3 (0,1) (1,2)
 *        d4 (1,1) (2,2)     d5 (1,0) (2,1)    d6 (1,0) (2,0)   d7 (1,0) (2,-1)
 *      and their negatives.  Secondary taps use directions d+2 and d-2.
 *  R8  Primary weights in 1/16: inner 4, outer 2 for even strength, 3 and 3
 *      for odd (Fig. 4 caption).  Secondary weights: inner 2, outer 1.
 *  R9  round() in Eq. (8) divides the weighted sum by 16 and rounds ties away
 *      from zero.
 *  R10 The clamp set R of Eq. (12) is the centre pixel plus every in-frame
 *      tap position (all taps have non-zero weight, whatever the strength).
 *  R11 Primary weight parity follows the strength actually used: the
 *      adjusted strength for luma, the signaled one for chroma.
 *  R12 For bit depth b > 8, the signaled luma strength is first adjusted by
 *      Eq. (13) in the 8-bit domain, the weights are picked by its parity,
 *      and then strengths are shifted left by b-8 and D raised by b-8.
 *  R13 Chroma damping: max(D - 1, floor(log2 S^(p)_chroma)) for both tap
 *      groups (D - 1 when S^(p)_chroma = 0).
 *  R14 Chroma at 4:2:0 uses the direction and skip flag of the co-located
 *      luma 8x8 block for each 4x4 chroma block; a chroma filter block is
 *      32x32.
 *  R15 skip = 1 marks an 8x8 block with no coded residual: it is copied, and
 *      so is its co-located chroma.
 *  R16 SSE counts in-frame pixels only and is per plane.
 *  R18 A preset holds, per plane group, a skip condition bit (Section 4),
 *      passed as bit 7 of the secondary-strength byte.  A filter block whose
 *      in-frame 8x8 blocks are all skipped is not filtered under any preset.
 *      Otherwise a skipped 8x8 block is filtered only when the bit is set.
 *      Strengths (0, 0) with the bit set stand for S^(p) = 19, S^(s) = 7 with
 *      the bit set.  19 goes through Eq. (13) and the weight parity rule like
 *      any primary strength; since D may never be lower than floor(log2 S),
 *      a luma block whose adjusted strength reaches 16..19 takes
 *      floor(log2 S) = 4 as its damping for both tap groups, as the chroma
 *      rule R13 does.
 *  R19 Eq. (14): the "8x8 block" is CDEF's filtering unit (an 8x8 luma
 *      block; at 4:2:0 its co-located 4x4 chroma block), over its in-frame
 *      pixels; sigma^2 are population variances (divided by the pixel
 *      count); C1 = 6.25 and C2 = 312.5 at 8 bits scale by 4^(b-8) and
 *      16^(b-8), the factors by which variances and their products grow, so
 *      that the weight of a frame does not change when every sample is
 *      multiplied by 2^(b-8).  Evaluated in double precision.
 *  R20 4:2:2 (chroma subsampled horizontally only): chroma is not filtered
 *      (Section 4) and so is copied, and the searches cover luma only.
 *  R21 4:4:4: each 8x8 chroma block takes the direction and skip flag of the
 *      co-located 8x8 luma block; chroma filter blocks are 64x64; strengths
 *      and damping follow the chroma rules of R13 as at 4:2:0.
 *  R22 Subset search (Section 5): a subset of the presets is the product of
 *      a set of S^(p) values, a set of S^(s) values and a set of skip
 *      condition bits; the presets outside it are not evaluated (their table
 *      entries hold the all-ones value) and the preset selection never
 *      chooses them.
 */
#include "cdef_oracle.h"

#include <math.h>
#include <stdlib.h>

/* ---- Section 2: direction search ---------------------------------------- */

/* R2: floor division for possibly negative numerators is not needed here
 * because i, j >= 0. */
int cdef_oracle_line_number(int d, int i, int j) {
  switch (d) {
    case 0: return i + j;
    case 1: return i + j / 2;
    case 2: return i;
    case 3: return i - j / 2 + 3;
    case 4: return i - j + 7;
    case 5: return j - i / 2 + 3;
    case 6: return j;
    default: return j + i / 2;
  }
}

/* Algorithm 1, first part: line sums, counts and s[d] (scaled by 840, the
 * least common multiple of 1..8, so that 840 / count is exact). */
void cdef_oracle_direction_costs(const uint16_t *px, int64_t stride, int bw, int bh,
                                 int bitdepth, int64_t cost[8]) {
  int shift = bitdepth - 8; /* R3 */
  for (int d = 0; d < 8; d++) {
    int64_t partial[15] = {0};
    int count[15] = {0};
    for (int i = 0; i < bh; i++) {
      for (int j = 0; j < bw; j++) {
        int L = cdef_oracle_line_number(d, i, j);
        int x = (int)(px[i * stride + j] >> shift) - 128;
        partial[L] += x;
        count[L] += 1;
      }
    }
    cost[d] = 0;
    for (int L = 0; L < 15; L++) {
      if (count[L] > 0) cost[d] += partial[L] * partial[L] * (840 / count[L]);
    }
  }
}

/* Algorithm 1, second part: strict '>' from best = 0, and the directional
 * contrast v = s[best] - s[best + 4 mod 8]. */
void cdef_oracle_find_dir(const uint16_t *luma, int64_t stride, int width, int height,
                          int bitdepth, uint8_t *dir, int32_t *var) {
  int bcols = (width + 7) / 8, brows = (height + 7) / 8;
  for (int by = 0; by < brows; by++) {
    for (int bx = 0; bx < bcols; bx++) {
      int bw = width - 8 * bx < 8 ? width - 8 * bx : 8;   /* R4 */
      int bh = height - 8 * by < 8 ? height - 8 * by : 8;
      int64_t cost[8];
      cdef_oracle_direction_costs(luma + (int64_t)8 * by * stride + 8 * bx, stride, bw, bh,
                                  bitdepth, cost);
      int best = 0;
      for (int d = 0; d < 8; d++)
        if (cost[d] > cost[best]) best = d;
      dir[by * bcols + bx] = (uint8_t)best;
      var[by * bcols + bx] = (int32_t)(cost[best] - cost[(best + 4) % 8]);
    }
  }
}

/* ---- Section 3: the constrained filter ---------------------------------- */

static int floor_log2(int v) { /* v >= 1 */
  int r = 0;
  while (v >= 2) {
    v /= 2;
    r++;
  }
  return r;
}

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }

/* Eq. (7), R6. */
int cdef_oracle_constrain(int diff, int strength, int damping) {
  if (strength == 0) return 0;
  int a = diff < 0 ? -diff : diff;
  int k = damping - floor_log2(strength); /* D >= floor(log2 S) keeps k >= 0 */
  int f = imin(a, imax(0, strength - a / (1 << k)));
  return diff < 0 ? -f : f;
}

/* Eq. (13), R5. */
int cdef_oracle_adjust_strength(int strength, int32_t var) {
  if (var < 1024) return 0;
  int q = var / 65536;
  int i = q == 0 ? 0 : imin(floor_log2(q), 12);
  return (strength * (4 + i) + 8) / 16;
}

/* Section 3.2, R13. */
int cdef_oracle_chroma_damping(int damping, int pri_strength) {
  int dc = damping - 1;
  if (pri_strength > 0 && floor_log2(pri_strength) > dc) dc = floor_log2(pri_strength);
  return dc;
}

/* R7 */
static const int TAPS[8][2][2] = {
    {{-1, 1}, {-2, 2}}, {{0, 1}, {-1, 2}}, {{0, 1}, {0, 2}}, {{0, 1}, {1, 2}},
    {{1, 1}, {2, 2}},   {{1, 0}, {2, 1}},  {{1, 0}, {2, 0}}, {{1, 0}, {2, -1}},
};

/* Eq. (8)-(12) at pixel (i, j).  Taps outside the plane are ignored
 * (Section 3.2: f = 0 for pixels outside the visible frame) and are not part
 * of the clamp set (R10). */
int cdef_oracle_filter_pixel(const uint16_t *p, int64_t stride, int pw, int ph, int i, int j,
                             int dir, int pri_strength, int pri_damping, int w1, int w2,
                             int sec_strength, int sec_damping) {
  int x = p[(int64_t)i * stride + j];
  int sum = 0, lo = x, hi = x;
  /* primary taps: along d */
  for (int k = 0; k < 2; k++) {
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int m = i + sgn * TAPS[dir][k][0], n = j + sgn * TAPS[dir][k][1];
      if (m < 0 || m >= ph || n < 0 || n >= pw) continue;
      int v = p[(int64_t)m * stride + n];
      sum += (k == 0 ? w1 : w2) * cdef_oracle_constrain(v - x, pri_strength, pri_damping);
      lo = imin(lo, v);
      hi = imax(hi, v);
    }
  }
  /* secondary taps: a cross at 45 degrees off d, i.e. directions d +- 2 */
  for (int s = 0; s < 2; s++) {
    int d2 = s == 0 ? (dir + 2) % 8 : (dir + 6) % 8;
    for (int k = 0; k < 2; k++) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int m = i + sgn * TAPS[d2][k][0], n = j + sgn * TAPS[d2][k][1];
        if (m < 0 || m >= ph || n < 0 || n >= pw) continue;
        int v = p[(int64_t)m * stride + n];
        sum += (k == 0 ? 2 : 1) * cdef_oracle_constrain(v - x, sec_strength, sec_damping);
        lo = imin(lo, v);
        hi = imax(hi, v);
      }
    }
  }
  /* R9: round(sum / 16), ties away from zero */
  int r = sum >= 0 ? (sum + 8) / 16 : -((-sum + 8) / 16);
  int y = x + r;
  return imin(hi, imax(lo, y)); /* Eq. (9)-(11) */
}

/* Filter parameters of one block of one plane (R11-R13). */
typedef struct {
  int pri_s, pri_d, w1, w2, sec_s, sec_d;
} block_params;

static block_params params_for(int plane, int bitdepth, int damping, int pri, int sec,
                               int32_t var) {
  block_params bp;
  int c = bitdepth - 8;
  int s, d;
  if (plane == 0) {
    s = cdef_oracle_adjust_strength(pri, var);
    d = damping;
    if (s > 0 && floor_log2(s) > d) d = floor_log2(s); /* R18 */
  } else {
    s = pri;
    d = cdef_oracle_chroma_damping(damping, pri);
  }
  bp.w1 = (s % 2) ? 3 : 4;
  bp.w2 = (s % 2) ? 3 : 2;
  bp.pri_s = s << c;
  bp.pri_d = d + c;
  bp.sec_s = sec << c;
  bp.sec_d = d + c;
  return bp;
}

/* Subsampling of a plane: chroma halves the width at 4:2:0 and 4:2:2 and
 * the height at 4:2:0. */
static void plane_geometry(const cdef_oracle_frame *f, int plane, int *pw, int *ph, int *ssx,
                           int *ssy) {
  *ssx = plane > 0 && (f->layout == CDEF_ORACLE_420 || f->layout == CDEF_ORACLE_422);
  *ssy = plane > 0 && f->layout == CDEF_ORACLE_420;
  *pw = (f->width + *ssx) >> *ssx;
  *ph = (f->height + *ssy) >> *ssy;
}

int cdef_oracle_search_planes(const cdef_oracle_frame *f) {
  return f->nplanes == 3 && f->layout != CDEF_ORACLE_422 ? 3 : 1;
}

/* R18: the preset of one plane group from a strengths entry. */
static void preset_of(const uint8_t *st, int plane, int *pri, int *sec, int *skipcond) {
  int sb = plane == 0 ? st[1] : st[3];
  *pri = plane == 0 ? st[0] : st[2];
  *sec = sb & 0x7f;
  *skipcond = sb >> 7;
  if (*pri == 0 && *sec == 0 && *skipcond) {
    *pri = 19;
    *sec = 7;
  }
}

/* R18: every in-frame 8x8 block of filter block (fby, fbx) is skipped. */
static int fb_skipped(const cdef_oracle_frame *f, const uint8_t *skip, int fby, int fbx) {
  if (!skip) return 0;
  int bcols = (f->width + 7) / 8, brows = (f->height + 7) / 8;
  for (int by = 8 * fby; by < imin(8 * fby + 8, brows); by++)
    for (int bx = 8 * fbx; bx < imin(8 * fbx + 8, bcols); bx++)
      if (!skip[by * bcols + bx]) return 0;
  return 1;
}

void cdef_oracle_filter_frame(const cdef_oracle_frame *in, uint16_t *const out[3],
                              const int64_t out_stride[3], const uint8_t *dir,
                              const int32_t *var, const uint8_t *skip, int damping,
                              const uint8_t *strengths) {
  int bcols = (in->width + 7) / 8;
  int fbcols = (in->width + 63) / 64;
  for (int p = 0; p < in->nplanes; p++) {
    int pw, ph, ssx, ssy;
    plane_geometry(in, p, &pw, &ph, &ssx, &ssy);
    int bw = 8 >> ssx, bh = 8 >> ssy, fw = 64 >> ssx, fh = 64 >> ssy;
    for (int i = 0; i < ph; i++) {
      for (int j = 0; j < pw; j++) {
        int b = (i / bh) * bcols + (j / bw);
        int x = in->plane[p][(int64_t)i * in->stride[p] + j];
        const uint8_t *st = strengths + 4 * ((i / fh) * fbcols + (j / fw));
        int pri, sec, skipcond;
        preset_of(st, p, &pri, &sec, &skipcond);
        int y;
        if ((p > 0 && in->layout == CDEF_ORACLE_422) || /* R20 */
            fb_skipped(in, skip, i / fh, j / fw) || (skip && skip[b] && !skipcond)) {
          y = x;
        } else {
          block_params bp = params_for(p, in->bitdepth, damping, pri, sec, var[b]);
          y = cdef_oracle_filter_pixel(in->plane[p], in->stride[p], pw, ph, i, j, dir[b],
                                       bp.pri_s, bp.pri_d, bp.w1, bp.w2, bp.sec_s, bp.sec_d);
        }
        out[p][(int64_t)i * out_stride[p] + j] = (uint16_t)y;
      }
    }
  }
}

/* ---- Section 5: the encoder's per-filter-block distortion ------------------ */

static const int SEC_STRENGTHS[4] = {0, 1, 2, 4};

/* R22: cand = S^(p) mask | S^(s) index mask << 16 | skip condition bit
 * mask << 20, 0 for every preset. */
static int candidate_in(uint32_t cand, int pri, int si, int k) {
  if (cand == 0) return 1;
  return ((cand >> pri) & 1) && ((cand >> (16 + si)) & 1) && ((cand >> (20 + k)) & 1);
}

/* Section 5: every candidate filters the whole filter block, as the filter
 * would with that preset (R18), and sums squared errors against the source.
 * Candidate (skip condition bit k, S^(p), S^(s) index) is at
 * sse[((p * nskip + k) * 16 + S^(p)) * 4 + index]. */
void cdef_oracle_search_fb3(const cdef_oracle_frame *recon, const cdef_oracle_frame *src,
                            const uint8_t *dir, const int32_t *var, const uint8_t *skip,
                            int damping, int nskip, uint32_t cand, int fby, int fbx,
                            uint64_t *sse) {
  int bcols = (recon->width + 7) / 8;
  int all_skipped = fb_skipped(recon, skip, fby, fbx);
  for (int p = 0; p < cdef_oracle_search_planes(recon); p++) {
    int pw, ph, ssx, ssy;
    plane_geometry(recon, p, &pw, &ph, &ssx, &ssy);
    int bw = 8 >> ssx, bh = 8 >> ssy, fw = 64 >> ssx, fh = 64 >> ssy;
    int i0 = fby * fh, j0 = fbx * fw;
    int i1 = imin(i0 + fh, ph), j1 = imin(j0 + fw, pw);
    for (int k = 0; k < nskip; k++) {
      for (int pri_sig = 0; pri_sig < 16; pri_sig++) {
        for (int si = 0; si < 4; si++) {
          if (!candidate_in(cand, pri_sig, si, k)) { /* R22 */
            sse[((p * nskip + k) * 16 + pri_sig) * 4 + si] = UINT64_MAX;
            continue;
          }
          uint8_t st[4] = {(uint8_t)pri_sig, (uint8_t)(SEC_STRENGTHS[si] | (k << 7)),
                           (uint8_t)pri_sig, (uint8_t)(SEC_STRENGTHS[si] | (k << 7))};
          int pri, sec, skipcond;
          preset_of(st, p, &pri, &sec, &skipcond);
          uint64_t acc = 0;
          for (int i = i0; i < i1; i++) {
            for (int j = j0; j < j1; j++) {
              int b = (i / bh) * bcols + (j / bw);
              int x = recon->plane[p][(int64_t)i * recon->stride[p] + j];
              int y;
              if (all_skipped || (skip && skip[b] && !skipcond)) {
                y = x;
              } else {
                block_params bp = params_for(p, recon->bitdepth, damping, pri, sec, var[b]);
                y = cdef_oracle_filter_pixel(recon->plane[p], recon->stride[p], pw, ph, i, j,
                                             dir[b], bp.pri_s, bp.pri_d, bp.w1, bp.w2,
                                             bp.sec_s, bp.sec_d);
              }
              int64_t e =
                  (int64_t)y - (int64_t)src->plane[p][(int64_t)i * src->stride[p] + j];
              acc += (uint64_t)(e * e);
            }
          }
          sse[((p * nskip + k) * 16 + pri_sig) * 4 + si] = acc;
        }
      }
    }
  }
}

/* Section 5, Eq. (14), R19: the contrast-weighted distortion of one filter
 * block for the 64 pairs (skip condition bit off).  Each pair filters the
 * whole block into a scratch copy, then every filtering unit contributes
 * (sigma_s^2 + sigma_d^2 + C1) / (2 sqrt(sigma_s^2 sigma_d^2 + C2)) ||s - d||^2. */
void cdef_oracle_search_fb_weighted(const cdef_oracle_frame *recon,
                                    const cdef_oracle_frame *src, const uint8_t *dir,
                                    const int32_t *var, const uint8_t *skip, int damping,
                                    int fby, int fbx, double *dist) {
  int bcols = (recon->width + 7) / 8;
  int c = recon->bitdepth - 8;
  double C1 = 6.25 * pow(4.0, c), C2 = 312.5 * pow(16.0, c);
  int all_skipped = fb_skipped(recon, skip, fby, fbx);
  int filtered[64 * 64];
  for (int p = 0; p < cdef_oracle_search_planes(recon); p++) {
    int pw, ph, ssx, ssy;
    plane_geometry(recon, p, &pw, &ph, &ssx, &ssy);
    int bw = 8 >> ssx, bh = 8 >> ssy, fw = 64 >> ssx, fh = 64 >> ssy;
    int i0 = fby * fh, j0 = fbx * fw;
    int i1 = imin(i0 + fh, ph), j1 = imin(j0 + fw, pw);
    for (int pri = 0; pri < 16; pri++) {
      for (int si = 0; si < 4; si++) {
        for (int i = i0; i < i1; i++) {
          for (int j = j0; j < j1; j++) {
            int b = (i / bh) * bcols + (j / bw);
            int x = recon->plane[p][(int64_t)i * recon->stride[p] + j];
            int y = x;
            if (!all_skipped && !(skip && skip[b])) {
              block_params bp =
                  params_for(p, recon->bitdepth, damping, pri, SEC_STRENGTHS[si], var[b]);
              y = cdef_oracle_filter_pixel(recon->plane[p], recon->stride[p], pw, ph, i, j,
                                           dir[b], bp.pri_s, bp.pri_d, bp.w1, bp.w2,
                                           bp.sec_s, bp.sec_d);
            }
            filtered[(i - i0) * 64 + (j - j0)] = y;
          }
        }
        double total = 0.0;
        for (int ui = i0; ui < i1; ui += bh) {
          for (int uj = j0; uj < j1; uj += bw) {
            int n = 0;
            double ms = 0.0, md = 0.0;
            for (int i = ui; i < imin(ui + bh, i1); i++)
              for (int j = uj; j < imin(uj + bw, j1); j++) {
                ms += src->plane[p][(int64_t)i * src->stride[p] + j];
                md += filtered[(i - i0) * 64 + (j - j0)];
                n++;
              }
            ms /= n;
            md /= n;
            double vs = 0.0, vd = 0.0, e2 = 0.0;
            for (int i = ui; i < imin(ui + bh, i1); i++)
              for (int j = uj; j < imin(uj + bw, j1); j++) {
                double sv = src->plane[p][(int64_t)i * src->stride[p] + j];
                double dv = filtered[(i - i0) * 64 + (j - j0)];
                vs += (sv - ms) * (sv - ms);
                vd += (dv - md) * (dv - md);
                e2 += (sv - dv) * (sv - dv);
              }
            vs /= n;
            vd /= n;
            total += (vs + vd + C1) / (2.0 * sqrt(vs * vd + C2)) * e2;
          }
        }
        dist[(p * 16 + pri) * 4 + si] = total;
      }
    }
  }
}

void cdef_oracle_search_fb2(const cdef_oracle_frame *recon, const cdef_oracle_frame *src,
                            const uint8_t *dir, const int32_t *var, const uint8_t *skip,
                            int damping, int nskip, int fby, int fbx, uint64_t *sse) {
  cdef_oracle_search_fb3(recon, src, dir, var, skip, damping, nskip, 0, fby, fbx, sse);
}

void cdef_oracle_search_fb(const cdef_oracle_frame *recon, const cdef_oracle_frame *src,
                           const uint8_t *dir, const int32_t *var, const uint8_t *skip,
                           int damping, int fby, int fbx, uint64_t *sse) {
  cdef_oracle_search_fb2(recon, src, dir, var, skip, damping, 1, fby, fbx, sse);
}

void cdef_oracle_search(const cdef_oracle_frame *recon, const cdef_oracle_frame *src,
                        const uint8_t *skip, int damping, uint64_t *sse, uint8_t *dir,
                        int32_t *var) {
  cdef_oracle_find_dir(recon->plane[0], recon->stride[0], recon->width, recon->height,
                       recon->bitdepth, dir, var);
  int fbr = (recon->height + 63) / 64, fbc = (recon->width + 63) / 64;
  uint64_t tmp[3 * 64];
  for (int by = 0; by < fbr; by++) {
    for (int bx = 0; bx < fbc; bx++) {
      cdef_oracle_search_fb(recon, src, dir, var, skip, damping, by, bx, tmp);
      for (int p = 0; p < cdef_oracle_search_planes(recon); p++)
        for (int k = 0; k < 64; k++)
          sse[(((int64_t)p * fbr + by) * fbc + bx) * 64 + k] = tmp[p * 64 + k];
    }
  }
}

/* ---- Section 5, Eq. (15): choosing the presets ---------------------------------
 * R17 Eq. (15) takes the minimum over P_luma and over P_chroma separately, as
 *     printed; B is the number of filter blocks.  The "optimal preset to add"
 *     is a candidate not yet in the set; ties go to the lowest candidate index
 *     (skip condition bit * 64 + S^(p) * 4 + index of S^(s); 64 candidates
 *     without the bit, 128 with it).  Re-optimization replaces one preset at a
 *     time by the best candidate not among the others, only when that strictly
 *     lowers the distortion. */

static uint64_t group_d(const uint64_t *sse, int nplanes, int nfb, int nc, int g, int b,
                        int p) {
  if (g == 0) return sse[(int64_t)b * nc + p];
  if (nplanes < 3) return 0;
  return sse[((int64_t)nfb + b) * nc + p] + sse[((int64_t)2 * nfb + b) * nc + p];
}

/* sum over blocks of the minimum distortion over set[0..n), with slot `skip`
 * replaced by candidate `with` (skip < 0: no replacement; with < 0: slot dropped) */
static uint64_t set_distortion(const uint64_t *sse, int nplanes, int nfb, int nc, int g,
                               const int *set, int n, int skip, int with) {
  uint64_t total = 0;
  for (int b = 0; b < nfb; b++) {
    uint64_t m = UINT64_MAX;
    for (int i = 0; i < n; i++) {
      int p = i == skip ? with : set[i];
      if (p < 0) continue;
      uint64_t d = group_d(sse, nplanes, nfb, nc, g, b, p);
      if (d < m) m = d;
    }
    total += m;
  }
  return total;
}

/* R22: candidates outside cand_mask (NULL: none) are never chosen. */
static int allowed(const uint64_t *cand_mask, int p) {
  return !cand_mask || ((cand_mask[p >> 6] >> (p & 63)) & 1);
}

static int in_set(const int *set, int n, int p, int except) {
  for (int i = 0; i < n; i++)
    if (i != except && set[i] == p) return 1;
  return 0;
}

void cdef_oracle_select_presets(const uint64_t *sse, int nplanes, int nfb, int ncand,
                                const uint64_t *cand_mask, double lambda, int refine_passes, int32_t *n_chosen, int32_t *sets_l,
                                int32_t *sets_c, uint64_t *dist, double *cost, uint8_t *fb_l,
                                uint8_t *fb_c) {
  static const int NS[4] = {1, 2, 4, 8};
  int best_sets[2][4][8];
  for (int g = 0; g < 2; g++) {
    int greedy[8];
    for (int step = 0; step < 8; step++) {
      int best = -1;
      uint64_t bestd = UINT64_MAX;
      for (int p = 0; p < ncand; p++) {
        if (in_set(greedy, step, p, -1) || !allowed(cand_mask, p)) continue;
        greedy[step] = p;
        uint64_t d = set_distortion(sse, nplanes, nfb, ncand, g, greedy, step + 1, -1, -1);
        if (best < 0 || d < bestd) {
          bestd = d;
          best = p;
        }
      }
      greedy[step] = best;
    }
    for (int k = 0; k < 4; k++) {
      int n = NS[k], set[8];
      for (int i = 0; i < 8; i++) set[i] = i < n ? greedy[i] : -1;
      for (int pass = 0; pass < refine_passes; pass++) {
        int changed = 0;
        for (int i = 0; i < n; i++) {
          uint64_t curd = set_distortion(sse, nplanes, nfb, ncand, g, set, n, -1, -1);
          int bestp = set[i];
          uint64_t bestd = curd;
          for (int p = 0; p < ncand; p++) {
            if (in_set(set, n, p, i) || !allowed(cand_mask, p)) continue;
            uint64_t d = set_distortion(sse, nplanes, nfb, ncand, g, set, n, i, p);
            if (d < bestd) {
              bestd = d;
              bestp = p;
            }
          }
          if (bestp != set[i]) {
            set[i] = bestp;
            changed = 1;
          }
        }
        if (!changed) break;
      }
      for (int i = 0; i < 8; i++) best_sets[g][k][i] = set[i];
      dist[g * 4 + k] = set_distortion(sse, nplanes, nfb, ncand, g, set, n, -1, -1);
    }
  }
  int chosen = 0;
  for (int k = 0; k < 4; k++) {
    cost[k] = lambda * (double)nfb * (double)k + (double)(dist[k] + dist[4 + k]);
    if (cost[k] < cost[chosen]) chosen = k;
  }
  *n_chosen = NS[chosen];
  for (int k = 0; k < 4; k++)
    for (int i = 0; i < 8; i++) {
      sets_l[k * 8 + i] = best_sets[0][k][i];
      sets_c[k * 8 + i] = best_sets[1][k][i];
    }
  for (int b = 0; b < nfb; b++) {
    for (int g = 0; g < 2; g++) {
      int bi = 0;
      uint64_t bd = UINT64_MAX;
      for (int i = 0; i < NS[chosen]; i++) {
        uint64_t d = group_d(sse, nplanes, nfb, ncand, g, b, best_sets[g][chosen][i]);
        if (d < bd) {
          bd = d;
          bi = i;
        }
      }
      (g == 0 ? fb_l : fb_c)[b] = (uint8_t)bi;
    }
  }
}
