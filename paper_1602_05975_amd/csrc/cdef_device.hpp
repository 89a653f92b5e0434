// Device-side building blocks of the gfx950 CDEF kernels.
//
// Paper: Midtskogen and Valin, "The AV1 Constrained Directional Enhancement
// Filter (CDEF)".  Section 2 (direction search, Eq. 1-5, Algorithm 1),
// Section 3 (constraint Eq. 7, 2-D filter Eq. 8-12, strengths and damping,
// adjustment Eq. 13), Section 4 (64x64 filter blocks, skip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdef {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Value stored in LDS for a position outside the visible frame.  As a signed
// 16-bit number it is the most negative value (never a signed maximum), as
// an unsigned one it is 32768 (never an unsigned minimum of valid samples),
// and its distance to any 10-bit sample is >= 31745, which no strength
// below 2^9 can pass through the constraint function.
constexpr uint16_t kOutside = 0x8000;

// ---- Direction geometry (the lost Fig. 1, 4, 5 read as documented) --------
// Direction 0 is the 45-degree line rising to the right; each step turns the
// line 22.5 degrees clockwise on screen (row index grows downward).

// Line number of pixel (i, j) of an 8x8 block for direction d.
__host__ __device__ __forceinline__ constexpr int line_key(int d, int i, int j) {
  return d == 0 ? i + j
       : d == 1 ? i + (j >> 1)
       : d == 2 ? i
       : d == 3 ? i - (j >> 1) + 3
       : d == 4 ? i - j + 7
       : d == 5 ? j - (i >> 1) + 3
       : d == 6 ? j
                : j + (i >> 1);
}

// Row/column offset of the inner (t = 0) and outer (t = 1) tap along d.
__host__ __device__ __forceinline__ constexpr int tap_dr(int d, int t) {
  return t == 0 ? (d == 0 ? -1 : d <= 3 ? 0 : 1)
                : (d == 0 ? -2 : d == 1 ? -1 : d == 2 ? 0 : d == 3 ? 1 : 2);
}
__host__ __device__ __forceinline__ constexpr int tap_dc(int d, int t) {
  return t == 0 ? (d <= 4 ? 1 : 0)
                : (d <= 4 ? 2 : d == 5 ? 1 : d == 6 ? 0 : -1);
}

__device__ __forceinline__ int floor_log2(int v) { return 31 - __clz(v); }  // v >= 1

// 840 / n for n = 1..8 (840 is the least common multiple of 1..8), looked
// up branch-free from 10-bit fields of two constants; n = 0 gives 0.
__device__ __forceinline__ int inv840(int n) {
  constexpr uint64_t lo = 840ull << 10 | 420ull << 20 | 280ull << 30 | 210ull << 40 |
                          168ull << 50;
  constexpr uint64_t hi = 140ull | 120ull << 10 | 105ull << 20;
  return n <= 5 ? (int)((lo >> (10 * n)) & 1023) : (int)((hi >> (10 * (n - 6))) & 1023);
}

// ---- Algorithm 1 in 32-bit lanes ---------------------------------------------
// The 64 centred values of a block in 64 registers, one 32-bit line sum per
// line.  Its adds and 24-bit multiplies issue as 2-cycle VOP2 instructions,
// so it is the cheaper form in issue cycles; the packed form below needs
// half the registers.  The search kernels, which are VALU-bound and whose
// task loops set their register budget anyway, use this one; the filter
// kernels and the stand-alone search, whose occupancy the direction search
// limits, use the packed one.  Both compute the same integers.

// Number of pixels on every line of every direction of a full 8x8 block,
// evaluated by the compiler.
struct LineCounts {
  int n[8][15];
};
__host__ __device__ constexpr LineCounts make_line_counts() {
  LineCounts t{};
  for (int d = 0; d < 8; ++d)
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) t.n[d][line_key(d, i, j)] += 1;
  return t;
}

// Algorithm 1 for one direction D of a full 8x8 block of centred 8-bit
// values: the 840-scaled s_D of Eq. (5).  D is a template parameter so that
// every line index and every 840 / N is a compile-time constant.
template <int D>
__device__ __forceinline__ int dir_cost_full(const int (&x)[64]) {
  constexpr LineCounts kN = make_line_counts();
  int part[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) part[k] = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) part[line_key(D, i, j)] += x[i * 8 + j];
  int c = 0;
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    const int n = kN.n[D][k];
    if (n > 0) c += __mul24(__mul24(part[k], part[k]), 840 / (n > 0 ? n : 1));
  }
  return c;
}

__device__ __forceinline__ void dir_costs_full(const int (&x)[64], int (&cost)[8]) {
  cost[0] = dir_cost_full<0>(x);
  cost[1] = dir_cost_full<1>(x);
  cost[2] = dir_cost_full<2>(x);
  cost[3] = dir_cost_full<3>(x);
  cost[4] = dir_cost_full<4>(x);
  cost[5] = dir_cost_full<5>(x);
  cost[6] = dir_cost_full<6>(x);
  cost[7] = dir_cost_full<7>(x);
}

// The same for a block cut by the frame edge: only the top-left bw x bh
// pixels exist, and line lengths are counted (840 / N stays exact).
template <int D>
__device__ __forceinline__ int dir_cost_partial(const int (&x)[64], int bw, int bh) {
  int part[15], cnt[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) part[k] = cnt[k] = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bool in = i < bh && j < bw;
      part[line_key(D, i, j)] += in ? x[i * 8 + j] : 0;
      cnt[line_key(D, i, j)] += in ? 1 : 0;
    }
  int c = 0;
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    c += __mul24(__mul24(part[k], part[k]), inv840(cnt[k]));
  }
  return c;
}

__device__ __forceinline__ void dir_costs_partial(const int (&x)[64], int bw, int bh,
                                                  int (&cost)[8]) {
  cost[0] = dir_cost_partial<0>(x, bw, bh);
  cost[1] = dir_cost_partial<1>(x, bw, bh);
  cost[2] = dir_cost_partial<2>(x, bw, bh);
  cost[3] = dir_cost_partial<3>(x, bw, bh);
  cost[4] = dir_cost_partial<4>(x, bw, bh);
  cost[5] = dir_cost_partial<5>(x, bw, bh);
  cost[6] = dir_cost_partial<6>(x, bw, bh);
  cost[7] = dir_cost_partial<7>(x, bw, bh);
}


// ---- Algorithm 1 on packed 16-bit halves ------------------------------------
// Row i of an 8x8 block is held as four 32-bit words; word m packs the
// centred 8-bit values of columns 2m (low half) and 2m + 1 (high half).  For
// direction D the halves of word (i, m) lie on lines line_key(D, i, 2m) and
// line_key(D, i, 2m + 1).  Words whose halves lie on the same pair of lines
// add into one packed accumulator (a line sum is at most 8 * 128 in
// magnitude, so 16 bits hold it), which makes the 64 pixel additions 32
// packed ones.  Each line then has at most one low-half and one high-half
// source (asserted below); v_dot2 with (1, 1) adds the two.

struct PackedLines {
  int nacc;            // packed accumulators
  int acc[8][4];       // accumulator of word (i, m)
  int nl;              // lines
  int lo[15], hi[15];  // per line: accumulator of its low / high half, -1 if none
  int nlo[15], nhi[15];
  int n[15];           // pixels on the line in a full block
};

__host__ __device__ constexpr PackedLines make_packed_lines(int d) {
  PackedLines t{};
  int kl[32] = {}, kh[32] = {};
  for (int l = 0; l < 15; ++l) t.lo[l] = t.hi[l] = -1;
  for (int i = 0; i < 8; ++i)
    for (int m = 0; m < 4; ++m) {
      const int a = line_key(d, i, 2 * m), b = line_key(d, i, 2 * m + 1);
      int id = -1;
      for (int k = 0; k < t.nacc; ++k)
        if (kl[k] == a && kh[k] == b) id = k;
      if (id < 0) {
        id = t.nacc++;
        kl[id] = a;
        kh[id] = b;
      }
      t.acc[i][m] = id;
      t.n[a] += 1;
      t.n[b] += 1;
      t.nl = a + 1 > t.nl ? a + 1 : t.nl;
      t.nl = b + 1 > t.nl ? b + 1 : t.nl;
    }
  for (int k = 0; k < t.nacc; ++k) {
    t.lo[kl[k]] = k;
    t.nlo[kl[k]] += 1;
    t.hi[kh[k]] = k;
    t.nhi[kh[k]] += 1;
  }
  return t;
}

constexpr bool packed_lines_ok() {
  for (int d = 0; d < 8; ++d) {
    const PackedLines t = make_packed_lines(d);
    if (t.nacc > 15) return false;
    for (int l = 0; l < t.nl; ++l)
      if (t.nlo[l] > 1 || t.nhi[l] > 1 || t.n[l] == 0) return false;
  }
  return true;
}
static_assert(packed_lines_ok(), "a line with two sources of one half, or an empty line");

// Line lengths of every direction for a block cut by the frame edge to its
// top-left bw x bh pixels: 4 bits per line (at most 8), lines 0..14 in one
// 64-bit word, indexed [d][bh - 1][bw - 1].  Evaluated by the compiler.
struct CutLineCounts {
  uint64_t w[8][8][8];
};
__host__ __device__ constexpr CutLineCounts make_cut_line_counts() {
  CutLineCounts t{};
  for (int d = 0; d < 8; ++d)
    for (int bh = 1; bh <= 8; ++bh)
      for (int bw = 1; bw <= 8; ++bw)
        for (int i = 0; i < bh; ++i)
          for (int j = 0; j < bw; ++j) t.w[d][bh - 1][bw - 1] += 1ull << (4 * line_key(d, i, j));
  return t;
}
static __constant__ CutLineCounts kCutLineCounts = make_cut_line_counts();

// Square of line l's value from its packed sources: with B = (low-half
// source, high-half source) and v = b0 + b1, v^2 = dot2(B, (v, v)), where
// (v, v) = B + B with its halves swapped.  Full-rate 16-bit work only; no
// 32-bit multiply.
template <int D>
__device__ __forceinline__ int line_square(const uint32_t (&A)[15], int l, int acc = 0) {
  constexpr PackedLines T = make_packed_lines(D);
  const int p = T.lo[l], q = T.hi[l];
  uint32_t w;
  if (p >= 0 && q >= 0)
    w = p == q ? A[p] : (A[p] & 0xFFFFu) | (A[q] & 0xFFFF0000u);
  else if (p >= 0)
    w = A[p] & 0xFFFFu;
  else
    w = A[q] & 0xFFFF0000u;
  const s16x2 b = __builtin_bit_cast(s16x2, w);
  return __builtin_amdgcn_sdot2(b, b + b.yx, acc, false);
}

// The 840-scaled s_D of Eq. (5) for one direction.  x: the 32 packed words of
// centred values (zero outside the frame); PARTIAL: the block is cut by the
// frame edge to its top-left bw x bh pixels (1..8 each), so line lengths are
// those of the cut block (840 / N stays exact).  D is a template parameter so that every
// accumulator index and every full-block 840 / N is a compile-time constant.
template <int D, bool PARTIAL>
__device__ __forceinline__ int dir_cost_packed(const uint32_t (&x)[32], int bw, int bh) {
  constexpr PackedLines T = make_packed_lines(D);
  uint32_t A[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) A[k] = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int a = T.acc[i][m];
      A[a] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(s16x2, A[a]) +
                                              __builtin_bit_cast(s16x2, x[4 * i + m]));
    }
  if constexpr (D == 6 && !PARTIAL) {
    // one half per line, every line 8 pixels: 105 * sum of squared halves
    int sq = 0;
#pragma unroll
    for (int k = 0; k < T.nacc; ++k)
      sq = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, A[k]),
                                  __builtin_bit_cast(s16x2, A[k]), sq, false);
    return __mul24(sq, 105);
  } else {
    // v^2 <= 1024^2 and 840 / N <= 840: both factors fit 24 bits
    int c = 0;
    if constexpr (PARTIAL) {
      const uint64_t cnt = kCutLineCounts.w[D][bh - 1][bw - 1];
#pragma unroll
      for (int l = 0; l < T.nl; ++l)
        c += __mul24(line_square<D>(A, l), inv840((int)(cnt >> (4 * l)) & 15));
    } else {
      // the squares of the lines of one length accumulate in v_dot2 and are
      // scaled by 840 / N once (at most 8 lines of 2^20: unsigned 24 bits)
      int sq[9];
#pragma unroll
      for (int n = 0; n < 9; ++n) sq[n] = 0;
#pragma unroll
      for (int l = 0; l < T.nl; ++l) sq[T.n[l]] = line_square<D>(A, l, sq[T.n[l]]);
#pragma unroll
      for (int n = 1; n < 9; ++n) {
        bool used = false;
        for (int l = 0; l < T.nl; ++l) used = used || T.n[l] == n;
        if (used) c = (int)__umul24((unsigned)sq[n], 840u / n) + c;
      }
    }
    return c;
  }
}

template <bool PARTIAL>
__device__ __forceinline__ void dir_costs_packed(const uint32_t (&x)[32], int bw, int bh,
                                                 int (&cost)[8]) {
  cost[0] = dir_cost_packed<0, PARTIAL>(x, bw, bh);
  cost[1] = dir_cost_packed<1, PARTIAL>(x, bw, bh);
  cost[2] = dir_cost_packed<2, PARTIAL>(x, bw, bh);
  cost[3] = dir_cost_packed<3, PARTIAL>(x, bw, bh);
  cost[4] = dir_cost_packed<4, PARTIAL>(x, bw, bh);
  cost[5] = dir_cost_packed<5, PARTIAL>(x, bw, bh);
  cost[6] = dir_cost_packed<6, PARTIAL>(x, bw, bh);
  cost[7] = dir_cost_packed<7, PARTIAL>(x, bw, bh);
}

// Centres a word of two raw samples for the search: (x >> c) - 128 per half
// (the downscale to 8 bits of Section 2 for c = bit depth - 8 > 0).
__device__ __forceinline__ uint32_t centre_word(uint32_t raw, int c) {
  const u16x2 v = __builtin_bit_cast(u16x2, raw) >> (u16x2){(unsigned short)c, (unsigned short)c};
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(s16x2, v) - (s16x2){128, 128});
}

// Keeps the halves of word (i, m) that lie inside the top-left bw x bh
// pixels of the block; zeroes the others.
__device__ __forceinline__ uint32_t mask_word(uint32_t w, int i, int m, int bw, int bh) {
  const uint32_t lo = (i < bh && 2 * m < bw) ? 0xFFFFu : 0u;
  const uint32_t hi = (i < bh && 2 * m + 1 < bw) ? 0xFFFF0000u : 0u;
  return w & (lo | hi);
}

// Argmax with a strict '>' from d = 0, and the directional contrast
// v = s_best - s_(best+4 mod 8).
__device__ __forceinline__ void pick_direction(const int (&cost)[8], int &dir, int &var) {
  int best = 0, bc = cost[0];
#pragma unroll
  for (int d = 1; d < 8; ++d)
    if (cost[d] > bc) {
      bc = cost[d];
      best = d;
    }
  int orth = cost[0];
#pragma unroll
  for (int d = 1; d < 8; ++d)
    if (((best + 4) & 7) == d) orth = cost[d];
  dir = best;
  var = bc - orth;
}

// Eq. (13): the luma primary strength adjusted by the contrast v, for all
// 16 signaled strengths, packed 4 bits each.
__device__ __forceinline__ uint64_t adjusted_strengths(int var) {
  if (var < 1024) return 0;
  const int q = var >> 16;
  const int i = q == 0 ? 0 : min(floor_log2(q), 12);
  uint64_t t = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) t |= (uint64_t)((s * (4 + i) + 8) >> 4) << (4 * s);
  return t;
}

// Eq. (13) for one signaled strength s (0..19).
__device__ __forceinline__ int adjust_strength(int s, int var) {
  if (var < 1024) return 0;
  const int q = var >> 16;
  const int i = q == 0 ? 0 : min(floor_log2(q), 12);
  return (s * (4 + i) + 8) >> 4;
}

// Section 4: the preset of one plane group from its two strength bytes:
// primary in the low 4 bits, secondary in bits 0-6 (values above 4 act as
// 4), the skip condition bit in bit 7.  Strengths 0, 0 with the bit set
// stand for S^(p) = 19, S^(s) = 7.
struct Preset {
  int pri, sec;
  bool skipcond;
};
__device__ __forceinline__ Preset decode_preset(int pri_byte, int sec_byte) {
  Preset p;
  p.pri = pri_byte & 15;
  p.sec = min(sec_byte & 0x7f, 4);
  p.skipcond = (sec_byte & 0x80) != 0;
  if (p.pri == 0 && p.sec == 0 && p.skipcond) {
    p.pri = 19;
    p.sec = 7;
  }
  return p;
}

// Luma damping of a block filtered with adjusted primary strength s: D,
// raised to floor(log2 s) when lower (D may never be below it; only the
// strength 19 of the special preset can reach 16 and up).
__device__ __forceinline__ int luma_damping(int D, int s) {
  return s > 0 ? max(D, floor_log2(s)) : D;
}

// ---- Tile staging ---------------------------------------------------------
// Copies rows y0-2 .. y0+TH+1 and columns x0-2 .. x0+TW+1 of a plane into an
// LDS tile whose column COL0 holds frame column x0.  Positions outside the
// plane get kOutside.  Threads walk consecutive columns, so global reads
// coalesce; the trip count is a compile-time constant so that every load is
// issued before the first LDS store (no load-to-store serialization).
template <int TH, int TW, int STRIDE, int COL0, int NT>
__device__ __forceinline__ void stage_recon(uint16_t *lds, const uint16_t *plane, int64_t stride,
                                            int pw, int ph, int y0, int x0, int tid) {
  constexpr int W = TW + 4, N = (TH + 4) * W, ITER = (N + NT - 1) / NT;
  uint16_t v[ITER];
#pragma unroll
  for (int k = 0; k < ITER; ++k) {
    const int e = tid + k * NT;
    const int r = e / W, c = e - r * W;
    const int y = y0 - 2 + r, x = x0 - 2 + c;
    v[k] = kOutside;
    if (e < N && y >= 0 && y < ph && x >= 0 && x < pw) v[k] = plane[(int64_t)y * stride + x];
  }
#pragma unroll
  for (int k = 0; k < ITER; ++k) {
    const int e = tid + k * NT;
    const int r = e / W, c = e - r * W;
    if (e < N) lds[r * STRIDE + COL0 - 2 + c] = v[k];
  }
}

// Copies the TH x TW interior (no halo) of a plane; outside positions get 0.
template <int TH, int TW, int NT>
__device__ __forceinline__ void stage_interior(uint16_t *lds, const uint16_t *plane,
                                               int64_t stride, int pw, int ph, int y0, int x0,
                                               int tid) {
  constexpr int ITER = (TH * TW + NT - 1) / NT;
  uint16_t v[ITER];
#pragma unroll
  for (int k = 0; k < ITER; ++k) {
    const int e = tid + k * NT;
    const int r = e / TW, c = e - r * TW;
    const int y = y0 + r, x = x0 + c;
    v[k] = (e < TH * TW && y < ph && x < pw) ? plane[(int64_t)y * stride + x] : (uint16_t)0;
  }
#pragma unroll
  for (int k = 0; k < ITER; ++k) {
    const int e = tid + k * NT;
    if (e < TH * TW) lds[e] = v[k];
  }
}

// Fast staging of ROWS rows of Q 16-byte chunks each, from a plane whose base
// and row pitch are 16-byte aligned, into LDS rows of LSTRIDE samples: row r,
// chunk q reads plane[(y0 + r) * stride + xs + 8 q .. + 7], xs a multiple of 8.
// The caller guarantees that the whole rectangle lies inside the plane.
// Frame planes live in device (global) memory: byte pointers into them in
// the global address space, so that loads and stores through them are
// global instructions with a scalar base, not flat ones.
using GlobalBytes = const __attribute__((address_space(1))) char *;
using GlobalBytesOut = __attribute__((address_space(1))) char *;
__device__ __forceinline__ GlobalBytes to_global(const uint16_t *p) {
  return (GlobalBytes)(reinterpret_cast<const char *>(p));
}
__device__ __forceinline__ GlobalBytesOut to_global_out(uint16_t *p) {
  return (GlobalBytesOut)(reinterpret_cast<char *>(p));
}
// 16- and 8-byte moves through such pointers (plain vector types: the HIP
// vector classes have no assignment in that address space)
using U32x4 = uint32_t __attribute__((ext_vector_type(4)));
using U32x2 = uint32_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint4 load16(GlobalBytes p) {
  return __builtin_bit_cast(uint4, *reinterpret_cast<const __attribute__((address_space(1))) U32x4 *>(p));
}
__device__ __forceinline__ void store16(GlobalBytesOut p, uint4 v) {
  *reinterpret_cast<__attribute__((address_space(1))) U32x4 *>(p) = __builtin_bit_cast(U32x4, v);
}
__device__ __forceinline__ void store8(GlobalBytesOut p, uint2 v) {
  *reinterpret_cast<__attribute__((address_space(1))) U32x2 *>(p) = __builtin_bit_cast(U32x2, v);
}

template <int ROWS, int Q, int LSTRIDE, int NT>
__device__ __forceinline__ void stage_rows16(uint16_t *lds, const uint16_t *plane, int64_t stride,
                                             int y0, int xs, int tid) {
  constexpr int N = ROWS * Q, ITER = (N + NT - 1) / NT;
  // global loads from a wave-uniform base at 32-bit byte offsets: the
  // callers take this path only for pitches below 2^23 samples, so a row
  // offset is a 24-bit product
  // offset, with e = r Q + q: r pitch + 16 q = r (pitch - 16 Q) + 16 e (the
  // callers' bounds keep the staged row inside the plane's row, so a pitch
  // holds at least its 16 Q bytes)
  const GlobalBytes base = to_global(plane + (int64_t)y0 * stride + xs);
  const uint32_t rstep = 2u * (uint32_t)stride - 16u * Q;
  uint4 v[ITER];
#pragma unroll
  for (int k = 0; k < ITER; ++k) {
    const int e = tid + k * NT;
    const int r = e / Q;
    v[k] = make_uint4(0, 0, 0, 0);
    if (e < N)
      v[k] = load16(base + (__umul24((uint32_t)r, rstep) + 16u * (uint32_t)e));
  }
  static_assert(LSTRIDE >= 8 * Q, "an LDS tile row holds the staged row");
#pragma unroll
  for (int k = 0; k < ITER; ++k) {
    const int e = tid + k * NT;
    const int r = e / Q;
    if (e < N) *reinterpret_cast<uint4 *>(lds + r * (LSTRIDE - 8 * Q) + 8 * e) = v[k];
  }
}

}  // namespace cdef
