// Fused CDEF kernel over 64x64 filter blocks (Section 4), one workgroup of
// four waves per filter block, in one of four modes:
//
//  * search (Section 5): direction search (Section 2, Algorithm 1), the
//    constrained filter (Section 3) under all 64 (S^(p), S^(s)) pairs and the
//    per-filter-block distortion D_{b,p} = ||s - d||^2 for every plane, with
//    filtered pixels never leaving registers;
//  * full search: the 64 pairs with and without the skip condition bit
//    (Section 4: skipped 8x8 blocks filtered too; strengths 0, 0 standing
//    for 19, 7), 128 in all;
//  * weighted search (Section 5, Eq. 14): the 64 pairs with the
//    contrast-weighted distortion instead of the SSE;
//  * filter: direction search and the filter (Eq. 7-13) at the block's own
//    preset, writing the filtered planes.
//
// A launch covers the filter blocks of one frame or of a batch of frames of
// any size, bit depth, chroma layout and damping; workgroup ids are remapped
// so that each XCD (one L2 each) walks a contiguous range of filter blocks
// and neighbouring blocks share their halo lines in L2.  Two sets of
// kernels are built from this source: the base kernels (3 waves per SIMD;
// 8/10-bit; 4:0:0, 4:2:0, 4:2:2) and the extended ones (2 waves per SIMD,
// more registers and LDS), which add 12-bit samples, 4:4:4 and the weighted
// search.
//
// Search decomposition per filter block:
//  * recon tiles with a 2-pixel halo (the taps reach +-2) and source tiles are
//    staged in LDS for luma and the chroma planes (4:2:2 chroma is never
//    filtered, Section 4, and is not staged);
//  * wave 0 runs Algorithm 1 for the 64 luma 8x8 blocks, one block per lane,
//    while waves 1-3 sum (x - s)^2 over skipped blocks (identical for every
//    pair);
//  * non-skipped blocks are compacted; a luma task is two 8x8 blocks held in
//    the two 16-bit halves of every lane (lane = pixel), so the per-block
//    strengths are wave-uniform scalars; a 4:2:0 chroma task is eight 4x4
//    blocks, Cb on waves 0-1 and Cr on waves 2-3; 4:4:4 chroma tasks are
//    shaped like luma tasks, one plane after the other on all four waves;
//  * per task and lane the candidate-independent work (12 tap magnitudes and
//    signs, clamp bounds) is done once; secondary sums for S^(s) = 1, 2, 4,
//    the primary sum once per S^(p), and per pair one packed
//    round/clamp/square-accumulate;
//  * the 64 per-lane accumulators are reduced across the wave by a
//    transposing butterfly built from lane swaps and DPP moves (lane k ends
//    with pair k), then across waves in LDS;
//  * the full search runs the same tasks a second time over the skipped
//    blocks, into separate sums, and evaluates (19, 7) in the slot of the
//    pair (0, 0), whose unfiltered distortion is summed while wave 0 runs
//    the direction search.  By 8x8 block the distortion splits: with the
//    bit, D = (blocks with residual at p) + (skipped blocks at p); without
//    it, (blocks with residual at p) + (skipped blocks unfiltered); a filter
//    block with every block skipped is never filtered.
//
// 12-bit samples: the packed arithmetic stays in 16 bits (tap differences
// and y - s below 2^12, strength sums below 2^13) but the source is no
// longer folded into the rounding offset (16 (x - s) would not fit), and the
// last two levels of the cross-lane sums run in 64 bits.
#include <atomic>
#include <cstddef>
#include <type_traits>

#include "cdef_device.hpp"
#include "cdef_launch.hpp"

// The kernels are built in sets, one translation unit of this source per
// set (CDEF_KSET = 0..8) so that they compile in parallel; without
// CDEF_KSET every set is built into one object.
#ifndef CDEF_KSET
#define CDEF_KSET -1
#endif
#define CDEF_IN_KSET(n) (CDEF_KSET < 0 || CDEF_KSET == (n))

namespace cdef {

namespace {

constexpr int kLS = 80;  // luma recon tile row stride in samples (68 used)
constexpr int kLC0 = 8;  // tile column that holds frame column x0 (16-byte aligned)
constexpr int kCS = 48;  // 4:2:0 chroma recon tile row stride (36 used)
constexpr int kCC0 = 8;

// LDS offsets of the six tap positions (inner, outer along d; along d+2;
// along d-2) in a tile of the given stride, per direction.
struct TapTable {
  int off[8][6];
};
__host__ __device__ constexpr TapTable make_tap_table(int stride) {
  TapTable t{};
  for (int d = 0; d < 8; ++d)
    for (int k = 0; k < 6; ++k) {
      const int dd = k < 2 ? d : k < 4 ? (d + 2) & 7 : (d + 6) & 7;
      t.off[d][k] = tap_dr(dd, k & 1) * stride + tap_dc(dd, k & 1);
    }
  return t;
}

// The 12 tap samples around LDS index b of a tile with the luma stride (also
// the 4:4:4 chroma tiles' stride), for a compile-time direction D: from a
// base moved back by the taps' largest reach (two rows and two columns),
// every tap is a positive load immediate, so the loads need no address
// arithmetic.  Order: primary +inner, -inner, +outer, -outer, then the same
// along d+2 and along d-2.
template <int D>
__device__ __forceinline__ void tap_samples(const uint16_t *rt, int b, uint32_t (&v)[12]) {
  constexpr TapTable T = make_tap_table(kLS);
  constexpr int kReach = 2 * kLS + 2;
  const uint16_t *p = rt + (b - kReach);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int slot = (k >> 1) * 4 + (k & 1) * 2;
    v[slot] = p[kReach + T.off[D][k]];
    v[slot + 1] = p[kReach - T.off[D][k]];
  }
}

// The same for a wave-uniform runtime direction: a scalar branch to the
// direction's loads.
__device__ __forceinline__ void tap_samples(int d, const uint16_t *rt, int b, uint32_t (&v)[12]) {
  switch (d) {
    case 0: tap_samples<0>(rt, b, v); break;
    case 1: tap_samples<1>(rt, b, v); break;
    case 2: tap_samples<2>(rt, b, v); break;
    case 3: tap_samples<3>(rt, b, v); break;
    case 4: tap_samples<4>(rt, b, v); break;
    case 5: tap_samples<5>(rt, b, v); break;
    case 6: tap_samples<6>(rt, b, v); break;
    default: tap_samples<7>(rt, b, v); break;
  }
}

__device__ __forceinline__ s16x2 as_s(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ s16x2 as_s(u16x2 v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ u16x2 as_u(s16x2 v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ u16x2 as_u(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ s16x2 splat(int v) { return s16x2{(short)v, (short)v}; }
__device__ __forceinline__ uint32_t splat32(uint32_t v) { return v | (v << 16); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return (uint64_t)(uint32_t)uniform((int)(uint32_t)v) |
         ((uint64_t)(uint32_t)uniform((int)(uint32_t)(v >> 32)) << 32);
}

// Per-lane, candidate-independent state of one task: two samples per lane.
struct Taps {
  u16x2 ad[12];  // |x_tap - x| (out-of-frame taps: >= 28673)
  s16x2 sg[12];  // sign of x_tap - x as +-1
  s16x2 X;       // 16 (x - s) + 8: the rounding offset with the source folded in (8/10-bit)
  s16x2 dxs;     // x - s
  s16x2 lo, hi;  // clamp range minus s
};

// Tap order: primary +inner, -inner, +outer, -outer; then for the two
// secondary directions d+2 and d-2 the same four.
template <bool B12>
__device__ __forceinline__ void prepare(Taps &t, uint32_t xv, uint32_t sv, const uint32_t (&tp)[12]) {
  const s16x2 X = as_s(xv);
  s16x2 hi = X;
  u16x2 lo = as_u(xv);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const s16x2 v = as_s(tp[k]);
    const s16x2 d = v - X;
    const s16x2 nd = X - v;
    t.ad[k] = as_u(__builtin_elementwise_max(d, nd));
    t.sg[k] = (d >> splat(15)) | splat(1);
    hi = __builtin_elementwise_max(hi, v);        // kOutside is the most negative int16
    lo = __builtin_elementwise_min(lo, as_u(v));  // and the largest uint16 here
  }
  const s16x2 S = as_s(sv);
  t.dxs = X - S;
  if (!B12) t.X = t.dxs * splat(16) + splat(8);
  t.lo = as_s(lo) - S;
  t.hi = hi - S;
}

// Weighted constrained sum over taps [k0, k0+4) with magnitudes already
// shifted (a): f = sign * min(|d|, max(0, S - (|d| >> shift))).
__device__ __forceinline__ s16x2 group_sum(const Taps &t, const u16x2 (&a)[4], int k0, uint32_t s,
                                           uint32_t wi, uint32_t wo) {
  s16x2 m[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    m[k] = as_s(__builtin_elementwise_min(__builtin_elementwise_sub_sat(as_u(s), a[k]),
                                          t.ad[k0 + k]));
  const s16x2 inner = m[0] * t.sg[k0] + m[1] * t.sg[k0 + 1];
  const s16x2 outer = m[2] * t.sg[k0 + 2] + m[3] * t.sg[k0 + 3];
  return inner * as_s(wi) + outer * as_s(wo);
}

// Secondary sum over the 8 secondary taps for strength `s` (scaled, both
// halves) and shift `sh` (both halves); weights 2 (inner) and 1 (outer).
__device__ __forceinline__ s16x2 secondary(const Taps &t, uint32_t s, uint32_t sh) {
  s16x2 q = splat(0);
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    u16x2 a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = t.ad[4 + 4 * g + k] >> as_u(sh);
    q = q + group_sum(t, a, 4 + 4 * g, s, splat32(2), splat32(1));
  }
  return q;
}

// round(v / 16), ties away from zero, as v + 8 - [v < 0] shifted right by 4.
__device__ __forceinline__ s16x2 round16(s16x2 v) {
  return (v + splat(8) + (v >> splat(15))) >> splat(4);
}

// One (S^(p), S^(s)) pair with both groups possibly active: round the sum
// of P and Q ties-away-from-zero, add to x - s, clamp; returns y - s.
template <bool B12>
__device__ __forceinline__ s16x2 err_both(const Taps &t, s16x2 P, s16x2 Q) {
  const s16x2 sum = P + Q;
  const s16x2 y = B12 ? t.dxs + round16(sum) : (t.X + sum + (sum >> splat(15))) >> splat(4);
  return __builtin_elementwise_min(__builtin_elementwise_max(y, t.lo), t.hi);
}

// A pair with only one tap group: its weights sum to 12/16 < 1, so the
// result cannot leave the clamp range and the clamp is skipped.
template <bool B12>
__device__ __forceinline__ s16x2 err_one(const Taps &t, s16x2 P) {
  return B12 ? t.dxs + round16(P) : (t.X + P + (P >> splat(15))) >> splat(4);
}

// The four pairs (S^(p), 0..3) of one primary strength: err_one for the
// first, err_both for the others, with the four dependency chains advanced
// step by step side by side, so that no packed result is read by the very
// next instruction (which costs a wait state).  Used by the extended
// kernels, whose two waves per SIMD hide few wait states (4:4:4 search
// +1 %); the base kernels, at three waves per SIMD, measured 0.3 % slower
// with it and keep the pair-by-pair order.
template <bool B12>
__device__ __forceinline__ void err_row(const Taps &t, s16x2 P, const s16x2 (&Q)[4],
                                        s16x2 (&e)[4]) {
  s16x2 v[4], r[4];
  v[0] = P;
#pragma unroll
  for (int i = 1; i < 4; ++i) v[i] = P + Q[i];
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = v[i] >> splat(15);
  if (B12) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = v[i] + splat(8);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = v[i] + r[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = v[i] >> splat(4);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = t.dxs + v[i];
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = t.X + v[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = v[i] + r[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = v[i] >> splat(4);
  }
  e[0] = v[0];
#pragma unroll
  for (int i = 1; i < 4; ++i) v[i] = __builtin_elementwise_max(v[i], t.lo);
#pragma unroll
  for (int i = 1; i < 4; ++i) e[i] = __builtin_elementwise_min(v[i], t.hi);
}

// Secondary sums for S^(s) = 1, 2, 4 at damping `damp` (8-bit domain).
__device__ __forceinline__ void secondaries(const Taps &t, int c, int damp, s16x2 (&Q)[4]) {
  Q[1] = secondary(t, splat32(1u << c), splat32((uint32_t)damp));
  Q[2] = secondary(t, splat32(2u << c), splat32((uint32_t)(damp - 1)));
  Q[3] = secondary(t, splat32(4u << c), splat32((uint32_t)(damp - 2)));
}

// The special preset (Section 4) on a luma task: S^(p) = 19 adjusted per
// block by Eq. (13) (a19A, a19B), S^(s) = 7, each block's damping raised to
// floor(log2 S) when lower.
template <bool B12>
__device__ __forceinline__ s16x2 luma_special(const Taps &t, int a19A, int a19B, int c, int D) {
  const int dA = luma_damping(D, a19A), dB = luma_damping(D, a19B);
  const uint32_t sp = ((uint32_t)a19A << c) | ((uint32_t)a19B << (16 + c));
  const uint32_t sh = (uint32_t)(a19A ? dA - floor_log2(a19A) : 0) |
                      ((uint32_t)(a19B ? dB - floor_log2(a19B) : 0) << 16);
  const uint32_t w1 = ((a19A & 1) ? 3u : 4u) | (((a19B & 1) ? 3u : 4u) << 16);
  const uint32_t w2 = ((a19A & 1) ? 3u : 2u) | (((a19B & 1) ? 3u : 2u) << 16);
  u16x2 a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = t.ad[k] >> as_u(sh);
  const s16x2 P = group_sum(t, a, 0, sp, w1, w2);
  const s16x2 Q = secondary(t, splat32(7u << c), (uint32_t)(dA - 2) | ((uint32_t)(dB - 2) << 16));
  return err_both<B12>(t, P, Q);
}

// The special preset on a chroma task: 19 (odd: weights 3, 3) and 7 at the
// chroma damping max(D - 1, floor(log2 19) = 4).
template <bool B12>
__device__ __forceinline__ s16x2 chroma_special(const Taps &t, int c, int D) {
  const int Dc = max(D - 1, 4);
  u16x2 a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = t.ad[k] >> as_u(splat32((uint32_t)(Dc - 4)));
  const s16x2 P = group_sum(t, a, 0, splat32(19u << c), splat32(3), splat32(3));
  const s16x2 Q = secondary(t, splat32(7u << c), splat32((uint32_t)(Dc - 2)));
  return err_both<B12>(t, P, Q);
}

// Luma task: 2 blocks (lo/hi half) with per-block adjusted primary
// strengths (Eq. 13).  Per-strength parameters are wave-uniform 32-bit
// scalars (low half: block A, high half: block B).  Each pair's y - s goes
// to sink(pair, e), pair = S^(p) * 4 + index of S^(s).
//
// SUB: only the strengths of a subset (pm: S^(p) mask, qm: S^(s) index mask,
// sp19: the special preset) are evaluated; the sink sees no other pair.
// QALL: the subset has every S^(s) (qm = 15), so no pair needs its own
// test.  Per block of the task (A: low halves, B: high halves): adj the
// adjusted strengths, lsh and par their shifts and parities
// (SmemCore::lsh, lpar).
template <bool FULL, bool B12, bool SUB, bool QALL = false, class Sink>
__device__ __forceinline__ void luma_pairs(const Taps &t, uint64_t adjA, uint64_t adjB,
                                           uint64_t lshA, uint64_t lshB, uint32_t parA,
                                           uint32_t parB, int a19A, int a19B, int c, int D,
                                           uint32_t pm, uint32_t qm, bool sp19, Sink &&sink) {
  if constexpr (QALL) qm = 15u;
  // pair (0, 0) filters nothing; in the full search its slot carries the
  // special preset instead (the unfiltered distortion is summed elsewhere)
  if (FULL) {
    if (!SUB || sp19) sink(0, luma_special<B12>(t, a19A, a19B, c, D));
  } else if (!SUB || (pm & qm & 1)) {
    sink(0, t.dxs);
  }
  s16x2 Q[4];
  secondaries(t, c, D, Q);
#pragma unroll
  for (int si = 1; si < 4; ++si)
    if (!SUB || ((pm & 1) && ((qm >> si) & 1))) sink(si, err_one<B12>(t, Q[si]));
#pragma unroll
  for (int S = 1; S < 16; ++S) {
    if (SUB && !((pm >> S) & 1)) continue;
    const uint32_t sa = (uint32_t)(adjA >> (4 * S)) & 15u, sb = (uint32_t)(adjB >> (4 * S)) & 15u;
    const uint32_t sp = (sa | (sb << 16)) << c;
    const uint32_t sh =
        ((uint32_t)(lshA >> (4 * S)) & 15u) | (((uint32_t)(lshB >> (4 * S)) & 15u) << 16);
    // weights 4, 2 at even strengths, 3, 3 at odd ones
    const uint32_t odd = ((parA >> S) & 1u) | (((parB >> S) & 1u) << 16);
    const uint32_t w1 = 0x00040004u - odd, w2 = 0x00020002u + odd;
    // the shift pair changes only a few times over S = 1..15, but skipping
    // the re-shift where it does not makes the magnitudes a value carried
    // across a branch at every strength, which the compiler copies (4
    // moves per strength, more than the 4 shifts)
    u16x2 a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = t.ad[k] >> as_u(sh);
    const s16x2 P = group_sum(t, a, 0, sp, w1, w2);
    if constexpr (!SUB && std::decay_t<Sink>::kRows) {
      s16x2 e[4];
      err_row<B12>(t, P, Q, e);
#pragma unroll
      for (int si = 0; si < 4; ++si) sink(4 * S + si, e[si]);
    } else {
      if (!SUB || (qm & 1)) sink(4 * S, err_one<B12>(t, P));
#pragma unroll
      for (int si = 1; si < 4; ++si)
        if (!SUB || ((qm >> si) & 1)) sink(4 * S + si, err_both<B12>(t, P, Q[si]));
    }
  }
}

// Chroma task: strengths are not adjusted (uniform over the plane); the
// chroma damping is max(D - 1, floor(log2 S^(p))) for both tap groups, which
// differs from D - 1 only for D = 3 and S^(p) >= 8.
// D3: D = 3, where the chroma damping of the secondary taps changes at
// S^(p) = 8.  Callers pick the variant outside their task loops (with_d3),
// so that no branch splits a loop's unrolled strength sequence.
template <bool FULL, bool B12, bool SUB, bool D3, bool QALL = false, class Sink>
__device__ __forceinline__ void chroma_pairs(const Taps &t, int c, int Drt, uint32_t pm,
                                             uint32_t qm, bool sp19, Sink &&sink) {
  const int D = D3 ? 3 : Drt;
  if constexpr (QALL) qm = 15u;  // as in luma_pairs
  if (FULL) {
    if (!SUB || sp19) sink(0, chroma_special<B12>(t, c, D));
  } else if (!SUB || (pm & qm & 1)) {
    sink(0, t.dxs);
  }
  s16x2 Q[4];
  secondaries(t, c, D - 1, Q);
#pragma unroll
  for (int si = 1; si < 4; ++si)
    if (!SUB || ((pm & 1) && ((qm >> si) & 1))) sink(si, err_one<B12>(t, Q[si]));
  u16x2 a[4];
#pragma unroll
  for (int S = 1; S < 16; ++S) {
    const int lg = S >= 8 ? 3 : S >= 4 ? 2 : S >= 2 ? 1 : 0;
    if (S == 8 && D3) secondaries(t, c, 3, Q);  // chroma damping becomes 3
    const int Dc = max(D - 1, lg);
    // the shift changes only where floor(log2 S) does (compile-time), so the
    // magnitudes are re-shifted there, also when a subset skips that S
    if (S == 1 || S == 2 || S == 4 || S == 8) {
#pragma unroll
      for (int k = 0; k < 4; ++k) a[k] = t.ad[k] >> as_u(splat32((uint32_t)(Dc - lg)));
    }
    if (SUB && !((pm >> S) & 1)) continue;
    const uint32_t w1 = splat32((S & 1) ? 3u : 4u), w2 = splat32((S & 1) ? 3u : 2u);
    const s16x2 P = group_sum(t, a, 0, splat32((uint32_t)S << c), w1, w2);
    if constexpr (!SUB && std::decay_t<Sink>::kRows) {
      s16x2 e[4];
      err_row<B12>(t, P, Q, e);
#pragma unroll
      for (int si = 0; si < 4; ++si) sink(4 * S + si, e[si]);
    } else {
      if (!SUB || (qm & 1)) sink(4 * S, err_one<B12>(t, P));
#pragma unroll
      for (int si = 1; si < 4; ++si)
        if (!SUB || ((qm >> si) & 1)) sink(4 * S + si, err_both<B12>(t, P, Q[si]));
    }
  }
}

// Runs f(std::true_type) when b holds, f(std::false_type) otherwise: a
// runtime choice made once, outside a task loop, between two instantiations.
template <class F>
__device__ __forceinline__ void with_flag(bool b, F &&f) {
  if (b)
    f(std::true_type{});
  else
    f(std::false_type{});
}

template <class F>
__device__ __forceinline__ void with_d3(int D, F &&f) {
  with_flag(D == 3, f);
}

// The subset of a job: S^(p) mask, S^(s) index mask, skip-bit mask (all
// presets when the job carries none).
struct Subset {
  uint32_t pm, qm, km;
  __device__ __forceinline__ explicit Subset(uint32_t cand)
      : pm(cand ? cand & 0xFFFF : 0xFFFF), qm(cand ? (cand >> 16) & 15 : 15),
        km(cand ? (cand >> 20) & 3 : 3) {}
  __device__ __forceinline__ bool has(int k, int pair) const {
    return ((pm >> (pair >> 2)) & (qm >> (pair & 3)) & (km >> k) & 1) != 0;
  }
};

// Square-accumulate sink of the SSE searches; ROWS: the pairs of a
// strength come through err_row (the extended kernels, two waves per SIMD).
template <bool ROWS>
struct SquareSum {
  static constexpr bool kRows = ROWS;
  int (&acc)[64];
  __device__ __forceinline__ void operator()(int k, s16x2 e) const {
    acc[k] = __builtin_amdgcn_sdot2(e, e, acc[k], false);
  }
};

// One butterfly level at lane distance 8, 4, 2 or 1: the partner lane (DPP
// `ctrl`) lies in the other half of the group; of the values v[0, 2 HALF)
// each lane keeps one half (the upper if `up`) and adds the partner's copy.
template <int HALF, int CTRL>
__device__ __forceinline__ void dpp_level(uint32_t (&v)[64], bool up) {
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const uint32_t a = v[i], b = v[i + HALF];
    const uint32_t send = up ? a : b;
    const uint32_t keep = up ? b : a;
    v[i] = keep + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)send, CTRL, 0xF, 0xF, false);
  }
}

// The same level on 64-bit values (two 32-bit DPP moves per value).
template <int HALF, int CTRL>
__device__ __forceinline__ void dpp_level64(uint64_t (&v)[4], bool up) {
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const uint64_t a = v[i], b = v[i + HALF];
    const uint64_t send = up ? a : b;
    const uint64_t keep = up ? b : a;
    const uint32_t lo =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)send, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(send >> 32),
                                                              CTRL, 0xF, 0xF, false);
    v[i] = keep + ((uint64_t)hi << 32 | lo);
  }
}

// Wave-wide sums of 64 per-lane 32-bit values (consumed); lane k returns
// the total of value k.  Each level halves the values kept per lane.  With
// B12 the last two levels (sums over 32 and 64 lanes) run in 64 bits: after
// 16 lanes a 12-bit sum is still below 2^32.
template <bool B12>
__device__ __forceinline__ uint64_t reduce_transpose_u(uint32_t (&v)[64], int lane) {
  // distance 32: lanes 0-31 keep value i, lanes 32-63 value i + 32
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(v[i], v[i + 32], false, false);
    v[i] = r[0] + r[1];
  }
  // distance 16: odd rows of 16 keep value i + 16
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(v[i], v[i + 16], false, false);
    v[i] = r[0] + r[1];
  }
  dpp_level<8, 0x140>(v, (lane & 8) != 0);  // row_mirror: 15 - l within a row
  dpp_level<4, 0x141>(v, (lane & 4) != 0);  // row_half_mirror: 7 - l within 8
  if constexpr (B12) {
    uint64_t w[4] = {v[0], v[1], v[2], v[3]};
    dpp_level64<2, 0x4E>(w, (lane & 2) != 0);  // quad_perm [2,3,0,1]
    dpp_level64<1, 0xB1>(w, (lane & 1) != 0);  // quad_perm [1,0,3,2]
    return w[0];
  } else {
    dpp_level<2, 0x4E>(v, (lane & 2) != 0);
    dpp_level<1, 0xB1>(v, (lane & 1) != 0);
    return v[0];
  }
}

template <bool B12>
__device__ __forceinline__ uint64_t reduce_transpose(const int (&acc)[64], int lane) {
  uint32_t v[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) v[i] = (uint32_t)acc[i];
  return reduce_transpose_u<B12>(v, lane);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Workgroup id -> work item: hardware deals workgroups to the 8 XCDs
// round-robin; give each XCD a contiguous range of items.
__device__ __forceinline__ int xcd_item(int wg, int n) {
  const int x = wg & 7, i = wg >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + i;
}

// Planes a search covers: luma only at 4:0:0 and 4:2:2.
__device__ __forceinline__ int search_planes(const JobDesc &J) {
  return J.nplanes == 3 && J.layout != kLayout422 ? 3 : 1;
}

// LDS of one workgroup.  X (extended kernels): chroma tiles as large as
// luma's for 4:4:4.  SmemCore: the tiles and per-block state every mode
// uses (the filter-only kernels hold just this); SmemT adds the searches'
// reduction buffers.
template <bool X>
struct SmemCore {
  static constexpr int kCT = X ? 68 * kLS : 36 * kCS;  // chroma recon tile
  static constexpr int kCSrc = X ? 64 * 64 : 32 * 32;  // chroma source tile
  uint16_t ry[68 * kLS];
  uint16_t sy[64 * 64];  // searches: source; filter: filtered luma
  uint16_t rc[2][kCT];
  uint16_t sc[2][kCSrc];  // searches: source; filter: filtered chroma
  uint64_t adj[64];
  union {
    // searches, per block and primary strength S = 1..15 of the adjusted
    // strength a_S: 4 bits of D - floor(log2 a_S) (0 where a_S = 0), and
    // bit S of its parity
    struct {
      uint64_t lsh[64];
      uint16_t lpar[64];
    };
    // filter mode, per block under the filter block's luma preset: word 0
    // holds the adjusted primary strength scaled to the bit depth (low half)
    // and its magnitude shift (high half), word 1 its parity (low half) and
    // the secondary taps' shift (high half)
    uint32_t fpar[64][2];
  };
  int32_t var[64];
  int16_t coff[8][6];  // 4:2:0 chroma tap offsets in bytes, per direction and tap position
  uint8_t dir[64];
  uint8_t list[64];   // blocks with residual, then (full search, filter) skipped blocks
  uint8_t adj19[64];  // Eq. (13) applied to 19 (full search, filter)
  uint8_t flag[64];   // bit 0: in frame, bit 1: skipped
  int n, nsk;
};

// Weighted search: per-wave moment scratch in chunks of 8 pairs (see
// ChunkMoments); waves 0-1 use `red`, idle in that mode, waves 2-3 `wb`.
constexpr int kWbPairs = 8;
constexpr int kWbRow = 8 * 16 + 8;                   // 8 blocks of 16 samples + padding
constexpr int kWbEntries = (kWbPairs + 1) * kWbRow;  // + the source samples

template <bool X>
struct SmemT : SmemCore<X> {
  alignas(16) uint64_t red[3][4][64];  // [plane][wave][pair]: blocks with residual
  union {
    uint64_t red2[3][4][64];  // the same over skipped blocks (full search)
    struct {
      // weighted search, per plane and filtering unit (8x8 luma and 4:4:4
      // chroma, 4x4 4:2:0 chroma): n, sum s, sum s^2, sum x, sum x^2, sum x s
      // over in-frame pixels
      uint32_t ustat[6][3][64];
      double wred[3][4][64];  // per wave and pair: Eq. (14) over its tasks' units
    } w;
  };
  uint64_t skipsse[3];  // per plane: sum of (x - s)^2 over skipped blocks
  uint64_t allsse[3];   // the same over every in-frame pixel (full search)
  double skipw[3];      // Eq. (14) over skipped units, per plane
  alignas(16) uint16_t wb[2 * kWbEntries];  // weighted search: waves 2-3's moment scratch
};

// Stage the recon tiles (all modes) and, for the searches, the source
// tiles; per-block flags for the 64 luma blocks.  Filter blocks whose tiles
// (with the 16-byte-rounded halo) lie inside aligned planes take 16-byte
// loads; the rest go sample by sample with the frame-edge sentinel.
template <bool X>
__device__ __forceinline__ void stage_item(SmemCore<X> &sm, const JobDesc &J, int fby, int fbx,
                                           int tid, bool search) {
  const int W = J.width, H = J.height, y0 = fby * 64, x0 = fbx * 64;
  const int cw = (W + 1) >> 1, ch = (H + 1) >> 1, cy0 = y0 >> 1, cx0 = x0 >> 1;
  const bool c420 = J.nplanes == 3 && J.layout == kLayout420;
  const bool c444 = X && J.nplanes == 3 && J.layout == kLayout444;
  const bool luma_fast = (J.flags & kAligned16) && y0 >= 2 && y0 + 66 <= H && x0 >= 8 &&
                         x0 + 72 <= W;
  const bool fast =
      luma_fast && (!c420 || (cy0 >= 2 && cy0 + 34 <= ch && cx0 >= 8 && cx0 + 40 <= cw));
  if (fast) {
    // luma: 68 rows of columns x0-8 .. x0+71 (the tile's full 80-sample rows)
    stage_rows16<68, 10, kLS, 256>(sm.ry, J.rec[0], J.rstride[0], y0 - 2, x0 - kLC0, tid);
    if (search) stage_rows16<64, 8, 64, 256>(sm.sy, J.src[0], J.sstride[0], y0, x0, tid);
    if (c420) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        stage_rows16<36, 6, kCS, 256>(sm.rc[p], J.rec[p + 1], J.rstride[p + 1], cy0 - 2,
                                      cx0 - kCC0, tid);
        if (search)
          stage_rows16<32, 4, 32, 256>(sm.sc[p], J.src[p + 1], J.sstride[p + 1], cy0, cx0, tid);
      }
    }
    if constexpr (X) {
      if (c444) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          stage_rows16<68, 10, kLS, 256>(sm.rc[p], J.rec[p + 1], J.rstride[p + 1], y0 - 2,
                                         x0 - kLC0, tid);
          if (search)
            stage_rows16<64, 8, 64, 256>(sm.sc[p], J.src[p + 1], J.sstride[p + 1], y0, x0, tid);
        }
      }
    }
  } else {
    stage_recon<64, 64, kLS, kLC0, 256>(sm.ry, J.rec[0], J.rstride[0], W, H, y0, x0, tid);
    if (search) stage_interior<64, 64, 256>(sm.sy, J.src[0], J.sstride[0], W, H, y0, x0, tid);
    if (c420) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        stage_recon<32, 32, kCS, kCC0, 256>(sm.rc[p], J.rec[p + 1], J.rstride[p + 1], cw, ch,
                                            cy0, cx0, tid);
        if (search)
          stage_interior<32, 32, 256>(sm.sc[p], J.src[p + 1], J.sstride[p + 1], cw, ch, cy0,
                                      cx0, tid);
      }
    }
    if constexpr (X) {
      if (c444) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          stage_recon<64, 64, kLS, kLC0, 256>(sm.rc[p], J.rec[p + 1], J.rstride[p + 1], W, H, y0,
                                              x0, tid);
          if (search)
            stage_interior<64, 64, 256>(sm.sc[p], J.src[p + 1], J.sstride[p + 1], W, H, y0, x0,
                                        tid);
        }
      }
    }
  }
  if (tid < 48) {
    const int d = tid / 6, k = tid - 6 * (tid / 6);
    const int dd = k < 2 ? d : k < 4 ? (d + 2) & 7 : (d + 6) & 7;
    sm.coff[d][k] = (int16_t)(2 * (tap_dr(dd, k & 1) * kCS + tap_dc(dd, k & 1)));
  }
  if (tid < 64) {
    const int by = fby * 8 + (tid >> 3), bx = fbx * 8 + (tid & 7);
    const bool in = by < J.brows && bx < J.bcols;
    const bool sk = in && J.skip && J.skip[(int64_t)by * J.bcols + bx];
    sm.flag[tid] = (uint8_t)((in ? 1 : 0) | (sk ? 2 : 0));
  }
}

// Algorithm 1 for the 64 luma blocks of the filter block, one per lane of
// wave 0; Eq. (13) adjusted strengths; compaction of the blocks to filter
// (the full search lists the skipped in-frame blocks after them).
// PACKED: Algorithm 1 on packed 16-bit halves (half the registers; the
// filter kernels), else in 32-bit lanes (fewer issue cycles; the searches).
template <bool FULL, bool X, bool PACKED = false, bool FILT = false>
__device__ __forceinline__ void direction_search(SmemCore<X> &sm, const JobDesc &J, int fby, int fbx,
                                                 int lane, const Preset &py = Preset{}) {
  const int b = lane;
  const int by = fby * 8 + (b >> 3), bx = fbx * 8 + (b & 7);
  const int c = J.bitdepth - 8;
  const bool in = sm.flag[b] & 1, sk = sm.flag[b] & 2;
  int d = 0, v = 0;
  if (in && (J.flags & kDirIn)) {
    // the caller's directions (masked to 0..7) and contrasts
    d = J.dir[(int64_t)by * J.bcols + bx] & 7;
    v = J.var[(int64_t)by * J.bcols + bx];
  } else if (in) {
    const int bw = min(8, J.width - 8 * bx), bh = min(8, J.height - 8 * by);
    const uint16_t *row0 = sm.ry + (2 + 8 * (b >> 3)) * kLS + kLC0 + 8 * (b & 7);
    int cost[8];
    if constexpr (PACKED) {
      uint32_t x[32];  // row i, word m: columns 2m and 2m + 1, centred
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint4 q = *reinterpret_cast<const uint4 *>(row0 + i * kLS);
        x[4 * i + 0] = centre_word(q.x, c);
        x[4 * i + 1] = centre_word(q.y, c);
        x[4 * i + 2] = centre_word(q.z, c);
        x[4 * i + 3] = centre_word(q.w, c);
      }
      if (bw == 8 && bh == 8) {
        dir_costs_packed<false>(x, 8, 8, cost);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int m = 0; m < 4; ++m) x[4 * i + m] = mask_word(x[4 * i + m], i, m, bw, bh);
        dir_costs_packed<true>(x, bw, bh, cost);
      }
    } else {
      int x[64];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint4 q = *reinterpret_cast<const uint4 *>(row0 + i * kLS);
        const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int px = (int)((w4[j >> 1] >> (16 * (j & 1))) & 0xFFFF);
          x[i * 8 + j] = (px >> c) - 128;
        }
      }
      if (bw == 8 && bh == 8) {
        dir_costs_full(x, cost);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (i >= bh || j >= bw) x[i * 8 + j] = 0;
        dir_costs_partial(x, bw, bh, cost);
      }
    }
    pick_direction(cost, d, v);
    if (J.dir) {
      J.dir[(int64_t)by * J.bcols + bx] = (uint8_t)d;
      J.var[(int64_t)by * J.bcols + bx] = v;
    }
  }
  sm.dir[b] = (uint8_t)d;
  sm.var[b] = v;
  const uint64_t adj = adjusted_strengths(v);
  sm.adj[b] = adj;
  if constexpr (FILT) {
    // the filter block's luma preset: per block the Eq. (13) strength (the
    // special preset's 19 adjusted the same way), its damping, shifts and
    // parity, once here instead of in every task
    const int a = py.pri == 19 ? adjust_strength(19, v) : (int)(adj >> (4 * py.pri)) & 15;
    const int Da = luma_damping(J.damping, a);
    const uint32_t sh = a ? (uint32_t)(Da - floor_log2(a)) : 0u;
    const uint32_t qsh = py.sec ? (uint32_t)(Da - floor_log2(py.sec)) : 0u;
    sm.fpar[b][0] = ((uint32_t)a << c) | (sh << 16);
    sm.fpar[b][1] = (uint32_t)(a & 1) | (qsh << 16);
  } else if constexpr (!PACKED) {
    const int D = J.damping;
    uint64_t shw = 0;
    uint32_t par = 0;
#pragma unroll
    for (int S = 1; S < 16; ++S) {
      const int a = (int)(adj >> (4 * S)) & 15;
      if (a) shw |= (uint64_t)(D - floor_log2(a)) << (4 * S);
      par |= (uint32_t)(a & 1) << S;
    }
    sm.lsh[b] = shw;
    sm.lpar[b] = (uint16_t)par;
  }
  const bool active = in && !sk;
  const uint64_t below = (1ull << lane) - 1ull;
  const uint64_t m = __ballot(active);
  if (active) sm.list[__popcll(m & below)] = (uint8_t)b;
  if (FULL) {
    sm.adj19[b] = (uint8_t)adjust_strength(19, v);
    const bool skipped = in && sk;
    const uint64_t ms = __ballot(skipped);
    if (skipped) sm.list[__popcll(m) + __popcll(ms & below)] = (uint8_t)b;
    if (lane == 0) sm.nsk = __popcll(ms);
  }
  if (lane == 0) sm.n = __popcll(m);
}

// Sum of (x - s)^2 over pixels of skipped blocks, for each searched plane,
// and in the full search also over every in-frame pixel; run by threads
// t0.. of the workgroup (nt of them).  The work unit is a block row (8
// samples of a luma-shaped plane, 4 of a 4:2:0 chroma plane), read as one
// 16- or 8-byte word from each tile; its squares go through v_dot2, two
// samples per instruction.  A row that the frame edge cuts takes the
// samples one by one.  Per-lane partial sums stay below 2^32 (at most 24
// samples of 12 bits); the wave sums are 64-bit.
template <bool FULL, bool X>
__device__ __forceinline__ void skipped_sse(SmemT<X> &sm, const JobDesc &J, int fby, int fbx,
                                            int t, int nt, int lane) {
  const int W = J.width, H = J.height, y0 = fby * 64, x0 = fbx * 64;
  uint32_t e[3] = {0, 0, 0}, a[3] = {0, 0, 0};
  const bool c444 = X && J.nplanes == 3 && J.layout == kLayout444;
  // squares of the differences of N 16-bit words pairs (2 samples each)
  auto sq = [](const uint32_t *xw, const uint32_t *sw, int n) {
    uint32_t q = 0;
    for (int w = 0; w < n; ++w) {
      const s16x2 d = as_s(xw[w]) - as_s(sw[w]);
      q = __builtin_amdgcn_sdot2(d, d, q, false);
    }
    return q;
  };
  // luma-shaped planes: 512 rows of 8 samples (row r, block column bc)
  auto plane8 = [&](const uint16_t *rt, const uint16_t *st, int P) {
    for (int i = t; i < 512; i += nt) {
      const int r = i >> 3, bc = i & 7, col = 8 * bc;
      const int fl = sm.flag[(r >> 3) * 8 + bc];
      if (!(fl & 1) || (!FULL && !(fl & 2)) || y0 + r >= H) continue;
      uint32_t q;
      if (x0 + col + 8 <= W) {
        const uint4 xv = *reinterpret_cast<const uint4 *>(rt + (r + 2) * kLS + kLC0 + col);
        const uint4 sv = *reinterpret_cast<const uint4 *>(st + r * 64 + col);
        const uint32_t xw[4] = {xv.x, xv.y, xv.z, xv.w}, sw[4] = {sv.x, sv.y, sv.z, sv.w};
        q = sq(xw, sw, 4);
      } else {
        q = 0;
        for (int j = 0; j < 8 && x0 + col + j < W; ++j) {
          const int dd = (int)rt[(r + 2) * kLS + kLC0 + col + j] - (int)st[r * 64 + col + j];
          q += (uint32_t)(dd * dd);
        }
      }
      if (fl & 2) e[P] += q;
      a[P] += q;
    }
  };
  plane8(sm.ry, sm.sy, 0);
  if constexpr (X) {
    if (c444) {
      plane8(sm.rc[0], sm.sc[0], 1);
      plane8(sm.rc[1], sm.sc[1], 2);
    }
  }
  if (J.nplanes == 3 && J.layout == kLayout420) {
    // 4:2:0 chroma: per plane 256 rows of 4 samples (4x4 blocks)
    const int cw = (W + 1) >> 1, ch = (H + 1) >> 1, cy0 = y0 >> 1, cx0 = x0 >> 1;
    for (int i = t; i < 512; i += nt) {
      const int p = i >> 8, r = (i >> 3) & 31, bc = i & 7, col = 4 * bc;
      const int fl = sm.flag[(r >> 2) * 8 + bc];
      if (!(fl & 1) || (!FULL && !(fl & 2)) || cy0 + r >= ch) continue;
      uint32_t q;
      if (cx0 + col + 4 <= cw) {
        const uint2 xv = *reinterpret_cast<const uint2 *>(sm.rc[p] + (r + 2) * kCS + kCC0 + col);
        const uint2 sv = *reinterpret_cast<const uint2 *>(sm.sc[p] + r * 32 + col);
        const uint32_t xw[2] = {xv.x, xv.y}, sw[2] = {sv.x, sv.y};
        q = sq(xw, sw, 2);
      } else {
        q = 0;
        for (int j = 0; j < 4 && cx0 + col + j < cw; ++j) {
          const int dd =
              (int)sm.rc[p][(r + 2) * kCS + kCC0 + col + j] - (int)sm.sc[p][r * 32 + col + j];
          q += (uint32_t)(dd * dd);
        }
      }
      if (fl & 2) e[1 + p] += q;
      a[1 + p] += q;
    }
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const uint64_t es = wave_sum64(e[p]);
    if (lane == 0) atomicAdd((unsigned long long *)&sm.skipsse[p], (unsigned long long)es);
    if (FULL) {
      const uint64_t as = wave_sum64(a[p]);
      if (lane == 0) atomicAdd((unsigned long long *)&sm.allsse[p], (unsigned long long)as);
    }
  }
}

// Tasks over list entries [first, first + count) of one plane shaped like
// luma (8x8 blocks, two per task, dealt round-robin to the four waves):
// plane 0 is luma, planes 1-2 are 4:4:4 chroma.  For each task,
// body(taps, A, B, hasB, packed source) consumes the pairs.
template <bool X, bool B12, int CH, bool SRC = true, class Body>
__device__ __forceinline__ void block_tasks(SmemCore<X> &sm, const JobDesc &J, int first, int count,
                                            int y0, int x0, int wave, int lane, Body &&body) {
  const int W = J.width, H = J.height;
  const uint16_t *rt = CH == 0 ? sm.ry : sm.rc[CH - 1];
  const uint16_t *st = CH == 0 ? sm.sy : sm.sc[CH - 1];
  const int ntask = (count + 1) >> 1;
  const int r = lane >> 3, col = lane & 7;
  // a sample's tile index is the lane's place in a block plus the block's
  // origin, which is wave-uniform: one add per block
  const int lr = (r + 2) * kLS + kLC0 + col, ls = r * 64 + col;
  for (int tk = wave; tk < ntask; tk += 4) {
    const int A = uniform(sm.list[first + 2 * tk]);
    const bool hasB = 2 * tk + 1 < count;
    const int B = hasB ? uniform(sm.list[first + 2 * tk + 1]) : A;
    const int dA = uniform(sm.dir[A]), dB = uniform(sm.dir[B]);
    const int rA = 8 * (A >> 3) + r, cA = 8 * (A & 7) + col;
    const int rB = 8 * (B >> 3) + r, cB = 8 * (B & 7) + col;
    const bool vA = y0 + rA < H && x0 + cA < W;
    const bool vB = hasB && y0 + rB < H && x0 + cB < W;
    // searches: lanes outside the frame see zeros and add nothing to a sum;
    // filter mode discards them (only in-frame pixels are copied out)
    const uint32_t vm = !SRC ? ~0u : (vA ? 0x0000FFFFu : 0u) | (vB ? 0xFFFF0000u : 0u);
    const int bA = lr + uniform(8 * (A >> 3) * kLS + 8 * (A & 7));
    const int bB = lr + uniform(8 * (B >> 3) * kLS + 8 * (B & 7));
    const uint32_t xv = ((uint32_t)rt[bA] | ((uint32_t)rt[bB] << 16)) & vm;
    // without a source (filter mode) y - s is y itself
    const uint32_t sv =
        SRC ? ((uint32_t)st[ls + uniform(512 * (A >> 3) + 8 * (A & 7))] |
               ((uint32_t)st[ls + uniform(512 * (B >> 3) + 8 * (B & 7))] << 16)) &
                  vm
            : 0u;
    uint32_t ta[12], tb[12], tp[12];
    tap_samples(dA, rt, bA, ta);
    tap_samples(dB, rt, bB, tb);
#pragma unroll
    for (int k = 0; k < 12; ++k) tp[k] = ta[k] | (tb[k] << 16);
    // the mask only where a lane is outside the frame or has no block B
    // (wave-uniform): most tasks skip it
    if (SRC && __builtin_amdgcn_read_exec() != __ballot(vA && vB)) {
#pragma unroll
      for (int k = 0; k < 12; ++k) tp[k] &= vm;
    }
    Taps t;
    prepare<B12>(t, xv, sv, tp);
    body(t, A, B, hasB, sv);
  }
}

// The pair generator of a luma-shaped task of plane CH (D3: see
// chroma_pairs; luma ignores it).
template <bool FULL, bool B12, int CH, bool SUB = false, bool D3 = false, bool QALL = false,
          bool X, class Sink>
__device__ __forceinline__ void block_pairs(SmemT<X> &sm, const JobDesc &J, const Taps &t, int A,
                                            int B, Sink &&sink) {
  const int c = J.bitdepth - 8, D = J.damping;
  const Subset sub(SUB ? J.cand : 0u);
  const bool sp19 = sub.has(1, 0);
  if (CH == 0) {
    const uint64_t adjA = uniform64(sm.adj[A]), adjB = uniform64(sm.adj[B]);
    const uint64_t lshA = uniform64(sm.lsh[A]), lshB = uniform64(sm.lsh[B]);
    const uint32_t parA = uniform(sm.lpar[A]), parB = uniform(sm.lpar[B]);
    const int a19A = FULL ? uniform(sm.adj19[A]) : 0, a19B = FULL ? uniform(sm.adj19[B]) : 0;
    luma_pairs<FULL, B12, SUB, QALL>(t, adjA, adjB, lshA, lshB, parA, parB, a19A, a19B, c, D,
                                     sub.pm, sub.qm, sp19, sink);
  } else {
    chroma_pairs<FULL, B12, SUB, D3, QALL>(t, c, D, sub.pm, sub.qm, sp19, sink);
  }
}

// SSE search over luma-shaped tasks; per-wave pair totals go to red[wave].
template <bool FULL, bool B12, bool SUB, int CH, bool X>
__device__ __forceinline__ void plane_tasks(SmemT<X> &sm, const JobDesc &J, int first, int count,
                                            int y0, int x0, int wave, int lane, uint64_t *red) {
  int acc[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) acc[i] = 0;
  auto run = [&](auto d3, auto qall) {
    block_tasks<X, B12, CH>(sm, J, first, count, y0, x0, wave, lane,
                            [&](const Taps &t, int A, int B, bool, uint32_t) {
                              block_pairs<FULL, B12, CH, SUB, decltype(d3)::value,
                                          decltype(qall)::value>(sm, J, t, A, B,
                                                                 SquareSum<X>{acc});
                            });
  };
  // a subset with every S^(s) takes loops without per-pair tests
  auto run_q = [&](auto d3) {
    if constexpr (SUB)
      with_flag(Subset(J.cand).qm == 15u, [&](auto qall) { run(d3, qall); });
    else
      run(d3, std::false_type{});
  };
  if constexpr (CH == 0)
    run_q(std::false_type{});
  else
    with_d3(J.damping, run_q);
  red[wave * 64 + lane] = reduce_transpose<B12>(acc, lane);
}

// 4:2:0 chroma tasks over list entries [first, first + count): eight 4x4
// blocks per task (four per half); waves 0-1 take Cb, waves 2-3 Cr.  For
// each task, body(taps, L, Hb, hasL, hasH, packed source) consumes the
// pairs.
template <bool X, bool B12, bool SRC = true, class Body>
__device__ __forceinline__ void chroma420_tasks(SmemCore<X> &sm, const JobDesc &J, int first,
                                                int count, int y0, int x0, int wave, int lane,
                                                Body &&body) {
  const int W = J.width, H = J.height;
  const int cw = (W + 1) >> 1, ch = (H + 1) >> 1, cy0 = y0 >> 1, cx0 = x0 >> 1;
  const int p = wave >> 1;
  const uint16_t *rt = sm.rc[p];
  const uint16_t *st = sm.sc[p];
  const int ntask = (count + 7) >> 3;
  const int sub = lane >> 4, r = (lane >> 2) & 3, col = lane & 3;
  for (int tk = wave & 1; tk < ntask; tk += 2) {
    const int iL = 8 * tk + sub, iH = 8 * tk + 4 + sub;
    const bool hasL = iL < count, hasH = iH < count;
    const int L = hasL ? sm.list[first + iL] : 0, Hb = hasH ? sm.list[first + iH] : 0;
    const int rL = 4 * (L >> 3) + r, cL = 4 * (L & 7) + col;
    const int rH = 4 * (Hb >> 3) + r, cH = 4 * (Hb & 7) + col;
    const bool vL = hasL && cy0 + rL < ch && cx0 + cL < cw;
    const bool vH = hasH && cy0 + rH < ch && cx0 + cH < cw;
    const uint32_t vm = !SRC ? ~0u : (vL ? 0x0000FFFFu : 0u) | (vH ? 0xFFFF0000u : 0u);
    const int bL = (rL + 2) * kCS + kCC0 + cL, bH = (rH + 2) * kCS + kCC0 + cH;
    const int dL = sm.dir[L], dH = sm.dir[Hb];
    const uint32_t xv = ((uint32_t)rt[bL] | ((uint32_t)rt[bH] << 16)) & vm;
    const uint32_t sv =
        SRC ? ((uint32_t)st[rL * 32 + cL] | ((uint32_t)st[rH * 32 + cH] << 16)) & vm : 0u;
    // the directions differ between lanes, so the tap addresses are formed
    // per lane: a byte offset from the table added to or subtracted from the
    // sample's byte address (one add per tap, the offset's sign extension
    // folded into it)
    const char *pL = reinterpret_cast<const char *>(rt + bL);
    const char *pH = reinterpret_cast<const char *>(rt + bH);
    auto at = [](const char *q) { return (uint32_t)*reinterpret_cast<const uint16_t *>(q); };
    uint32_t tp[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int oL = sm.coff[dL][k], oH = sm.coff[dH][k];
      const int slot = (k >> 1) * 4 + (k & 1) * 2;
      tp[slot] = at(pL + oL) | (at(pH + oH) << 16);
      tp[slot + 1] = at(pL - oL) | (at(pH - oH) << 16);
    }
    // as for luma tasks: the mask only where a lane is outside the frame or
    // past the list's end (wave-uniform)
    if (SRC && __builtin_amdgcn_read_exec() != __ballot(vL && vH)) {
#pragma unroll
      for (int k = 0; k < 12; ++k) tp[k] &= vm;
    }
    Taps t;
    prepare<B12>(t, xv, sv, tp);
    body(t, L, Hb, hasL, hasH, sv);
  }
}

// The same tasks with a lane's two samples side by side in one block row:
// lane (b, r, j) = (lane >> 3, (lane >> 1) & 3, lane & 1) holds columns 2j
// and 2j + 1 of row r of list entry first + 8 tk + b.  Both samples share
// the block's direction and their taps sit side by side too, so each tap of
// the pair is one 32-bit LDS read (at 2-byte alignment for odd offsets) and
// no halves are merged.  The searches, with 64 pairs of arithmetic per
// read, gain from it; the filter mode, with little arithmetic per read,
// measured 7 % slower with the unaligned reads and keeps the layout above.
// For each task, body(taps, block, has block, packed source) consumes the
// pairs.
template <bool X, bool B12, bool SRC = true, class Body>
__device__ __forceinline__ void chroma420_row_tasks(SmemCore<X> &sm, const JobDesc &J, int first,
                                                    int count, int y0, int x0, int wave,
                                                    int lane, Body &&body) {
  const int W = J.width, H = J.height;
  const int cw = (W + 1) >> 1, ch = (H + 1) >> 1, cy0 = y0 >> 1, cx0 = x0 >> 1;
  const int p = wave >> 1;
  const uint16_t *rt = sm.rc[p];
  const uint16_t *st = sm.sc[p];
  const int ntask = (count + 7) >> 3;
  const int sub = lane >> 3, r = (lane >> 1) & 3, col = 2 * (lane & 1);
  auto pair_at = [](const char *q) {
    uint32_t v;
    __builtin_memcpy(&v, __builtin_assume_aligned(q, 2), 4);
    return v;
  };
  for (int tk = wave & 1; tk < ntask; tk += 2) {
    const int i = 8 * tk + sub;
    const bool has = i < count;
    const int L = has ? sm.list[first + i] : 0;
    const int rL = 4 * (L >> 3) + r, cL = 4 * (L & 7) + col;
    const bool rin = has && cy0 + rL < ch;
    const bool v0 = rin && cx0 + cL < cw, v1 = rin && cx0 + cL + 1 < cw;
    const uint32_t vm = !SRC ? ~0u : (v0 ? 0x0000FFFFu : 0u) | (v1 ? 0xFFFF0000u : 0u);
    // an even sample index: the pair is one aligned word
    const int b = (rL + 2) * kCS + kCC0 + cL;
    const int d = sm.dir[L];
    const uint32_t xv = *reinterpret_cast<const uint32_t *>(rt + b) & vm;
    const uint32_t sv = SRC ? *reinterpret_cast<const uint32_t *>(st + rL * 32 + cL) & vm : 0u;
    const char *pb = reinterpret_cast<const char *>(rt + b);
    uint32_t tp[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int o = sm.coff[d][k];
      const int slot = (k >> 1) * 4 + (k & 1) * 2;
      tp[slot] = pair_at(pb + o);
      tp[slot + 1] = pair_at(pb - o);
    }
    if (SRC && __builtin_amdgcn_read_exec() != __ballot(v0 && v1)) {
#pragma unroll
      for (int k = 0; k < 12; ++k) tp[k] &= vm;
    }
    Taps t;
    prepare<B12>(t, xv, sv, tp);
    body(t, L, has, sv);
  }
}

// SSE search over 4:2:0 chroma tasks; plane 1 + p's totals go to
// red[1 + p][wave & 1].
template <bool FULL, bool B12, bool SUB, bool X>
__device__ __forceinline__ void chroma420_sse(SmemT<X> &sm, const JobDesc &J, int first, int count,
                                              int y0, int x0, int wave, int lane,
                                              uint64_t (*red)[4][64]) {
  const int c = J.bitdepth - 8, D = J.damping;
  const Subset sub(SUB ? J.cand : 0u);
  const bool sp19 = sub.has(1, 0);
  int acc[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) acc[i] = 0;
  auto run = [&](auto d3, auto qall) {
    chroma420_row_tasks<X, B12>(sm, J, first, count, y0, x0, wave, lane,
                                [&](const Taps &t, int, bool, uint32_t) {
                                  chroma_pairs<FULL, B12, SUB, decltype(d3)::value,
                                               decltype(qall)::value>(
                                      t, c, D, sub.pm, sub.qm, sp19, SquareSum<X>{acc});
                                });
  };
  with_d3(D, [&](auto d3) {
    if constexpr (SUB)
      with_flag(sub.qm == 15u, [&](auto qall) { run(d3, qall); });
    else
      run(d3, std::false_type{});
  });
  red[1 + (wave >> 1)][wave & 1][lane] = reduce_transpose<B12>(acc, lane);
}

// Waves whose per-wave sums make up plane P's totals.
__device__ __forceinline__ int plane_waves(const JobDesc &J, int P) {
  return P == 0 || J.layout == kLayout444 ? 4 : 2;
}

template <bool FULL, bool B12, bool SUB, bool X>
__device__ __forceinline__ void search_item(SmemT<X> &sm, const JobDesc &J, int fby, int fbx,
                                            int tid) {
  const int lane = tid & 63, wave = uniform(tid >> 6);  // scalar task loops
  const int y0 = fby * 64, x0 = fbx * 64;
  const bool c420 = J.nplanes == 3 && J.layout == kLayout420;
  const bool c444 = X && J.nplanes == 3 && J.layout == kLayout444;

  // Staging and the direction search run at raised wave priority: the
  // other workgroups on the CU are in their task loops, and issuing this
  // one's loads and wave-0 work first brings its four waves to the task
  // loops sooner (measured: +5 % on 8 x 4K frames).
  __builtin_amdgcn_s_setprio(2);
  stage_item<X>(sm, J, fby, fbx, tid, true);
  if (tid < 3) {
    sm.skipsse[tid] = 0;
    sm.allsse[tid] = 0;
  }
  __syncthreads();
  if (wave == 0)
    direction_search<FULL>(sm, J, fby, fbx, lane);
  else
    skipped_sse<FULL>(sm, J, fby, fbx, tid - 64, 192, lane);
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);
  const int n = sm.n;

  const Subset sub(SUB ? J.cand : 0u);
  plane_tasks<FULL, B12, SUB, 0>(sm, J, 0, n, y0, x0, wave, lane, &sm.red[0][0][0]);
  if (c420) chroma420_sse<FULL, B12, SUB>(sm, J, 0, n, y0, x0, wave, lane, sm.red);
  if constexpr (X) {
    if (c444) {
      plane_tasks<FULL, B12, SUB, 1>(sm, J, 0, n, y0, x0, wave, lane, &sm.red[1][0][0]);
      plane_tasks<FULL, B12, SUB, 2>(sm, J, 0, n, y0, x0, wave, lane, &sm.red[2][0][0]);
    }
  }
  // skipped blocks matter only where some block has residual, and only for
  // the presets with the skip condition bit
  if (FULL && n > 0 && (!SUB || (sub.km & 2))) {
    const int nsk = sm.nsk;
    plane_tasks<FULL, B12, SUB, 0>(sm, J, n, nsk, y0, x0, wave, lane, &sm.red2[0][0][0]);
    if (c420) chroma420_sse<FULL, B12, SUB>(sm, J, n, nsk, y0, x0, wave, lane, sm.red2);
    if constexpr (X) {
      if (c444) {
        plane_tasks<FULL, B12, SUB, 1>(sm, J, n, nsk, y0, x0, wave, lane, &sm.red2[1][0][0]);
        plane_tasks<FULL, B12, SUB, 2>(sm, J, n, nsk, y0, x0, wave, lane, &sm.red2[2][0][0]);
      }
    }
  }
  __syncthreads();

  const int P = tid >> 6, k = lane;
  if (P >= search_planes(J)) return;
  const int nw = plane_waves(J, P);
  uint64_t A = 0, Bf = 0;
  for (int w = 0; w < nw; ++w) {
    A += sm.red[P][w][k];
    if (FULL) Bf += sm.red2[P][w][k];
  }
  const int64_t fbi = (int64_t)fby * J.fbc + fbx;
  const int64_t nfb = (int64_t)J.fbr * J.fbc;
  const uint64_t U = sm.skipsse[P];
  // presets outside a subset read 2^64 - 1 (12-bit jobs evaluate them all
  // and mark them here)
  const Subset out(J.cand);
  if (!FULL) {
    J.sse[(P * nfb + fbi) * 64 + k] = out.has(0, k) ? A + U : UINT64_MAX;
  } else {
    // slot 0 holds the special preset; (0, 0) itself is the unfiltered sum
    uint64_t *o = J.sse + (P * nfb + fbi) * 128;
    o[k] = out.has(0, k) ? (k == 0 ? sm.allsse[P] : A + U) : UINT64_MAX;
    // every block skipped: nothing is filtered
    o[64 + k] = out.has(1, k) ? (n > 0 ? A + Bf : U) : UINT64_MAX;
  }
}

// ---- Weighted search (Eq. 14) ---------------------------------------------

// Eq. (14) for one filtering unit from exact integer moments: n pixels,
// sums of s, s^2, d, d^2 and the unit's SSE.  With V = n sum x^2 - (sum x)^2
// = n^2 sigma^2, the weight is (Vs + Vd + C1 n^2) / (2 sqrt(Vs Vd + C2 n^4)).
// The unit's part (n, Vs and the constants times powers of n) is formed
// once per unit; per pair, Vd is exact in double (its terms are integers
// below 2^53) and 1 / sqrt comes from the hardware estimate refined by two
// Newton steps (relative error a few units in the last place).
struct Eq14Unit {
  double n, vs, a, b;  // a = (Vs + C1 n^2) / 2, b = C2 n^4
};

__device__ __forceinline__ Eq14Unit eq14_unit(int n, uint32_t ss, uint32_t ss2, double C1,
                                              double C2) {
  const double nn = (double)n * (double)n;
  const double vs = (double)((int64_t)n * ss2 - (int64_t)ss * ss);
  return {(double)n, vs, 0.5 * (vs + C1 * nn), C2 * nn * nn};
}

__device__ __forceinline__ double eq14(const Eq14Unit &u, uint32_t sd, uint32_t sd2,
                                       uint32_t sse) {
  const double dd = (double)sd;
  const double vd = fma(u.n, (double)sd2, -(dd * dd));
  const double x = fma(u.vs, vd, u.b);
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return fma(0.5, vd, u.a) * y * (double)sse;
}

__device__ __forceinline__ double eq14(int n, uint32_t ss, uint32_t ss2, uint32_t sd, uint32_t sd2,
                                       uint32_t sse, double C1, double C2) {
  return eq14(eq14_unit(n, ss, ss2, C1, C2), sd, sd2, sse);
}

// Per-unit moments of the source and the unfiltered reconstruction, one
// unit row (8 or 4 pixels) per step; run by threads t0.. (nt of them) while
// wave 0 runs the direction search.  Unit rows are dealt so that
// neighbouring threads add into different units.
template <bool X>
__device__ __forceinline__ void unit_stats(SmemT<X> &sm, const JobDesc &J, int fby, int fbx, int t,
                                           int nt) {
  const int W = J.width, H = J.height, y0 = fby * 64, x0 = fbx * 64;
  const int cw = (W + 1) >> 1, ch = (H + 1) >> 1, cy0 = y0 >> 1, cx0 = x0 >> 1;
  const int planes = search_planes(J);
  const bool c444 = X && J.layout == kLayout444;
  // unit rows: 512 luma, then per chroma plane 256 (4x4 units) or 512 (8x8)
  const int crows = c444 ? 512 : 256;
  const int nrows = 512 + (planes - 1) * crows;
  for (int k = t; k < nrows; k += nt) {
    int P, u, row;
    if (k < 512) {
      P = 0;
      u = k & 63;
      row = k >> 6;
    } else {
      const int kk = k - 512;
      P = 1 + kk / crows;
      u = kk & 63;
      row = (kk % crows) >> 6;
    }
    uint32_t cnt = 0, a = 0, a2 = 0, b = 0, b2 = 0, ab = 0;
    if (P == 0 || c444) {
      const uint16_t *rt = P == 0 ? sm.ry : sm.rc[P - 1];
      const uint16_t *st = P == 0 ? sm.sy : sm.sc[P - 1];
      const int r = 8 * (u >> 3) + row, c0 = 8 * (u & 7);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (y0 + r < H && x0 + c0 + j < W) {
          const uint32_t sv = st[r * 64 + c0 + j], xv = rt[(r + 2) * kLS + kLC0 + c0 + j];
          ++cnt;
          a += sv;
          a2 += sv * sv;
          b += xv;
          b2 += xv * xv;
          ab += xv * sv;
        }
      }
    } else {
      const int r = 4 * (u >> 3) + row, c0 = 4 * (u & 7);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (cy0 + r < ch && cx0 + c0 + j < cw) {
          const uint32_t sv = sm.sc[P - 1][r * 32 + c0 + j];
          const uint32_t xv = sm.rc[P - 1][(r + 2) * kCS + kCC0 + c0 + j];
          ++cnt;
          a += sv;
          a2 += sv * sv;
          b += xv;
          b2 += xv * xv;
          ab += xv * sv;
        }
      }
    }
    if (cnt) {
      atomicAdd(&sm.w.ustat[0][P][u], cnt);
      atomicAdd(&sm.w.ustat[1][P][u], a);
      atomicAdd(&sm.w.ustat[2][P][u], a2);
      atomicAdd(&sm.w.ustat[3][P][u], b);
      atomicAdd(&sm.w.ustat[4][P][u], b2);
      atomicAdd(&sm.w.ustat[5][P][u], ab);
    }
  }
}

// ---- Weighted-search moments through LDS ----------------------------------
// A task's e = y - s for its 64 pairs is transposed through a per-wave LDS
// scratch, 8 pairs at a time, so that a lane holds samples of one pair and
// one filtering unit: sum d, sum d^2 and sum e^2 then accumulate inside the
// lane, two samples of the same unit per 32-bit word (v_dot2 squares and adds
// both halves), instead of one transposing cross-lane reduction per moment and
// unit.  Scratch layout, per wave: a row per pair of 8 blocks of 16 samples
// (16-bit) and 8 entries of padding, then a row of the source samples.  A
// task's lane k writes its low-half sample at entry k and its high-half
// sample at 64 + k of each row: a luma task's unit A (blocks 0-3, a quarter
// of the unit each) then unit B (blocks 4-7); a 4:2:0 chroma task's units 0-3
// (low halves of lane rows 0-3) then 4-7 (high halves).  The pairs are
// written as the pair generator produces them, 8 at a time, so no lane holds
// more than 8 errors, and the scratch fits beside the base layout at three
// workgroups per CU.  4:4:4 chroma planes are shaped like luma.

template <bool X>
__device__ __forceinline__ uint16_t *moment_scratch(SmemT<X> &sm, int wave) {
  return wave < 2 ? reinterpret_cast<uint16_t *>(&sm.red[0][0][0]) + wave * kWbEntries
                  : sm.wb + (wave - 2) * kWbEntries;
}
static_assert(2 * kWbEntries * 2 <= (int)sizeof(uint64_t) * 3 * 4 * 64, "scratch in red");
static_assert((kWbEntries * 2) % 16 == 0 && (kWbRow * 2) % 16 == 0, "16-byte aligned rows");
static_assert(offsetof(SmemT<false>, red) % 16 == 0 && offsetof(SmemT<false>, wb) % 16 == 0 &&
                  offsetof(SmemT<true>, red) % 16 == 0 && offsetof(SmemT<true>, wb) % 16 == 0,
              "16-byte aligned scratch");

// Entries another lane of the wave wrote before this point are read after
// it: the LDS serves one wave's accesses in order, and the fences keep the
// compiler from moving them across.
__device__ __forceinline__ void wave_lds_exchange() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  asm volatile("" ::: "memory");
}

// The 8 words of a 16-sample block of the scratch.
__device__ __forceinline__ void wb_read8(const uint16_t *ws, int at, uint32_t (&v)[8]) {
  const uint4 *p = reinterpret_cast<const uint4 *>(ws + at);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const uint4 x = p[i];
    v[4 * i] = x.x;
    v[4 * i + 1] = x.y;
    v[4 * i + 2] = x.z;
    v[4 * i + 3] = x.w;
  }
}

// sum d, sum d^2, sum e^2 over the 16 samples of 8 words (d = e + s).
__device__ __forceinline__ void block_moments(const uint32_t (&E)[8], const uint32_t (&S)[8],
                                              uint32_t (&m)[3]) {
  u16x2 s = {0, 0};
  uint32_t a = 0;
  int b = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const u16x2 d = as_u(E[k]) + as_u(S[k]);  // in [0, 2^b)
    s += d;
    a = __builtin_amdgcn_udot2(d, d, a, false);
    b = __builtin_amdgcn_sdot2(as_s(E[k]), as_s(E[k]), b, false);
  }
  m[0] = (uint32_t)s.x + (uint32_t)s.y;
  m[1] = a;
  m[2] = (uint32_t)b;
}

// Pair sink of the base-layout weighted search: keeps the errors of the
// current chunk of 8 pairs; after a chunk's last pair it writes them to the
// wave's scratch and the reading lane takes the moments of its block
// (m[chunk]).  k is a compile-time constant at every call (the pair loops
// are unrolled), so the chunk logic folds away.
template <bool X>
struct ChunkMoments {
  static constexpr bool kRows = X;
  uint16_t *ws;
  int lane, rd, rq;         // this lane's entry in a row; the block and the row it reads
  const uint32_t (&S)[8];   // the source words of the lane's block
  uint32_t (&m)[8][3];
  s16x2 ev[kWbPairs];
  __device__ __forceinline__ void operator()(int k, s16x2 e) {
    ev[k & 7] = e;
    if ((k & 7) != 7) return;
#pragma unroll
    for (int i = 0; i < kWbPairs; ++i) {
      const uint32_t v = __builtin_bit_cast(uint32_t, ev[i]);
      ws[kWbRow * i + lane] = (uint16_t)v;
      ws[kWbRow * i + 64 + lane] = (uint16_t)(v >> 16);
    }
    wave_lds_exchange();
    uint32_t E[8];
    wb_read8(ws, rq + rd, E);
    block_moments(E, S, m[k >> 3]);
    wave_lds_exchange();  // read before the next chunk overwrites
  }
};

// The source row of a task, and each lane's source words.
__device__ __forceinline__ void wb_source(uint16_t *ws, int lane, int rd, uint32_t sv,
                                          uint32_t (&S)[8]) {
  ws[kWbPairs * kWbRow + lane] = (uint16_t)sv;
  ws[kWbPairs * kWbRow + 64 + lane] = (uint16_t)(sv >> 16);
  wave_lds_exchange();
  wb_read8(ws, kWbPairs * kWbRow + rd, S);
}

// One reduce-scatter level over the lanes of a quad: of the chunk sets
// [c] and [c ^ BIT], each lane keeps the one whose bit matches its own
// (`up`) and adds the partner lane's copy (DPP quad_perm CTRL).
template <int BIT, int CTRL>
__device__ __forceinline__ void quad_level(uint32_t (&m)[8][3], bool up) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (c & BIT) continue;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const uint32_t lo = m[c][j], hi = m[c | BIT][j];
      const uint32_t keep = up ? hi : lo, send = up ? lo : hi;
      m[c][j] = keep + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)send, CTRL, 0xF, 0xF, false);
    }
  }
}

// Luma-shaped tasks of plane CH (luma, 4:4:4 chroma).  Lane (q, h, r) =
// (lane >> 3, (lane >> 2) & 1, lane & 3) reads quarter r of unit h of pair
// 8 c + q in chunk c; after the task the quad's four lanes reduce-scatter
// their eight chunks' partial moments so that lane r holds chunks r and
// r + 4 whole: pairs 8 r + q and 32 + 8 r + q of unit h.
template <bool X, bool B12, int CH>
__device__ __forceinline__ void plane_tasks_wb(SmemT<X> &sm, const JobDesc &J, int n, int y0,
                                               int x0, int wave, int lane, double C1,
                                               double C2) {
  uint16_t *ws = moment_scratch(sm, wave);
  const int q = lane >> 3, h = (lane >> 2) & 1, r = lane & 3;
  const int rd = 16 * (lane & 7), rq = kWbRow * q;  // block 4 h + r of pair row q
  double acc[2] = {0.0, 0.0};
  auto run = [&](auto d3) {
    block_tasks<X, B12, CH>(
        sm, J, 0, n, y0, x0, wave, lane,
        [&](const Taps &t, int A, int B, bool hasB, uint32_t sv) {
          uint32_t S[8], m[8][3];
          wb_source(ws, lane, rd, sv, S);
          ChunkMoments<X> sink{ws, lane, rd, rq, S, m, {}};
          block_pairs<false, B12, CH, false, decltype(d3)::value>(sm, J, t, A, B, sink);
          quad_level<2, 0x4E>(m, (r & 2) != 0);  // quad_perm [2, 3, 0, 1]: lane ^ 2
          quad_level<1, 0xB1>(m, (r & 1) != 0);  // quad_perm [1, 0, 3, 2]: lane ^ 1
          if (h == 0 || hasB) {
            const int u = h ? B : A;
            const Eq14Unit e = eq14_unit((int)sm.w.ustat[0][CH][u], sm.w.ustat[1][CH][u],
                                         sm.w.ustat[2][CH][u], C1, C2);
            acc[0] += eq14(e, m[0][0], m[0][1], m[0][2]);  // chunk r
            acc[1] += eq14(e, m[4][0], m[4][1], m[4][2]);  // chunk r + 4
          }
        });
  };
  if constexpr (CH == 0)
    run(std::false_type{});
  else
    with_d3(J.damping, run);
  // units A and B (h = 0, 1) hold the same pairs
#pragma unroll
  for (int j = 0; j < 2; ++j) acc[j] += __shfl_xor(acc[j], 4, 64);
  if (h == 0) {
    sm.w.wred[CH][wave][8 * r + q] = acc[0];
    sm.w.wred[CH][wave][32 + 8 * r + q] = acc[1];
  }
}

// 4:2:0 chroma tasks: lane (q, u) = (lane >> 3, lane & 7) reads unit u of
// pair 8 c + q whole (16 samples), so it completes the moments alone and
// adds the unit's Eq. (14) term to pair 8 c + q; the eight lanes u of a pair
// are summed at the end.
template <bool X, bool B12>
__device__ __forceinline__ void chroma420_wb(SmemT<X> &sm, const JobDesc &J, int n, int y0,
                                             int x0, int wave, int lane, double C1, double C2) {
  const int c = J.bitdepth - 8, D = J.damping;
  const int P = 1 + (wave >> 1);
  uint16_t *ws = moment_scratch(sm, wave);
  const int q = lane >> 3, u = lane & 7;
  const int rd = 16 * u, rq = kWbRow * q;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  with_d3(D, [&](auto d3) {
    chroma420_tasks<X, B12>(
        sm, J, 0, n, y0, x0, wave, lane,
        [&](const Taps &t, int L, int Hb, bool hasL, bool hasH, uint32_t sv) {
          // unit u: the low half (u < 4) or the high half of lane row u & 3
          const int src = (u & 3) << 4;
          const int uL = __shfl(L, src, 64), uH = __shfl(Hb, src, 64);
          const int has = __shfl((hasL ? 1 : 0) | (hasH ? 2 : 0), src, 64);
          const bool mine = (has >> (u >> 2)) & 1;
          const int unit = u < 4 ? uL : uH;
          const Eq14Unit e = eq14_unit((int)sm.w.ustat[0][P][unit], sm.w.ustat[1][P][unit],
                                       sm.w.ustat[2][P][unit], C1, C2);
          uint32_t S[8], m[8][3];
          wb_source(ws, lane, rd, sv, S);
          ChunkMoments<X> sink{ws, lane, rd, rq, S, m, {}};
          chroma_pairs<false, B12, false, decltype(d3)::value>(t, c, D, 0xFFFFu, 15u, false,
                                                               sink);
          if (mine) {
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += eq14(e, m[k][0], m[k][1], m[k][2]);
          }
        });
  });
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    acc[k] += __shfl_xor(acc[k], 1, 64);
    acc[k] += __shfl_xor(acc[k], 2, 64);
    acc[k] += __shfl_xor(acc[k], 4, 64);
  }
  if (u == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) sm.w.wred[P][wave & 1][8 * k + q] = acc[k];
  }
}

template <bool X, bool B12>
__device__ __forceinline__ void search_item_weighted(SmemT<X> &sm, const JobDesc &J, int fby,
                                                     int fbx, int tid) {
  const int lane = tid & 63, wave = uniform(tid >> 6);  // scalar task loops
  const int y0 = fby * 64, x0 = fbx * 64;
  const bool c420 = J.nplanes == 3 && J.layout == kLayout420;
  const bool c444 = J.nplanes == 3 && J.layout == kLayout444;
  const int c = J.bitdepth - 8;
  // C1 = 6.25 and C2 = 312.5 at 8 bits, scaled like variances and their
  // products (exact powers of two)
  const double C1 = 6.25 * (double)(1 << (2 * c)), C2 = 312.5 * (double)(1 << (4 * c));

  __builtin_amdgcn_s_setprio(2);  // as in the SSE search
  stage_item<X>(sm, J, fby, fbx, tid, true);
  for (int i = tid; i < 6 * 3 * 64; i += 256) (&sm.w.ustat[0][0][0])[i] = 0;
  __syncthreads();
  if (wave == 0)
    direction_search<false>(sm, J, fby, fbx, lane);
  else
    unit_stats(sm, J, fby, fbx, tid - 64, 192);
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);
  const int n = sm.n;
  const int planes = search_planes(J);

  // skipped units are not filtered under any pair: wave P sums plane P's
  if (wave < 3) {
    const int P = wave, u = lane;
    double w = 0.0;
    if (P < planes && (sm.flag[u] & 2)) {
      const uint32_t cnt = sm.w.ustat[0][P][u];
      const uint32_t ss = sm.w.ustat[1][P][u], ss2 = sm.w.ustat[2][P][u];
      const uint32_t sx = sm.w.ustat[3][P][u], sx2 = sm.w.ustat[4][P][u];
      const uint32_t sxs = sm.w.ustat[5][P][u];
      if (cnt) w = eq14((int)cnt, ss, ss2, sx, sx2, sx2 + ss2 - 2 * sxs, C1, C2);
    }
    w = wave_sum_f64(w);
    if (lane == 0) sm.skipw[P] = w;
  }

  // the same code on both layouts, so that a job's table does not depend on
  // the kernel its batch runs on
  plane_tasks_wb<X, B12, 0>(sm, J, n, y0, x0, wave, lane, C1, C2);
  if (c420) chroma420_wb<X, B12>(sm, J, n, y0, x0, wave, lane, C1, C2);
  if constexpr (X) {
    if (c444) {
      plane_tasks_wb<X, B12, 1>(sm, J, n, y0, x0, wave, lane, C1, C2);
      plane_tasks_wb<X, B12, 2>(sm, J, n, y0, x0, wave, lane, C1, C2);
    }
  }
  __syncthreads();

  const int P = tid >> 6, k = lane;
  if (P >= planes) return;
  const int nw = plane_waves(J, P);
  double total = sm.skipw[P];
  for (int w = 0; w < nw; ++w) total += sm.w.wred[P][w][k];
  const int64_t fbi = (int64_t)fby * J.fbc + fbx;
  const int64_t nfb = (int64_t)J.fbr * J.fbc;
  reinterpret_cast<double *>(J.sse)[(P * nfb + fbi) * 64 + k] = total;
}

// Filter mode: the block's own preset (Section 3.2 ranges, Section 4 skip
// rules; bad values are masked / clamped so the kernel stays defined).  The
// filtered blocks (with residual, and under the skip condition bit the
// skipped ones too; none when every in-frame block is skipped) go through
// the searches' task loops, two samples per lane, with the source taken as 0
// so that a pair's "y - s" is y; results land in the idle source tiles, and
// every in-frame pixel is then copied out, filtered or not.  4:2:2 chroma is
// copied.
// PACKED: the packed direction search (the filter-only kernels, whose
// occupancy it sets); the search kernels' filter mode keeps the 32-bit one.
template <bool X, bool B12, bool PACKED>
__device__ __forceinline__ void filter_item(SmemCore<X> &sm, const JobDesc &J, int fby, int fbx,
                                            int tid) {
  const int wave = uniform(tid >> 6), lane = tid & 63;  // scalar task loops
  const int W = J.width, H = J.height, y0 = fby * 64, x0 = fbx * 64;
  const int c = J.bitdepth - 8, D = J.damping;
  __builtin_amdgcn_s_setprio(2);  // as in the searches
  const uint8_t *st = J.strengths + 4 * ((int64_t)fby * J.fbc + fbx);
  // the filter block's four strength bytes are wave-uniform: read once and
  // decoded in scalar registers, so that every per-task quantity derived
  // from them (dampings, shifts, weights, the tap groups in use) stays
  // scalar too
  const uint32_t sw = (uint32_t)uniform(
      (int)((uint32_t)st[0] | ((uint32_t)st[1] << 8) | ((uint32_t)st[2] << 16) |
            ((uint32_t)st[3] << 24)));
  const Preset py = decode_preset(sw & 255, (sw >> 8) & 255);
  const Preset pc = decode_preset((sw >> 16) & 255, sw >> 24);
  stage_item<X>(sm, J, fby, fbx, tid, false);
  __syncthreads();
  if (wave == 0) direction_search<true, X, PACKED, true>(sm, J, fby, fbx, lane, py);
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);
  const int n = sm.n, nsk = sm.nsk;
  const int ny = n == 0 ? 0 : n + (py.skipcond ? nsk : 0);
  const int nc = n == 0 ? 0 : n + (pc.skipcond ? nsk : 0);
  const bool c420 = J.nplanes == 3 && J.layout == kLayout420;
  const bool c444 = X && J.nplanes == 3 && J.layout == kLayout444;
  const int ly = (lane >> 3) * 64 + (lane & 7);  // a lane's place in a block of a 64-wide tile

  // luma: per-block adjusted primary strength (Eq. 13), its parity weights
  // and damping (raised for 16..19), per 16-bit half.  A tap group at
  // strength 0 adds nothing (f = 0), and with one group the clamp cannot
  // bind (its weights sum to 12/16 < 1), so the groups in use are decided
  // per filter block (a task-loop instantiation each).  A block whose
  // adjusted primary strength is 0 under a preset with S^(p) > 0 still runs
  // the primary group, at strength 0: it adds 0, and the clamp it brings
  // cannot bind either.
  with_flag(py.pri != 0, [&](auto pri_used) {
    with_flag(py.sec != 0, [&](auto sec_used) {
      constexpr bool prim = decltype(pri_used)::value, secd = decltype(sec_used)::value;
      block_tasks<X, B12, 0, false>(
          sm, J, 0, ny, y0, x0, wave, lane,
          [&](const Taps &t, int A, int B, bool hasB, uint32_t) {
            // per-block words from the direction search, halves paired
            const uint32_t fA0 = (uint32_t)uniform((int)sm.fpar[A][0]);
            const uint32_t fB0 = (uint32_t)uniform((int)sm.fpar[B][0]);
            const uint32_t fA1 = (uint32_t)uniform((int)sm.fpar[A][1]);
            const uint32_t fB1 = (uint32_t)uniform((int)sm.fpar[B][1]);
            const uint32_t sp = (fA0 & 0xFFFFu) | (fB0 << 16);
            const uint32_t sh = (fA0 >> 16) | (fB0 & 0xFFFF0000u);
            const uint32_t odd = (fA1 & 0xFFFFu) | (fB1 << 16);
            // weights 4, 2 at even strengths, 3, 3 at odd ones
            const uint32_t w1 = 0x00040004u - odd, w2 = 0x00020002u + odd;
            s16x2 P = splat(0), Q = splat(0);
            if constexpr (prim) {
              u16x2 a[4];
#pragma unroll
              for (int k = 0; k < 4; ++k) a[k] = t.ad[k] >> as_u(sh);
              P = group_sum(t, a, 0, sp, w1, w2);
            }
            if constexpr (secd) {
              const uint32_t qsh = (fA1 >> 16) | (fB1 & 0xFFFF0000u);
              Q = secondary(t, splat32((uint32_t)py.sec << c), qsh);
            }
            const uint32_t y = __builtin_bit_cast(
                uint32_t, prim && secd ? err_both<B12>(t, P, Q)
                                       : prim || secd ? err_one<B12>(t, prim ? P : Q) : t.dxs);
            sm.sy[ly + uniform(512 * (A >> 3) + 8 * (A & 7))] = (uint16_t)y;
            if (hasB) sm.sy[ly + uniform(512 * (B >> 3) + 8 * (B & 7))] = (uint16_t)(y >> 16);
          });
    });
  });

  // chroma: one preset for both planes; damping max(D - 1, floor(log2 S^(p)))
  const int Dc = pc.pri ? max(D - 1, floor_log2(pc.pri)) : D - 1;
  const uint32_t csp = splat32((uint32_t)pc.pri << c);
  const uint32_t csh = splat32((uint32_t)(pc.pri ? Dc - floor_log2(pc.pri) : 0));
  const uint32_t cw1 = splat32((pc.pri & 1) ? 3u : 4u), cw2 = splat32((pc.pri & 1) ? 3u : 2u);
  const uint32_t css = splat32((uint32_t)pc.sec << c);
  const uint32_t cqsh = splat32((uint32_t)(pc.sec ? Dc - floor_log2(pc.sec) : 0));
  // as for luma, but both groups' use is the filter block's: one loop
  // instantiation per combination
  auto chroma_y = [&](const Taps &t, auto pri_used, auto sec_used) {
    constexpr bool prim = decltype(pri_used)::value, secd = decltype(sec_used)::value;
    s16x2 P = splat(0), Q = splat(0);
    if constexpr (prim) {
      u16x2 a[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) a[k] = t.ad[k] >> as_u(csh);
      P = group_sum(t, a, 0, csp, cw1, cw2);
    }
    if constexpr (secd) Q = secondary(t, css, cqsh);
    return __builtin_bit_cast(uint32_t, prim && secd ? err_both<B12>(t, P, Q)
                                        : prim || secd ? err_one<B12>(t, prim ? P : Q)
                                                       : t.dxs);
  };
  with_flag(pc.pri != 0, [&](auto pri_used) {
    with_flag(pc.sec != 0, [&](auto sec_used) {
      if (c420) {
        const int p = wave >> 1, r4 = (lane >> 2) & 3, col4 = lane & 3;
        chroma420_tasks<X, B12, false>(
            sm, J, 0, nc, y0, x0, wave, lane,
            [&](const Taps &t, int L, int Hb, bool hasL, bool hasH, uint32_t) {
              const uint32_t y = chroma_y(t, pri_used, sec_used);
              if (hasL) sm.sc[p][(4 * (L >> 3) + r4) * 32 + 4 * (L & 7) + col4] = (uint16_t)y;
              if (hasH)
                sm.sc[p][(4 * (Hb >> 3) + r4) * 32 + 4 * (Hb & 7) + col4] = (uint16_t)(y >> 16);
            });
      }
      if constexpr (X) {
        if (c444) {
          auto plane444 = [&](auto ch) {
            constexpr int CH = decltype(ch)::value;
            block_tasks<X, B12, CH, false>(
                sm, J, 0, nc, y0, x0, wave, lane,
                [&](const Taps &t, int A, int B, bool hasB, uint32_t) {
                  const uint32_t y = chroma_y(t, pri_used, sec_used);
                  sm.sc[CH - 1][ly + uniform(512 * (A >> 3) + 8 * (A & 7))] = (uint16_t)y;
                  if (hasB)
                    sm.sc[CH - 1][ly + uniform(512 * (B >> 3) + 8 * (B & 7))] =
                        (uint16_t)(y >> 16);
                });
          };
          plane444(std::integral_constant<int, 1>{});
          plane444(std::integral_constant<int, 2>{});
        }
      }
    });
  });
  __syncthreads();

  // copy-out: filtered pixels from the result tiles, the rest unchanged.
  // Aligned outputs move a block row at a time (16 bytes; 8 for 4:2:0
  // chroma): every sample of it shares the block's decision.
  const bool out16 = J.flags & kOut16;
  // aligned outputs: a wave-uniform base per plane and 32-bit byte offsets
  // (their pitches are below 2^23 samples)
  auto out_row = [&](int p, int y, int x) {
    return to_global_out(J.out[p] + (int64_t)y * J.ostride[p] + x);
  };
  if (out16 && x0 + 64 <= W) {
    GlobalBytesOut ob = out_row(0, y0, x0);
    const uint32_t pitch = 2u * (uint32_t)J.ostride[0];
    for (int e = tid; e < 64 * 8; e += 256) {
      const int r = e >> 3, q = e & 7;
      if (y0 + r >= H) continue;
      const bool filt = n > 0 && (!(sm.flag[(r >> 3) * 8 + q] & 2) || py.skipcond);
      const uint4 v = filt ? *reinterpret_cast<const uint4 *>(&sm.sy[r * 64 + 8 * q])
                           : *reinterpret_cast<const uint4 *>(&sm.ry[(r + 2) * kLS + kLC0 + 8 * q]);
      store16(ob + (__umul24((uint32_t)r, pitch) + 16u * q), v);
    }
  } else {
    for (int e = tid; e < 64 * 64; e += 256) {
      const int r = e >> 6, col = e & 63;
      if (y0 + r >= H || x0 + col >= W) continue;
      const int b = (r >> 3) * 8 + (col >> 3);
      const bool filt = n > 0 && (!(sm.flag[b] & 2) || py.skipcond);
      J.out[0][(int64_t)(y0 + r) * J.ostride[0] + x0 + col] =
          filt ? sm.sy[e] : sm.ry[(r + 2) * kLS + kLC0 + col];
    }
  }
  if (J.nplanes != 3) return;
  if (J.layout == kLayout422) {
    // Section 4: chroma subsampled horizontally only is never filtered
    const int cw = (W + 1) >> 1, cx0 = x0 >> 1;
    for (int e = tid; e < 2 * 64 * 32; e += 256) {
      const int p = e >> 11, r = (e >> 5) & 63, col = e & 31;
      if (y0 + r >= H || cx0 + col >= cw) continue;
      J.out[1 + p][(int64_t)(y0 + r) * J.ostride[1 + p] + cx0 + col] =
          J.rec[1 + p][(int64_t)(y0 + r) * J.rstride[1 + p] + cx0 + col];
    }
    return;
  }
  if constexpr (X) {
    if (c444) {
      if (out16 && x0 + 64 <= W) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          GlobalBytesOut ob = out_row(1 + p, y0, x0);
          const uint32_t pitch = 2u * (uint32_t)J.ostride[1 + p];
          for (int e = tid; e < 64 * 8; e += 256) {
            const int r = e >> 3, q = e & 7;
            if (y0 + r >= H) continue;
            const bool filt = n > 0 && (!(sm.flag[(r >> 3) * 8 + q] & 2) || pc.skipcond);
            const uint4 v =
                filt ? *reinterpret_cast<const uint4 *>(&sm.sc[p][r * 64 + 8 * q])
                     : *reinterpret_cast<const uint4 *>(&sm.rc[p][(r + 2) * kLS + kLC0 + 8 * q]);
            store16(ob + (__umul24((uint32_t)r, pitch) + 16u * q), v);
          }
        }
        return;
      }
      for (int e = tid; e < 2 * 64 * 64; e += 256) {
        const int p = e >> 12, r = (e >> 6) & 63, col = e & 63;
        if (y0 + r >= H || x0 + col >= W) continue;
        const int b = (r >> 3) * 8 + (col >> 3);
        const bool filt = n > 0 && (!(sm.flag[b] & 2) || pc.skipcond);
        J.out[1 + p][(int64_t)(y0 + r) * J.ostride[1 + p] + x0 + col] =
            filt ? sm.sc[p][r * 64 + col] : sm.rc[p][(r + 2) * kLS + kLC0 + col];
      }
      return;
    }
  }
  const int cw = (W + 1) >> 1, ch = (H + 1) >> 1, cy0 = y0 >> 1, cx0 = x0 >> 1;
  if (out16 && cx0 + 32 <= cw) {
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
      GlobalBytesOut ob = out_row(1 + pl, cy0, cx0);
      const uint32_t pitch = 2u * (uint32_t)J.ostride[1 + pl];
      for (int e = tid; e < 32 * 8; e += 256) {
        const int r = e >> 3, q = e & 7;
        if (cy0 + r >= ch) continue;
        const bool filt = n > 0 && (!(sm.flag[(r >> 2) * 8 + q] & 2) || pc.skipcond);
        const uint2 v =
            filt ? *reinterpret_cast<const uint2 *>(&sm.sc[pl][r * 32 + 4 * q])
                 : *reinterpret_cast<const uint2 *>(&sm.rc[pl][(r + 2) * kCS + kCC0 + 4 * q]);
        store8(ob + (__umul24((uint32_t)r, pitch) + 8u * q), v);
      }
    }
    return;
  }
  for (int e = tid; e < 2 * 32 * 32; e += 256) {
    const int p = e >> 10, r = (e >> 5) & 31, col = e & 31;
    if (cy0 + r >= ch || cx0 + col >= cw) continue;
    const int b = (r >> 2) * 8 + (col >> 2);
    const bool filt = n > 0 && (!(sm.flag[b] & 2) || pc.skipcond);
    J.out[1 + p][(int64_t)(cy0 + r) * J.ostride[1 + p] + cx0 + col] =
        filt ? sm.sc[p][r * 32 + col] : sm.rc[p][(r + 2) * kCS + kCC0 + col];
  }
}

// X: the extended kernels (4:4:4, the weighted search).  FILTER: the kernel
// also runs filter jobs (batches that mix them with searches; single filter
// jobs and filter-only batches have kernels of their own).
template <bool X, bool FILTER = true>
__device__ __forceinline__ void run_item(SmemT<X> &sm, const JobDesc &J, int item, int tid) {
  const int fby = item / J.fbc, fbx = item - fby * J.fbc;
  if (J.mode == kModeSearchWeighted) {
    if (J.bitdepth == 12)
      search_item_weighted<X, true>(sm, J, fby, fbx, tid);
    else
      search_item_weighted<X, false>(sm, J, fby, fbx, tid);
    return;
  }
  if (J.bitdepth == 12) {
    if (J.mode == kModeSearch)
      search_item<false, true, false>(sm, J, fby, fbx, tid);
    else if (J.mode == kModeSearchFull)
      search_item<true, true, false>(sm, J, fby, fbx, tid);
    else if constexpr (FILTER)
      filter_item<X, true, false>(sm, J, fby, fbx, tid);
    return;
  }
  if (J.mode == kModeSearch) {
    if (J.cand)
      search_item<false, false, true>(sm, J, fby, fbx, tid);
    else
      search_item<false, false, false>(sm, J, fby, fbx, tid);
  } else if (J.mode == kModeSearchFull) {
    if (J.cand)
      search_item<true, false, true>(sm, J, fby, fbx, tid);
    else
      search_item<true, false, false>(sm, J, fby, fbx, tid);
  } else if constexpr (FILTER) {
    filter_item<X, false, false>(sm, J, fby, fbx, tid);
  }
}

}  // namespace

// One search job; the descriptor is a kernel argument.
#if CDEF_IN_KSET(0)
__global__ __launch_bounds__(256, 3) void k_fused_one(const JobDesc J) {
  __shared__ __align__(16) SmemT<false> sm;
  run_item<false, false>(sm, J, xcd_item(blockIdx.x, gridDim.x), threadIdx.x);
}
#endif

// One frame on the extended kernel (2 waves per SIMD: 256 VGPRs).  The
// descriptor is read through a global-memory view of the argument segment:
// as with the batch kernel's table, its fields are then reloaded where used
// instead of being held in registers for the whole kernel.
#if CDEF_IN_KSET(1)
__global__ __launch_bounds__(256, 2) void k_fused_one_x(const JobDesc J) {
  __shared__ __align__(16) SmemT<true> sm;
  (void)J;
  const uintptr_t args = reinterpret_cast<uintptr_t>(__builtin_amdgcn_kernarg_segment_ptr());
  const JobDesc *__restrict__ jp = reinterpret_cast<const JobDesc *>(args);
  run_item<true, false>(sm, *jp, xcd_item(blockIdx.x, gridDim.x), threadIdx.x);
}

hipError_t launch_one_ext(const JobDesc &job, hipStream_t s) {
  hipLaunchKernelGGL(k_fused_one_x, dim3(job.fbc * job.fbr), dim3(256), 0, s, job);
  return hipGetLastError();
}
#endif

// Index of the job that holds batch item `item`: the last job with
// item0 <= item.
__device__ __forceinline__ int job_of_item(const JobDesc *__restrict__ jobs, int njobs,
                                           int item) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].item0 <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// A batch: descriptors in device memory, items numbered across jobs.
// OCC bounds the waves per SIMD (and so the VGPR budget); XCD selects the
// XCD-contiguous order of filter blocks.
template <int OCC, bool XCD, bool X>
__global__ __launch_bounds__(256, OCC) void k_fused_batch(const JobDesc *__restrict__ jobs,
                                                          int njobs) {
  __shared__ __align__(16) SmemT<X> sm;
  const int item = XCD ? xcd_item(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const JobDesc &J = jobs[job_of_item(jobs, njobs, item)];
  run_item<X>(sm, J, item - J.item0, threadIdx.x);
}

// One launcher per instantiation; the two orders of a set may sit in
// different translation units.
#define CDEF_BATCH_LAUNCHER(NAME, OCC, XCD, X)                                          \
  hipError_t NAME(const JobDesc *jobs, int njobs, int nitems, hipStream_t s) {      \
    hipLaunchKernelGGL((k_fused_batch<OCC, XCD, X>), dim3(nitems), dim3(256), 0, s, \
                       jobs, njobs);                                               \
    return hipGetLastError();                                                      \
  }
#if CDEF_IN_KSET(2)
CDEF_BATCH_LAUNCHER(launch_batch_base3_xcd, 3, true, false)
CDEF_BATCH_LAUNCHER(launch_batch_base3_seq, 3, false, false)
#endif
#if CDEF_IN_KSET(3)
CDEF_BATCH_LAUNCHER(launch_batch_base2_xcd, 2, true, false)
CDEF_BATCH_LAUNCHER(launch_batch_base2_seq, 2, false, false)
#endif
#if CDEF_IN_KSET(4)
CDEF_BATCH_LAUNCHER(launch_batch_ext_xcd, 2, true, true)
#endif
#if CDEF_IN_KSET(6)
CDEF_BATCH_LAUNCHER(launch_batch_ext_seq, 2, false, true)
#endif
#undef CDEF_BATCH_LAUNCHER

// Persistent batch: as many workgroups as fit on the device at once, each
// taking filter blocks from a work queue until none is left.  The items are
// split into 8 contiguous ranges, one per XCD (workgroups are dealt to the
// XCDs round-robin, so workgroup w runs on XCD w mod 8 and its range's halo
// rows stay in that XCD's L2); a workgroup whose range is used up goes on
// to the next ranges in turn, so no XCD idles while another still has
// items.  Claims are atomic increments of one counter per range; a range
// that returned an index past its end is never asked again.  The last
// workgroup to leave resets the counters, so launches of one batch must not
// overlap.
template <int OCC, bool X>
__global__ __launch_bounds__(256, OCC) void k_fused_batch_queue(const JobDesc *__restrict__ jobs,
                                                                int njobs, int nitems,
                                                                BatchQueue *q) {
  __shared__ __align__(16) SmemT<X> sm;
  __shared__ int claimed;
  const int per = nitems >> 3, rem = nitems & 7;
  int r = blockIdx.x & 7;  // thread 0: the range it is drawing from
  int ranges_left = 8;
  for (;;) {
    if (threadIdx.x == 0) {
      int item = -1;
      while (ranges_left > 0) {
        const int len = per + (r < rem);
        const uint32_t k = atomicAdd(&q->next[r][0], 1u);
        if ((int)k < len) {
          item = r * per + min(r, rem) + (int)k;
          break;
        }
        r = (r + 1) & 7;
        --ranges_left;
      }
      claimed = item;
    }
    __syncthreads();
    const int item = claimed;
    if (item < 0) break;
    // a fresh, opaque thread index each time round: values derived from it
    // are then recomputed per item instead of being hoisted out of the loop
    // and held in registers across the whole item
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const JobDesc &J = jobs[job_of_item(jobs, njobs, item)];
    run_item<X>(sm, J, item - J.item0, tid);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // every claim of this workgroup precedes its departure; the last one to
    // leave knows that no claim is still to come
    __threadfence();
    if (atomicAdd(&q->done[0], 1u) == gridDim.x - 1) {
      for (int x = 0; x < 8; ++x) atomicExch(&q->next[x][0], 0u);
      atomicExch(&q->done[0], 0u);
    }
  }
}

// Resident workgroups of a kernel per device (queried once per device).
template <class K>
int resident_workgroups(K kernel) {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int c = cache[dev].load(std::memory_order_relaxed);
  if (c == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
        cus < 1 || per_cu < 1)
      return 256;
    c = cus * per_cu;
    cache[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

template <int OCC, bool X>
hipError_t launch_queue_kernel(const JobDesc *jobs, int njobs, int nitems, BatchQueue *q,
                               hipStream_t s) {
  const int g = min(nitems, resident_workgroups(k_fused_batch_queue<OCC, X>));
  hipLaunchKernelGGL((k_fused_batch_queue<OCC, X>), dim3(g), dim3(256), 0, s, jobs, njobs,
                     nitems, q);
  return hipGetLastError();
}

#if CDEF_IN_KSET(7)
hipError_t launch_batch_queue_base(int occ, const JobDesc *jobs, int njobs, int nitems,
                                   BatchQueue *q, hipStream_t s) {
  return occ == 2 ? launch_queue_kernel<2, false>(jobs, njobs, nitems, q, s)
                  : launch_queue_kernel<3, false>(jobs, njobs, nitems, q, s);
}
#endif
#if CDEF_IN_KSET(8)
hipError_t launch_batch_queue_ext(const JobDesc *jobs, int njobs, int nitems, BatchQueue *q,
                                  hipStream_t s) {
  return launch_queue_kernel<2, true>(jobs, njobs, nitems, q, s);
}
#endif

#if CDEF_IN_KSET(5)
// Filter-only kernels: the LDS holds just the tiles and per-block state
// (31 KB without the 4:4:4 chroma tiles) and the code just the filter mode.
// The direction search's registers keep them at 3 waves per SIMD.
template <bool X>
__device__ __forceinline__ void filter_run(SmemCore<X> &sm, const JobDesc &J, int item,
                                           int tid) {
  const int fby = item / J.fbc, fbx = item - fby * J.fbc;
  if (J.bitdepth == 12)
    filter_item<X, true, true>(sm, J, fby, fbx, tid);
  else
    filter_item<X, false, true>(sm, J, fby, fbx, tid);
}

__global__ __launch_bounds__(256, 5) void k_filter_one(const JobDesc J) {
  __shared__ __align__(16) SmemCore<false> sm;
  filter_run<false>(sm, J, xcd_item(blockIdx.x, gridDim.x), threadIdx.x);
}

__global__ __launch_bounds__(256, 2) void k_filter_one_x(const JobDesc J) {
  __shared__ __align__(16) SmemCore<true> sm;
  filter_run<true>(sm, J, xcd_item(blockIdx.x, gridDim.x), threadIdx.x);
}

template <bool X>
__global__ __launch_bounds__(256, X ? 2 : 5) void k_filter_batch(const JobDesc *__restrict__ jobs,
                                                                 int njobs) {
  __shared__ __align__(16) SmemCore<X> sm;
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const JobDesc &J = jobs[job_of_item(jobs, njobs, item)];
  filter_run<X>(sm, J, item - J.item0, threadIdx.x);
}

hipError_t launch_filter_one(const JobDesc &job, bool extended, hipStream_t s) {
  const dim3 g(job.fbc * job.fbr), b(256);
  if (extended)
    hipLaunchKernelGGL(k_filter_one_x, g, b, 0, s, job);
  else
    hipLaunchKernelGGL(k_filter_one, g, b, 0, s, job);
  return hipGetLastError();
}

hipError_t launch_filter_batch(bool extended, const JobDesc *jobs, int njobs, int nitems,
                               hipStream_t s) {
  const dim3 g(nitems), b(256);
  if (extended)
    hipLaunchKernelGGL((k_filter_batch<true>), g, b, 0, s, jobs, njobs);
  else
    hipLaunchKernelGGL((k_filter_batch<false>), g, b, 0, s, jobs, njobs);
  return hipGetLastError();
}
#endif

#if CDEF_IN_KSET(0)
void fill_job_geometry(JobDesc &j) {
  j.bcols = (j.width + 7) / 8;
  j.brows = (j.height + 7) / 8;
  j.fbc = (j.width + 63) / 64;
  j.fbr = (j.height + 63) / 64;
}

bool job_needs_extended(const JobDesc &j) {
  return j.nplanes == 3 && j.layout == kLayout444;
}

hipError_t launch_fused_one(const JobDesc &job, hipStream_t s) {
  if (job.mode == kModeFilter) return launch_filter_one(job, job_needs_extended(job), s);
  if (job_needs_extended(job)) return launch_one_ext(job, s);
  hipLaunchKernelGGL(k_fused_one, dim3(job.fbc * job.fbr), dim3(256), 0, s, job);
  return hipGetLastError();
}

hipError_t launch_batch_queue(int occ, bool extended, const JobDesc *jobs, int njobs, int nitems,
                              BatchQueue *queue, hipStream_t s) {
  return extended ? launch_batch_queue_ext(jobs, njobs, nitems, queue, s)
                  : launch_batch_queue_base(occ, jobs, njobs, nitems, queue, s);
}

hipError_t launch_fused_batch(const JobDesc *jobs, int njobs, int nitems, int variant,
                              bool extended, bool filter_only, BatchQueue *queue,
                              hipStream_t s) {
  // the variant picks the occupancy bound (3 or 2 waves per SIMD; the
  // extended kernels always run at 2), the filter-block order and a flat
  // grid or persistent workgroups; it does not apply to filter-only batches
  if (filter_only) return launch_filter_batch(extended, jobs, njobs, nitems, s);
  if (variant == 4 || variant == 5)
    return launch_batch_queue(variant == 4 ? 3 : 2, extended, jobs, njobs, nitems, queue, s);
  const bool xcd = variant == 0 || variant == 1;
  if (extended)
    return xcd ? launch_batch_ext_xcd(jobs, njobs, nitems, s)
               : launch_batch_ext_seq(jobs, njobs, nitems, s);
  if (variant == 1 || variant == 3)
    return xcd ? launch_batch_base2_xcd(jobs, njobs, nitems, s)
               : launch_batch_base2_seq(jobs, njobs, nitems, s);
  return xcd ? launch_batch_base3_xcd(jobs, njobs, nitems, s)
             : launch_batch_base3_seq(jobs, njobs, nitems, s);
}
#endif

}  // namespace cdef
