// Fused encoder strength search (Section 5): direction search (Section 2),
// constrained filter (Section 3) under all 64 (S^(p), S^(s)) pairs, and the
// per-filter-block SSE D_{b,p} = ||s - d||^2, without filtered pixels ever
// leaving registers.
//
// Work decomposition (one workgroup = one 64x64 filter block, 4 waves):
//  * the recon tile plus a 2-pixel halo (the taps reach +-2) and the source
//    tile are staged in LDS for luma and both 4:2:0 chroma planes;
//  * wave 0 runs Algorithm 1 for the 64 luma 8x8 blocks, one block per lane;
//  * non-skipped blocks are compacted into a list; a luma task is a pair of
//    8x8 blocks held in the two 16-bit halves of every lane (lane = pixel),
//    so the per-block strength tables are wave-uniform scalars; a chroma task
//    is eight 4x4 blocks (four per half);
//  * per task and lane the candidate-independent work (12 tap differences,
//    magnitudes, signs, clamp bounds) is done once; the secondary sums are
//    formed for S^(s) = 1, 2, 4, the primary sum once per S^(p), and every
//    pair costs one packed round/clamp/square-accumulate sequence;
//  * 64 per-lane accumulators are reduced across the wave by a transposing
//    butterfly (lane k ends with pair k), then across waves in LDS.
#include "cdef_device.hpp"
#include "cdef_launch.hpp"

namespace cdef {

struct SearchArgs {
  const uint16_t *rec[3];
  int64_t rstride[3];
  const uint16_t *src[3];
  int64_t sstride[3];
  int width, height, nplanes;
  int bcols, brows, fbc, fbr;
  const uint8_t *skip;
  uint64_t *sse;
  uint8_t *dir;
  int32_t *var;
};

namespace {

constexpr int kLS = 80;  // luma recon tile row stride in samples (68 used)
constexpr int kLC0 = 8;  // tile column that holds frame column x0 (16-byte aligned)
constexpr int kCS = 48;  // chroma recon tile row stride (36 used)
constexpr int kCC0 = 8;

// LDS offsets of the six tap positions (inner, outer along d; along d+2;
// along d-2) in the luma tile, per direction.  Indexed with wave-uniform
// directions, so the reads are scalar loads.
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
__constant__ TapTable kLumaTaps = make_tap_table(kLS);

__device__ __forceinline__ s16x2 as_s(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ s16x2 as_s(u16x2 v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ u16x2 as_u(s16x2 v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ u16x2 as_u(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_w(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t as_w(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

__device__ __forceinline__ s16x2 splat(int v) { return s16x2{(short)v, (short)v}; }
__device__ __forceinline__ u16x2 splatu(int v) {
  return u16x2{(unsigned short)v, (unsigned short)v};
}
__device__ __forceinline__ u16x2 pair_u(int lo, int hi) {
  return u16x2{(unsigned short)lo, (unsigned short)hi};
}
__device__ __forceinline__ s16x2 pair_s(int lo, int hi) { return s16x2{(short)lo, (short)hi}; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per-lane, candidate-independent state of one task: two samples per lane.
struct Taps {
  u16x2 ad[12];  // |x_tap - x| (out-of-frame taps: >= 31745)
  s16x2 sg[12];  // sign of x_tap - x as +-1
  s16x2 X;       // 16 (x - s) + 8: the rounding offset with the source folded in
  s16x2 dxs;     // x - s
  s16x2 lo, hi;  // clamp range minus s
};

// Tap order: primary +inner, -inner, +outer, -outer; then for the two
// secondary directions d+2 and d-2 the same four.
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
    hi = __builtin_elementwise_max(hi, v);         // kOutside is the most negative int16
    lo = __builtin_elementwise_min(lo, as_u(v));   // and the largest uint16 here
  }
  const s16x2 S = as_s(sv);
  t.dxs = X - S;
  t.X = t.dxs * splat(16) + splat(8);
  t.lo = as_s(lo) - S;
  t.hi = hi - S;
}

// Weighted constrained sum over taps [k0, k0+4): inner pair weight wi, outer
// pair weight wo, strength s, shift sh (per half).
__device__ __forceinline__ s16x2 group_sum(const Taps &t, int k0, u16x2 s, u16x2 sh, s16x2 wi,
                                           s16x2 wo) {
  s16x2 m[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const u16x2 a = t.ad[k0 + k] >> sh;
    const u16x2 g = __builtin_elementwise_sub_sat(s, a);  // max(0, S - (|d| >> sh))
    m[k] = as_s(__builtin_elementwise_min(g, t.ad[k0 + k]));
  }
  const s16x2 inner = m[0] * t.sg[k0] + m[1] * t.sg[k0 + 1];
  const s16x2 outer = m[2] * t.sg[k0 + 2] + m[3] * t.sg[k0 + 3];
  return inner * wi + outer * wo;
}

// Secondary sum for a compile-time strength and damping (same both halves).
template <int BD, int SEC, int DAMP>
__device__ __forceinline__ s16x2 secondary(const Taps &t) {
  constexpr int lg = SEC == 4 ? 2 : SEC == 2 ? 1 : 0;
  const u16x2 s = splatu(SEC << (BD - 8));
  const u16x2 sh = splatu(DAMP - lg);
  return group_sum(t, 4, s, sh, splat(2), splat(1)) + group_sum(t, 8, s, sh, splat(2), splat(1));
}

// One (S^(p), S^(s)) pair with both groups possibly active: round the sum
// of P and Q ties-away-from-zero, add to x - s, clamp, square-accumulate.
__device__ __forceinline__ int pair_both(const Taps &t, s16x2 P, s16x2 Q, int acc) {
  const s16x2 sum = P + Q;
  s16x2 y = (t.X + sum + (sum >> splat(15))) >> splat(4);
  y = __builtin_elementwise_min(__builtin_elementwise_max(y, t.lo), t.hi);
  return __builtin_amdgcn_sdot2(y, y, acc, false);
}

// A pair with only one tap group: its weights sum to 12/16 < 1, so the
// result cannot leave the clamp range and the clamp is skipped.
__device__ __forceinline__ int pair_one(const Taps &t, s16x2 P, int acc) {
  const s16x2 y = (t.X + P + (P >> splat(15))) >> splat(4);
  return __builtin_amdgcn_sdot2(y, y, acc, false);
}

// Luma task: 2 blocks (lo/hi half), per-block adjusted primary strengths.
// The per-strength parameters are wave-uniform; they are built as 32-bit
// scalars (low half: block A, high half: block B) so that they stay in SGPRs.
template <int BD, int D>
__device__ __forceinline__ void luma_task(const Taps &t, uint64_t adjA, uint64_t adjB,
                                          int (&acc)[64]) {
  constexpr int c = BD - 8;
  s16x2 Q[4];
  Q[1] = secondary<BD, 1, D>(t);
  Q[2] = secondary<BD, 2, D>(t);
  Q[3] = secondary<BD, 4, D>(t);
  acc[0] = __builtin_amdgcn_sdot2(t.dxs, t.dxs, acc[0], false);
#pragma unroll
  for (int si = 1; si < 4; ++si) acc[si] = pair_one(t, Q[si], acc[si]);
  uint32_t prev_sh = 0xFFFFFFFFu;
  u16x2 a[4];
#pragma unroll
  for (int S = 1; S < 16; ++S) {
    const uint32_t sa = (uint32_t)(adjA >> (4 * S)) & 15u, sb = (uint32_t)(adjB >> (4 * S)) & 15u;
    const uint32_t sp = (sa << c) | (sb << (16 + c));
    const uint32_t sha = sa ? (uint32_t)(D - floor_log2((int)sa)) : 0u;
    const uint32_t shb = sb ? (uint32_t)(D - floor_log2((int)sb)) : 0u;
    const uint32_t sh = sha | (shb << 16);
    const uint32_t w1 = ((sa & 1) ? 3u : 4u) | (((sb & 1) ? 3u : 4u) << 16);
    const uint32_t w2 = ((sa & 1) ? 3u : 2u) | (((sb & 1) ? 3u : 2u) << 16);
    if (sh != prev_sh) {  // the shift changes at most a few times over S = 1..15
      prev_sh = sh;
#pragma unroll
      for (int k = 0; k < 4; ++k) a[k] = t.ad[k] >> as_u(sh);
    }
    s16x2 m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      m[k] = as_s(__builtin_elementwise_min(__builtin_elementwise_sub_sat(as_u(sp), a[k]), t.ad[k]));
    const s16x2 inner = m[0] * t.sg[0] + m[1] * t.sg[1];
    const s16x2 outer = m[2] * t.sg[2] + m[3] * t.sg[3];
    const s16x2 P = inner * as_s(w1) + outer * as_s(w2);
    acc[4 * S] = pair_one(t, P, acc[4 * S]);
#pragma unroll
    for (int si = 1; si < 4; ++si) acc[4 * S + si] = pair_both(t, P, Q[si], acc[4 * S + si]);
  }
}

// Chroma task: strengths are not adjusted, so every parameter is a
// compile-time constant; damping max(D - 1, floor(log2 S^(p))) splits the
// secondary sums in two when D = 3.
template <int BD, int D>
__device__ __forceinline__ void chroma_task(const Taps &t, int (&acc)[64]) {
  constexpr int c = BD - 8;
  constexpr int Dlo = D - 1;   // chroma damping while floor(log2 S^(p)) <= D - 1
  s16x2 Qa[4], Qb[4];          // Qa: damping D - 1; Qb: damping 3 (only when D = 3)
  Qa[1] = secondary<BD, 1, Dlo>(t);
  Qa[2] = secondary<BD, 2, Dlo>(t);
  Qa[3] = secondary<BD, 4, Dlo>(t);
  if constexpr (D == 3) {
    Qb[1] = secondary<BD, 1, 3>(t);
    Qb[2] = secondary<BD, 2, 3>(t);
    Qb[3] = secondary<BD, 4, 3>(t);
  }
  acc[0] = __builtin_amdgcn_sdot2(t.dxs, t.dxs, acc[0], false);
#pragma unroll
  for (int si = 1; si < 4; ++si) acc[si] = pair_one(t, Qa[si], acc[si]);
#pragma unroll
  for (int S = 1; S < 16; ++S) {
    const int lg = S >= 8 ? 3 : S >= 4 ? 2 : S >= 2 ? 1 : 0;
    const int Dc = lg > Dlo ? lg : Dlo;
    const u16x2 s = splatu(S << c);
    const u16x2 sh = splatu(Dc - lg);
    const s16x2 w1 = splat((S & 1) ? 3 : 4), w2 = splat((S & 1) ? 3 : 2);
    const s16x2 P = group_sum(t, 0, s, sh, w1, w2);
    acc[4 * S] = pair_one(t, P, acc[4 * S]);
#pragma unroll
    for (int si = 1; si < 4; ++si) {
      s16x2 Q = Qa[si];
      if constexpr (D == 3) {
        if (Dc != Dlo) Q = Qb[si];
      }
      acc[4 * S + si] = pair_both(t, P, Q, acc[4 * S + si]);
    }
  }
}

// Wave-wide sum of 64 per-lane accumulators; lane k returns the total of
// accumulator k.  Each step halves the values kept per lane.
__device__ __forceinline__ uint32_t reduce_transpose(int (&acc)[64], int lane) {
  uint32_t v[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) v[i] = (uint32_t)acc[i];
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1) {
    const bool up = (lane & step) != 0;
#pragma unroll
    for (int i = 0; i < step; ++i) {
      const uint32_t a = v[i], b = v[i + step];
      const uint32_t send = up ? a : b;
      const uint32_t keep = up ? b : a;
      v[i] = keep + (uint32_t)__shfl_xor((int)send, step, 64);
    }
  }
  return v[0];
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += (uint32_t)__shfl_xor((int)v, m, 64);
  return v;
}

}  // namespace

template <int BD, int D>
__global__ __launch_bounds__(256, 3) void k_search(const SearchArgs a) {
  __shared__ __align__(16) uint16_t ry[68 * kLS];
  __shared__ __align__(16) uint16_t sy[64 * 64];
  __shared__ __align__(16) uint16_t rc[2][36 * kCS];
  __shared__ __align__(16) uint16_t sc[2][32 * 32];
  __shared__ uint64_t s_adj[64];
  __shared__ uint8_t s_dir[64];
  __shared__ uint8_t s_list[64];
  __shared__ uint8_t s_skip[64];
  __shared__ int s_n;
  __shared__ uint32_t s_red[4][64];
  __shared__ uint32_t s_skipsse[3];
  __shared__ int16_t s_coff[8][6];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fby = blockIdx.x / a.fbc, fbx = blockIdx.x - fby * a.fbc;
  const int y0 = fby * 64, x0 = fbx * 64;
  const int W = a.width, H = a.height;
  const int cw = (W + 1) >> 1, ch = (H + 1) >> 1, cy0 = y0 >> 1, cx0 = x0 >> 1;
  const bool chroma = a.nplanes == 3;

  // ---- a1: stage recon tiles (with halo) and source tiles ----
  stage_recon<64, 64, kLS, kLC0, 256>(ry, a.rec[0], a.rstride[0], W, H, y0, x0, tid);
  stage_interior<64, 64, 256>(sy, a.src[0], a.sstride[0], W, H, y0, x0, tid);
  if (chroma) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      stage_recon<32, 32, kCS, kCC0, 256>(rc[p], a.rec[p + 1], a.rstride[p + 1], cw, ch, cy0,
                                          cx0, tid);
      stage_interior<32, 32, 256>(sc[p], a.src[p + 1], a.sstride[p + 1], cw, ch, cy0, cx0, tid);
    }
  }
  if (tid < 48) {
    const int d = tid / 6, k = tid - 6 * (tid / 6);
    const int dd = k < 2 ? d : k < 4 ? (d + 2) & 7 : (d + 6) & 7;
    s_coff[d][k] = (int16_t)(tap_dr(dd, k & 1) * kCS + tap_dc(dd, k & 1));
  }
  if (tid < 3) s_skipsse[tid] = 0;
  __syncthreads();

  // ---- a2: direction search, one 8x8 luma block per lane of wave 0 ----
  if (wave == 0) {
    const int b = lane;
    const int by = fby * 8 + (b >> 3), bx = fbx * 8 + (b & 7);
    const bool in = by < a.brows && bx < a.bcols;
    const bool sk = in && a.skip && a.skip[(int64_t)by * a.bcols + bx];
    int d = 0, v = 0;
    if (in) {
      const int bw = min(8, W - 8 * bx), bh = min(8, H - 8 * by);
      int x[64];
      const uint16_t *row0 = ry + (2 + 8 * (b >> 3)) * kLS + kLC0 + 8 * (b & 7);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint4 q = *reinterpret_cast<const uint4 *>(row0 + i * kLS);
        const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int px = (int)((w4[j >> 1] >> (16 * (j & 1))) & 0xFFFF);
          x[i * 8 + j] = (px >> (BD - 8)) - 128;
        }
      }
      int cost[8];
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
      pick_direction(cost, d, v);
      if (a.dir) {
        a.dir[(int64_t)by * a.bcols + bx] = (uint8_t)d;
        a.var[(int64_t)by * a.bcols + bx] = v;
      }
    }
    s_dir[b] = (uint8_t)d;
    s_adj[b] = adjusted_strengths(v);
    s_skip[b] = (uint8_t)(!in || sk);
    const bool active = in && !sk;
    const uint64_t m = __ballot(active);
    const int pos = __popcll(m & ((1ull << lane) - 1ull));
    if (active) s_list[pos] = (uint8_t)b;
    if (lane == 0) s_n = __popcll(m);
  }
  __syncthreads();
  const int n = s_n;

  // ---- SSE of skipped (unfiltered) pixels, identical for all 64 pairs ----
  {
    uint32_t e0 = 0, e1 = 0, e2 = 0;
    for (int e = tid; e < 64 * 64; e += 256) {
      const int r = e >> 6, col = e & 63;
      if (s_skip[(r >> 3) * 8 + (col >> 3)] && y0 + r < H && x0 + col < W) {
        const int dd = (int)ry[(r + 2) * kLS + kLC0 + col] - (int)sy[e];
        e0 += (uint32_t)(dd * dd);
      }
    }
    if (chroma) {
      for (int e = tid; e < 32 * 32; e += 256) {
        const int r = e >> 5, col = e & 31;
        if (s_skip[(r >> 2) * 8 + (col >> 2)] && cy0 + r < ch && cx0 + col < cw) {
          const int i = (r + 2) * kCS + kCC0 + col;
          const int d1 = (int)rc[0][i] - (int)sc[0][e];
          const int d2 = (int)rc[1][i] - (int)sc[1][e];
          e1 += (uint32_t)(d1 * d1);
          e2 += (uint32_t)(d2 * d2);
        }
      }
    }
    e0 = wave_sum(e0);
    e1 = wave_sum(e1);
    e2 = wave_sum(e2);
    if (lane == 0) {
      atomicAdd(&s_skipsse[0], e0);
      atomicAdd(&s_skipsse[1], e1);
      atomicAdd(&s_skipsse[2], e2);
    }
  }

  const int64_t fbi = (int64_t)fby * a.fbc + fbx;
  const int64_t plane_stride = (int64_t)a.fbr * a.fbc * 64;

  // ---- a3-a7 luma: tasks of two 8x8 blocks ----
  {
    int acc[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) acc[i] = 0;
    const int ntask = (n + 1) >> 1;
    const int r = lane >> 3, col = lane & 7;
    for (int tk = wave; tk < ntask; tk += 4) {
      const int A = uniform(s_list[2 * tk]);
      const bool hasB = 2 * tk + 1 < n;
      const int B = hasB ? uniform(s_list[2 * tk + 1]) : A;
      const int dA = uniform(s_dir[A]), dB = uniform(s_dir[B]);
      const uint64_t adjA = ((uint64_t)(uint32_t)uniform((int)(uint32_t)s_adj[A])) |
                            ((uint64_t)(uint32_t)uniform((int)(uint32_t)(s_adj[A] >> 32)) << 32);
      const uint64_t adjB = ((uint64_t)(uint32_t)uniform((int)(uint32_t)s_adj[B])) |
                            ((uint64_t)(uint32_t)uniform((int)(uint32_t)(s_adj[B] >> 32)) << 32);
      const int rA = 8 * (A >> 3) + r, cA = 8 * (A & 7) + col;
      const int rB = 8 * (B >> 3) + r, cB = 8 * (B & 7) + col;
      const bool vA = y0 + rA < H && x0 + cA < W;
      const bool vB = hasB && y0 + rB < H && x0 + cB < W;
      const uint32_t vm = (vA ? 0x0000FFFFu : 0u) | (vB ? 0xFFFF0000u : 0u);
      const int bA = (rA + 2) * kLS + kLC0 + cA, bB = (rB + 2) * kLS + kLC0 + cB;
      int oA[6], oB[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        oA[k] = kLumaTaps.off[dA][k];
        oB[k] = kLumaTaps.off[dB][k];
      }
      const uint32_t xv = ((uint32_t)ry[bA] | ((uint32_t)ry[bB] << 16)) & vm;
      const uint32_t sv = ((uint32_t)sy[rA * 64 + cA] | ((uint32_t)sy[rB * 64 + cB] << 16)) & vm;
      uint32_t tp[12];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        // k: 0 inner, 1 outer of d; 2, 3 of d+2; 4, 5 of d-2
        const int slot = (k >> 1) * 4 + (k & 1) * 2;
        tp[slot] = ((uint32_t)ry[bA + oA[k]] | ((uint32_t)ry[bB + oB[k]] << 16)) & vm;
        tp[slot + 1] = ((uint32_t)ry[bA - oA[k]] | ((uint32_t)ry[bB - oB[k]] << 16)) & vm;
      }
      Taps t;
      prepare(t, xv, sv, tp);
      luma_task<BD, D>(t, adjA, adjB, acc);
    }
    const uint32_t tot = reduce_transpose(acc, lane);
    s_red[wave][lane] = tot;
    __syncthreads();
    if (tid < 64) {
      const uint64_t s = (uint64_t)s_red[0][tid] + s_red[1][tid] + s_red[2][tid] +
                         s_red[3][tid] + s_skipsse[0];
      a.sse[fbi * 64 + tid] = s;
    }
  }

  if (!chroma) return;

  // ---- a3-a7 chroma (4:2:0): tasks of eight 4x4 blocks, four per half ----
  const int ntask = (n + 7) >> 3;
  const int sub = lane >> 4, r = (lane >> 2) & 3, col = lane & 3;
  for (int p = 0; p < 2; ++p) {
    int acc[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) acc[i] = 0;
    const uint16_t *rt = rc[p];
    const uint16_t *stl = sc[p];
    for (int tk = wave; tk < ntask; tk += 4) {
      const int iL = 8 * tk + sub, iH = 8 * tk + 4 + sub;
      const bool hasL = iL < n, hasH = iH < n;
      const int L = hasL ? s_list[iL] : 0, Hb = hasH ? s_list[iH] : 0;
      const int rL = 4 * (L >> 3) + r, cL = 4 * (L & 7) + col;
      const int rH = 4 * (Hb >> 3) + r, cH = 4 * (Hb & 7) + col;
      const bool vL = hasL && cy0 + rL < ch && cx0 + cL < cw;
      const bool vH = hasH && cy0 + rH < ch && cx0 + cH < cw;
      const uint32_t vm = (vL ? 0x0000FFFFu : 0u) | (vH ? 0xFFFF0000u : 0u);
      const int bL = (rL + 2) * kCS + kCC0 + cL, bH = (rH + 2) * kCS + kCC0 + cH;
      const int dL = s_dir[L], dH = s_dir[Hb];
      const uint32_t xv = ((uint32_t)rt[bL] | ((uint32_t)rt[bH] << 16)) & vm;
      const uint32_t sv =
          ((uint32_t)stl[rL * 32 + cL] | ((uint32_t)stl[rH * 32 + cH] << 16)) & vm;
      uint32_t tp[12];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const int oL = s_coff[dL][k], oH = s_coff[dH][k];
        const int slot = (k >> 1) * 4 + (k & 1) * 2;
        tp[slot] = ((uint32_t)rt[bL + oL] | ((uint32_t)rt[bH + oH] << 16)) & vm;
        tp[slot + 1] = ((uint32_t)rt[bL - oL] | ((uint32_t)rt[bH - oH] << 16)) & vm;
      }
      Taps t;
      prepare(t, xv, sv, tp);
      chroma_task<BD, D>(t, acc);
    }
    const uint32_t tot = reduce_transpose(acc, lane);
    __syncthreads();  // previous readers of s_red are done
    s_red[wave][lane] = tot;
    __syncthreads();
    if (tid < 64) {
      const uint64_t s = (uint64_t)s_red[0][tid] + s_red[1][tid] + s_red[2][tid] +
                         s_red[3][tid] + s_skipsse[1 + p];
      a.sse[(1 + p) * plane_stride + fbi * 64 + tid] = s;
    }
  }
}

template <int BD>
static hipError_t launch_search_bd(const SearchArgs &a, int damping, int grid, hipStream_t s) {
  switch (damping) {
    case 3: hipLaunchKernelGGL((k_search<BD, 3>), dim3(grid), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_search<BD, 4>), dim3(grid), dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_search<BD, 5>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_search<BD, 6>), dim3(grid), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_search(const FrameDesc &rec, const FrameDesc &src, const uint8_t *skip,
                         int damping, uint64_t *sse, uint8_t *dir, int32_t *var, hipStream_t s) {
  SearchArgs a{};
  for (int p = 0; p < 3; ++p) {
    a.rec[p] = rec.plane[p];
    a.rstride[p] = rec.stride[p];
    a.src[p] = src.plane[p];
    a.sstride[p] = src.stride[p];
  }
  a.width = rec.width;
  a.height = rec.height;
  a.nplanes = rec.nplanes;
  a.bcols = (rec.width + 7) / 8;
  a.brows = (rec.height + 7) / 8;
  a.fbc = (rec.width + 63) / 64;
  a.fbr = (rec.height + 63) / 64;
  a.skip = skip;
  a.sse = sse;
  a.dir = dir;
  a.var = var;
  const int grid = a.fbc * a.fbr;
  return rec.bitdepth == 8 ? launch_search_bd<8>(a, damping, grid, s)
                           : launch_search_bd<10>(a, damping, grid, s);
}

}  // namespace cdef
