// Preset selection on the strength-search table (Section 5, Eq. 15).
//
// D^luma_{b,p} is the luma SSE of filter block b under pair p (p = S^(p) * 4
// + index of S^(s)); D^chroma_{b,p} is the Cb + Cr SSE.  For each group a
// greedy sequence of 8 presets is built, each step adding the candidate not
// yet chosen that most lowers sum_b min over the set (lowest index on ties);
// for N = 1, 2, 4, 8 the greedy prefix is re-optimized one preset at a time
// (a slot takes the best candidate not among the others, on a strict
// improvement) for up to `refine` passes; J(N) = lambda * B * log2 N +
// D^luma(N) + D^chroma(N), the smallest N of minimal J wins, and every filter
// block gets the slot of its smallest distortion (lowest slot on ties).
//
// One workgroup of 1024 threads per group: thread (p = t % 64, q = t / 64)
// sums min(m_b, D_{b,p}) over blocks b = q mod 16, where m_b, the minimum
// over the presets held fixed, is staged in LDS 4096 blocks at a time; the
// 16 partial sums per candidate are added in LDS.
#include "cdef_launch.hpp"

#include <stdint.h>

namespace cdef {

namespace {

constexpr int kChunk = 4096;
constexpr int kNT = 1024;

__device__ __forceinline__ uint64_t dist_of(const uint64_t *sse, int nplanes, int nfb, int g,
                                            int b, int p) {
  if (g == 0) return sse[(int64_t)b * 64 + p];
  if (nplanes < 3) return 0;
  return sse[((int64_t)nfb + b) * 64 + p] + sse[((int64_t)2 * nfb + b) * 64 + p];
}

struct PresetSmem {
  uint64_t m[kChunk];
  uint64_t part[16][64];
  uint64_t cost[64];
  int set[8];
  int greedy[8];
  int changed;
};

// cost[p] = sum_b min(min_{i < n, i != excl} D_{b,S[i]}, D_{b,p}) for all 64 p.
__device__ void evaluate(PresetSmem &sm, const uint64_t *sse, int nplanes, int nfb, int g,
                         const int *S, int n, int excl) {
  const int tid = threadIdx.x, p = tid & 63, q = tid >> 6;
  uint64_t acc = 0;
  for (int c0 = 0; c0 < nfb; c0 += kChunk) {
    const int cn = min(kChunk, nfb - c0);
    for (int i = tid; i < cn; i += kNT) {
      uint64_t mm = UINT64_MAX;
      for (int k = 0; k < n; ++k) {
        if (k == excl) continue;
        const uint64_t d = dist_of(sse, nplanes, nfb, g, c0 + i, S[k]);
        mm = d < mm ? d : mm;
      }
      sm.m[i] = mm;
    }
    __syncthreads();
    for (int i = q; i < cn; i += 16) {
      const uint64_t d = dist_of(sse, nplanes, nfb, g, c0 + i, p);
      acc += d < sm.m[i] ? d : sm.m[i];
    }
    __syncthreads();
  }
  sm.part[q][p] = acc;
  __syncthreads();
  if (tid < 64) {
    uint64_t s = 0;
    for (int k = 0; k < 16; ++k) s += sm.part[k][tid];
    sm.cost[tid] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ bool in_set(const int *S, int n, int p, int except) {
  for (int i = 0; i < n; ++i)
    if (i != except && S[i] == p) return true;
  return false;
}

__global__ __launch_bounds__(kNT) void k_preset_search(const uint64_t *__restrict__ sse,
                                                       int nplanes, int nfb, int refine,
                                                       PresetResult *out) {
  __shared__ PresetSmem sm;
  const int g = blockIdx.x, tid = threadIdx.x;
  for (int step = 0; step < 8; ++step) {
    evaluate(sm, sse, nplanes, nfb, g, sm.greedy, step, -1);
    if (tid == 0) {
      int best = -1;
      for (int p = 0; p < 64; ++p) {
        if (in_set(sm.greedy, step, p, -1)) continue;
        if (best < 0 || sm.cost[p] < sm.cost[best]) best = p;
      }
      sm.greedy[step] = best;
    }
    __syncthreads();
  }
  for (int k = 0; k < 4; ++k) {
    const int n = 1 << k;
    if (tid < 8) sm.set[tid] = tid < n ? sm.greedy[tid] : -1;
    __syncthreads();
    for (int pass = 0; pass < refine; ++pass) {
      if (tid == 0) sm.changed = 0;
      __syncthreads();
      for (int i = 0; i < n; ++i) {
        evaluate(sm, sse, nplanes, nfb, g, sm.set, n, i);
        if (tid == 0) {
          int bp = sm.set[i];
          uint64_t bd = sm.cost[bp];
          for (int p = 0; p < 64; ++p) {
            if (in_set(sm.set, n, p, i)) continue;
            if (sm.cost[p] < bd) {
              bd = sm.cost[p];
              bp = p;
            }
          }
          if (bp != sm.set[i]) {
            sm.set[i] = bp;
            sm.changed = 1;
          }
        }
        __syncthreads();
      }
      // every thread reads the flag before thread 0 may clear it again
      const int changed = sm.changed;
      __syncthreads();
      if (!changed) break;
    }
    evaluate(sm, sse, nplanes, nfb, g, sm.set, n, -1);
    if (tid == 0) {
      uint64_t *dist = g == 0 ? out->dist_luma : out->dist_chroma;
      int32_t *sets = g == 0 ? &out->luma[0][0] : &out->chroma[0][0];
      dist[k] = sm.cost[sm.set[0]];  // min(m_b, D_{b,S[0]}) = m_b
      for (int i = 0; i < 8; ++i) sets[k * 8 + i] = sm.set[i];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kNT) void k_preset_finish(const uint64_t *__restrict__ sse,
                                                       int nplanes, int nfb, double lambda,
                                                       PresetResult *out, uint8_t *fb_luma,
                                                       uint8_t *fb_chroma) {
  __shared__ int chosen;
  if (threadIdx.x == 0) {
    // J(N) is evaluated as written, one rounding per operation (no fused
    // multiply-add), so that equal inputs give the same choice everywhere.
#pragma clang fp contract(off)
    int c = 0;
    for (int k = 0; k < 4; ++k) {
      out->cost[k] = lambda * (double)nfb * (double)k +
                     (double)(out->dist_luma[k] + out->dist_chroma[k]);
      if (out->cost[k] < out->cost[c]) c = k;
    }
    out->n = 1 << c;
    out->reserved = 0;
    chosen = c;
  }
  __syncthreads();
  const int c = chosen, n = 1 << c;
  for (int b = blockIdx.x * kNT + threadIdx.x; b < nfb; b += gridDim.x * kNT) {
    for (int g = 0; g < 2; ++g) {
      const int32_t *sets = g == 0 ? &out->luma[c][0] : &out->chroma[c][0];
      int bi = 0;
      uint64_t bd = UINT64_MAX;
      for (int i = 0; i < n; ++i) {
        const uint64_t d = dist_of(sse, nplanes, nfb, g, b, sets[i]);
        if (d < bd) {
          bd = d;
          bi = i;
        }
      }
      (g == 0 ? fb_luma : fb_chroma)[b] = (uint8_t)bi;
    }
  }
}

}  // namespace

hipError_t launch_select_presets(const uint64_t *sse, int nplanes, int nfb, double lambda,
                                 int refine, PresetResult *out, uint8_t *fb_luma,
                                 uint8_t *fb_chroma, hipStream_t s) {
  hipLaunchKernelGGL(k_preset_search, dim3(2), dim3(kNT), 0, s, sse, nplanes, nfb, refine, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // one workgroup: every thread of it needs the chosen N computed by thread 0
  hipLaunchKernelGGL(k_preset_finish, dim3(1), dim3(kNT), 0, s, sse, nplanes, nfb, lambda, out,
                     fb_luma, fb_chroma);
  return hipGetLastError();
}

}  // namespace cdef
