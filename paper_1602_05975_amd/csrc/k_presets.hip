// Preset selection on the strength-search table (Section 5, Eq. 15).
//
// D^luma_{b,p} is the luma SSE of filter block b under candidate p (p =
// skip condition bit * 64 + S^(p) * 4 + index of S^(s); 64 candidates
// without the bit, 128 with it); D^chroma_{b,p} is the Cb + Cr SSE.  A
// candidate mask restricts the choice to a subset (the low-complexity
// search leaves the others unevaluated).  For each group a
// greedy sequence of 8 presets is built, each step adding the candidate not
// yet chosen that most lowers sum_b min over the set (lowest index on ties);
// for N = 1, 2, 4, 8 the greedy prefix is re-optimized one preset at a time
// (a slot takes the best candidate not among the others, on a strict
// improvement) for up to `refine` passes; J(N) = lambda * B * log2 N +
// D^luma(N) + D^chroma(N), the smallest N of minimal J wins, and every filter
// block gets the slot of its smallest distortion (lowest slot on ties).
//
// Layout of the work.  Each group (luma, chroma) is spread over G workgroups;
// workgroup w owns a contiguous slice of filter blocks (96 at 64 candidates,
// 48 at 128) and keeps its slice of D (chroma already summed) in LDS.  Every step of the search is a
// "round": each workgroup evaluates, for up to three candidate sets at once,
// the partial sums sum_{b in slice} min(m_b, D_{b,p}) (m_b the minimum over
// the presets held fixed), adds them atomically into the round's totals in
// the workspace and waits until all G workgroups of its group have done so.
// Every workgroup then reads the same integer totals and takes the same
// decisions without further communication.  The greedy
// takes 8 rounds; the refinements of N = 2, 4 and 8 advance together, one
// slot per round.  Two facts keep this exact with fewer rounds: the N = 1
// refinement can never change the set (the greedy first pick is the exact
// minimum of the same sums, lowest index first), and a refined set's
// distortion is the smaller of the two costs compared at its last slot
// decision, so it needs no extra evaluation.
//
// Waits are bounded in time: a workgroup that waited more than a second marks
// the selection failed and leaves, every other one leaves at its next wait,
// and the result then reports n = 0.
#include "cdef_launch.hpp"

#include <stdint.h>

#include <mutex>

namespace cdef {

namespace {

constexpr int kNT = 256;        // threads per workgroup
constexpr int kLdsEntries = 6144;  // D values per workgroup kept in LDS
constexpr int kMaxG = 128;      // workgroups per group
constexpr int kQ = 3;           // candidate sets evaluated per round
constexpr int kMaxNC = 128;     // candidates
constexpr uint64_t kWaitTicks = 100000000ull;  // 1 s of the 100 MHz wall clock

template <int NC>
constexpr int slice_blocks() { return kLdsEntries / NC; }

struct PresetWork {
  uint32_t arrive[2];  // per-group arrival counters (G per round)
  uint32_t failed;
  uint32_t pad[61];
  uint64_t total[3][2][kQ][kMaxNC];  // [round mod 3][group][set][p]
};

template <int NC>
__device__ __forceinline__ uint64_t group_dist(const uint64_t *sse, int nfb, int g, int b, int p) {
  if (g == 0) return sse[(int64_t)b * NC + p];
  return sse[((int64_t)nfb + b) * NC + p] + sse[((int64_t)2 * nfb + b) * NC + p];
}

struct Query {
  int set[8];
  int n, excl;
};

// Candidates outside the caller's subset are never chosen.
struct CandMask {
  uint64_t w[2];
  __device__ __forceinline__ bool allowed(int p) const { return (w[p >> 6] >> (p & 63)) & 1; }
};

template <int NC>
struct CoopSmem {
  static constexpr int kSlice = slice_blocks<NC>(), kRows = kNT / NC;
  uint64_t d[kSlice][NC];
  uint64_t m[kQ][kSlice];
  uint64_t red[kRows][kQ][NC];
  uint64_t cost[kQ][NC];
  uint64_t best_cost[kQ];
  int best_p[kQ];
  Query q[kQ];
  int qowner[kQ];  // refinement (0: N = 2, 1: N = 4, 2: N = 8) of each query
  int nq, last, ok;
  // search state, identical in every workgroup of the group
  int step;
  int greedy[8];
  uint64_t greedy_cost[8];
  int rset[3][8];
  int slot[3], pass[3], changed[3], done[3];
  uint64_t rdist[3];
};

__device__ __forceinline__ bool excluded(const Query &q, int p) {
  for (int i = 0; i < q.n; ++i)
    if (i != q.excl && q.set[i] == p) return true;
  return false;
}

__device__ __forceinline__ void argmin2(uint64_t &c, int &p, uint64_t oc, int op) {
  if (oc < c || (oc == c && op < p)) {
    c = oc;
    p = op;
  }
}

// Lexicographic (cost, p) minimum over the 64 lanes of a wave; excluded
// candidates carry UINT64_MAX and an index past the last candidate.
__device__ __forceinline__ void wave_argmin(uint64_t &c, int &p) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint64_t oc = __shfl_xor(c, off, 64);
    const int op = __shfl_xor(p, off, 64);
    argmin2(c, p, oc, op);
  }
}

// The workgroup's partial sums for this round are in sm.red.  They are added
// atomically into the round's totals, then the workgroup counts its arrival
// and waits for the group's other workgroups.  Totals rotate over three
// buffers: the last arrival of round r clears the buffer of round r - 1
// (= r + 2 mod 3), which every workgroup has read before arriving at round r
// and none adds to before round r + 2.  Everything that passes between
// workgroups (totals, counters, the failure flag) is accessed only by
// device-scope atomics, so ordering needs no cache write-back or
// invalidation: each wave waits until its own atomics have returned before
// the arrival is counted, and totals are read only after the count is seen
// complete.  On return sm.cost holds the group's totals; false if the wait
// timed out.
template <int NC>
__device__ bool round_totals(CoopSmem<NC> &sm, PresetWork *work, int g, int G, int nq,
                             uint32_t round) {
  constexpr int R = CoopSmem<NC>::kRows;
  const int tid = threadIdx.x;
  const uint32_t buf = round % 3;
  uint64_t before = 0;
  for (int i = tid; i < nq * NC; i += kNT) {
    const int s = i / NC, p = i % NC;
    uint64_t v = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) v += sm.red[r][s][p];
    before += __hip_atomic_fetch_add(&work->total[buf][g][s][p], v, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
  }
  // consuming the returned values makes the wave wait for the adds to complete
  __asm__ volatile("" : : "v"(before));
  __syncthreads();
  if (tid == 0) {
    const uint32_t target = (uint32_t)G * (round + 1);
    const uint32_t old =
        __hip_atomic_fetch_add(&work->arrive[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    if (old + 1 != target) {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&work->arrive[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
             target) {
        if (__hip_atomic_load(&work->failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            wall_clock64() - t0 > kWaitTicks) {
          __hip_atomic_store(&work->failed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    sm.last = old + 1 == target;
    sm.ok = ok;
  }
  __syncthreads();
  if (!sm.ok) return false;
  for (int i = tid; i < nq * NC; i += kNT)
    sm.cost[i / NC][i % NC] = __hip_atomic_load(&work->total[buf][g][i / NC][i % NC],
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (sm.last)
    for (int i = tid; i < kQ * NC; i += kNT)
      __hip_atomic_store(&work->total[(round + 2) % 3][g][i / NC][i % NC], (uint64_t)0,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // the clearing stores complete before this workgroup's next arrival
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  return true;
}

template <int NC, bool LDS>
__global__ __launch_bounds__(kNT) void k_preset_coop(const uint64_t *__restrict__ sse,
                                                     int nplanes, int nfb, int G, int refine,
                                                     CandMask cm, PresetWork *work,
                                                     PresetResult *out) {
  using Smem = CoopSmem<NC>;
  constexpr int R = Smem::kRows;
  __shared__ Smem sm;
  const int g = blockIdx.x / G, w = blockIdx.x % G, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int pc = tid % NC, row = tid / NC;  // candidate and block row of this thread
  if (g == 1 && nplanes == 1) {
    // all-zero chroma: every candidate ties, so the greedy takes 0, 1, ..., 7
    // and no refinement finds a strict improvement
    if (w == 0 && tid < 32) {
      const int k = tid >> 3, i = tid & 7;
      out->chroma[k][i] = i < (1 << k) ? i : -1;
      if (i == 0) out->dist_chroma[k] = 0;
    }
    return;
  }
  const int per = (nfb + G - 1) / G;
  const int b0 = min(nfb, w * per), cnt = min(nfb, b0 + per) - b0;

  if (LDS) {
    for (int i = tid; i < cnt * NC; i += kNT)
      sm.d[i / NC][i % NC] = group_dist<NC>(sse, nfb, g, b0 + i / NC, i % NC);
  }
  if (tid == 0) {
    sm.step = 0;
    for (int r = 0; r < 3; ++r) sm.done[r] = 0;
  }
  __syncthreads();

  for (uint32_t round = 0;; ++round) {
    // ---- the candidate sets evaluated in this round
    if (tid == 0) {
      int nq = 0;
      if (sm.step < 8) {
        Query &q = sm.q[0];
        for (int i = 0; i < 8; ++i) q.set[i] = sm.greedy[i];
        q.n = sm.step;
        q.excl = -1;
        sm.qowner[0] = -1;
        nq = 1;
      } else {
        for (int r = 0; r < 3; ++r) {
          if (sm.done[r]) continue;
          Query &q = sm.q[nq];
          for (int i = 0; i < 8; ++i) q.set[i] = sm.rset[r][i];
          q.n = 2 << r;
          q.excl = sm.slot[r];
          sm.qowner[nq] = r;
          ++nq;
        }
      }
      sm.nq = nq;
    }
    __syncthreads();
    const int nq = sm.nq;
    if (nq == 0) break;

    // ---- partial sums: thread (candidate pc, row) over blocks row, row + R, ...
    uint64_t acc[kQ] = {0, 0, 0};
    if (LDS) {
      for (int i = tid; i < nq * cnt; i += kNT) {
        const int s = i / cnt, bl = i - s * cnt;
        const Query &q = sm.q[s];
        uint64_t mm = UINT64_MAX;
        for (int k = 0; k < q.n; ++k) {
          if (k == q.excl) continue;
          const uint64_t d = sm.d[bl][q.set[k]];
          mm = d < mm ? d : mm;
        }
        sm.m[s][bl] = mm;
      }
      __syncthreads();
      for (int bl = row; bl < cnt; bl += R) {
        const uint64_t d = sm.d[bl][pc];
#pragma unroll
        for (int s = 0; s < kQ; ++s) {
          if (s < nq) {
            const uint64_t mm = sm.m[s][bl];
            acc[s] += d < mm ? d : mm;
          }
        }
      }
    } else {
      for (int bl = row; bl < cnt; bl += R) {
        const uint64_t d = group_dist<NC>(sse, nfb, g, b0 + bl, pc);
        for (int s = 0; s < nq; ++s) {
          const Query &q = sm.q[s];
          uint64_t mm = UINT64_MAX;
          for (int k = 0; k < q.n; ++k) {
            if (k == q.excl) continue;
            const uint64_t e = group_dist<NC>(sse, nfb, g, b0 + bl, q.set[k]);
            mm = e < mm ? e : mm;
          }
          acc[s] += d < mm ? d : mm;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kQ; ++s) sm.red[row][s][pc] = acc[s];
    __syncthreads();
    if (!round_totals<NC>(sm, work, g, G, nq, round)) return;

    // ---- one decision per candidate set: wave s scans the NC candidates,
    // NC / 64 per lane
    if (wave < nq) {
      const Query &q = sm.q[wave];
      uint64_t c = UINT64_MAX;
      int p = NC;
#pragma unroll
      for (int h = 0; h < NC / 64; ++h) {
        const int cand = lane + 64 * h;
        if (!excluded(q, cand) && cm.allowed(cand)) argmin2(c, p, sm.cost[wave][cand], cand);
      }
      wave_argmin(c, p);
      if (lane == 0) {
        sm.best_cost[wave] = c;
        sm.best_p[wave] = p;
      }
    }
    __syncthreads();

    // ---- state update (thread 0; every workgroup does the same)
    if (tid == 0) {
      if (sm.step < 8) {
        sm.greedy[sm.step] = sm.best_p[0];
        sm.greedy_cost[sm.step] = sm.best_cost[0];
        if (++sm.step == 8) {
          for (int r = 0; r < 3; ++r) {
            const int n = 2 << r;
            for (int i = 0; i < 8; ++i) sm.rset[r][i] = i < n ? sm.greedy[i] : -1;
            sm.slot[r] = sm.pass[r] = sm.changed[r] = 0;
            sm.rdist[r] = sm.greedy_cost[n - 1];
            sm.done[r] = refine == 0;
          }
        }
      } else {
        for (int s = 0; s < nq; ++s) {
          const int r = sm.qowner[s], n = 2 << r, i = sm.slot[r];
          const uint64_t cur = sm.cost[s][sm.rset[r][i]];
          if (sm.best_cost[s] < cur) {
            sm.rset[r][i] = sm.best_p[s];
            sm.changed[r] = 1;
            sm.rdist[r] = sm.best_cost[s];
          } else {
            sm.rdist[r] = cur;
          }
          if (++sm.slot[r] == n) {
            sm.slot[r] = 0;
            ++sm.pass[r];
            if (!sm.changed[r] || sm.pass[r] == refine) sm.done[r] = 1;
            sm.changed[r] = 0;
          }
        }
      }
    }
    __syncthreads();
  }

  if (w == 0 && tid == 0) {
    int32_t *sets = g == 0 ? &out->luma[0][0] : &out->chroma[0][0];
    uint64_t *dist = g == 0 ? out->dist_luma : out->dist_chroma;
    sets[0] = sm.greedy[0];
    for (int i = 1; i < 8; ++i) sets[i] = -1;
    dist[0] = sm.greedy_cost[0];
    for (int r = 0; r < 3; ++r) {
      for (int i = 0; i < 8; ++i) sets[(r + 1) * 8 + i] = sm.rset[r][i];
      dist[r + 1] = sm.rdist[r];
    }
  }
}

// Counters and the totals of rounds 0 and 1 start at zero.
__global__ void k_preset_reset(PresetWork *work) {
  const int t = threadIdx.x;
  if (t < 2) work->arrive[t] = 0;
  if (t == 0) work->failed = 0;
  uint64_t *tot = &work->total[0][0][0][0];
  for (int i = t; i < 2 * 2 * kQ * kMaxNC; i += blockDim.x) tot[i] = 0;
}

template <int NC>
__global__ __launch_bounds__(kNT) void k_preset_finish(const uint64_t *__restrict__ sse,
                                                       int nplanes, int nfb, double lambda,
                                                       const PresetWork *work, PresetResult *out,
                                                       uint8_t *fb_luma, uint8_t *fb_chroma) {
  __shared__ int chosen;
  if (work->failed) {
    if (blockIdx.x == 0 && threadIdx.x == 0) out->n = 0;
    return;
  }
  if (threadIdx.x == 0) {
    // J(N) is evaluated as written, one rounding per operation (no fused
    // multiply-add), so that equal inputs give the same choice everywhere.
#pragma clang fp contract(off)
    double cost[4];
    int c = 0;
    for (int k = 0; k < 4; ++k) {
      cost[k] = lambda * (double)nfb * (double)k +
                (double)(out->dist_luma[k] + out->dist_chroma[k]);
      if (cost[k] < cost[c]) c = k;
    }
    if (blockIdx.x == 0) {
      for (int k = 0; k < 4; ++k) out->cost[k] = cost[k];
      out->n = 1 << c;
      out->reserved = 0;
    }
    chosen = c;
  }
  __syncthreads();
  const int c = chosen, n = 1 << c;
  const int b = blockIdx.x * kNT + threadIdx.x;
  if (b >= nfb) return;
  for (int g = 0; g < 2; ++g) {
    const int32_t *sets = g == 0 ? &out->luma[c][0] : &out->chroma[c][0];
    int bi = 0;
    if (g == 0 || nplanes == 3) {
      uint64_t bd = UINT64_MAX;
      for (int i = 0; i < n; ++i) {
        const uint64_t d = group_dist<NC>(sse, nfb, g, b, sets[i]);
        if (d < bd) {
          bd = d;
          bi = i;
        }
      }
    }
    (g == 0 ? fb_luma : fb_chroma)[b] = (uint8_t)bi;
  }
}

}  // namespace

size_t preset_workspace_bytes() { return sizeof(PresetWork); }

// Workspace of the allocation-free selection (cdef_select_presets_noalloc):
// a file-scope device array instead of caller memory.  Every device holds
// its own copy, at its own address, until the process ends.  On the host
// the array's name is only a stand-in for the symbol: kernels get the
// address hipGetSymbolAddress returns for the device, never the name.
static_assert(sizeof(PresetWork) <= kPresetScratchBytes, "selection workspace exceeds scratch");
static __device__ __align__(256) unsigned char scratch[kPresetScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

hipError_t preset_scratch(hipStream_t s, void **ptr) {
  int dev = 0;
  hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    // the symbol's address on `dev`, looked up with `dev` current
    int cur = 0;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (((uintptr_t)p & 255) != 0) return hipErrorInvalidValue;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

namespace {

template <int NC>
hipError_t select_presets_nc(const uint64_t *sse, int nplanes, int nfb, CandMask cm,
                             double lambda, int refine, PresetResult *out, uint8_t *fb_luma,
                             uint8_t *fb_chroma, PresetWork *work, hipStream_t s) {
  constexpr int kSlice = slice_blocks<NC>();
  const int G = min(kMaxG, (nfb + kSlice - 1) / kSlice);
  const int per = (nfb + G - 1) / G;
  hipLaunchKernelGGL(k_preset_reset, dim3(1), dim3(256), 0, s, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // 2 G <= 256 workgroups of 256 threads: all of them fit on the device at
  // once, so every wait for the last arrival of a round ends.
  if (per <= kSlice)
    hipLaunchKernelGGL((k_preset_coop<NC, true>), dim3(2 * G), dim3(kNT), 0, s, sse, nplanes, nfb,
                       G, refine, cm, work, out);
  else
    hipLaunchKernelGGL((k_preset_coop<NC, false>), dim3(2 * G), dim3(kNT), 0, s, sse, nplanes,
                       nfb, G, refine, cm, work, out);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_preset_finish<NC>, dim3((nfb + kNT - 1) / kNT), dim3(kNT), 0, s, sse,
                     nplanes, nfb, lambda, work, out, fb_luma, fb_chroma);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_select_presets(const uint64_t *sse, int nplanes, int nfb, int ncand,
                                 const uint64_t mask[2], double lambda, int refine,
                                 PresetResult *out, uint8_t *fb_luma, uint8_t *fb_chroma,
                                 void *workspace, hipStream_t s) {
  PresetWork *work = static_cast<PresetWork *>(workspace);
  const CandMask cm{{mask[0], mask[1]}};
  if (ncand == 128)
    return select_presets_nc<128>(sse, nplanes, nfb, cm, lambda, refine, out, fb_luma, fb_chroma,
                                  work, s);
  return select_presets_nc<64>(sse, nplanes, nfb, cm, lambda, refine, out, fb_luma, fb_chroma,
                               work, s);
}

}  // namespace cdef
