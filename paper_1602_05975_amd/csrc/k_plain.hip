// The stand-alone direction search (Section 2, Algorithm 1), one thread per
// 8x8 luma block.  The frame filter (cdef_filter_frame) runs on the fused
// kernel's filter mode with the caller's directions.
#include "cdef_device.hpp"
#include "cdef_launch.hpp"

namespace cdef {

// Two raw samples of a row as one word (low half: the left one).
__device__ __forceinline__ uint32_t pair_at(const uint16_t *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 16);
}

// One thread per 8x8 luma block.  A whole block reads its rows as 16-byte
// loads when they are 16-byte aligned (as 4-byte ones when 4-byte
// aligned); a block cut by the frame edge reads only its in-frame samples.
template <int BD>
__global__ __launch_bounds__(256) void k_find_dir(const uint16_t *__restrict__ luma,
                                                  int64_t stride, int w, int h, int bcols,
                                                  int nblocks, uint8_t *__restrict__ dir,
                                                  int32_t *__restrict__ var) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= nblocks) return;
  const int by = b / bcols, bx = b - by * bcols;
  const int bw = min(8, w - 8 * bx), bh = min(8, h - 8 * by);
  const uint16_t *p = luma + (int64_t)8 * by * stride + 8 * bx;
  constexpr int c = BD - 8;
  uint32_t x[32];
  int cost[8];
  if (bw == 8 && bh == 8) {
    const bool a16 = (((uintptr_t)p | (uintptr_t)(stride * 2)) & 15) == 0;
    const bool a4 = (((uintptr_t)p | (uintptr_t)(stride * 2)) & 3) == 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint16_t *r = p + i * stride;
      uint32_t q[4];
      if (a16) {
        const uint4 v = *reinterpret_cast<const uint4 *>(r);
        q[0] = v.x, q[1] = v.y, q[2] = v.z, q[3] = v.w;
      } else if (a4) {
#pragma unroll
        for (int m = 0; m < 4; ++m) q[m] = reinterpret_cast<const uint32_t *>(r)[m];
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) q[m] = pair_at(r + 2 * m);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) x[4 * i + m] = centre_word(q[m], c);
    }
    dir_costs_packed<false>(x, 8, 8, cost);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int j = 2 * m;
        const uint32_t lo = (i < bh && j < bw) ? p[i * stride + j] : 0u;
        const uint32_t hi = (i < bh && j + 1 < bw) ? p[i * stride + j + 1] : 0u;
        x[4 * i + m] = mask_word(centre_word(lo | (hi << 16), c), i, m, bw, bh);
      }
    dir_costs_packed<true>(x, bw, bh, cost);
  }
  int d, v;
  pick_direction(cost, d, v);
  dir[b] = (uint8_t)d;
  var[b] = v;
}

hipError_t launch_find_dir(const FrameDesc &f, uint8_t *dir, int32_t *var, hipStream_t s) {
  const int bcols = (f.width + 7) / 8, brows = (f.height + 7) / 8;
  const int nb = bcols * brows;
  const int grid = (nb + 255) / 256;
  if (f.bitdepth == 8)
    hipLaunchKernelGGL(k_find_dir<8>, dim3(grid), dim3(256), 0, s, f.plane[0], f.stride[0],
                       f.width, f.height, bcols, nb, dir, var);
  else if (f.bitdepth == 10)
    hipLaunchKernelGGL(k_find_dir<10>, dim3(grid), dim3(256), 0, s, f.plane[0], f.stride[0],
                       f.width, f.height, bcols, nb, dir, var);
  else
    hipLaunchKernelGGL(k_find_dir<12>, dim3(grid), dim3(256), 0, s, f.plane[0], f.stride[0],
                       f.width, f.height, bcols, nb, dir, var);
  return hipGetLastError();
}

}  // namespace cdef
