// The stand-alone direction search (Section 2, Algorithm 1), one thread per
// 8x8 luma block.  The frame filter (cdef_filter_frame) runs on the fused
// kernel's filter mode with the caller's directions.
#include "cdef_device.hpp"
#include "cdef_launch.hpp"

namespace cdef {

// One thread per 8x8 luma block.
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
  int x[64];
  int cost[8];
  if (bw == 8 && bh == 8) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) x[i * 8 + j] = (int)(p[i * stride + j] >> (BD - 8)) - 128;
    dir_costs_full(x, cost);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        x[i * 8 + j] = (i < bh && j < bw) ? (int)(p[i * stride + j] >> (BD - 8)) - 128 : 0;
    dir_costs_partial(x, bw, bh, cost);
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
