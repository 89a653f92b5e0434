// Plain (one strength set per filter block) path: the stand-alone direction
// search and the frame filter.
//
// Direction search: Section 2, Algorithm 1.  Filter: Section 3, Eq. (7)-(13);
// filter blocks and skip: Section 4.
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

struct FilterArgs {
  const uint16_t *in[3];
  int64_t istride[3];
  uint16_t *out[3];
  int64_t ostride[3];
  int width, height, nplanes, layout;
  int bcols, fbc;
  int damping;
  const uint8_t *dir;
  const int32_t *var;
  const uint8_t *skip;
  const uint8_t *strengths;  // [fbr][fbc][4]
};

constexpr int kLS = 80;  // luma tile row stride (68 used)
constexpr int kLC0 = 8;  // tile column of frame column x0
constexpr int kCS = 48;  // chroma tile row stride (36 used)
constexpr int kCC0 = 8;

// One workgroup per 64x64 filter block; every pixel reads unfiltered input
// from the LDS tile, so no ordering between blocks matters.  Section 4: a
// skipped 8x8 block is filtered only under a preset with the skip condition
// bit, and a filter block whose blocks are all skipped is not filtered.
template <int BD>
__global__ __launch_bounds__(256) void k_filter(const FilterArgs a) {
  __shared__ __align__(16) uint16_t ry[68 * kLS];
  __shared__ __align__(16) uint16_t rc[68 * kLS];  // one chroma plane (4:4:4 size)
  // per 8x8 block: dir, primary strength, primary shift, w1 | w2 << 8,
  // skipped, secondary shift (luma)
  __shared__ int s_par[64][6];
  constexpr int c = BD - 8;
  const int tid = threadIdx.x;
  const int fby = blockIdx.x / a.fbc, fbx = blockIdx.x - fby * a.fbc;
  const int y0 = fby * 64, x0 = fbx * 64;
  const int W = a.width, H = a.height;
  const uint8_t *st = a.strengths + 4 * blockIdx.x;
  const Preset py = decode_preset(st[0], st[1]);
  const Preset pc = decode_preset(st[2], st[3]);
  const int D = a.damping;

  stage_recon<64, 64, kLS, kLC0, 256>(ry, a.in[0], a.istride[0], W, H, y0, x0, tid);
  int active = 0;
  if (tid < 64) {
    const int by = fby * 8 + (tid >> 3), bx = fbx * 8 + (tid & 7);
    int d = 0, sk = 1, v = 0;
    if (by * 8 < H && bx * 8 < W) {
      const int b = by * a.bcols + bx;
      d = a.dir[b];
      v = a.var[b];
      sk = a.skip ? (a.skip[b] != 0) : 0;
      active = !sk;
    }
    const int adj = adjust_strength(py.pri, v);  // Eq. (13)
    const int Dl = luma_damping(D, adj);
    s_par[tid][0] = d & 7;
    s_par[tid][1] = adj << c;
    s_par[tid][2] = adj ? Dl - floor_log2(adj) : 0;
    s_par[tid][3] = (adj & 1) ? (3 | (3 << 8)) : (4 | (2 << 8));
    s_par[tid][4] = sk;
    s_par[tid][5] = py.sec ? Dl - floor_log2(py.sec) : 0;
  }
  // a filter block with no block left to filter is copied
  const bool fb_skipped = !__syncthreads_or(active);
  {
    const int ss = py.sec << c;
    for (int e = tid; e < 64 * 64; e += 256) {
      const int r = e >> 6, col = e & 63;
      if (y0 + r >= H || x0 + col >= W) continue;
      const int b = (r >> 3) * 8 + (col >> 3);
      const int base = (r + 2) * kLS + kLC0 + col;
      int y;
      if (fb_skipped || (s_par[b][4] && !py.skipcond)) {
        y = ry[base];
      } else {
        const int w12 = s_par[b][3];
        y = filter_pixel(ry, base, kLS, s_par[b][0], s_par[b][1], s_par[b][2], w12 & 255,
                         w12 >> 8, ss, s_par[b][5]);
      }
      a.out[0][(int64_t)(y0 + r) * a.ostride[0] + x0 + col] = (uint16_t)y;
    }
  }
  if (a.nplanes == 1) return;
  if (a.layout == kLayout422) {
    // Section 4: chroma subsampled horizontally only is never filtered
    const int cw = (W + 1) >> 1, cx0 = x0 >> 1;
    for (int p = 1; p < 3; ++p)
      for (int e = tid; e < 64 * 32; e += 256) {
        const int r = e >> 5, col = e & 31;
        if (y0 + r >= H || cx0 + col >= cw) continue;
        a.out[p][(int64_t)(y0 + r) * a.ostride[p] + cx0 + col] =
            a.in[p][(int64_t)(y0 + r) * a.istride[p] + cx0 + col];
      }
    return;
  }
  // Chroma: unadjusted strength, damping max(D - 1, floor(log2 S)); 4:2:0
  // 4x4 blocks in a 32x32 filter block, 4:4:4 8x8 blocks in 64x64.
  const int Dc = pc.pri ? max(D - 1, floor_log2(pc.pri)) : D - 1;
  const int ps = pc.pri << c, pshift = pc.pri ? Dc - floor_log2(pc.pri) : 0;
  const int w1 = (pc.pri & 1) ? 3 : 4, w2 = (pc.pri & 1) ? 3 : 2;
  const int ss = pc.sec << c, sshift = pc.sec ? Dc - floor_log2(pc.sec) : 0;
  const bool c444 = a.layout == kLayout444;
  const int sh = c444 ? 0 : 1;  // subsampling shift
  const int cw = (W + sh) >> sh, ch = (H + sh) >> sh, cy0 = y0 >> sh, cx0 = x0 >> sh;
  const int side = 64 >> sh, bsh = 3 - sh;  // filter block side, log2 block side
  const int ts = c444 ? kLS : kCS, t0 = c444 ? kLC0 : kCC0;
  for (int p = 1; p < 3; ++p) {
    __syncthreads();
    if (c444)
      stage_recon<64, 64, kLS, kLC0, 256>(rc, a.in[p], a.istride[p], cw, ch, cy0, cx0, tid);
    else
      stage_recon<32, 32, kCS, kCC0, 256>(rc, a.in[p], a.istride[p], cw, ch, cy0, cx0, tid);
    __syncthreads();
    for (int e = tid; e < side * side; e += 256) {
      const int r = e / side, col = e - r * side;
      if (cy0 + r >= ch || cx0 + col >= cw) continue;
      const int b = (r >> bsh) * 8 + (col >> bsh);
      const int base = (r + 2) * ts + t0 + col;
      const int y = (fb_skipped || (s_par[b][4] && !pc.skipcond))
                        ? (int)rc[base]
                        : filter_pixel(rc, base, ts, s_par[b][0], ps, pshift, w1, w2, ss, sshift);
      a.out[p][(int64_t)(cy0 + r) * a.ostride[p] + cx0 + col] = (uint16_t)y;
    }
  }
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

hipError_t launch_filter(const FrameDesc &in, uint16_t *const out[3], const int64_t out_stride[3],
                         const uint8_t *dir, const int32_t *var, const uint8_t *skip, int damping,
                         const uint8_t *strengths, hipStream_t s) {
  FilterArgs a{};
  for (int p = 0; p < 3; ++p) {
    a.in[p] = in.plane[p];
    a.istride[p] = in.stride[p];
    a.out[p] = out[p];
    a.ostride[p] = out_stride[p];
  }
  a.width = in.width;
  a.height = in.height;
  a.nplanes = in.nplanes;
  a.layout = in.layout;
  a.bcols = (in.width + 7) / 8;
  a.fbc = (in.width + 63) / 64;
  a.damping = damping;
  a.dir = dir;
  a.var = var;
  a.skip = skip;
  a.strengths = strengths;
  const int grid = a.fbc * ((in.height + 63) / 64);
  if (in.bitdepth == 8)
    hipLaunchKernelGGL(k_filter<8>, dim3(grid), dim3(256), 0, s, a);
  else if (in.bitdepth == 10)
    hipLaunchKernelGGL(k_filter<10>, dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_filter<12>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace cdef
