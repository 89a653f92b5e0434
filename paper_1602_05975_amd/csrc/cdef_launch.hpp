// Host-side launch wrappers shared by the C ABI (cdef_api.hip) and the
// kernels' translation units.  Arguments are validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdef {

struct FrameDesc {
  const uint16_t *plane[3];
  int64_t stride[3];
  int width, height;  // luma
  int bitdepth;       // 8 or 10
  int nplanes;        // 1 (4:0:0) or 3 (4:2:0)
};

hipError_t launch_find_dir(const FrameDesc &f, uint8_t *dir, int32_t *var, hipStream_t s);

hipError_t launch_filter(const FrameDesc &in, uint16_t *const out[3], const int64_t out_stride[3],
                         const uint8_t *dir, const int32_t *var, const uint8_t *skip, int damping,
                         const uint8_t *strengths, hipStream_t s);

hipError_t launch_search(const FrameDesc &rec, const FrameDesc &src, const uint8_t *skip,
                         int damping, uint64_t *sse, uint8_t *dir, int32_t *var, hipStream_t s);

}  // namespace cdef
