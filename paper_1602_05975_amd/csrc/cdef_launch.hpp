// Host-side launch wrappers shared by the C ABI (cdef_api.hip) and the
// kernels' translation units.  Arguments are validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdef {

// Chroma layouts (the values of CDEF_LAYOUT_*).
enum Layout : int32_t { kLayout400 = 0, kLayout420 = 1, kLayout422 = 2, kLayout444 = 3 };

struct FrameDesc {
  const uint16_t *plane[3];
  int64_t stride[3];
  int width, height;  // luma
  int bitdepth;       // 8, 10 or 12
  int nplanes;        // 1 (4:0:0) or 3
  int layout;
};

enum JobMode : int32_t {
  kModeSearch = 0,
  kModeFilter = 1,
  kModeSearchFull = 2,
  kModeSearchWeighted = 3
};
// kDirIn: filter mode takes dir / var as inputs (cdef_filter_frame) instead
// of running the direction search and optionally writing them.
// kAligned16: every plane the job reads has a 16-byte aligned base and row
// pitch, and a pitch below kPitch16Max samples.
// kOut16: the same for filter mode's output planes.
enum JobFlags : int32_t { kAligned16 = 1, kDirIn = 2, kOut16 = 4 };
// Pitch limit of the 16-byte paths: 68 rows of a tile then span less than
// 2^31 bytes and a row offset is a 24-bit product (samples, 2 bytes each).
constexpr int32_t kPitch16Max = 1 << 23;

// One frame of work as the fused kernel reads it (kernel argument for a
// single frame, or an element of a device-resident table for a batch).
// Strides are in samples and fit 32 bits (frames are at most 65536 wide).
struct JobDesc {
  const uint16_t *rec[3];
  const uint16_t *src[3];  // search mode
  uint16_t *out[3];        // filter mode
  const uint8_t *skip;     // may be null
  const uint8_t *strengths;  // filter mode: [fbr][fbc][4]
  uint64_t *sse;           // search modes: [nplanes][fbr][fbc][64] (full: [..][2][64];
                           // weighted: double [..][64])
  uint8_t *dir;            // optional outputs (inputs with kDirIn)
  int32_t *var;
  int32_t rstride[3], sstride[3], ostride[3];
  int32_t width, height, bitdepth, damping, nplanes, mode;
  int32_t fbc, fbr, bcols, brows;
  int32_t item0;  // first work item (filter block) of this job in the batch
  int32_t flags;  // JobFlags
  int32_t layout;
  uint32_t cand;  // searches: preset subset (S^(p) | S^(s) << 16 | skip bit << 20), 0 = all
};

hipError_t launch_find_dir(const FrameDesc &f, uint8_t *dir, int32_t *var, hipStream_t s);

// One frame, job descriptor passed by value.
hipError_t launch_fused_one(const JobDesc &job, hipStream_t s);

// Many frames: `jobs` is a device array of njobs descriptors (item0 set),
// nitems the total number of filter blocks.
// extended: some job needs the extended kernels (4:4:4);
// filter_only: every job is a filter job (the filter-only kernels run it).
// Work-queue counters of the persistent batch kernels, in the caller's
// workspace after the job table: next[x][0] counts the items claimed from
// XCD x's range, done[0] the workgroups that have left; each on its own
// 128-byte line.  Zero before a launch; the last workgroup to leave sets
// them back to zero.
struct BatchQueue {
  uint32_t next[8][32];
  uint32_t done[32];
};
// Byte offset of the queue in a batch workspace of njobs descriptors.
inline size_t batch_queue_offset(int njobs) {
  return ((size_t)njobs * sizeof(JobDesc) + 255) & ~(size_t)255;
}

// variant: 0..3 flat grids (see cdef.h), 4 / 5 persistent workgroups at 3 /
// 2 waves per SIMD taking items from `queue`.
hipError_t launch_fused_batch(const JobDesc *jobs, int njobs, int nitems, int variant,
                              bool extended, bool filter_only, BatchQueue *queue,
                              hipStream_t s);
bool job_needs_extended(const JobDesc &j);

// The kernels behind launch_fused_one / launch_fused_batch, built in sets of
// one translation unit each.  Batch kernels: base3 / base2 = base LDS layout
// at 3 / 2 waves per SIMD, ext = extended layout; _xcd = XCD-contiguous
// filter-block order, _seq = plain order.
hipError_t launch_one_ext(const JobDesc &job, hipStream_t s);
hipError_t launch_filter_one(const JobDesc &job, bool extended, hipStream_t s);
hipError_t launch_filter_batch(bool extended, const JobDesc *jobs, int njobs, int nitems,
                               hipStream_t s);
hipError_t launch_batch_base3_xcd(const JobDesc *jobs, int njobs, int nitems, hipStream_t s);
hipError_t launch_batch_base3_seq(const JobDesc *jobs, int njobs, int nitems, hipStream_t s);
hipError_t launch_batch_base2_xcd(const JobDesc *jobs, int njobs, int nitems, hipStream_t s);
hipError_t launch_batch_base2_seq(const JobDesc *jobs, int njobs, int nitems, hipStream_t s);
hipError_t launch_batch_ext_xcd(const JobDesc *jobs, int njobs, int nitems, hipStream_t s);
hipError_t launch_batch_ext_seq(const JobDesc *jobs, int njobs, int nitems, hipStream_t s);
hipError_t launch_batch_queue_base(int occ, const JobDesc *jobs, int njobs, int nitems,
                                   BatchQueue *queue, hipStream_t s);
hipError_t launch_batch_queue_ext(const JobDesc *jobs, int njobs, int nitems, BatchQueue *queue,
                                  hipStream_t s);

void fill_job_geometry(JobDesc &j);

// Result of the preset selection; same layout as cdef_preset_result.
struct PresetResult {
  int32_t n, reserved;
  int32_t luma[4][8], chroma[4][8];
  uint64_t dist_luma[4], dist_chroma[4];
  double cost[4];
};

size_t preset_workspace_bytes();
hipError_t launch_select_presets(const uint64_t *sse, int nplanes, int nfb, int ncand,
                                 const uint64_t mask[2], double lambda, int refine,
                                 PresetResult *out, uint8_t *fb_luma, uint8_t *fb_chroma,
                                 void *workspace, hipStream_t s);

// The library-owned workspace of the allocation-free selection: bytes of
// device memory it holds per device, and its address on the device of
// stream `s` (looked up on the first call for that device).
constexpr size_t kPresetScratchBytes = 20480;
hipError_t preset_scratch(hipStream_t s, void **ptr);

}  // namespace cdef
