// C ABI of the gfx950 CDEF library: argument checks on the host, then one
// kernel launch per call.  See include/cdef.h for the contract of each entry
// point.
#include "../../include/cdef.h"
#include "cdef_launch.hpp"

#include <stdint.h>

namespace {

using cdef::FrameDesc;

bool ranges_overlap(const void *a, size_t an, const void *b, size_t bn) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bn && b0 < a0 + an;
}

int nplanes_of(int32_t layout) { return layout == CDEF_LAYOUT_420 ? 3 : 1; }

void plane_dims(const cdef_frame *f, int p, int *w, int *h) {
  *w = p == 0 ? f->width : (f->width + 1) / 2;
  *h = p == 0 ? f->height : (f->height + 1) / 2;
}

size_t plane_bytes(const cdef_frame *f, int p) {
  int w, h;
  plane_dims(f, p, &w, &h);
  return ((size_t)(h - 1) * (size_t)f->stride[p] + (size_t)w) * sizeof(uint16_t);
}

// Checks shared by every entry point; fills `d` on success.
cdef_status check_frame(const cdef_frame *f, FrameDesc *d) {
  if (!f) return CDEF_E_INVAL;
  if (f->layout != CDEF_LAYOUT_400 && f->layout != CDEF_LAYOUT_420) return CDEF_E_INVAL;
  if (f->width < 1 || f->height < 1) return CDEF_E_INVAL;
  if (f->width > (1 << 16) || f->height > (1 << 16)) return CDEF_E_UNSUPPORTED;
  if (f->bitdepth == 12) return CDEF_E_UNSUPPORTED;
  if (f->bitdepth != 8 && f->bitdepth != 10) return CDEF_E_INVAL;
  const int np = nplanes_of(f->layout);
  for (int p = 0; p < np; ++p) {
    int w, h;
    plane_dims(f, p, &w, &h);
    if (!f->plane[p]) return CDEF_E_INVAL;
    if (f->stride[p] < w) return CDEF_E_INVAL;
  }
  for (int p = 0; p < 3; ++p) {
    d->plane[p] = p < np ? f->plane[p] : nullptr;
    d->stride[p] = p < np ? f->stride[p] : 0;
  }
  d->width = f->width;
  d->height = f->height;
  d->bitdepth = f->bitdepth;
  d->nplanes = np;
  return CDEF_OK;
}

cdef_status from_hip(hipError_t e) { return e == hipSuccess ? CDEF_OK : CDEF_E_HIP; }

bool same_geometry(const cdef_frame *a, const cdef_frame *b) {
  return a->width == b->width && a->height == b->height && a->bitdepth == b->bitdepth &&
         a->layout == b->layout;
}

}  // namespace

extern "C" {

cdef_status cdef_find_dir(const cdef_frame *f, uint8_t *dir, int32_t *var, void *stream) {
  FrameDesc d;
  const cdef_status st = check_frame(f, &d);
  if (st != CDEF_OK) return st;
  if (!dir || !var) return CDEF_E_INVAL;
  return from_hip(cdef::launch_find_dir(d, dir, var, (hipStream_t)stream));
}

cdef_status cdef_filter_frame(const cdef_frame *in, const cdef_frame_out *out, const uint8_t *dir,
                              const int32_t *var, const uint8_t *skip8x8, int32_t damping,
                              const cdef_strength *fb, void *stream) {
  FrameDesc d;
  const cdef_status st = check_frame(in, &d);
  if (st != CDEF_OK) return st;
  if (!out || !dir || !var || !fb) return CDEF_E_INVAL;
  if (damping < 3 || damping > 6) return CDEF_E_INVAL;
  uint16_t *outp[3] = {nullptr, nullptr, nullptr};
  int64_t outs[3] = {0, 0, 0};
  for (int p = 0; p < d.nplanes; ++p) {
    int w, h;
    plane_dims(in, p, &w, &h);
    if (!out->plane[p] || out->stride[p] < w) return CDEF_E_INVAL;
    cdef_frame o = *in;
    o.stride[p] = out->stride[p];
    for (int q = 0; q < d.nplanes; ++q)
      if (ranges_overlap(out->plane[p], plane_bytes(&o, p), in->plane[q], plane_bytes(in, q)))
        return CDEF_E_INVAL;
    outp[p] = out->plane[p];
    outs[p] = out->stride[p];
  }
  return from_hip(cdef::launch_filter(d, outp, outs, dir, var, skip8x8, damping,
                                      reinterpret_cast<const uint8_t *>(fb),
                                      (hipStream_t)stream));
}

cdef_status cdef_search_strengths(const cdef_frame *recon, const cdef_frame *src,
                                  const uint8_t *skip8x8, int32_t damping, uint64_t *sse,
                                  uint8_t *dir, int32_t *var, void *stream) {
  FrameDesc r, s;
  cdef_status st = check_frame(recon, &r);
  if (st != CDEF_OK) return st;
  st = check_frame(src, &s);
  if (st != CDEF_OK) return st;
  if (!same_geometry(recon, src)) return CDEF_E_INVAL;
  if (!sse) return CDEF_E_INVAL;
  if ((dir == nullptr) != (var == nullptr)) return CDEF_E_INVAL;
  if (damping < 3 || damping > 6) return CDEF_E_INVAL;
  return from_hip(cdef::launch_search(r, s, skip8x8, damping, sse, dir, var, (hipStream_t)stream));
}

const char *cdef_status_str(cdef_status s) {
  switch (s) {
    case CDEF_OK: return "ok";
    case CDEF_E_INVAL: return "invalid argument";
    case CDEF_E_UNSUPPORTED: return "unsupported input";
    case CDEF_E_HIP: return "HIP runtime error";
    case CDEF_E_NOMEM: return "workspace too small";
  }
  return "unknown status";
}

int32_t cdef_abi_version(void) { return CDEF_ABI_VERSION; }

}  // extern "C"
