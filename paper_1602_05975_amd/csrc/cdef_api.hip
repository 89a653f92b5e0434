// C ABI of the gfx950 CDEF library: argument checks on the host, then one
// kernel launch per call.  See include/cdef.h for the contract of each entry
// point.
#include "cdef.h"
#include "cdef_launch.hpp"

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static_assert(sizeof(cdef_preset_result) == sizeof(cdef::PresetResult), "preset result layout");
static_assert(offsetof(cdef_preset_result, cost) == offsetof(cdef::PresetResult, cost),
              "preset result layout");
static_assert(CDEF_PRESET_SCRATCH_BYTES == cdef::kPresetScratchBytes, "preset scratch size");
static_assert(CDEF_LAYOUT_400 == cdef::kLayout400 && CDEF_LAYOUT_420 == cdef::kLayout420 &&
                  CDEF_LAYOUT_422 == cdef::kLayout422 && CDEF_LAYOUT_444 == cdef::kLayout444,
              "layouts");
static_assert(CDEF_MODE_SEARCH == cdef::kModeSearch && CDEF_MODE_FILTER == cdef::kModeFilter &&
                  CDEF_MODE_SEARCH128 == cdef::kModeSearchFull &&
                  CDEF_MODE_SEARCH_WEIGHTED == cdef::kModeSearchWeighted,
              "job modes");

namespace {

using cdef::FrameDesc;

bool ranges_overlap(const void *a, size_t an, const void *b, size_t bn) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bn && b0 < a0 + an;
}

int nplanes_of(int32_t layout) { return layout == CDEF_LAYOUT_400 ? 1 : 3; }

// Chroma halves the width at 4:2:0 and 4:2:2, the height at 4:2:0.
void plane_dims(const cdef_frame *f, int p, int *w, int *h) {
  const int sx = p > 0 && (f->layout == CDEF_LAYOUT_420 || f->layout == CDEF_LAYOUT_422);
  const int sy = p > 0 && f->layout == CDEF_LAYOUT_420;
  *w = (f->width + sx) >> sx;
  *h = (f->height + sy) >> sy;
}

size_t plane_bytes(const cdef_frame *f, int p) {
  int w, h;
  plane_dims(f, p, &w, &h);
  return ((size_t)(h - 1) * (size_t)f->stride[p] + (size_t)w) * sizeof(uint16_t);
}

// Checks shared by every entry point; fills `d` on success.
cdef_status check_frame(const cdef_frame *f, FrameDesc *d) {
  if (!f) return CDEF_E_INVAL;
  if (f->layout < CDEF_LAYOUT_400 || f->layout > CDEF_LAYOUT_444) return CDEF_E_INVAL;
  if (f->width < 1 || f->height < 1) return CDEF_E_INVAL;
  if (f->width > (1 << 16) || f->height > (1 << 16)) return CDEF_E_UNSUPPORTED;
  if (f->bitdepth != 8 && f->bitdepth != 10 && f->bitdepth != 12) return CDEF_E_INVAL;
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
  d->layout = f->layout;
  return CDEF_OK;
}

cdef_status from_hip(hipError_t e) { return e == hipSuccess ? CDEF_OK : CDEF_E_HIP; }

bool same_geometry(const cdef_frame *a, const cdef_frame *b) {
  return a->width == b->width && a->height == b->height && a->bitdepth == b->bitdepth &&
         a->layout == b->layout;
}

bool stride32(int64_t s) { return s >= 0 && s <= INT32_MAX; }

// A preset subset: non-empty S^(p), S^(s) and skip-bit masks, no other
// bits; the skip condition bit only in the 128-combination search.
bool candidates_valid(uint32_t cand, int32_t mode) {
  if (cand >> 22) return false;
  if (!(cand & 0xFFFF) || !((cand >> 16) & 15) || !((cand >> 20) & 3)) return false;
  if (mode == CDEF_MODE_SEARCH) return ((cand >> 20) & 3) == 1;
  return mode == CDEF_MODE_SEARCH128;
}

// Host-side checks of one job plus its descriptor for the fused kernel.
cdef_status make_job(const cdef_job *j, cdef::JobDesc *o) {
  FrameDesc r;
  cdef_status st = check_frame(&j->recon, &r);
  if (st != CDEF_OK) return st;
  if (j->damping < 3 || j->damping > 6) return CDEF_E_INVAL;
  if (j->candidates && !candidates_valid(j->candidates, j->mode)) return CDEF_E_INVAL;
  if ((j->dir == nullptr) != (j->var == nullptr)) return CDEF_E_INVAL;
  memset(o, 0, sizeof(*o));
  for (int p = 0; p < r.nplanes; ++p) {
    if (!stride32(r.stride[p])) return CDEF_E_UNSUPPORTED;
    o->rec[p] = r.plane[p];
    o->rstride[p] = (int32_t)r.stride[p];
  }
  const bool search = j->mode == CDEF_MODE_SEARCH || j->mode == CDEF_MODE_SEARCH128 ||
                      j->mode == CDEF_MODE_SEARCH_WEIGHTED;
  if (search) {
    FrameDesc s;
    st = check_frame(&j->src, &s);
    if (st != CDEF_OK) return st;
    if (!same_geometry(&j->recon, &j->src) || !j->sse) return CDEF_E_INVAL;
    for (int p = 0; p < s.nplanes; ++p) {
      if (!stride32(s.stride[p])) return CDEF_E_UNSUPPORTED;
      o->src[p] = s.plane[p];
      o->sstride[p] = (int32_t)s.stride[p];
    }
  } else if (j->mode == CDEF_MODE_FILTER) {
    if (!j->fb) return CDEF_E_INVAL;
    for (int p = 0; p < r.nplanes; ++p) {
      int w, h;
      plane_dims(&j->recon, p, &w, &h);
      if (!j->out.plane[p] || j->out.stride[p] < w) return CDEF_E_INVAL;
      if (!stride32(j->out.stride[p])) return CDEF_E_UNSUPPORTED;
      cdef_frame o2 = j->recon;
      o2.stride[p] = j->out.stride[p];
      for (int q = 0; q < r.nplanes; ++q)
        if (ranges_overlap(j->out.plane[p], plane_bytes(&o2, p), j->recon.plane[q],
                           plane_bytes(&j->recon, q)))
          return CDEF_E_INVAL;
      o->out[p] = j->out.plane[p];
      o->ostride[p] = (int32_t)j->out.stride[p];
    }
  } else {
    return CDEF_E_INVAL;
  }
  o->skip = j->skip8x8;
  o->strengths = reinterpret_cast<const uint8_t *>(j->fb);
  o->sse = j->sse;
  o->dir = j->dir;
  o->var = j->var;
  o->width = r.width;
  o->height = r.height;
  o->bitdepth = r.bitdepth;
  o->damping = j->damping;
  o->nplanes = r.nplanes;
  o->layout = r.layout;
  o->mode = j->mode;
  o->cand = j->candidates;
  cdef::fill_job_geometry(*o);
  // 16-byte staging is possible when every plane read starts 16-byte aligned
  // and every row pitch keeps it so (and is small enough for the 32-bit row
  // offsets of that path)
  auto fits16 = [](const void *base, int32_t pitch) {
    return ((uintptr_t)base & 15) == 0 && (pitch & 7) == 0 && pitch < cdef::kPitch16Max;
  };
  bool al = true;
  for (int p = 0; p < r.nplanes; ++p) {
    al = al && fits16(o->rec[p], o->rstride[p]);
    if (search) al = al && fits16(o->src[p], o->sstride[p]);
  }
  o->flags = al ? cdef::kAligned16 : 0;
  if (j->mode == CDEF_MODE_FILTER) {
    bool ao = true;
    for (int p = 0; p < r.nplanes; ++p) ao = ao && fits16(o->out[p], o->ostride[p]);
    if (ao) o->flags |= cdef::kOut16;
  }
  return CDEF_OK;
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
  if (!in || !out || !dir || !var || !fb) return CDEF_E_INVAL;
  // the fused kernel's filter mode, with the caller's directions
  cdef_job j;
  memset(&j, 0, sizeof(j));
  j.recon = *in;
  j.out = *out;
  j.skip8x8 = skip8x8;
  j.fb = fb;
  j.dir = const_cast<uint8_t *>(dir);
  j.var = const_cast<int32_t *>(var);
  j.damping = damping;
  j.mode = CDEF_MODE_FILTER;
  cdef::JobDesc d;
  const cdef_status st = make_job(&j, &d);
  if (st != CDEF_OK) return st;
  d.flags |= cdef::kDirIn;
  return from_hip(cdef::launch_fused_one(d, (hipStream_t)stream));
}

namespace {

cdef_status search_one(const cdef_frame *recon, const cdef_frame *src, const uint8_t *skip8x8,
                       int32_t damping, uint64_t *sse, uint8_t *dir, int32_t *var, int32_t mode,
                       void *stream, uint32_t candidates = 0) {
  if (!recon || !src) return CDEF_E_INVAL;
  cdef_job j;
  memset(&j, 0, sizeof(j));
  j.recon = *recon;
  j.src = *src;
  j.skip8x8 = skip8x8;
  j.sse = sse;
  j.dir = dir;
  j.var = var;
  j.damping = damping;
  j.mode = mode;
  j.candidates = candidates;
  cdef::JobDesc d;
  const cdef_status st = make_job(&j, &d);
  if (st != CDEF_OK) return st;
  return from_hip(cdef::launch_fused_one(d, (hipStream_t)stream));
}

}  // namespace

cdef_status cdef_search_strengths(const cdef_frame *recon, const cdef_frame *src,
                                  const uint8_t *skip8x8, int32_t damping, uint64_t *sse,
                                  uint8_t *dir, int32_t *var, void *stream) {
  return search_one(recon, src, skip8x8, damping, sse, dir, var, CDEF_MODE_SEARCH, stream);
}

cdef_status cdef_search_strengths128(const cdef_frame *recon, const cdef_frame *src,
                                     const uint8_t *skip8x8, int32_t damping, uint64_t *sse,
                                     uint8_t *dir, int32_t *var, void *stream) {
  return search_one(recon, src, skip8x8, damping, sse, dir, var, CDEF_MODE_SEARCH128, stream);
}

cdef_status cdef_search_subset(const cdef_frame *recon, const cdef_frame *src,
                               const uint8_t *skip8x8, int32_t damping, uint32_t candidates,
                               uint64_t *sse, uint8_t *dir, int32_t *var, void *stream) {
  const int32_t mode = ((candidates >> 20) & 2) ? CDEF_MODE_SEARCH128 : CDEF_MODE_SEARCH;
  if (!candidates_valid(candidates, mode)) return CDEF_E_INVAL;
  return search_one(recon, src, skip8x8, damping, sse, dir, var, mode, stream, candidates);
}

void cdef_candidate_mask(uint32_t candidates, uint64_t mask[2]) {
  mask[0] = mask[1] = 0;
  for (int k = 0; k < 2; ++k)
    for (int p = 0; p < 64; ++p) {
      const bool in = candidates == 0 || (((candidates >> (p >> 2)) & 1) &&
                                          ((candidates >> (16 + (p & 3))) & 1) &&
                                          ((candidates >> (20 + k)) & 1));
      if (in) mask[k] |= 1ull << p;
    }
}

cdef_status cdef_search_weighted(const cdef_frame *recon, const cdef_frame *src,
                                 const uint8_t *skip8x8, int32_t damping, double *dist,
                                 uint8_t *dir, int32_t *var, void *stream) {
  return search_one(recon, src, skip8x8, damping, reinterpret_cast<uint64_t *>(dist), dir, var,
                    CDEF_MODE_SEARCH_WEIGHTED, stream);
}

cdef_status cdef_job_validate(const cdef_job *job) {
  if (!job) return CDEF_E_INVAL;
  cdef::JobDesc d;
  return make_job(job, &d);
}

size_t cdef_batch_workspace_bytes(int32_t njobs) {
  return njobs < 1 ? 0 : cdef::batch_queue_offset(njobs) + sizeof(cdef::BatchQueue);
}

cdef_status cdef_batch_prepare(const cdef_job *jobs, int32_t njobs, void *host_staging,
                               void *workspace, size_t workspace_bytes, cdef_batch_plan *plan,
                               void *stream) {
  if (!jobs || njobs < 1 || !workspace || !plan) return CDEF_E_INVAL;
  const size_t need = cdef_batch_workspace_bytes(njobs);
  if (workspace_bytes < need) return CDEF_E_NOMEM;
  cdef::JobDesc *table = host_staging ? (cdef::JobDesc *)host_staging
                                      : (cdef::JobDesc *)malloc(need);
  if (!table) return CDEF_E_NOMEM;
  // the persistent kernels' queue counters start at zero
  memset((char *)table + cdef::batch_queue_offset(njobs), 0, sizeof(cdef::BatchQueue));
  int64_t items = 0;
  int32_t flags = 2;
  cdef_status st = CDEF_OK;
  for (int32_t i = 0; i < njobs && st == CDEF_OK; ++i) {
    st = make_job(&jobs[i], &table[i]);
    if (st == CDEF_OK && cdef::job_needs_extended(table[i])) flags |= 1;
    if (st == CDEF_OK && table[i].mode != CDEF_MODE_FILTER) flags &= ~2;
    if (st == CDEF_OK) {
      table[i].item0 = (int32_t)items;
      items += (int64_t)table[i].fbc * table[i].fbr;
      if (items > INT32_MAX / 2) st = CDEF_E_UNSUPPORTED;
    }
  }
  if (st == CDEF_OK) {
    // ordered on `stream` after the work already there (an earlier launch
    // may still read a table in this workspace); without staging the call
    // waits for the copy, so the temporary table can be freed
    hipError_t e =
        hipMemcpyAsync(workspace, table, need, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess && !host_staging) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) st = CDEF_E_HIP;
  }
  if (!host_staging) free(table);
  if (st != CDEF_OK) return st;
  plan->table = workspace;
  plan->njobs = njobs;
  plan->nitems = (int32_t)items;
  plan->variant = 0;
  plan->flags = flags;
  return CDEF_OK;
}

cdef_status cdef_batch_launch(const cdef_batch_plan *plan, void *stream) {
  if (!plan || !plan->table || plan->njobs < 1 || plan->nitems < 1) return CDEF_E_INVAL;
  if (plan->variant < 0 || plan->variant >= CDEF_BATCH_VARIANTS) return CDEF_E_INVAL;
  cdef::BatchQueue *queue = reinterpret_cast<cdef::BatchQueue *>(
      (char *)const_cast<void *>(plan->table) + cdef::batch_queue_offset(plan->njobs));
  return from_hip(cdef::launch_fused_batch((const cdef::JobDesc *)plan->table, plan->njobs,
                                           plan->nitems, plan->variant, (plan->flags & 1) != 0,
                                           (plan->flags & 2) != 0, queue, (hipStream_t)stream));
}

cdef_status cdef_tuning_variant(const cdef_tuning *t, int32_t *variant) {
  if (!t || !variant) return CDEF_E_INVAL;
  if ((t->tile_w != 0 && t->tile_w != 64) || (t->tile_h != 0 && t->tile_h != 64))
    return CDEF_E_UNSUPPORTED;
  if (t->cand_group != 0 && t->cand_group != 64) return CDEF_E_UNSUPPORTED;
  if (t->wg_per_cu != 0 && t->wg_per_cu != 2 && t->wg_per_cu != 3) return CDEF_E_UNSUPPORTED;
  if (t->order != 0 && t->order != 1) return CDEF_E_INVAL;
  if (t->persistent != 0 && t->persistent != 1) return CDEF_E_INVAL;
  const int two = t->wg_per_cu == 2;
  if (t->persistent) {
    if (t->order != 0) return CDEF_E_UNSUPPORTED;  // the queues are XCD-contiguous
    *variant = two ? 5 : 4;
  } else {
    *variant = (t->order ? 2 : 0) + two;
  }
  return CDEF_OK;
}

cdef_status cdef_search_batch(const cdef_job *jobs, int32_t n, const cdef_tuning *t,
                              void *workspace, size_t workspace_bytes, void *stream) {
  int32_t variant = 0;
  if (t) {
    const cdef_status st = cdef_tuning_variant(t, &variant);
    if (st != CDEF_OK) return st;
  }
  cdef_batch_plan plan;
  const cdef_status st =
      cdef_batch_prepare(jobs, n, nullptr, workspace, workspace_bytes, &plan, stream);
  if (st != CDEF_OK) return st;
  plan.variant = variant;
  return cdef_batch_launch(&plan, stream);
}

size_t cdef_select_presets_workspace_bytes(void) { return cdef::preset_workspace_bytes(); }

}  // extern "C"

namespace {

// Host-side checks of a selection's arguments other than the workspace;
// fills the candidate mask and the number of filter blocks.
cdef_status check_selection(const uint64_t *sse, int32_t nplanes, int32_t fb_rows,
                            int32_t fb_cols, int32_t ncand, const uint64_t *cand_mask,
                            double lambda, int32_t refine_passes, cdef_preset_result *result,
                            uint8_t *fb_luma, uint8_t *fb_chroma, uint64_t mask[2],
                            int *nfb) {
  if (!sse || !result || !fb_luma || !fb_chroma) return CDEF_E_INVAL;
  if (nplanes != 1 && nplanes != 3) return CDEF_E_INVAL;
  if (ncand != 64 && ncand != 128) return CDEF_E_INVAL;
  mask[0] = ~0ull;
  mask[1] = ncand == 128 ? ~0ull : 0ull;
  if (cand_mask) {
    mask[0] = cand_mask[0];
    mask[1] = ncand == 128 ? cand_mask[1] : 0ull;
  }
  if (__builtin_popcountll(mask[0]) + __builtin_popcountll(mask[1]) < 8) return CDEF_E_INVAL;
  if (fb_rows < 1 || fb_cols < 1) return CDEF_E_INVAL;
  if (!(lambda >= 0.0) || !isfinite(lambda)) return CDEF_E_INVAL;
  if (refine_passes < 0 || refine_passes > 16) return CDEF_E_INVAL;
  const int64_t n = (int64_t)fb_rows * fb_cols;
  if (n > (1 << 24)) return CDEF_E_UNSUPPORTED;
  *nfb = (int)n;
  return CDEF_OK;
}

}  // namespace

extern "C" {

cdef_status cdef_select_presets(const uint64_t *sse, int32_t nplanes, int32_t fb_rows,
                                int32_t fb_cols, int32_t ncand, const uint64_t *cand_mask,
                                double lambda, int32_t refine_passes,
                                cdef_preset_result *result, uint8_t *fb_luma,
                                uint8_t *fb_chroma, void *workspace, size_t workspace_bytes,
                                void *stream) {
  if (!workspace) return CDEF_E_INVAL;
  if (workspace_bytes < cdef::preset_workspace_bytes() || ((uintptr_t)workspace & 255))
    return CDEF_E_INVAL;
  uint64_t mask[2];
  int nfb = 0;
  const cdef_status st = check_selection(sse, nplanes, fb_rows, fb_cols, ncand, cand_mask,
                                         lambda, refine_passes, result, fb_luma, fb_chroma,
                                         mask, &nfb);
  if (st != CDEF_OK) return st;
  return from_hip(cdef::launch_select_presets(
      sse, nplanes, nfb, ncand, mask, lambda, refine_passes,
      reinterpret_cast<cdef::PresetResult *>(result), fb_luma, fb_chroma, workspace,
      (hipStream_t)stream));
}

cdef_status cdef_select_presets_noalloc(const uint64_t *sse, int32_t nplanes, int32_t fb_rows,
                                        int32_t fb_cols, int32_t ncand,
                                        const uint64_t *cand_mask, double lambda,
                                        int32_t refine_passes, cdef_preset_result *result,
                                        uint8_t *fb_luma, uint8_t *fb_chroma, void *stream) {
  uint64_t mask[2];
  int nfb = 0;
  const cdef_status st = check_selection(sse, nplanes, fb_rows, fb_cols, ncand, cand_mask,
                                         lambda, refine_passes, result, fb_luma, fb_chroma,
                                         mask, &nfb);
  if (st != CDEF_OK) return st;
  // the workspace has one size for every table, which the fixed scratch holds
  if (cdef::preset_workspace_bytes() > cdef::kPresetScratchBytes) return CDEF_E_NOMEM;
  void *scratch = nullptr;
  if (cdef::preset_scratch((hipStream_t)stream, &scratch) != hipSuccess) return CDEF_E_HIP;
  return from_hip(cdef::launch_select_presets(
      sse, nplanes, nfb, ncand, mask, lambda, refine_passes,
      reinterpret_cast<cdef::PresetResult *>(result), fb_luma, fb_chroma, scratch,
      (hipStream_t)stream));
}

const char *cdef_status_str(cdef_status s) {
  switch (s) {
    case CDEF_OK: return "ok";
    case CDEF_E_INVAL: return "invalid argument";
    case CDEF_E_UNSUPPORTED: return "unsupported input";
    case CDEF_E_HIP: return "HIP runtime error";
    case CDEF_E_NOMEM: return "workspace too small";
    case CDEF_E_TIMEOUT: return "a bounded device-side wait gave up";
  }
  return "unknown status";
}

int32_t cdef_abi_version(void) { return CDEF_ABI_VERSION; }

}  // extern "C"
