// HIP-event timing of the hot-path kernels, recorded on the context's stream
// when enabled with efe_timing.
#include "efe_internal.h"

int efe_timer_begin(efe_ctx *c, int which) {
  if (!c->timing) return -1;
  std::vector<hipEvent_t> &v = c->tev[which];
  const int64_t slot = c->tused[which];
  while ((int64_t)v.size() < 2 * (slot + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    v.push_back(e);
  }
  if (hipEventRecord(v[2 * slot], c->stream) != hipSuccess) return -1;
  c->tused[which] = slot + 1;
  return (int)slot;
}

void efe_timer_end(efe_ctx *c, int which, int slot) {
  if (slot < 0) return;
  (void)hipEventRecord(c->tev[which][2 * slot + 1], c->stream);
}

extern "C" efe_status efe_timing(efe_ctx *c, int32_t enable) {
  if (!c) return EFE_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->timing = enable != 0;
  if (enable)
    for (int w = 0; w < EFE_T_N; ++w) c->tused[w] = 0;
  return EFE_OK;
}

extern "C" efe_status efe_timing_get(efe_ctx *c, int32_t which, int64_t *launches,
                                     double *total_ms) {
  if (!c) return EFE_EINVAL;
  if (which < 0 || which >= EFE_T_N || !launches || !total_ms) EFE_FAIL(c, EFE_EINVAL, "bad timer");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (int64_t s = 0; s < c->tused[which]; ++s) {
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->tev[which][2 * s], c->tev[which][2 * s + 1]));
    tot += ms;
  }
  *launches = c->tused[which];
  *total_ms = tot;
  return EFE_OK;
}
