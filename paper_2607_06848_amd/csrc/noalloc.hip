// Chebyshev filter that allocates nothing, for callers that cannot call the
// device allocator (code under stream capture, tight serving loops).  Its
// workspaces come from `scratch`, a fixed region of device memory that every
// GPU the library runs on holds until the process ends; its address on each
// device is taken once, when the first context on that device is set up.
#include <mutex>

#include "efe_internal.h"

static __device__ __align__(256) unsigned char scratch[EFE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

efe_status efe_scratch_attach(efe_ctx *c) {
  if (c->device < 0 || c->device >= kMaxDevices) EFE_FAIL(c, EFE_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[c->device]) return EFE_OK;
  // the context's device is the current one here (efe_setup_mesh)
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    c->err = std::string("hipGetSymbolAddress of the scratch region failed: ") + hipGetErrorString(e);
    return EFE_EHIP;
  }
  g_scratch_ptr[c->device] = p;
  return EFE_OK;
}

// Workspace bytes of one filter call, an upper bound of what its slots take
// (the first column chunk is the widest): G, Z_{k-1}, Z_{k-2}, H V, the
// enrichment rows of M~^-1 Z, the C_k(lambda) and sigma tables; inside each
// apply the even-width copies of the CFE and enrichment rows, the projector
// coefficients, the cells' partial enrichment rows and the dense-block
// products; 256-byte alignment of every slot.
static size_t filter_scratch_bytes(const efe_ctx *c, int32_t ncols, int m) {
  const size_t nc = (size_t)std::min<int32_t>(ncols, EFE_COL_CHUNK);
  const size_t ldc = (nc + 1) & ~(size_t)1;
  const size_t rows = (size_t)c->rows, nn = (size_t)c->n_nodes;
  const size_t ne = (size_t)c->n_enr, ne1 = std::max<size_t>(ne, 1);
  size_t b = 4 * rows * nc * 8 + ne1 * nc * 8 + (size_t)(m + 1) * nc * 8 + (size_t)(m + 1) * 8;
  b += nn * ldc * 8 + ne * ldc * 8 + (size_t)c->nproj * nc * 8 +
       (size_t)c->nf * (size_t)std::max<int64_t>(c->ncpairs, 1) * nc * 8 + ne * nc * 8;
  return b + 16 * 256;
}

extern "C" efe_status efe_cheb_filter_noalloc(efe_ctx *c, double *V, const double *lambda,
                                              int32_t ncols, int64_t ld,
                                              const efe_cheb_params *prm) {
  efe_status s = efe_filter_check(c, V, lambda, ncols, ld, prm);
  if (s) return s;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices) base = g_scratch_ptr[c->device];
  }
  if (!base) EFE_FAIL(c, EFE_ESTATE, "no scratch region on this device");
  const size_t need = filter_scratch_bytes(c, ncols, prm->degree);
  if (need > (size_t)EFE_NOALLOC_SCRATCH_BYTES)
    EFE_FAIL(c, EFE_EINVAL,
             "filter needs " + std::to_string(need) + " bytes of scratch, more than the " +
                 std::to_string((size_t)EFE_NOALLOC_SCRATCH_BYTES) + " the region holds");
  // every workspace slot from the region; timing would create events, so it
  // is off for the call
  const bool timing = c->timing;
  c->timing = false;
  c->arena = (char *)base;
  c->arena_cap = EFE_NOALLOC_SCRATCH_BYTES;
  c->arena_used = 0;
  for (int i = 0; i < efe_ctx::kArenaSlots; ++i) c->arena_len[i] = 0;
  s = efe_filter_run(c, V, lambda, ncols, ld, prm);
  c->arena = nullptr;
  c->arena_cap = 0;
  c->timing = timing;
  return s;
}
