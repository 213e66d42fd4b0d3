// C-ABI plumbing of the gridding library: error messages, device checks,
// the registry of live plans, plan inspection and destruction.
#include <cstring>
#include <mutex>
#include <set>
#include <string>

#include "hcg_internal.h"

namespace hcg {

static thread_local std::string g_last_error;
static std::mutex g_mu;
static std::set<const hcg_plan_s*>* g_live = nullptr;

hcg_status fail(hcg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

hcg_status check_device_arch() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HCG_E_DEVICE, "no HIP device: %s", hipGetErrorString(e));
  static std::mutex mu;
  static int checked[64] = {0};  // 0 unknown, 1 ok, 2 unsupported
  std::lock_guard<std::mutex> lk(mu);
  if (dev < 0 || dev >= 64) return fail(HCG_E_DEVICE, "device index %d out of range", dev);
  if (checked[dev] == 0) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(HCG_E_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    checked[dev] = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : 2;
    if (checked[dev] == 2)
      return fail(HCG_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", dev,
                  prop.gcnArchName);
  }
  if (checked[dev] == 2) return fail(HCG_E_UNSUPPORTED, "device %d is not gfx950", dev);
  return HCG_OK;
}

bool plan_is_live(const hcg_plan_s* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_live && g_live->count(p) && p->magic == kPlanMagic;
}

void plan_register(hcg_plan_s* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_live) g_live = new std::set<const hcg_plan_s*>();
  g_live->insert(p);
}

void plan_unregister(hcg_plan_s* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_live) g_live->erase(p);
}

}  // namespace hcg

using namespace hcg;

extern "C" const char* hcg_last_error(void) { return g_last_error.c_str(); }

extern "C" hcg_status hcg_destroy(hcg_plan_t plan) {
  if (!plan) return HCG_OK;
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_destroy: not a live plan");
  if (plan->batch_owned)
    return fail(HCG_E_STATE, "hcg_destroy: the plan belongs to a batch (hcg_destroy_batch frees it)");
  plan_unregister(plan);
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != plan->device) (void)hipSetDevice(plan->device);
  // (a plan of a batch has no arena of its own: the batch frees the shared one)
  hipError_t e1 = plan->arena ? hipDeviceSynchronize() : hipSuccess;
  // (a pooled arena goes back to the library's pool, kept there for the next plan)
  hipError_t e2 = !plan->arena        ? hipSuccess
                  : plan->arena_pooled ? hipFreeAsync(plan->arena, nullptr)
                                       : hipFree(plan->arena);
  if (cur != plan->device && cur >= 0) (void)hipSetDevice(cur);
  plan->magic = 0;
  delete plan;
  if (e1 != hipSuccess) return fail(HCG_E_DEVICE, "hcg_destroy: %s", hipGetErrorString(e1));
  if (e2 != hipSuccess) return fail(HCG_E_DEVICE, "hcg_destroy: %s", hipGetErrorString(e2));
  return HCG_OK;
}

extern "C" hcg_status hcg_get_plan_info(hcg_plan_t plan, hcg_plan_info* info) {
  if (!plan || !info) return fail(HCG_E_ARG, "hcg_get_plan_info: NULL pointer");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_get_plan_info: not a live plan");
  const hcg_plan_s* p = plan;
  info->n = p->n;
  info->nside = p->nside;
  info->key_bits = p->key_bits;
  info->pix_base = p->pix_base;
  info->pix_max = p->pix_max;
  info->ring_first = p->ring_first;
  info->ring_last = p->ring_last;
  info->tile_x = kTileX;
  info->tile_y = kTileY;
  info->ntiles_x = p->ntx;
  info->ntiles_y = p->nty;
  info->max_ranges = p->maxr;
  info->sort_passes = p->passes;
  info->sigma_rad = p->sigma_rad;
  info->support_rad = p->support_rad;
  return HCG_OK;
}

static hcg_status array_of(const hcg_plan_s* p, hcg_array which, const void** src,
                           int64_t* bytes) {
  const int64_t ntiles = (int64_t)p->ntx * p->nty;
  switch (which) {
    case HCG_ARR_KEYS: *src = p->keys; *bytes = 4 * p->n; return HCG_OK;
    case HCG_ARR_PERM: *src = p->perm; *bytes = 4 * p->n; return HCG_OK;
    case HCG_ARR_RING_CSR:
      *src = p->csr;
      *bytes = 4 * (int64_t)(p->ring_last - p->ring_first + 2);
      return HCG_OK;
    case HCG_ARR_TILE_NRANGES: *src = p->nranges; *bytes = 4 * ntiles; return HCG_OK;
    case HCG_ARR_TILE_RANGES: *src = p->ranges; *bytes = 8 * ntiles * p->maxr; return HCG_OK;
  }
  return fail(HCG_E_ARG, "unknown array %d", (int)which);
}

extern "C" hcg_status hcg_export_size(hcg_plan_t plan, hcg_array which, int64_t* bytes) {
  if (!plan || !bytes) return fail(HCG_E_ARG, "hcg_export_size: NULL pointer");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_export_size: not a live plan");
  const void* src;
  return array_of(plan, which, &src, bytes);
}

extern "C" hcg_status hcg_export(hcg_plan_t plan, hcg_array which, void* dst, int64_t bytes,
                                 void* hip_stream) {
  if (!plan || !dst) return fail(HCG_E_ARG, "hcg_export: NULL pointer");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_export: not a live plan");
  const void* src;
  int64_t need;
  hcg_status st = array_of(plan, which, &src, &need);
  if (st != HCG_OK) return st;
  if (bytes != need) return fail(HCG_E_ARG, "hcg_export: %lld bytes given, %lld needed",
                                 (long long)bytes, (long long)need);
  HCG_HIP(hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, (hipStream_t)hip_stream));
  return HCG_OK;
}
