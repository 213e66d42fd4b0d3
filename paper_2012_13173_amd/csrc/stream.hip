// Out-of-core gridding: spectra and cube in host memory, streamed through the
// device one channel slab at a time (the CUDA-streams overlap of copy and
// compute that Section 5 names as future work, for cubes larger than HBM).
//
// One plan serves every slab.  Three streams overlap the three stages of
// consecutive slabs: the host-to-device copy of slab s + 1, the gather of
// slab s and the device-to-host copy of slab s - 1.  Two device buffers per
// stage (double buffering) and events order them:
//   in[s]   waits until the gather of slab s - 2 has read its buffer;
//   grid[s] waits for in[s] and for the copy-out of slab s - 2;
//   out[s]  waits for grid[s].
// A slab of spectra is a strided host region (n rows of slab channels, row
// pitch nchan floats), copied with one 2-D copy into a dense [n][slab] device
// buffer, which is what hcg_grid takes.
#include <algorithm>

#include "hcg_internal.h"

using namespace hcg;

namespace {

struct StreamRes {
  hipStream_t s_in = nullptr, s_out = nullptr;
  hipEvent_t ev_in[2] = {nullptr, nullptr}, ev_grid[2] = {nullptr, nullptr},
             ev_out[2] = {nullptr, nullptr};
  void* dspec[2] = {nullptr, nullptr};
  void* dcube[2] = {nullptr, nullptr};
  float* dw = nullptr;
  ~StreamRes() {
    // every stage has been waited for before the resources go
    for (int b = 0; b < 2; ++b) {
      if (ev_in[b]) (void)hipEventDestroy(ev_in[b]);
      if (ev_grid[b]) (void)hipEventDestroy(ev_grid[b]);
      if (ev_out[b]) (void)hipEventDestroy(ev_out[b]);
      if (dspec[b]) (void)hipFree(dspec[b]);
      if (dcube[b]) (void)hipFree(dcube[b]);
    }
    if (dw) (void)hipFree(dw);
    if (s_in) (void)hipStreamDestroy(s_in);
    if (s_out) (void)hipStreamDestroy(s_out);
  }
};

}  // namespace

extern "C" hcg_status hcg_grid_host(hcg_plan_t plan, const float* spectra_host, int64_t nchan,
                                    int64_t slab_chan, float* cube_host, float* weights_host,
                                    void* hip_stream) {
  if (!plan) return fail(HCG_E_ARG, "hcg_grid_host: plan is NULL");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_grid_host: not a live plan");
  if (!spectra_host || !cube_host) return fail(HCG_E_ARG, "hcg_grid_host: NULL pointer");
  if (nchan < 1) return fail(HCG_E_ARG, "hcg_grid_host: nchan must be >= 1");
  if (slab_chan < 0) return fail(HCG_E_ARG, "hcg_grid_host: slab_chan must be >= 0");
  const hcg_plan_s* p = plan;
  const int64_t n = p->n;
  const int64_t G = (int64_t)p->grid.nx * p->grid.ny;
  // default slab: 512 channels, or fewer so that one spectra buffer stays
  // within 4 GiB
  int64_t cs = slab_chan ? slab_chan : 512;
  const int64_t cap = std::max<int64_t>(1, ((int64_t)4 << 30) / (4 * std::max<int64_t>(n, G)));
  if (!slab_chan) cs = std::min(cs, cap);
  cs = std::min(cs, nchan);
  const int64_t nslab = (nchan + cs - 1) / cs;
  hipStream_t s_grid = (hipStream_t)hip_stream;

  StreamRes r;
  HCG_HIP(hipStreamCreateWithFlags(&r.s_in, hipStreamNonBlocking));
  HCG_HIP(hipStreamCreateWithFlags(&r.s_out, hipStreamNonBlocking));
  for (int b = 0; b < 2; ++b) {
    HCG_HIP(hipEventCreateWithFlags(&r.ev_in[b], hipEventDisableTiming));
    HCG_HIP(hipEventCreateWithFlags(&r.ev_grid[b], hipEventDisableTiming));
    HCG_HIP(hipEventCreateWithFlags(&r.ev_out[b], hipEventDisableTiming));
    if (hipMalloc(&r.dspec[b], sizeof(float) * n * cs) != hipSuccess ||
        hipMalloc(&r.dcube[b], sizeof(float) * G * cs) != hipSuccess) {
      (void)hipGetLastError();
      return fail(HCG_E_NOMEM, "hcg_grid_host: cannot allocate two slabs of %lld channels",
                  (long long)cs);
    }
  }
  if (weights_host && hipMalloc(&r.dw, sizeof(float) * G) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "hcg_grid_host: cannot allocate the weight map");
  }
  // the caller's earlier work on its stream comes first
  HCG_HIP(hipEventRecord(r.ev_grid[1], s_grid));
  HCG_HIP(hipStreamWaitEvent(r.s_in, r.ev_grid[1], 0));

  hcg_status st = HCG_OK;
  for (int64_t s = 0; s < nslab && st == HCG_OK; ++s) {
    const int b = (int)(s & 1);
    const int64_t c0 = s * cs, cn = std::min(cs, nchan - c0);
    // in: the buffer was last read by the gather of slab s - 2
    if (s >= 2) HCG_HIP(hipStreamWaitEvent(r.s_in, r.ev_grid[b], 0));
    HCG_HIP(hipMemcpy2DAsync(r.dspec[b], sizeof(float) * cn, spectra_host + c0,
                             sizeof(float) * nchan, sizeof(float) * cn, n,
                             hipMemcpyHostToDevice, r.s_in));
    HCG_HIP(hipEventRecord(r.ev_in[b], r.s_in));
    // gather: after the copy-in, and after the copy-out of slab s - 2
    HCG_HIP(hipStreamWaitEvent(s_grid, r.ev_in[b], 0));
    if (s >= 2) HCG_HIP(hipStreamWaitEvent(s_grid, r.ev_out[b], 0));
    st = hcg_grid(plan, r.dspec[b], cn, HCG_F32, nullptr, (float*)r.dcube[b],
                  s == 0 ? r.dw : nullptr, s_grid);
    if (st != HCG_OK) break;
    HCG_HIP(hipEventRecord(r.ev_grid[b], s_grid));
    // out: the cube slab is contiguous in [C][ny][nx]
    HCG_HIP(hipStreamWaitEvent(r.s_out, r.ev_grid[b], 0));
    HCG_HIP(hipMemcpyAsync(cube_host + c0 * G, r.dcube[b], sizeof(float) * cn * G,
                           hipMemcpyDeviceToHost, r.s_out));
    if (s == 0 && weights_host)
      HCG_HIP(hipMemcpyAsync(weights_host, r.dw, sizeof(float) * G, hipMemcpyDeviceToHost,
                             r.s_out));
    HCG_HIP(hipEventRecord(r.ev_out[b], r.s_out));
  }
  // drain every stage before the buffers are freed (also after an error)
  const hipError_t e1 = hipStreamSynchronize(r.s_in);
  const hipError_t e2 = hipStreamSynchronize(s_grid);
  const hipError_t e3 = hipStreamSynchronize(r.s_out);
  if (st != HCG_OK) return st;
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
    return fail(HCG_E_DEVICE, "hcg_grid_host: %s",
                hipGetErrorString(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3));
  return HCG_OK;
}
