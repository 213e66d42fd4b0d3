// Internal definitions shared by the HIP sources of the gridding library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "hcg.h"

namespace hcg {

constexpr double kDeg2Rad = 0.017453292519943295;
constexpr double kPi = 3.141592653589793;
constexpr uint64_t kPlanMagic = 0x48434750'4c414e31ull;  // "HCGPLAN1"

// Output-cell tile of the gather kernels: 8 x 8 cells, four 4 x 4 blocks.
constexpr int kTileX = 8;
constexpr int kTileY = 8;
constexpr int kTileCells = kTileX * kTileY;
constexpr int kMaxRangesLimit = 1024;

// ---------------------------------------------------------------------------
// HEALPix ring scheme (Section 3.2; Gorski et al. 2005).  Rings are numbered
// 1 .. 4 Ns - 1 from the north pole: 4i pixels in the polar-cap rings i < Ns
// (and mirrored in the south), 4 Ns in the equatorial belt Ns <= i <= 3 Ns.
// ---------------------------------------------------------------------------
__host__ __device__ inline int64_t hpx_ring_npix(int64_t ns, int64_t i) {
  if (i < ns) return 4 * i;
  if (i <= 3 * ns) return 4 * ns;
  return 4 * (4 * ns - i);
}

__host__ __device__ inline int64_t hpx_ring_start(int64_t ns, int64_t i) {
  if (i <= ns) return 2 * i * (i - 1);
  if (i <= 3 * ns) return 2 * ns * (ns - 1) + 4 * ns * (i - ns);
  const int64_t s = 4 * ns - i;
  return 12 * ns * ns - 2 * s * (s + 1);
}

// z = sin(latitude) of the pixel centres of ring i; z(0) = 1, z(4Ns) = -1.
__host__ __device__ inline double hpx_ring_z(int64_t ns, int64_t i) {
  if (i <= 0) return 1.0;
  if (i >= 4 * ns) return -1.0;
  const double n = (double)ns;
  if (i < ns) return 1.0 - (double)(i * i) / (3.0 * n * n);
  if (i <= 3 * ns) return 4.0 / 3.0 - 2.0 * (double)i / (3.0 * n);
  const int64_t s = 4 * ns - i;
  return (double)(s * s) / (3.0 * n * n) - 1.0;
}

// Continuous ring coordinate of latitude z (inverse of hpx_ring_z).
__host__ __device__ inline double hpx_ring_of_z(int64_t ns, double z) {
  const double n = (double)ns;
  if (z > 2.0 / 3.0) return n * sqrt(3.0 * (1.0 - z));
  if (z < -2.0 / 3.0) return 4.0 * n - n * sqrt(3.0 * (1.0 + z));
  return n * (2.0 - 1.5 * z);
}

// Ring holding pixel p.
__host__ __device__ inline int64_t hpx_pix2ring(int64_t ns, int64_t p) {
  int64_t lo = 1, hi = 4 * ns - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (hpx_ring_start(ns, mid) <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Device-side grid geometry (degrees, as given by the caller).
struct GridGeom {
  int32_t nx, ny;
  double lon0, lat0, dlon, dlat;
};

__host__ __device__ inline double cell_lon_deg(const GridGeom& g, int ix) {
  return g.lon0 + ((double)ix - 0.5 * (double)(g.nx - 1)) * g.dlon;
}
__host__ __device__ inline double cell_lat_deg(const GridGeom& g, int iy) {
  return g.lat0 + ((double)iy - 0.5 * (double)(g.ny - 1)) * g.dlat;
}

// First position in [lo, hi) whose key is >= target.
__device__ inline uint32_t lower_bound_u32(const uint32_t* __restrict__ keys, uint32_t lo,
                                           uint32_t hi, int64_t target) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if ((int64_t)keys[mid] < target) lo = mid + 1; else hi = mid;
  }
  return lo;
}

}  // namespace hcg

// The plan object behind hcg_plan_t.  Every device array lives in one arena.
struct hcg_plan_s {
  uint64_t magic;
  int device;
  int64_t n;
  int32_t nside;
  uint32_t pix_base, pix_max;
  int32_t key_bits, passes;
  int32_t ring_first, ring_last;
  hcg::GridGeom grid;
  double fwhm_deg, support_deg, sigma_rad, support_rad;
  int32_t ntx, nty, maxr;
  void* arena;
  size_t arena_bytes;
  double4* trig;       // [n] sorted: sin(lat/2), cos(lat/2), sin(lon/2), cos(lon/2)
  uint32_t* keys;      // [n] sorted pixel - pix_base
  uint32_t* perm;      // [n] input index of each sorted sample
  uint32_t* csr;       // [nrings + 1]
  uint2* ranges;       // [ntiles][maxr] candidate ranges [a, b)
  uint32_t* nranges;   // [ntiles]
  uint32_t* ncand;     // [ntiles] candidates per tile
  uint32_t* flags;     // [4] device status words
};

namespace hcg {

// Error plumbing: every entry point returns a status and leaves a message.
hcg_status fail(hcg_status st, const char* fmt, ...);
hcg_status check_device_arch();
bool plan_is_live(const hcg_plan_s* p);
void plan_register(hcg_plan_s* p);
void plan_unregister(hcg_plan_s* p);

// Step launchers (plan.hip); all asynchronous on `stream`.
hcg_status launch_ang2pix(const double* lon, const double* lat, int64_t n, int nside,
                          uint32_t* pix, uint32_t* stat, hipStream_t stream);
size_t radix_sort_temp_bytes(int64_t n);
hcg_status launch_radix_sort(const uint32_t* keys_in, int64_t n, int key_bits, uint32_t* keys_out,
                             uint32_t* perm_out, void* temp, hipStream_t stream);

}  // namespace hcg

#define HCG_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::hcg::fail(HCG_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define HCG_LAUNCH_CHECK(name)                                                          \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      return ::hcg::fail(HCG_E_DEVICE, "launch of %s failed: %s", name,                \
                         hipGetErrorString(e_));                                       \
  } while (0)
