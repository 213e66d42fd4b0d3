// Internal definitions shared by the HIP sources of the gridding library.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>
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

// Device-side grid geometry (degrees, as given by the caller).  A plan whose
// cells were given by their centres keeps nx, ny here and zeros elsewhere;
// every gather reads the cell centres from the plan's unit-vector array.
struct GridGeom {
  int32_t nx, ny;
  double lon0, lat0, dlon, dlat;
};

// Kernel of the plan (Section 3.6 (iii)): the weight of a pair at distance d
// (d <= R), all factors precomputed on the host.
//   kGauss      exp2(d^2 wscale)
//   kElliptic   exp2(d^2 (a^2 kmaj + b^2 kmin) / (a^2 + b^2)), (a, b) the
//               sample's offset along the major / minor axis in the tangent
//               plane of the cell: a = xn cpa + xe spa, b = xe cpa - xn spa
//               (xe, xn its east / north components); weight 1 at d = 0
//   kSinc       sin(d sinc_k) / (d sinc_k) exp2(d^2 taper_k)
enum KernelType : int32_t { kGauss = 0, kElliptic = 1, kSinc = 2 };
struct KernelParams {
  int32_t type;
  int32_t pad_;
  double wscale;          // Gaussian: -log2(e) / (2 sigma^2)
  double kmaj, kmin;      // elliptic: -log2(e) / (2 sigma^2) of each axis
  double cpa, spa;        // elliptic: cos / sin of the major axis' position angle
  double sinc_k, taper_k; // sinc: pi / b and -log2(e) / a^2
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

// ---------------------------------------------------------------------------
// Element encodings of the low-precision forms (round to nearest even).
// ---------------------------------------------------------------------------
// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint32_t f32_to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ uint32_t f32_to_f16(float x) {
  const _Float16 h = (_Float16)x;  // round to nearest even
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

// float -> OCP FP8 E4M3 (bias 7, no infinities, max 448, 0x7F = NaN), round
// to nearest even, saturating at 448.
__device__ __forceinline__ uint32_t f32_to_e4m3(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7FFFFFFFu;
  if (a > 0x7F800000u) return sign | 0x7Fu;
  const float fa = __uint_as_float(a);
  if (fa < 0.015625f) {  // below 2^-6: subnormal steps of 2^-9
    const uint32_t m = (uint32_t)rintf(fa * 512.0f);  // 0 .. 8 (8 = smallest normal)
    return sign | m;
  }
  // keep 3 mantissa bits with round to nearest even
  const uint32_t r = a + 0x7FFFFu + ((a >> 20) & 1u);
  const int e = (int)(r >> 23) - 127;
  const uint32_t m = (r >> 20) & 7u;
  if (e > 8 || (e == 8 && m == 7u)) return sign | 0x7Eu;  // saturate to 448
  return sign | ((uint32_t)(e + 7) << 3) | m;
}
__device__ __forceinline__ float e4m3_to_f32(uint32_t c) {
  const uint32_t e = (c >> 3) & 15u, m = c & 7u;
  const float v = (e == 0) ? (float)m * 0.001953125f
                           : __uint_as_float(((e + 120u) << 23) | (m << 20));
  return (c & 0x80u) ? -v : v;
}

// The same two conversions through the gfx950 conversion instructions (OCP
// E4M3, round to nearest even): equal to f32_to_e4m3 / e4m3_to_f32 for every
// |x| <= 448, subnormals included (checked on the device over that range),
// one instruction each.  Callers keep their arguments within +-448.
__device__ __forceinline__ uint32_t f32_to_e4m3_cvt(float x) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xFFu;
}
__device__ __forceinline__ float e4m3_cvt_to_f32(uint32_t c) {
  return __builtin_amdgcn_cvt_f32_fp8((int)c, 0);
}

}  // namespace hcg

// The plan object behind hcg_plan_t.  Every device array lives in one arena.
struct hcg_plan_s {
  uint64_t magic;
  int device;
  int batch_owned;  // a plan of a batch: freed with the batch only
  int arena_pooled;  // the arena came from the library's pool (freed stream-ordered)
  int64_t n;
  int32_t nside;
  uint32_t pix_base, pix_max;
  int32_t key_bits, passes;
  int32_t ring_first, ring_last;
  hcg::GridGeom grid;
  int32_t centres;     // 1: cells given by their centres (no linear geometry)
  double fwhm_deg, support_deg, sigma_rad, support_rad;
  hcg::KernelParams kern;
  int32_t ntx, nty, maxr;
  void* arena;
  size_t arena_bytes;
  double4* xyz;        // [n + 8] sorted unit vectors (cos b cos l, cos b sin l, sin b, 0);
                       // entries n .. n + 7: NaN (sentinels)
  uint32_t* keys;      // [n] sorted pixel - pix_base
  uint32_t* perm;      // [n + 1] input index of each sorted sample; entry n: 0 (sentinel)
  uint32_t* csr;       // [nrings + 1]
  uint2* ranges;       // [ntiles][maxr] candidate ranges [a, b)
  uint32_t* nranges;   // [ntiles]
  uint32_t* ncand;     // [ntiles] candidates per tile
  uint32_t* flags;     // [4] device status words
  double4* cells;      // [ny * nx] unit vectors of the cell centres (NaN: no cell)
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

// Arguments of the gather for one plan and one spectra buffer (gather.hip).
struct GatherArgs {
  const double4* cells; // [ny][nx] unit vectors of the cell centres
  KernelParams kern;
  float* wcube;         // masked form: per-channel weights [C][ny][nx] or NULL
  const double4* xyz;
  const uint32_t* perm;
  const uint2* ranges;
  const uint32_t* nranges;
  int maxr;
  uint32_t sentinel;    // n: index of the first sentinel entry of xyz and perm
  const void* spec;     // [n][C] in the form's storage type
  const void* spec_lo;  // low plane for the split form
  const float* scale;   // [C] per-channel scale for the scaled forms
  int64_t C;
  GridGeom g;
  int ntx, ntiles, tiles_per_xcd;
  int vec;  // rows can be read 4 elements at a time
  double c2R;     // squared chord of the support radius, 4 sin^2(R / 2)
  float* cube;
  float* wmap;
};

// The host fills GatherArgs tables that kernels index; the layout is fixed
// (both compilation passes see these checks).
static_assert(sizeof(KernelParams) == 64, "KernelParams layout changed");
static_assert(sizeof(GatherArgs) == 232, "GatherArgs layout changed");
static_assert(offsetof(GatherArgs, kern) == 8 && offsetof(GatherArgs, wcube) == 72 &&
                  offsetof(GatherArgs, sentinel) == 116 && offsetof(GatherArgs, C) == 144 &&
                  offsetof(GatherArgs, g) == 152 &&
                  offsetof(GatherArgs, c2R) == 208 && offsetof(GatherArgs, wmap) == 224,
              "GatherArgs layout changed");

// Batched gather (gather.hip): one work item = (field, tile, channel slab).
// Field f owns the items [base, base + ntiles * slabs) of the item space,
// item base + s * ntiles + t being slab s of tile t.  Segments are listed in
// increasing base.  The persistent kernel reads device arrays of GatherArgs
// (one per field) and BatchSeg, and a control block of kBatchCtl words.
// Largest squared support chord of the narrow-support gather kernels.
constexpr double kNarrowChord2 = 1e-4;

// The library's stream-ordered memory pool on the current device (NULL if
// it cannot be created): plan arenas and per-call scratch, kept for reuse
// up to a release threshold instead of being handed back to the driver
// at every synchronisation.  Lives until the process ends.
hipMemPool_t plan_pool();

struct BatchSeg {
  uint32_t base, ntiles, slabs, field;
};
constexpr int kBatchXcds = 8;
constexpr int kBatchCtl = 16;
hcg_status plan_build_fields(int32_t nf, const hcg_field_desc* fd, const hcg_opts* opts,
                             hipStream_t stream, hcg_plan_t* plans, void** arena_out,
                             std::vector<std::vector<uint32_t>>* ncand, int32_t* failed);
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
