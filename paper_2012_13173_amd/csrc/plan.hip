// Plan stage of the gridding library: everything that depends on sample
// positions and the target grid but not on the spectra (HCGrid Section 3.3 -
// 3.4, moved onto the GPU).
//
//   k_ang2pix        HEALPix ring-scheme pixel of every sample (Section 3.2)
//   k_radix_*        stable LSD radix sort of (pixel, sample) (Section 3.3 I)
//   k_permute_xyz    sorted unit vector of every sample
//   k_ring_csr       start of every ring in the sorted order (Section 3.3 III)
//   k_tile_ranges    per tile of output cells, the sorted-sample ranges that
//                    can lie within the support (Section 3.4 steps i-iv)
#include <algorithm>
#include <cmath>
#include <mutex>
#include <set>

#include "hcg_internal.h"
#include "sphere.h"

namespace hcg {

// ---------------------------------------------------------------------------
// a1: ang2pix.  t = 2 phi / pi, z = sin(lat).  In the equatorial belt the
// pixel edges are the lines Ns (1/2 + t -+ 3z/4) = integer, so the integer
// parts of those two quantities give the ring (their difference) and the
// position along it (their sum).  In the polar caps the edges are
// tau q = integer and (1 - tau) q = integer with tau = frac(t) and
// q = Ns sqrt(3 (1 - |z|)); the ring from the pole is the sum of the integer
// parts plus one and the pixel along it is floor(t * ring).
// Evaluated without FMA contraction so that the result is a function of the
// IEEE operations alone.
// ---------------------------------------------------------------------------
__device__ __noinline__ uint32_t ang2pix_ring(int ns_i, double lon_deg, double lat_deg) {
#pragma clang fp contract(off)
  const int64_t ns = ns_i;
  double lon = fmod(lon_deg, 360.0);
  if (lon < 0.0) lon += 360.0;
  if (lon >= 360.0) lon -= 360.0;
  const double t = lon / 90.0;
  const double z = sin(lat_deg * kDeg2Rad);
  const double za = fabs(z);
  const double n = (double)ns;
  if (za <= 2.0 / 3.0) {
    const double a = n * (0.5 + t);
    const double b = n * z * 0.75;
    const int64_t jp = (int64_t)floor(a - b);
    const int64_t jm = (int64_t)floor(a + b);
    const int64_t ir = ns + 1 + jp - jm;  // 1 .. 2Ns+1 counted from z = 2/3
    const int64_t kshift = 1 - (ir & 1);
    int64_t ip = (jp + jm - ns + kshift + 1);
    ip = (ip >= 0) ? (ip >> 1) : -((-ip + 1) >> 1);
    ip %= 4 * ns;
    if (ip < 0) ip += 4 * ns;
    return (uint32_t)(2 * ns * (ns - 1) + (ir - 1) * 4 * ns + ip);
  }
  const double tau = t - floor(t);
  const double q = n * sqrt(3.0 * (1.0 - za));
  const int64_t jp = (int64_t)floor(tau * q);
  const int64_t jm = (int64_t)floor((1.0 - tau) * q);
  const int64_t ir = jp + jm + 1;  // ring counted from the nearest pole
  int64_t ip = (int64_t)floor(t * (double)ir);
  ip %= 4 * ir;
  if (ip < 0) ip += 4 * ir;
  if (z > 0.0) return (uint32_t)(2 * ir * (ir - 1) + ip);
  return (uint32_t)(12 * ns * ns - 2 * ir * (ir + 1) + ip);
}

// stat[0] = min pixel, stat[1] = max pixel, stat[2] = count of bad inputs.
// Grid-stride over the samples; one set of atomics per block.
__global__ void __launch_bounds__(256) k_ang2pix(const double* __restrict__ lon,
                                                 const double* __restrict__ lat, int64_t n,
                                                 int ns, uint32_t* __restrict__ pix,
                                                 uint32_t* __restrict__ stat) {
  __shared__ uint32_t s_red[3][4];
  uint32_t vmin = 0xFFFFFFFFu, vmax = 0u, bad = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double lo = lon[i], la = lat[i];
    uint32_t p;
    if (!isfinite(lo) || !isfinite(la) || fabs(la) > 90.0) {
      p = 0xFFFFFFFFu;
      bad += 1;
    } else {
      p = ang2pix_ring(ns, lo, la);
      vmin = min(vmin, p);
      vmax = max(vmax, p);
    }
    pix[i] = p;
  }
  for (int off = 32; off > 0; off >>= 1) {
    vmin = min(vmin, (uint32_t)__shfl_xor((int)vmin, off));
    vmax = max(vmax, (uint32_t)__shfl_xor((int)vmax, off));
    bad += (uint32_t)__shfl_xor((int)bad, off);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_red[0][wave] = vmin;
    s_red[1][wave] = vmax;
    s_red[2][wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      vmin = min(vmin, s_red[0][w]);
      vmax = max(vmax, s_red[1][w]);
      bad += s_red[2][w];
    }
    atomicMin(&stat[0], vmin);
    atomicMax(&stat[1], vmax);
    if (bad) atomicAdd(&stat[2], bad);
  }
}

hcg_status launch_ang2pix(const double* lon, const double* lat, int64_t n, int nside,
                          uint32_t* pix, uint32_t* stat, hipStream_t stream) {
  const uint32_t init[4] = {0xFFFFFFFFu, 0u, 0u, 0u};
  HCG_HIP(hipMemcpyAsync(stat, init, sizeof(init), hipMemcpyHostToDevice, stream));
  if (n == 0) return HCG_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
  k_ang2pix<<<(unsigned)blocks, 256, 0, stream>>>(lon, lat, n, nside, pix, stat);
  HCG_LAUNCH_CHECK("k_ang2pix");
  return HCG_OK;
}

// ---------------------------------------------------------------------------
// a2: stable LSD radix sort, 8-bit digits.  A tile of 4096 keys per block;
// per pass: digit histogram per tile, exclusive scan over (digit, tile), then
// a scatter that ranks equal digits inside the tile in input order (round by
// round, wave ballots for lanes of one wave, per-wave counters for the rest).
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kScanChunk = 4096;

__global__ void __launch_bounds__(kRsThreads) k_radix_hist(const uint32_t* __restrict__ keys,
                                                           int64_t n, int shift,
                                                           uint32_t* __restrict__ hist,
                                                           int ntiles) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    const int64_t idx = base + r * kRsThreads + tid;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// Exclusive scan of a 256-thread block; returns the block total in *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh_wave, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh_wave[wave] = x;
  __syncthreads();
  uint32_t wave_off = 0, tot = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) wave_off += sh_wave[w];
    tot += sh_wave[w];
  }
  __syncthreads();
  *total = tot;
  return wave_off + x - v;
}

__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t* __restrict__ in, int64_t m,
                                                     uint32_t* __restrict__ partial) {
  __shared__ uint32_t sh[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t s = 0;
  for (int r = 0; r < kScanChunk / 256; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    if (i < m) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_scan_top(uint32_t* __restrict__ partial, int64_t np) {
  __shared__ uint32_t sh[4];
  uint32_t carry = 0;
  for (int64_t base = 0; base < np; base += 256) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = (i < np) ? partial[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < np) partial[i] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(256) k_scan_apply(const uint32_t* __restrict__ in, int64_t m,
                                                    const uint32_t* __restrict__ partial,
                                                    uint32_t* __restrict__ out) {
  __shared__ uint32_t sh[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t carry = partial[blockIdx.x];
  for (int r = 0; r < kScanChunk / 256; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    const uint32_t v = (i < m) ? in[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < m) out[i] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(kRsThreads) k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t n, int shift,
    const uint32_t* __restrict__ offs, int ntiles) {
  __shared__ uint32_t base_off[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base_off[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
  run[tid] = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile_base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    const int64_t idx = tile_base + r * kRsThreads + tid;
    const bool valid = idx < n;
    const uint32_t key = valid ? keys_in[idx] : 0u;
    const uint32_t val = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
    const uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base_off[d] + run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
    __syncthreads();
  }
}

static inline int64_t rs_ntiles(int64_t n) { return (n + kRsTile - 1) / kRsTile; }
static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t radix_sort_temp_bytes(int64_t n) {
  const int64_t nt = std::max<int64_t>(rs_ntiles(n), 1);
  const int64_t m = 256 * nt;
  const int64_t np = (m + kScanChunk - 1) / kScanChunk;
  return 2 * align256(sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1))  // ping-pong keys, vals
         + 2 * align256(sizeof(uint32_t) * (size_t)m)                      // hist, offsets
         + align256(sizeof(uint32_t) * (size_t)np);
}

// keys_out / perm_out receive the result; temp holds radix_sort_temp_bytes(n).
hcg_status launch_radix_sort(const uint32_t* keys_in, int64_t n, int key_bits, uint32_t* keys_out,
                             uint32_t* perm_out, void* temp, hipStream_t stream) {
  if (n == 0) return HCG_OK;
  const int passes = (key_bits + 7) / 8;
  const int64_t nt = rs_ntiles(n);
  const int64_t m = 256 * nt;
  const int64_t np = (m + kScanChunk - 1) / kScanChunk;
  char* t = (char*)temp;
  uint32_t* k_alt = (uint32_t*)t;
  t += align256(sizeof(uint32_t) * (size_t)n);
  uint32_t* v_alt = (uint32_t*)t;
  t += align256(sizeof(uint32_t) * (size_t)n);
  uint32_t* hist = (uint32_t*)t;
  t += align256(sizeof(uint32_t) * (size_t)m);
  uint32_t* offs = (uint32_t*)t;
  t += align256(sizeof(uint32_t) * (size_t)m);
  uint32_t* partial = (uint32_t*)t;
  // Ping-pong so that the final pass lands in keys_out / perm_out.
  const int npass = passes;
  const uint32_t* src_k = keys_in;
  const uint32_t* src_v = nullptr;
  for (int p = 0; p < npass; ++p) {
    // pass p writes to out if (npass - 1 - p) is even, else to alt
    const bool to_out = ((npass - 1 - p) % 2) == 0;
    uint32_t* dk = to_out ? keys_out : k_alt;
    uint32_t* dv = to_out ? perm_out : v_alt;
    const int shift = 8 * p;
    k_radix_hist<<<(unsigned)nt, kRsThreads, 0, stream>>>(src_k, n, shift, hist, (int)nt);
    HCG_LAUNCH_CHECK("k_radix_hist");
    k_scan_reduce<<<(unsigned)np, 256, 0, stream>>>(hist, m, partial);
    k_scan_top<<<1, 256, 0, stream>>>(partial, np);
    k_scan_apply<<<(unsigned)np, 256, 0, stream>>>(hist, m, partial, offs);
    HCG_LAUNCH_CHECK("k_scan");
    k_radix_scatter<<<(unsigned)nt, kRsThreads, 0, stream>>>(src_k, src_v, dk, dv, n, shift, offs,
                                                            (int)nt);
    HCG_LAUNCH_CHECK("k_radix_scatter");
    src_k = dk;
    src_v = dv;
  }
  return HCG_OK;
}

__global__ void __launch_bounds__(256) k_rel_keys(const uint32_t* __restrict__ pix, uint32_t base,
                                                  int64_t n, uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = pix[i] - base;
}

// ---------------------------------------------------------------------------
// a3: sorted coordinates as unit vectors (FP64): the gather measures the
// great-circle distance through the chord between two of them.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_permute_xyz(const double* __restrict__ lon,
                                                     const double* __restrict__ lat,
                                                     const uint32_t* __restrict__ perm, int64_t n,
                                                     double4* __restrict__ xyz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = perm[i];
  double sb, cb, sl, cl;
  sincos(lat[s] * kDeg2Rad, &sb, &cb);
  sincos(lon[s] * kDeg2Rad, &sl, &cl);
  xyz[i] = make_double4(cb * cl, cb * sl, sb, 0.0);
}

// ---------------------------------------------------------------------------
// a4: ring lookup table.  csr[r] = first sorted position whose pixel is in
// ring ring_first + r or later; csr[nrings] = n.
// ---------------------------------------------------------------------------
__global__ void k_ring_csr(const uint32_t* __restrict__ keys, int64_t n, int ns, int ring_first,
                           int nrings, uint32_t pix_base, uint32_t* __restrict__ csr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > nrings) return;
  if (r == nrings) { csr[r] = (uint32_t)n; return; }
  const int64_t target = hpx_ring_start(ns, ring_first + r) - (int64_t)pix_base;
  csr[r] = (target <= 0) ? 0u : lower_bound_u32(keys, 0u, (uint32_t)n, target);
}

// ---------------------------------------------------------------------------
// a5: candidate ranges per tile of output cells: ring_ranges (sphere.h) for
// every ring that can hold a sample within R of the tile.
// ---------------------------------------------------------------------------
// One wave per tile; lane r handles ring i_lo + r (+64, ...).  Ranges are
// written in ring order, two slots at most per ring.
__global__ void __launch_bounds__(256) k_tile_ranges(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ csr, int ns, int ring_first,
    int ring_last, uint32_t pix_base, GridGeom g, int ntx, int nty, double support_rad, int maxr,
    uint2* __restrict__ ranges, uint32_t* __restrict__ nranges, uint32_t* __restrict__ ncand,
    uint32_t* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntx * nty) return;
  const int tx = tile % ntx, ty = tile / ntx;
  const int ix0 = tx * kTileX, ix1 = min(g.nx, ix0 + kTileX) - 1;
  const int iy0 = ty * kTileY, iy1 = min(g.ny, iy0 + kTileY) - 1;
  double lon_a = cell_lon_deg(g, ix0) * kDeg2Rad, lon_b = cell_lon_deg(g, ix1) * kDeg2Rad;
  double lat_a = cell_lat_deg(g, iy0) * kDeg2Rad, lat_b = cell_lat_deg(g, iy1) * kDeg2Rad;
  if (lon_a > lon_b) { const double t = lon_a; lon_a = lon_b; lon_b = t; }
  if (lat_a > lat_b) { const double t = lat_a; lat_a = lat_b; lat_b = t; }
  const double half_pi = 0.5 * kPi;
  lat_a = fmax(-half_pi, fmin(half_pi, lat_a));
  lat_b = fmax(-half_pi, fmin(half_pi, lat_b));
  // conservative support: absorbs rounding of every bound below
  const double Rs = support_rad * (1.0 + 1e-9) + 1e-12;
  const double sR = sin(0.5 * Rs);
  const double hR = sR * sR;
  const double cos_g = cos(fmax(fabs(lat_a), fabs(lat_b)));
  const double z_top = sin(fmin(half_pi, lat_b + Rs));
  const double z_bot = sin(fmax(-half_pi, lat_a - Rs));
  const int i_lo = max(ring_first, (int)floor(hpx_ring_of_z(ns, z_top)) - 2);
  const int i_hi = min(ring_last, (int)ceil(hpx_ring_of_z(ns, z_bot)) + 2);
  uint2* out = ranges + (int64_t)tile * maxr;
  uint32_t count = 0, total = 0;
  bool overflow = false;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int base = i_lo; base <= i_hi; base += 64) {
    const int i = base + lane;
    RingRanges rr{0u, 0u, 0u, 0u};
    if (i <= i_hi)
      rr = ring_ranges(i, keys, csr, ns, ring_first, pix_base, lon_a, lon_b, lat_a, lat_b, Rs,
                       hR, cos_g);
    const bool h0 = rr.b0 > rr.a0, h1 = rr.b1 > rr.a1;
    const uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
    const uint32_t off = count + (uint32_t)__popcll(m0 & lt_mask) + (uint32_t)__popcll(m1 & lt_mask);
    uint32_t slot = off;
    if (h0) {
      if (slot < (uint32_t)maxr) out[slot] = make_uint2(rr.a0, rr.b0); else overflow = true;
      ++slot;
    }
    if (h1) {
      if (slot < (uint32_t)maxr) out[slot] = make_uint2(rr.a1, rr.b1); else overflow = true;
    }
    uint32_t len = (h0 ? rr.b0 - rr.a0 : 0u) + (h1 ? rr.b1 - rr.a1 : 0u);
    for (int o = 32; o > 0; o >>= 1) len += (uint32_t)__shfl_xor((int)len, o);
    total += len;
    count += (uint32_t)(__popcll(m0) + __popcll(m1));
  }
  if (__ballot(overflow) && lane == 0) atomicOr(&flags[0], 1u);
  if (lane == 0) {
    nranges[tile] = min(count, (uint32_t)maxr);
    ncand[tile] = total;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int auto_nside(double sigma_rad) {
  int ns = 1;
  while (ns < 16384 && std::sqrt(4.0 * kPi / (12.0 * (double)ns * ns)) > 0.5 * sigma_rad) ns *= 2;
  return ns;
}

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

static int bit_length(uint32_t v) {
  int b = 0;
  while (v) { ++b; v >>= 1; }
  return b;
}

// Owns device allocations until released.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
  void* release() { void* q = p; p = nullptr; return q; }
};

}  // namespace hcg

using namespace hcg;

extern "C" hcg_status hcg_ang2pix(const double* lon_deg, const double* lat_deg, int64_t n,
                                  int32_t nside, uint32_t* pix, void* hip_stream) {
  if (n < 0) return fail(HCG_E_ARG, "hcg_ang2pix: n < 0");
  if (n > 0 && (!lon_deg || !lat_deg || !pix)) return fail(HCG_E_ARG, "hcg_ang2pix: NULL pointer");
  if (!is_pow2(nside) || nside > 16384)
    return fail(HCG_E_ARG, "hcg_ang2pix: nside %d is not a power of two in 1..16384", nside);
  hcg_status st = check_device_arch();
  if (st != HCG_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;
  DevBuf stat;
  HCG_HIP(hipMalloc(&stat.p, 16));
  st = launch_ang2pix(lon_deg, lat_deg, n, nside, pix, (uint32_t*)stat.p, stream);
  if (st != HCG_OK) return st;
  uint32_t h[4];
  HCG_HIP(hipMemcpyAsync(h, stat.p, sizeof(h), hipMemcpyDeviceToHost, stream));
  HCG_HIP(hipStreamSynchronize(stream));
  if (h[2]) return fail(HCG_E_ARG, "hcg_ang2pix: %u non-finite or out-of-range coordinates", h[2]);
  return HCG_OK;
}

extern "C" hcg_status hcg_sort_keys(const uint32_t* keys_in, int64_t n, int32_t key_bits,
                                    uint32_t* keys_out, uint32_t* perm_out, void* hip_stream) {
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(HCG_E_ARG, "hcg_sort_keys: n out of range");
  if (key_bits < 1 || key_bits > 32) return fail(HCG_E_ARG, "hcg_sort_keys: key_bits must be 1..32");
  if (n > 0 && (!keys_in || !keys_out || !perm_out))
    return fail(HCG_E_ARG, "hcg_sort_keys: NULL pointer");
  if (n > 0 && (keys_in == keys_out)) return fail(HCG_E_ARG, "hcg_sort_keys: in-place not supported");
  hcg_status st = check_device_arch();
  if (st != HCG_OK) return st;
  if (n == 0) return HCG_OK;
  hipStream_t stream = (hipStream_t)hip_stream;
  DevBuf temp;
  HCG_HIP(hipMalloc(&temp.p, radix_sort_temp_bytes(n)));
  st = launch_radix_sort(keys_in, n, key_bits, keys_out, perm_out, temp.p, stream);
  if (st != HCG_OK) return st;
  HCG_HIP(hipStreamSynchronize(stream));
  return HCG_OK;
}

extern "C" hcg_status hcg_plan(hcg_plan_t* out, const double* lon_deg, const double* lat_deg,
                               int64_t n, const hcg_grid_desc* grid, double fwhm_deg,
                               double support_deg, const hcg_opts* opts, void* hip_stream) {
  if (!out) return fail(HCG_E_ARG, "hcg_plan: out is NULL");
  *out = nullptr;
  if (!lon_deg || !lat_deg || !grid) return fail(HCG_E_ARG, "hcg_plan: NULL pointer");
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(HCG_E_ARG, "hcg_plan: n must be in 1..2^31-1");
  if (grid->nx < 1 || grid->ny < 1) return fail(HCG_E_ARG, "hcg_plan: grid nx, ny must be >= 1");
  if ((int64_t)grid->nx * grid->ny > INT32_MAX) return fail(HCG_E_ARG, "hcg_plan: grid too large");
  if (!std::isfinite(grid->lon0_deg) || !std::isfinite(grid->lat0_deg) ||
      !std::isfinite(grid->dlon_deg) || !std::isfinite(grid->dlat_deg) || grid->dlon_deg == 0.0 ||
      grid->dlat_deg == 0.0)
    return fail(HCG_E_ARG, "hcg_plan: grid origin and steps must be finite, steps non-zero");
  {
    const double la = grid->lat0_deg - 0.5 * (grid->ny - 1) * grid->dlat_deg;
    const double lb = grid->lat0_deg + 0.5 * (grid->ny - 1) * grid->dlat_deg;
    if (std::fabs(la) > 90.0 || std::fabs(lb) > 90.0)
      return fail(HCG_E_ARG, "hcg_plan: grid cell latitudes leave [-90, 90]");
  }
  if (!(fwhm_deg > 0.0) || !std::isfinite(fwhm_deg)) return fail(HCG_E_ARG, "hcg_plan: fwhm must be > 0");
  if (!(support_deg >= 0.0) || !(support_deg < 90.0))
    return fail(HCG_E_ARG, "hcg_plan: support must be in [0, 90) degrees");
  hcg_opts o = {};
  if (opts) o = *opts;
  if ((o.tile_x && o.tile_x != kTileX) || (o.tile_y && o.tile_y != kTileY))
    return fail(HCG_E_UNSUPPORTED, "hcg_plan: only 8 x 8 cell tiles are built");
  if (o.coarsen || o.chan_tile || o.flags)
    return fail(HCG_E_UNSUPPORTED, "hcg_plan: coarsen, chan_tile and flags must be 0");
  const double sigma = fwhm_deg * kDeg2Rad / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  int nside = o.nside ? o.nside : auto_nside(sigma);
  if (!is_pow2(nside) || nside > 16384)
    return fail(HCG_E_ARG, "hcg_plan: nside %d is not a power of two in 1..16384", nside);
  hcg_status st = check_device_arch();
  if (st != HCG_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;

  // candidate-range slots per tile: rings in the tile's latitude span + 2R,
  // two ranges per ring; rings are at least 2/(3 Ns) apart in latitude
  const double R = support_deg * kDeg2Rad;
  const double tile_span = (kTileY - 1) * std::fabs(grid->dlat_deg) * kDeg2Rad;
  const double rings_d = (tile_span + 2.0 * R) / (2.0 / (3.0 * nside)) + 6.0;
  if (rings_d > kMaxRangesLimit / 2)
    return fail(HCG_E_UNSUPPORTED,
                "hcg_plan: support too wide for nside %d (%.0f rings per tile; at most %d)", nside,
                rings_d, kMaxRangesLimit / 2);
  const int maxr = 2 * (int)std::ceil(rings_d);
  const int ntx = (grid->nx + kTileX - 1) / kTileX, nty = (grid->ny + kTileY - 1) / kTileY;
  const int64_t ntiles = (int64_t)ntx * nty;

  // pass 1: pixels and their range (one small read-back)
  DevBuf pixbuf, statbuf;
  HCG_HIP(hipMalloc(&pixbuf.p, sizeof(uint32_t) * n));
  HCG_HIP(hipMalloc(&statbuf.p, 16));
  st = launch_ang2pix(lon_deg, lat_deg, n, nside, (uint32_t*)pixbuf.p, (uint32_t*)statbuf.p, stream);
  if (st != HCG_OK) return st;
  uint32_t hs[4];
  HCG_HIP(hipMemcpyAsync(hs, statbuf.p, sizeof(hs), hipMemcpyDeviceToHost, stream));
  HCG_HIP(hipStreamSynchronize(stream));
  if (hs[2]) return fail(HCG_E_ARG, "hcg_plan: %u sample coordinates are non-finite or |lat| > 90", hs[2]);
  const uint32_t pix_base = hs[0], pix_max = hs[1];
  const int ring_first = (int)hpx_pix2ring(nside, pix_base);
  const int ring_last = (int)hpx_pix2ring(nside, pix_max);
  const int nrings = ring_last - ring_first + 1;
  const int key_bits = bit_length(pix_max - pix_base);

  // plan arena
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off += align256(bytes); return at; };
  // xyz carries eight sentinel entries from n (NaN vectors) and perm one
  // (row 0): the gather reads them for candidate lists widened to whole
  // groups of 8 sorted positions
  const size_t o_xyz = take(sizeof(double4) * (n + 8));
  const size_t o_keys = take(sizeof(uint32_t) * n);
  const size_t o_perm = take(sizeof(uint32_t) * (n + 1));
  const size_t o_csr = take(sizeof(uint32_t) * (nrings + 1));
  const size_t o_rng = take(sizeof(uint2) * (size_t)ntiles * maxr);
  const size_t o_nr = take(sizeof(uint32_t) * ntiles);
  const size_t o_nc = take(sizeof(uint32_t) * ntiles);
  const size_t o_flags = take(16);
  const size_t arena_bytes = off;
  DevBuf arena, temp;
  if (hipMalloc(&arena.p, arena_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "hcg_plan: cannot allocate %zu bytes for the plan", arena_bytes);
  }
  const size_t temp_bytes = radix_sort_temp_bytes(n) + align256(sizeof(uint32_t) * n);
  if (hipMalloc(&temp.p, temp_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "hcg_plan: cannot allocate %zu bytes of scratch", temp_bytes);
  }
  char* A = (char*)arena.p;
  auto* p = new hcg_plan_s{};
  p->magic = kPlanMagic;
  HCG_HIP(hipGetDevice(&p->device));
  p->n = n;
  p->nside = nside;
  p->pix_base = pix_base;
  p->pix_max = pix_max;
  p->key_bits = key_bits;
  p->passes = (key_bits + 7) / 8;
  p->ring_first = ring_first;
  p->ring_last = ring_last;
  p->grid = GridGeom{grid->nx, grid->ny, grid->lon0_deg, grid->lat0_deg, grid->dlon_deg,
                     grid->dlat_deg};
  p->fwhm_deg = fwhm_deg;
  p->support_deg = support_deg;
  p->sigma_rad = sigma;
  p->support_rad = R;
  p->ntx = ntx;
  p->nty = nty;
  p->maxr = maxr;
  p->arena_bytes = arena_bytes;
  p->xyz = (double4*)(A + o_xyz);
  p->keys = (uint32_t*)(A + o_keys);
  p->perm = (uint32_t*)(A + o_perm);
  p->csr = (uint32_t*)(A + o_csr);
  p->ranges = (uint2*)(A + o_rng);
  p->nranges = (uint32_t*)(A + o_nr);
  p->ncand = (uint32_t*)(A + o_nc);
  p->flags = (uint32_t*)(A + o_flags);
  struct PlanGuard {
    hcg_plan_s* p;
    ~PlanGuard() { delete p; }
  } guard{p};

  // keys relative to the smallest pixel, then the stable sort
  uint32_t* rel = (uint32_t*)((char*)temp.p + radix_sort_temp_bytes(n));
  k_rel_keys<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>((const uint32_t*)pixbuf.p,
                                                               pix_base, n, rel);
  HCG_LAUNCH_CHECK("k_rel_keys");
  st = launch_radix_sort(rel, n, key_bits == 0 ? 1 : key_bits, p->keys, p->perm, temp.p, stream);
  if (st != HCG_OK) return st;
  k_permute_xyz<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(lon_deg, lat_deg, p->perm, n,
                                                                p->xyz);
  HCG_LAUNCH_CHECK("k_permute_xyz");
  HCG_HIP(hipMemsetAsync(p->xyz + n, 0xFF, 8 * sizeof(double4), stream));  // all-ones: NaN
  HCG_HIP(hipMemsetAsync(p->perm + n, 0, sizeof(uint32_t), stream));
  k_ring_csr<<<(unsigned)((nrings + 1 + 255) / 256), 256, 0, stream>>>(
      p->keys, n, nside, ring_first, nrings, pix_base, p->csr);
  HCG_LAUNCH_CHECK("k_ring_csr");
  HCG_HIP(hipMemsetAsync(p->flags, 0, 16, stream));
  k_tile_ranges<<<(unsigned)((ntiles + 3) / 4), 256, 0, stream>>>(
      p->keys, p->csr, nside, ring_first, ring_last, pix_base, p->grid, ntx, nty, R, maxr,
      p->ranges, p->nranges, p->ncand, p->flags);
  HCG_LAUNCH_CHECK("k_tile_ranges");
  uint32_t fl[4];
  HCG_HIP(hipMemcpyAsync(fl, p->flags, sizeof(fl), hipMemcpyDeviceToHost, stream));
  HCG_HIP(hipStreamSynchronize(stream));
  if (fl[0]) return fail(HCG_E_DEVICE, "hcg_plan: candidate-range slots overflowed (internal bound)");
  p->arena = arena.release();
  guard.p = nullptr;
  plan_register(p);
  *out = p;
  return HCG_OK;
}
