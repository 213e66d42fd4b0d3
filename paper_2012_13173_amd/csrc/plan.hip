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
// Block `bx` of `nb` strides over the samples; one set of atomics per block.
__device__ inline void ang2pix_block(const double* __restrict__ lon,
                                     const double* __restrict__ lat, int64_t n, int ns,
                                     uint32_t* __restrict__ pix, uint32_t* __restrict__ stat,
                                     uint32_t bx, uint32_t nb) {
  __shared__ uint32_t s_red[3][4];
  uint32_t vmin = 0xFFFFFFFFu, vmax = 0u, bad = 0u;
  for (int64_t i = (int64_t)bx * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)nb * blockDim.x) {
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

__global__ void __launch_bounds__(256) k_ang2pix(const double* __restrict__ lon,
                                                 const double* __restrict__ lat, int64_t n,
                                                 int ns, uint32_t* __restrict__ pix,
                                                 uint32_t* __restrict__ stat) {
  ang2pix_block(lon, lat, n, ns, pix, stat, blockIdx.x, gridDim.x);
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

__device__ inline void radix_hist_block(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                        uint32_t* __restrict__ hist, int ntiles, uint32_t bx) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)bx * kRsTile;
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    const int64_t idx = base + r * kRsThreads + tid;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * ntiles + bx] = h[tid];
}

__global__ void __launch_bounds__(kRsThreads) k_radix_hist(const uint32_t* __restrict__ keys,
                                                           int64_t n, int shift,
                                                           uint32_t* __restrict__ hist,
                                                           int ntiles) {
  radix_hist_block(keys, n, shift, hist, ntiles, blockIdx.x);
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

__device__ inline void scan_reduce_block(const uint32_t* __restrict__ in, int64_t m,
                                         uint32_t* __restrict__ partial, uint32_t bx) {
  __shared__ uint32_t sh[4];
  const int64_t base = (int64_t)bx * kScanChunk;
  uint32_t s = 0;
  for (int r = 0; r < kScanChunk / 256; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    if (i < m) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) partial[bx] = tot;
}

__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t* __restrict__ in, int64_t m,
                                                     uint32_t* __restrict__ partial) {
  scan_reduce_block(in, m, partial, blockIdx.x);
}

__device__ inline void scan_top_block(uint32_t* __restrict__ partial, int64_t np) {
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

__global__ void __launch_bounds__(256) k_scan_top(uint32_t* __restrict__ partial, int64_t np) {
  scan_top_block(partial, np);
}

__device__ inline void scan_apply_block(const uint32_t* __restrict__ in, int64_t m,
                                        const uint32_t* __restrict__ partial,
                                        uint32_t* __restrict__ out, uint32_t bx) {
  __shared__ uint32_t sh[4];
  const int64_t base = (int64_t)bx * kScanChunk;
  uint32_t carry = partial[bx];
  for (int r = 0; r < kScanChunk / 256; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    const uint32_t v = (i < m) ? in[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < m) out[i] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(256) k_scan_apply(const uint32_t* __restrict__ in, int64_t m,
                                                    const uint32_t* __restrict__ partial,
                                                    uint32_t* __restrict__ out) {
  scan_apply_block(in, m, partial, out, blockIdx.x);
}

__device__ inline void radix_scatter_block(const uint32_t* __restrict__ keys_in,
                                           const uint32_t* __restrict__ vals_in,
                                           uint32_t* __restrict__ keys_out,
                                           uint32_t* __restrict__ vals_out, int64_t n, int shift,
                                           const uint32_t* __restrict__ offs, int ntiles,
                                           uint32_t bx) {
  __shared__ uint32_t base_off[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base_off[tid] = offs[(int64_t)tid * ntiles + bx];
  run[tid] = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile_base = (int64_t)bx * kRsTile;
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

__global__ void __launch_bounds__(kRsThreads) k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t n, int shift,
    const uint32_t* __restrict__ offs, int ntiles) {
  radix_scatter_block(keys_in, vals_in, keys_out, vals_out, n, shift, offs, ntiles, blockIdx.x);
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
// Cell centres as unit vectors (FP64), one per cell of the target grid: from
// the linear lon/lat geometry, or from caller arrays of centres (a projected
// map).  A centre that is not finite or has |lat| > 90 gives a NaN vector: a
// cell that no sample reaches.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cell_vecs_linear(GridGeom g, double4* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)g.nx * g.ny) return;
  const CellVec c = cell_vec(g, (int)(i % g.nx), (int)(i / g.nx));
  out[i] = make_double4(c.x, c.y, c.z, 0.0);
}

__global__ void __launch_bounds__(256) k_cell_vecs_arrays(const double* __restrict__ lon,
                                                          const double* __restrict__ lat,
                                                          int64_t ncell,
                                                          double4* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const double lo = lon[i], la = lat[i];
  if (!isfinite(lo) || !isfinite(la) || fabs(la) > 90.0) {
    const double nan = __builtin_nan("");
    out[i] = make_double4(nan, nan, nan, 0.0);
    return;
  }
  double sb, cb, sl, cl;
  sincos(la * kDeg2Rad, &sb, &cb);
  sincos(lo * kDeg2Rad, &sl, &cl);
  out[i] = make_double4(cb * cl, cb * sl, sb, 0.0);
}

// ---------------------------------------------------------------------------
// a5: candidate ranges per tile of output cells: ring_ranges (sphere.h) for
// every ring that can hold a sample within R of the tile.
// ---------------------------------------------------------------------------
// One wave per tile; lane r handles ring i_lo + r (+64, ...).  Ranges are
// written in ring order, two slots at most per ring.  The tile is the
// lon/lat box [lon_a, lon_b] x [lat_a, lat_b] (radians) of its cells, or a
// point (a degenerate box) with the support widened by the radius of a cap
// holding its cells; Rs is the (widened, conservative) support.
__device__ void tile_ranges_wave(const uint32_t* __restrict__ keys,
                                 const uint32_t* __restrict__ csr, int ns, int ring_first,
                                 int ring_last, uint32_t pix_base, double lon_a, double lon_b,
                                 double lat_a, double lat_b, double Rs, int maxr,
                                 uint2* __restrict__ out, uint32_t* nranges_out,
                                 uint32_t* ncand_out, uint32_t* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const double half_pi = 0.5 * kPi;
  const double sR = sin(0.5 * fmin(Rs, kPi));
  const double hR = sR * sR;
  const double cos_g = cos(fmax(fabs(lat_a), fabs(lat_b)));
  const double z_top = sin(fmin(half_pi, lat_b + Rs));
  const double z_bot = sin(fmax(-half_pi, lat_a - Rs));
  const int i_lo = max(ring_first, (int)floor(hpx_ring_of_z(ns, z_top)) - 2);
  const int i_hi = min(ring_last, (int)ceil(hpx_ring_of_z(ns, z_bot)) + 2);
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
    *nranges_out = min(count, (uint32_t)maxr);
    *ncand_out = total;
  }
}

// Linear lon/lat grid: the box of the tile's cell centres (one wave per
// tile; block bx holds tiles 4 bx .. 4 bx + 3).
__device__ inline void tile_ranges_linear(const uint32_t* __restrict__ keys,
                                          const uint32_t* __restrict__ csr, int ns,
                                          int ring_first, int ring_last, uint32_t pix_base,
                                          const GridGeom& g, int ntx, int nty, double support_rad,
                                          int maxr, uint2* __restrict__ ranges,
                                          uint32_t* __restrict__ nranges,
                                          uint32_t* __restrict__ ncand,
                                          uint32_t* __restrict__ flags, uint32_t bx) {
  const int tile = (int)bx * 4 + (threadIdx.x >> 6);
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
  tile_ranges_wave(keys, csr, ns, ring_first, ring_last, pix_base, lon_a, lon_b, lat_a, lat_b, Rs,
                   maxr, ranges + (int64_t)tile * maxr, &nranges[tile], &ncand[tile], flags);
}

__global__ void __launch_bounds__(256) k_tile_ranges(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ csr, int ns, int ring_first,
    int ring_last, uint32_t pix_base, GridGeom g, int ntx, int nty, double support_rad, int maxr,
    uint2* __restrict__ ranges, uint32_t* __restrict__ nranges, uint32_t* __restrict__ ncand,
    uint32_t* __restrict__ flags) {
  tile_ranges_linear(keys, csr, ns, ring_first, ring_last, pix_base, g, ntx, nty, support_rad,
                     maxr, ranges, nranges, ncand, flags, blockIdx.x);
}

// Cells given by their centres: per tile (one wave), the cap around the
// normalised mean of its cells' unit vectors that holds them all; caps[t] =
// (centre lon, centre lat, radius) in radians, radius < 0 for a tile
// without cells.  The largest radius goes to *rmax (as the bits of a
// non-negative double, which order like the values).
__global__ void __launch_bounds__(256) k_tile_caps(const double4* __restrict__ cells, int nx,
                                                   int ny, int ntx, int nty,
                                                   double4* __restrict__ caps,
                                                   unsigned long long* __restrict__ rmax) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntx * nty) return;
  const int x = (tile % ntx) * kTileX + (lane & 7), y = (tile / ntx) * kTileY + (lane >> 3);
  double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
  if (x < nx && y < ny) v = cells[(int64_t)y * nx + x];
  const bool valid = (x < nx && y < ny) && v.x == v.x;
  double sx = valid ? v.x : 0.0, sy = valid ? v.y : 0.0, sz = valid ? v.z : 0.0;
  for (int o = 1; o < 64; o <<= 1) {
    sx += __shfl_xor(sx, o);
    sy += __shfl_xor(sy, o);
    sz += __shfl_xor(sz, o);
  }
  const double nrm = sqrt(sx * sx + sy * sy + sz * sz);
  // a tile of cells spread over a hemisphere or more has no useful centre:
  // take any and the whole sphere as its cap
  const bool degenerate = !(nrm > 1e-6);
  const double cx = degenerate ? 0.0 : sx / nrm, cy = degenerate ? 0.0 : sy / nrm,
               cz = degenerate ? 1.0 : sz / nrm;
  double c2 = 0.0;
  if (valid) {
    const double dx = v.x - cx, dy = v.y - cy, dz = v.z - cz;
    c2 = dx * dx + dy * dy + dz * dz;
  }
  for (int o = 1; o < 64; o <<= 1) c2 = fmax(c2, __shfl_xor(c2, o));
  const bool any = __ballot(valid) != 0ull;
  if (lane == 0) {
    double r = 2.0 * asin(fmin(0.5 * sqrt(c2), 1.0));
    if (degenerate) r = kPi;
    if (!any) r = -1.0;
    caps[tile] = make_double4(atan2(cy, cx), asin(fmax(-1.0, fmin(1.0, cz))), r, 0.0);
    if (r > 0.0) atomicMax(rmax, (unsigned long long)__double_as_longlong(r));
  }
}

__global__ void __launch_bounds__(256) k_tile_ranges_cap(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ csr, int ns, int ring_first,
    int ring_last, uint32_t pix_base, const double4* __restrict__ caps, int ntiles,
    double support_rad, int maxr, uint2* __restrict__ ranges, uint32_t* __restrict__ nranges,
    uint32_t* __restrict__ ncand, uint32_t* __restrict__ flags) {
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;
  const double4 cap = caps[tile];
  if (cap.z < 0.0) {
    if ((threadIdx.x & 63) == 0) {
      nranges[tile] = 0u;
      ncand[tile] = 0u;
    }
    return;
  }
  // every cell is within cap.z of the centre, so every sample within R of a
  // cell is within R + cap.z of it (triangle inequality); slack for rounding
  const double Rs = (support_rad + cap.z) * (1.0 + 1e-9) + 1e-12;
  tile_ranges_wave(keys, csr, ns, ring_first, ring_last, pix_base, cap.x, cap.x, cap.y, cap.y, Rs,
                   maxr, ranges + (int64_t)tile * maxr, &nranges[tile], &ncand[tile], flags);
}

// ---------------------------------------------------------------------------
// Many plans at once (batches of fields on linear grids): every step runs
// for all fields in one launch.  A launch's blocks are the fields' blocks
// laid end to end; block b finds its field by binary search in the launch
// kind's prefix table (fields_blocks[kind][0..nf]) and runs the step's
// block body for that field's arrays.
// ---------------------------------------------------------------------------
enum FieldBlockKind : int {
  kFbSamples = 0,    // ceil(n / 256)
  kFbSortTiles = 1,  // radix-sort tiles of 4096 keys
  kFbScan = 2,       // scan chunks of the digit histogram
  kFbOne = 3,        // one block per field
  kFbCells = 4,      // ceil(cells / 256)
  kFbRings = 5,      // ceil((rings + 1) / 256)
  kFbTiles = 6,      // ceil(tiles / 4)
  kFbKinds = 7
};

struct PlanField {
  // first step
  const double* lon;
  const double* lat;
  int64_t n;
  int nside;
  uint32_t* pix;
  uint32_t* stat;
  // second step
  GridGeom grid;
  int ntx, nty, maxr, ring_first, ring_last, nrings;
  uint32_t pix_base;
  double support_rad;
  int64_t rs_ntiles, rs_m, rs_np;
  uint32_t *rel, *k_alt, *v_alt, *hist, *offs, *partial;
  uint32_t *keys, *perm, *csr, *nranges, *ncand, *flags;
  uint2* ranges;
  double4 *xyz, *cells;
};

// The field of flattened block b of launch kind `kind`, and its block there.
__device__ inline int field_of_block(const uint32_t* __restrict__ prefix, int nf, uint32_t b,
                                     uint32_t* local) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  *local = b - prefix[lo];
  return lo;
}

#define HCG_FIELD_BLOCK(kind)                                                     \
  uint32_t lb;                                                                   \
  const int fi = field_of_block(prefix + (size_t)(kind) * (nf + 1), nf, blockIdx.x, &lb); \
  const PlanField& F = fields[fi];

__global__ void __launch_bounds__(256) k_stat_init_fields(const PlanField* __restrict__ fields,
                                                          const uint32_t* __restrict__ prefix,
                                                          int nf) {
  HCG_FIELD_BLOCK(kFbOne);
  (void)lb;
  if (threadIdx.x < 4) F.stat[threadIdx.x] = (threadIdx.x == 0) ? 0xFFFFFFFFu : 0u;
}

__global__ void __launch_bounds__(256) k_ang2pix_fields(const PlanField* __restrict__ fields,
                                                        const uint32_t* __restrict__ prefix,
                                                        int nf) {
  HCG_FIELD_BLOCK(kFbSamples);
  const uint32_t nb = prefix[kFbSamples * (nf + 1) + fi + 1] - prefix[kFbSamples * (nf + 1) + fi];
  ang2pix_block(F.lon, F.lat, F.n, F.nside, F.pix, F.stat, lb, nb);
}

__global__ void __launch_bounds__(256) k_cells_rel_fields(const PlanField* __restrict__ fields,
                                                          const uint32_t* __restrict__ prefix,
                                                          int nf) {
  // cell vectors into the plan, then (from block kFbCells onward) the keys
  // relative to the smallest pixel: one launch of kFbCells + kFbSamples blocks
  const uint32_t ncb = prefix[kFbCells * (nf + 1) + nf];
  if (blockIdx.x < ncb) {
    HCG_FIELD_BLOCK(kFbCells);
    const int64_t i = (int64_t)lb * 256 + threadIdx.x;
    if (i < (int64_t)F.grid.nx * F.grid.ny) {
      const CellVec c = cell_vec(F.grid, (int)(i % F.grid.nx), (int)(i / F.grid.nx));
      F.cells[i] = make_double4(c.x, c.y, c.z, 0.0);
    }
    return;
  }
  uint32_t lb;
  const int fi = field_of_block(prefix + (size_t)kFbSamples * (nf + 1), nf, blockIdx.x - ncb, &lb);
  const PlanField& F = fields[fi];
  const int64_t i = (int64_t)lb * 256 + threadIdx.x;
  if (i < F.n) F.rel[i] = F.pix[i] - F.pix_base;
}

// Pass p of `passes` (every field takes the same number; a digit that is
// zero for all keys of a field leaves its order as it is): the pass reads the
// previous pass's output (the relative keys and no values for p = 0) and
// writes to the plan's keys and permutation on the last pass, ping-pong
// before it.
__device__ inline void sort_pass_arrays(const PlanField& F, int p, int passes,
                                        const uint32_t** sk, const uint32_t** sv, uint32_t** dk,
                                        uint32_t** dv) {
  auto out_of = [&](int q, uint32_t** k, uint32_t** v) {
    const bool to_out = ((passes - 1 - q) % 2) == 0;
    *k = to_out ? F.keys : F.k_alt;
    *v = to_out ? F.perm : F.v_alt;
  };
  out_of(p, dk, dv);
  if (p == 0) {
    *sk = F.rel;
    *sv = nullptr;
  } else {
    uint32_t *k, *v;
    out_of(p - 1, &k, &v);
    *sk = k;
    *sv = v;
  }
}

__global__ void __launch_bounds__(kRsThreads) k_radix_hist_fields(
    const PlanField* __restrict__ fields, const uint32_t* __restrict__ prefix, int nf, int p,
    int passes) {
  HCG_FIELD_BLOCK(kFbSortTiles);
  const uint32_t *sk, *sv;
  uint32_t *dk, *dv;
  sort_pass_arrays(F, p, passes, &sk, &sv, &dk, &dv);
  radix_hist_block(sk, F.n, 8 * p, F.hist, (int)F.rs_ntiles, lb);
}

__global__ void __launch_bounds__(256) k_scan_reduce_fields(const PlanField* __restrict__ fields,
                                                            const uint32_t* __restrict__ prefix,
                                                            int nf) {
  HCG_FIELD_BLOCK(kFbScan);
  scan_reduce_block(F.hist, F.rs_m, F.partial, lb);
}

__global__ void __launch_bounds__(256) k_scan_top_fields(const PlanField* __restrict__ fields,
                                                         const uint32_t* __restrict__ prefix,
                                                         int nf) {
  HCG_FIELD_BLOCK(kFbOne);
  (void)lb;
  scan_top_block(F.partial, F.rs_np);
}

__global__ void __launch_bounds__(256) k_scan_apply_fields(const PlanField* __restrict__ fields,
                                                           const uint32_t* __restrict__ prefix,
                                                           int nf) {
  HCG_FIELD_BLOCK(kFbScan);
  scan_apply_block(F.hist, F.rs_m, F.partial, F.offs, lb);
}

__global__ void __launch_bounds__(kRsThreads) k_radix_scatter_fields(
    const PlanField* __restrict__ fields, const uint32_t* __restrict__ prefix, int nf, int p,
    int passes) {
  HCG_FIELD_BLOCK(kFbSortTiles);
  const uint32_t *sk, *sv;
  uint32_t *dk, *dv;
  sort_pass_arrays(F, p, passes, &sk, &sv, &dk, &dv);
  radix_scatter_block(sk, sv, dk, dv, F.n, 8 * p, F.offs, (int)F.rs_ntiles, lb);
}

__global__ void __launch_bounds__(256) k_permute_xyz_fields(const PlanField* __restrict__ fields,
                                                            const uint32_t* __restrict__ prefix,
                                                            int nf) {
  HCG_FIELD_BLOCK(kFbSamples);
  const int64_t i = (int64_t)lb * 256 + threadIdx.x;
  if (i < F.n) {
    const uint32_t s = F.perm[i];
    double sb, cb, sl, cl;
    sincos(F.lat[s] * kDeg2Rad, &sb, &cb);
    sincos(F.lon[s] * kDeg2Rad, &sl, &cl);
    F.xyz[i] = make_double4(cb * cl, cb * sl, sb, 0.0);
  }
  // the sentinels past n: eight NaN vectors, permutation entry 0, flags 0
  if (lb == 0 && threadIdx.x < 8) {
    const double nan = __builtin_nan("");
    F.xyz[F.n + threadIdx.x] = make_double4(nan, nan, nan, nan);
    if (threadIdx.x == 0) F.perm[F.n] = 0u;
    if (threadIdx.x < 4) F.flags[threadIdx.x] = 0u;
  }
}

__global__ void __launch_bounds__(256) k_ring_csr_fields(const PlanField* __restrict__ fields,
                                                         const uint32_t* __restrict__ prefix,
                                                         int nf) {
  HCG_FIELD_BLOCK(kFbRings);
  const int r = (int)lb * 256 + threadIdx.x;
  if (r > F.nrings) return;
  if (r == F.nrings) {
    F.csr[r] = (uint32_t)F.n;
    return;
  }
  const int64_t target = hpx_ring_start(F.nside, F.ring_first + r) - (int64_t)F.pix_base;
  F.csr[r] = (target <= 0) ? 0u : lower_bound_u32(F.keys, 0u, (uint32_t)F.n, target);
}

__global__ void __launch_bounds__(256) k_tile_ranges_fields(const PlanField* __restrict__ fields,
                                                            const uint32_t* __restrict__ prefix,
                                                            int nf) {
  HCG_FIELD_BLOCK(kFbTiles);
  tile_ranges_linear(F.keys, F.csr, F.nside, F.ring_first, F.ring_last, F.pix_base, F.grid, F.ntx,
                     F.nty, F.support_rad, F.maxr, F.ranges, F.nranges, F.ncand, F.flags, lb);
}
#undef HCG_FIELD_BLOCK

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

// Freed memory the pool keeps for reuse (a plan of the 20M-sample cube
// takes about 1.2 GB of arena and scratch).
constexpr uint64_t kPoolKeepBytes = 2ull << 30;
constexpr int kMaxDevices = 64;

hipMemPool_t plan_pool() {
  static std::mutex mu;
  static hipMemPool_t pools[kMaxDevices] = {};
  static bool tried[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!tried[dev]) {
    tried[dev] = true;
    hipMemPoolProps props = {};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
      uint64_t keep = kPoolKeepBytes;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      pools[dev] = pool;
    } else {
      (void)hipGetLastError();
    }
  }
  return pools[dev];
}

// Owns a device allocation until released.  Scratch that lives only for
// one call is stream-ordered (alloc_async): hipFree would synchronise the
// whole device, which serialises plans built on several streams at once.
struct DevBuf {
  void* p = nullptr;
  hipStream_t s = nullptr;
  bool async = false;
  ~DevBuf() {
    if (!p) return;
    if (async) (void)hipFreeAsync(p, s);
    else (void)hipFree(p);
  }
  void* release() { void* q = p; p = nullptr; return q; }
  hipError_t alloc_async(size_t bytes, hipStream_t stream) {
    hipMemPool_t pool = plan_pool();
    const hipError_t e = pool ? hipMallocFromPoolAsync(&p, bytes, pool, stream)
                              : hipMallocAsync(&p, bytes, stream);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    s = stream;
    async = true;
    return e;
  }
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
  HCG_HIP(stat.alloc_async(16, stream));
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
  HCG_HIP(temp.alloc_async(radix_sort_temp_bytes(n), stream));
  st = launch_radix_sort(keys_in, n, key_bits, keys_out, perm_out, temp.p, stream);
  if (st != HCG_OK) return st;
  HCG_HIP(hipStreamSynchronize(stream));
  return HCG_OK;
}

namespace {

// What a plan's target and kernel come down to once the arguments are
// checked: the linear grid or the caller's centre arrays, the kernel's
// precomputed factors and the sigma that picks the automatic nside.
struct PlanTarget {
  const hcg_grid_desc* grid;  // linear lon/lat grid, or NULL
  const double* clon;         // or: device centre arrays [ny][nx]
  const double* clat;
  int32_t nx, ny;
};

hcg_status check_grid(const hcg_grid_desc* grid, const char* who) {
  if (grid->nx < 1 || grid->ny < 1) return fail(HCG_E_ARG, "%s: grid nx, ny must be >= 1", who);
  if ((int64_t)grid->nx * grid->ny > INT32_MAX) return fail(HCG_E_ARG, "%s: grid too large", who);
  if (!std::isfinite(grid->lon0_deg) || !std::isfinite(grid->lat0_deg) ||
      !std::isfinite(grid->dlon_deg) || !std::isfinite(grid->dlat_deg) || grid->dlon_deg == 0.0 ||
      grid->dlat_deg == 0.0)
    return fail(HCG_E_ARG, "%s: grid origin and steps must be finite, steps non-zero", who);
  const double la = grid->lat0_deg - 0.5 * (grid->ny - 1) * grid->dlat_deg;
  const double lb = grid->lat0_deg + 0.5 * (grid->ny - 1) * grid->dlat_deg;
  if (std::fabs(la) > 90.0 || std::fabs(lb) > 90.0)
    return fail(HCG_E_ARG, "%s: grid cell latitudes leave [-90, 90]", who);
  return HCG_OK;
}

double sigma_of_fwhm(double fwhm_deg) {
  return fwhm_deg * kDeg2Rad / (2.0 * std::sqrt(2.0 * std::log(2.0)));
}

// Kernel factors (Section 3.6 (iii)) and the width that sets the automatic
// nside: sigma of the Gaussian, of the minor axis of the elliptical one, and
// half the smaller of the sinc's zero and taper widths.
hcg_status kernel_params(const hcg_kernel* k, const char* who, KernelParams* kp,
                         double* sigma_nside, double* fwhm_nominal) {
  const double l2e = 1.4426950408889634;
  memset(kp, 0, sizeof(*kp));
  kp->type = k->type;
  auto bad = [&](double v) { return !(v > 0.0) || !std::isfinite(v); };
  switch (k->type) {
    case HCG_KERNEL_GAUSS: {
      if (bad(k->fwhm_deg)) return fail(HCG_E_ARG, "%s: fwhm must be > 0", who);
      const double sg = sigma_of_fwhm(k->fwhm_deg);
      kp->wscale = -l2e / (2.0 * sg * sg);
      *sigma_nside = sg;
      *fwhm_nominal = k->fwhm_deg;
      return HCG_OK;
    }
    case HCG_KERNEL_ELLIPTIC_GAUSS: {
      if (bad(k->fwhm_deg) || bad(k->fwhm_minor_deg) || !std::isfinite(k->pa_deg))
        return fail(HCG_E_ARG, "%s: elliptical kernel needs fwhm, fwhm_minor > 0 and a finite pa", who);
      const double sa = sigma_of_fwhm(k->fwhm_deg), sb = sigma_of_fwhm(k->fwhm_minor_deg);
      kp->kmaj = -l2e / (2.0 * sa * sa);
      kp->kmin = -l2e / (2.0 * sb * sb);
      kp->cpa = std::cos(k->pa_deg * kDeg2Rad);
      kp->spa = std::sin(k->pa_deg * kDeg2Rad);
      kp->wscale = kp->kmaj;
      *sigma_nside = std::min(sa, sb);
      *fwhm_nominal = k->fwhm_deg;
      return HCG_OK;
    }
    case HCG_KERNEL_TAPERED_SINC: {
      if (bad(k->sinc_deg) || bad(k->taper_deg))
        return fail(HCG_E_ARG, "%s: tapered sinc needs sinc_deg, taper_deg > 0", who);
      const double b = k->sinc_deg * kDeg2Rad, a = k->taper_deg * kDeg2Rad;
      kp->sinc_k = kPi / b;
      kp->taper_k = -l2e / (a * a);
      *sigma_nside = 0.5 * std::min(a, b);
      *fwhm_nominal = k->sinc_deg;
      return HCG_OK;
    }
    default:
      return fail(HCG_E_UNSUPPORTED, "%s: unknown kernel type %d", who, (int)k->type);
  }
}

// A plan is built in three steps with a host read between them: begin (cell
// vectors and the samples' pixels, whose range comes back to the host),
// middle (the sizes from that range; the sorted samples, ring table and tile
// ranges; an overflow flag comes back) and finish (the flag checked, the
// plan registered).  hcg_plan runs the steps with a stream synchronisation
// after each; hcg_plan_batch runs each step for every field and
// synchronises once per step.  host: 64 bytes of host memory that the
// device writes between the steps (page-locked for the batch).
struct PlanBuilder {
  const char* who = "";
  const double* lon_deg = nullptr;
  const double* lat_deg = nullptr;
  int64_t n = 0;
  PlanTarget tg{};
  double support_deg = 0.0;
  KernelParams kp{};
  double sigma = 0.0, fwhm_nominal = 0.0;
  int nside = 0;
  hipStream_t stream = nullptr;
  uint32_t* host = nullptr;  // [0..7] pixel stats, [8..11] flags
  int nx = 0, ny = 0, ntx = 0, nty = 0;
  int64_t ntiles = 0, ncell = 0;
  double R = 0.0;
  DevBuf pixbuf, statbuf, cellbuf, capbuf, arena, temp;
  hcg_plan_s* p = nullptr;

  ~PlanBuilder() { delete p; }

  hcg_status begin(const double* lon, const double* lat, int64_t n_, const PlanTarget& tg_,
                   const hcg_kernel* kernel, double support, const hcg_opts* opts,
                   hipStream_t s, uint32_t* host_, const char* who_) {
    who = who_;
    lon_deg = lon;
    lat_deg = lat;
    n = n_;
    tg = tg_;
    support_deg = support;
    stream = s;
    host = host_;
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(HCG_E_ARG, "%s: n must be in 1..2^31-1", who);
    if (!(support_deg >= 0.0) || !(support_deg < 90.0))
      return fail(HCG_E_ARG, "%s: support must be in [0, 90) degrees", who);
    hcg_status st = kernel_params(kernel, who, &kp, &sigma, &fwhm_nominal);
    if (st != HCG_OK) return st;
    hcg_opts o = {};
    if (opts) o = *opts;
    if ((o.tile_x && o.tile_x != kTileX) || (o.tile_y && o.tile_y != kTileY))
      return fail(HCG_E_UNSUPPORTED, "%s: only 8 x 8 cell tiles are built", who);
    if (o.coarsen || o.chan_tile || o.flags)
      return fail(HCG_E_UNSUPPORTED, "%s: coarsen, chan_tile and flags must be 0", who);
    nside = o.nside ? o.nside : auto_nside(sigma);
    if (!is_pow2(nside) || nside > 16384)
      return fail(HCG_E_ARG, "%s: nside %d is not a power of two in 1..16384", who, nside);
    st = check_device_arch();
    if (st != HCG_OK) return st;
    nx = tg.grid ? tg.grid->nx : tg.nx;
    ny = tg.grid ? tg.grid->ny : tg.ny;
    ntx = (nx + kTileX - 1) / kTileX;
    nty = (ny + kTileY - 1) / kTileY;
    ntiles = (int64_t)ntx * nty;
    ncell = (int64_t)nx * ny;
    R = support_deg * kDeg2Rad;

    // pixels and their range; for centre arrays also the cell vectors and
    // the tile caps, whose largest radius sizes the candidate-range slots
    HCG_HIP(pixbuf.alloc_async(sizeof(uint32_t) * n, stream));
    HCG_HIP(statbuf.alloc_async(32, stream));
    if (cellbuf.alloc_async(sizeof(double4) * ncell, stream) != hipSuccess) {
      (void)hipGetLastError();
      return fail(HCG_E_NOMEM, "%s: cannot allocate the cell vectors", who);
    }
    double4* cells = (double4*)cellbuf.p;
    const unsigned cell_blocks = (unsigned)((ncell + 255) / 256);
    if (tg.grid) {
      const GridGeom gg{tg.grid->nx, tg.grid->ny, tg.grid->lon0_deg, tg.grid->lat0_deg,
                        tg.grid->dlon_deg, tg.grid->dlat_deg};
      k_cell_vecs_linear<<<cell_blocks, 256, 0, stream>>>(gg, cells);
      HCG_LAUNCH_CHECK("k_cell_vecs_linear");
    } else {
      k_cell_vecs_arrays<<<cell_blocks, 256, 0, stream>>>(tg.clon, tg.clat, ncell, cells);
      HCG_LAUNCH_CHECK("k_cell_vecs_arrays");
      HCG_HIP(capbuf.alloc_async(sizeof(double4) * ntiles, stream));
      HCG_HIP(hipMemsetAsync((char*)statbuf.p + 16, 0, 8, stream));
      k_tile_caps<<<(unsigned)((ntiles + 3) / 4), 256, 0, stream>>>(
          cells, nx, ny, ntx, nty, (double4*)capbuf.p,
          (unsigned long long*)((char*)statbuf.p + 16));
      HCG_LAUNCH_CHECK("k_tile_caps");
    }
    st = launch_ang2pix(lon_deg, lat_deg, n, nside, (uint32_t*)pixbuf.p, (uint32_t*)statbuf.p,
                        stream);
    if (st != HCG_OK) return st;
    HCG_HIP(hipMemcpyAsync(host, statbuf.p, 32, hipMemcpyDeviceToHost, stream));
    return HCG_OK;
  }

  // after the pixel statistics have reached host[0..7]
  hcg_status middle() {
    const uint32_t* hs = host;
    if (hs[2]) return fail(HCG_E_ARG, "%s: %u sample coordinates are non-finite or |lat| > 90", who, hs[2]);
    const uint32_t pix_base = hs[0], pix_max = hs[1];
    const int ring_first = (int)hpx_pix2ring(nside, pix_base);
    const int ring_last = (int)hpx_pix2ring(nside, pix_max);
    const int nrings = ring_last - ring_first + 1;
    const int key_bits = bit_length(pix_max - pix_base);

    // candidate-range slots per tile: rings in the tile's latitude span + 2R,
    // two ranges per ring; rings are at least 2/(3 Ns) apart in latitude
    double tile_span = 0.0;
    if (tg.grid) {
      tile_span = (kTileY - 1) * std::fabs(tg.grid->dlat_deg) * kDeg2Rad;
    } else {
      double rmax = 0.0;
      memcpy(&rmax, &hs[4], sizeof(double));
      tile_span = 2.0 * std::min(rmax, kPi);
    }
    const double rings_d = (tile_span + 2.0 * R) / (2.0 / (3.0 * nside)) + 6.0;
    if (rings_d > kMaxRangesLimit / 2)
      return fail(HCG_E_UNSUPPORTED,
                  "%s: support or tile too wide for nside %d (%.0f rings per tile; at most %d)", who,
                  nside, rings_d, kMaxRangesLimit / 2);
    const int maxr = 2 * (int)std::ceil(rings_d);

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
    const size_t o_cells = take(sizeof(double4) * ncell);
    const size_t arena_bytes = off;
    if (arena.alloc_async(arena_bytes, stream) != hipSuccess) {
      (void)hipGetLastError();
      return fail(HCG_E_NOMEM, "%s: cannot allocate %zu bytes for the plan", who, arena_bytes);
    }
    const size_t temp_bytes = radix_sort_temp_bytes(n) + align256(sizeof(uint32_t) * n);
    if (temp.alloc_async(temp_bytes, stream) != hipSuccess) {
      (void)hipGetLastError();
      return fail(HCG_E_NOMEM, "%s: cannot allocate %zu bytes of scratch", who, temp_bytes);
    }
    char* A = (char*)arena.p;
    p = new hcg_plan_s{};
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
    if (tg.grid)
      p->grid = GridGeom{tg.grid->nx, tg.grid->ny, tg.grid->lon0_deg, tg.grid->lat0_deg,
                         tg.grid->dlon_deg, tg.grid->dlat_deg};
    else
      p->grid = GridGeom{nx, ny, 0.0, 0.0, 0.0, 0.0};
    p->centres = tg.grid ? 0 : 1;
    p->fwhm_deg = fwhm_nominal;
    p->support_deg = support_deg;
    p->sigma_rad = sigma;
    p->support_rad = R;
    p->kern = kp;
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
    p->cells = (double4*)(A + o_cells);

    HCG_HIP(hipMemcpyAsync(p->cells, cellbuf.p, sizeof(double4) * ncell, hipMemcpyDeviceToDevice,
                           stream));
    // keys relative to the smallest pixel, then the stable sort
    uint32_t* rel = (uint32_t*)((char*)temp.p + radix_sort_temp_bytes(n));
    k_rel_keys<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>((const uint32_t*)pixbuf.p,
                                                                 pix_base, n, rel);
    HCG_LAUNCH_CHECK("k_rel_keys");
    hcg_status st =
        launch_radix_sort(rel, n, key_bits == 0 ? 1 : key_bits, p->keys, p->perm, temp.p, stream);
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
    if (tg.grid) {
      k_tile_ranges<<<(unsigned)((ntiles + 3) / 4), 256, 0, stream>>>(
          p->keys, p->csr, nside, ring_first, ring_last, pix_base, p->grid, ntx, nty, R, maxr,
          p->ranges, p->nranges, p->ncand, p->flags);
      HCG_LAUNCH_CHECK("k_tile_ranges");
    } else {
      k_tile_ranges_cap<<<(unsigned)((ntiles + 3) / 4), 256, 0, stream>>>(
          p->keys, p->csr, nside, ring_first, ring_last, pix_base, (const double4*)capbuf.p,
          (int)ntiles, R, maxr, p->ranges, p->nranges, p->ncand, p->flags);
      HCG_LAUNCH_CHECK("k_tile_ranges_cap");
    }
    HCG_HIP(hipMemcpyAsync(host + 8, p->flags, 16, hipMemcpyDeviceToHost, stream));
    return HCG_OK;
  }

  // after the flags have reached host[8..11]
  hcg_status finish(hcg_plan_t* out) {
    if (host[8]) return fail(HCG_E_DEVICE, "%s: candidate-range slots overflowed (internal bound)", who);
    p->arena_pooled = arena.async ? 1 : 0;
    p->arena = arena.release();
    plan_register(p);
    *out = p;
    p = nullptr;
    return HCG_OK;
  }
};

hcg_status plan_build(hcg_plan_t* out, const double* lon_deg, const double* lat_deg, int64_t n,
                      const PlanTarget& tg, const hcg_kernel* kernel, double support_deg,
                      const hcg_opts* opts, void* hip_stream, const char* who) {
  hipStream_t stream = (hipStream_t)hip_stream;
  // the two reads between the steps land in page-locked memory (a copy to
  // pageable memory is staged by the runtime: about 0.1-0.2 ms each)
  thread_local uint32_t* pinned = nullptr;
  thread_local bool tried = false;
  if (!tried) {
    tried = true;
    if (hipHostMalloc((void**)&pinned, sizeof(uint32_t) * 16, hipHostMallocPortable) != hipSuccess) {
      (void)hipGetLastError();
      pinned = nullptr;
    }
  }
  uint32_t stack_words[16] = {0};
  uint32_t* host = pinned ? pinned : stack_words;
  memset(host, 0, sizeof(uint32_t) * 16);
  PlanBuilder b;
  hcg_status st = b.begin(lon_deg, lat_deg, n, tg, kernel, support_deg, opts, stream, host, who);
  if (st != HCG_OK) return st;
  HCG_HIP(hipStreamSynchronize(stream));
  st = b.middle();
  if (st != HCG_OK) return st;
  HCG_HIP(hipStreamSynchronize(stream));
  return b.finish(out);
}

}  // namespace

namespace hcg {

// Plans of many fields on linear grids (the batch), built together: the
// pixels of every field in one launch, one read of their ranges, then every
// further step for all fields in one launch each (the sort with the largest
// number of passes any field needs), one read of the overflow flags.  The
// plans' arrays share one allocation, *arena_out, which the caller frees
// after destroying the plans (their own arena pointers are NULL).  On
// failure *failed is the first failing field (or -1) and nothing is left
// allocated.
hcg_status plan_build_fields(int32_t nf, const hcg_field_desc* fd, const hcg_opts* opts,
                             hipStream_t stream, hcg_plan_t* plans, void** arena_out,
                             std::vector<std::vector<uint32_t>>* ncand, int32_t* failed) {
  *failed = -1;
  *arena_out = nullptr;
  for (int32_t f = 0; f < nf; ++f) plans[f] = nullptr;
  hcg_opts o = {};
  if (opts) o = *opts;
  if ((o.tile_x && o.tile_x != kTileX) || (o.tile_y && o.tile_y != kTileY))
    return fail(HCG_E_UNSUPPORTED, "hcg_plan: only 8 x 8 cell tiles are built");
  if (o.coarsen || o.chan_tile || o.flags)
    return fail(HCG_E_UNSUPPORTED, "hcg_plan: coarsen, chan_tile and flags must be 0");
  hcg_status st = check_device_arch();
  if (st != HCG_OK) return st;

  // ---- argument checks and first-step sizes
  std::vector<PlanField> F(nf);
  std::vector<KernelParams> kp(nf);
  std::vector<double> sigma(nf), fwhm_nom(nf);
  hcg_kernel k{};
  k.type = HCG_KERNEL_GAUSS;
  for (int32_t f = 0; f < nf; ++f) {
    const hcg_field_desc& d = fd[f];
    *failed = f;
    if (!d.lon_deg || !d.lat_deg) return fail(HCG_E_ARG, "hcg_plan: NULL pointer");
    st = check_grid(&d.grid, "hcg_plan");
    if (st != HCG_OK) return st;
    if (d.n < 1 || d.n >= (int64_t(1) << 31)) return fail(HCG_E_ARG, "hcg_plan: n must be in 1..2^31-1");
    if (!(d.support_deg >= 0.0) || !(d.support_deg < 90.0))
      return fail(HCG_E_ARG, "hcg_plan: support must be in [0, 90) degrees");
    k.fwhm_deg = d.fwhm_deg;
    st = kernel_params(&k, "hcg_plan", &kp[f], &sigma[f], &fwhm_nom[f]);
    if (st != HCG_OK) return st;
    const int nside = o.nside ? o.nside : auto_nside(sigma[f]);
    if (!is_pow2(nside) || nside > 16384)
      return fail(HCG_E_ARG, "hcg_plan: nside %d is not a power of two in 1..16384", nside);
    PlanField& P = F[f];
    memset(&P, 0, sizeof(P));
    P.lon = d.lon_deg;
    P.lat = d.lat_deg;
    P.n = d.n;
    P.nside = nside;
    P.grid = GridGeom{d.grid.nx, d.grid.ny, d.grid.lon0_deg, d.grid.lat0_deg, d.grid.dlon_deg,
                      d.grid.dlat_deg};
    P.ntx = (d.grid.nx + kTileX - 1) / kTileX;
    P.nty = (d.grid.ny + kTileY - 1) / kTileY;
    P.support_rad = d.support_deg * kDeg2Rad;
  }
  *failed = -1;

  // page-locked host block: the field table, the launch prefix tables, and
  // what comes back (pixel statistics, flags)
  const size_t tab_bytes = align256(sizeof(PlanField) * nf);
  const size_t pre_bytes = align256(sizeof(uint32_t) * kFbKinds * (nf + 1));
  const size_t back_bytes = align256(sizeof(uint32_t) * 4 * nf);
  char* host = nullptr;
  if (hipHostMalloc((void**)&host, tab_bytes + pre_bytes + back_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "cannot allocate page-locked host memory for %d plans", nf);
  }
  struct HostFree {
    char* h;
    ~HostFree() { (void)hipHostFree(h); }
  } hf{host};
  PlanField* h_tab = (PlanField*)host;
  uint32_t* h_pre = (uint32_t*)(host + tab_bytes);
  uint32_t* h_back = (uint32_t*)(host + tab_bytes + pre_bytes);
  auto prefix = [&](int kind, auto blocks_of) {
    uint32_t* pr = h_pre + (size_t)kind * (nf + 1);
    uint64_t acc = 0;
    for (int32_t f = 0; f < nf; ++f) {
      pr[f] = (uint32_t)acc;
      acc += blocks_of(F[f]);
    }
    pr[nf] = (uint32_t)acc;
    return acc;
  };

  // ---- first step: pixels and their range
  size_t t1 = 0;
  std::vector<size_t> o_pix(nf);
  for (int32_t f = 0; f < nf; ++f) {
    o_pix[f] = t1;
    t1 += align256(sizeof(uint32_t) * F[f].n);
  }
  const size_t o_stat = t1;
  t1 += align256(sizeof(uint32_t) * 4 * nf);
  const size_t o_tab = t1;
  t1 += tab_bytes + pre_bytes;
  DevBuf temp1;
  if (temp1.alloc_async(t1, stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "cannot allocate %zu bytes of scratch for %d plans", t1, nf);
  }
  char* T1 = (char*)temp1.p;
  for (int32_t f = 0; f < nf; ++f) {
    F[f].pix = (uint32_t*)(T1 + o_pix[f]);
    F[f].stat = (uint32_t*)(T1 + o_stat) + 4 * f;
  }
  const uint64_t nb_samples = prefix(kFbSamples, [](const PlanField& P) { return (uint64_t)((P.n + 255) / 256); });
  prefix(kFbOne, [](const PlanField&) { return (uint64_t)1; });
  if (nb_samples >= 0xFFFFFFF0ull) return fail(HCG_E_UNSUPPORTED, "hcg_plan_batch: too many samples");
  memcpy(h_tab, F.data(), sizeof(PlanField) * nf);
  PlanField* d_tab = (PlanField*)(T1 + o_tab);
  uint32_t* d_pre = (uint32_t*)(T1 + o_tab + tab_bytes);
  HCG_HIP(hipMemcpyAsync(d_tab, host, tab_bytes + pre_bytes, hipMemcpyHostToDevice, stream));
  k_stat_init_fields<<<(unsigned)nf, 256, 0, stream>>>(d_tab, d_pre, nf);
  HCG_LAUNCH_CHECK("k_stat_init_fields");
  k_ang2pix_fields<<<(unsigned)nb_samples, 256, 0, stream>>>(d_tab, d_pre, nf);
  HCG_LAUNCH_CHECK("k_ang2pix_fields");
  HCG_HIP(hipMemcpyAsync(h_back, T1 + o_stat, sizeof(uint32_t) * 4 * nf, hipMemcpyDeviceToHost,
                         stream));
  HCG_HIP(hipStreamSynchronize(stream));

  // ---- sizes, the plans' arena and the sort scratch
  int passes = 1;
  std::vector<size_t> o_ar(nf);
  std::vector<int> key_bits(nf);
  std::vector<uint32_t> pix_max_of(nf);
  size_t arena_bytes = 0, t2 = 0;
  std::vector<size_t> o_t2(nf);
  struct Off { size_t xyz, keys, perm, csr, rng, nr, nc, flags, cells, bytes; };
  std::vector<Off> off(nf);
  for (int32_t f = 0; f < nf; ++f) {
    PlanField& P = F[f];
    const uint32_t* hs = h_back + 4 * f;
    if (hs[2]) {
      *failed = f;
      return fail(HCG_E_ARG, "hcg_plan: %u sample coordinates are non-finite or |lat| > 90", hs[2]);
    }
    P.pix_base = hs[0];
    const uint32_t pix_max = hs[1];
    pix_max_of[f] = pix_max;
    P.ring_first = (int)hpx_pix2ring(P.nside, P.pix_base);
    P.ring_last = (int)hpx_pix2ring(P.nside, pix_max);
    P.nrings = P.ring_last - P.ring_first + 1;
    key_bits[f] = bit_length(pix_max - P.pix_base);
    passes = std::max(passes, (key_bits[f] + 7) / 8);
    const double tile_span = (kTileY - 1) * std::fabs(P.grid.dlat) * kDeg2Rad;
    const double rings_d = (tile_span + 2.0 * P.support_rad) / (2.0 / (3.0 * P.nside)) + 6.0;
    if (rings_d > kMaxRangesLimit / 2) {
      *failed = f;
      return fail(HCG_E_UNSUPPORTED,
                  "hcg_plan: support or tile too wide for nside %d (%.0f rings per tile; at most %d)",
                  P.nside, rings_d, kMaxRangesLimit / 2);
    }
    P.maxr = 2 * (int)std::ceil(rings_d);
    const int64_t ntiles = (int64_t)P.ntx * P.nty, ncell = (int64_t)P.grid.nx * P.grid.ny;
    Off& a = off[f];
    size_t at = 0;
    auto take = [&](size_t bytes) { size_t r = at; at += align256(bytes); return r; };
    a.xyz = take(sizeof(double4) * (P.n + 8));
    a.keys = take(sizeof(uint32_t) * P.n);
    a.perm = take(sizeof(uint32_t) * (P.n + 1));
    a.csr = take(sizeof(uint32_t) * (P.nrings + 1));
    a.rng = take(sizeof(uint2) * (size_t)ntiles * P.maxr);
    a.nr = take(sizeof(uint32_t) * ntiles);
    a.nc = take(sizeof(uint32_t) * ntiles);
    a.flags = take(16);
    a.cells = take(sizeof(double4) * ncell);
    a.bytes = at;
    o_ar[f] = arena_bytes;
    arena_bytes += at;
    P.rs_ntiles = std::max<int64_t>(rs_ntiles(P.n), 1);
    P.rs_m = 256 * P.rs_ntiles;
    P.rs_np = (P.rs_m + kScanChunk - 1) / kScanChunk;
    o_t2[f] = t2;
    t2 += radix_sort_temp_bytes(P.n) + align256(sizeof(uint32_t) * P.n);
  }
  DevBuf arena, temp2;
  if (hipMalloc(&arena.p, arena_bytes) != hipSuccess) {
    (void)hipGetLastError();
    arena.p = nullptr;
    return fail(HCG_E_NOMEM, "cannot allocate %zu bytes for %d plans", arena_bytes, nf);
  }
  if (temp2.alloc_async(t2, stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "cannot allocate %zu bytes of scratch for %d plans", t2, nf);
  }
  for (int32_t f = 0; f < nf; ++f) {
    PlanField& P = F[f];
    char* A = (char*)arena.p + o_ar[f];
    const Off& a = off[f];
    P.xyz = (double4*)(A + a.xyz);
    P.keys = (uint32_t*)(A + a.keys);
    P.perm = (uint32_t*)(A + a.perm);
    P.csr = (uint32_t*)(A + a.csr);
    P.ranges = (uint2*)(A + a.rng);
    P.nranges = (uint32_t*)(A + a.nr);
    P.ncand = (uint32_t*)(A + a.nc);
    P.flags = (uint32_t*)(A + a.flags);
    P.cells = (double4*)(A + a.cells);
    char* t = (char*)temp2.p + o_t2[f];
    P.k_alt = (uint32_t*)t;
    t += align256(sizeof(uint32_t) * P.n);
    P.v_alt = (uint32_t*)t;
    t += align256(sizeof(uint32_t) * P.n);
    P.hist = (uint32_t*)t;
    t += align256(sizeof(uint32_t) * P.rs_m);
    P.offs = (uint32_t*)t;
    t += align256(sizeof(uint32_t) * P.rs_m);
    P.partial = (uint32_t*)t;
    P.rel = (uint32_t*)((char*)temp2.p + o_t2[f] + radix_sort_temp_bytes(P.n));
  }

  // ---- second step: every remaining build step, one launch each
  const uint64_t nb_cells = prefix(kFbCells, [](const PlanField& P) { return (uint64_t)(((int64_t)P.grid.nx * P.grid.ny + 255) / 256); });
  prefix(kFbSamples, [](const PlanField& P) { return (uint64_t)((P.n + 255) / 256); });
  const uint64_t nb_sort = prefix(kFbSortTiles, [](const PlanField& P) { return (uint64_t)P.rs_ntiles; });
  const uint64_t nb_scan = prefix(kFbScan, [](const PlanField& P) { return (uint64_t)P.rs_np; });
  prefix(kFbOne, [](const PlanField&) { return (uint64_t)1; });
  const uint64_t nb_rings = prefix(kFbRings, [](const PlanField& P) { return (uint64_t)((P.nrings + 1 + 255) / 256); });
  const uint64_t nb_tiles = prefix(kFbTiles, [](const PlanField& P) { return (uint64_t)(((int64_t)P.ntx * P.nty + 3) / 4); });
  if (nb_cells + nb_samples >= 0xFFFFFFF0ull || nb_tiles >= 0xFFFFFFF0ull)
    return fail(HCG_E_UNSUPPORTED, "hcg_plan_batch: too many cells");
  memcpy(h_tab, F.data(), sizeof(PlanField) * nf);
  HCG_HIP(hipMemcpyAsync(d_tab, host, tab_bytes + pre_bytes, hipMemcpyHostToDevice, stream));
  k_cells_rel_fields<<<(unsigned)(nb_cells + nb_samples), 256, 0, stream>>>(d_tab, d_pre, nf);
  HCG_LAUNCH_CHECK("k_cells_rel_fields");
  for (int p = 0; p < passes; ++p) {
    k_radix_hist_fields<<<(unsigned)nb_sort, kRsThreads, 0, stream>>>(d_tab, d_pre, nf, p, passes);
    k_scan_reduce_fields<<<(unsigned)nb_scan, 256, 0, stream>>>(d_tab, d_pre, nf);
    k_scan_top_fields<<<(unsigned)nf, 256, 0, stream>>>(d_tab, d_pre, nf);
    k_scan_apply_fields<<<(unsigned)nb_scan, 256, 0, stream>>>(d_tab, d_pre, nf);
    k_radix_scatter_fields<<<(unsigned)nb_sort, kRsThreads, 0, stream>>>(d_tab, d_pre, nf, p,
                                                                         passes);
    HCG_LAUNCH_CHECK("k_radix_*_fields");
  }
  k_permute_xyz_fields<<<(unsigned)nb_samples, 256, 0, stream>>>(d_tab, d_pre, nf);
  HCG_LAUNCH_CHECK("k_permute_xyz_fields");
  k_ring_csr_fields<<<(unsigned)nb_rings, 256, 0, stream>>>(d_tab, d_pre, nf);
  HCG_LAUNCH_CHECK("k_ring_csr_fields");
  k_tile_ranges_fields<<<(unsigned)nb_tiles, 256, 0, stream>>>(d_tab, d_pre, nf);
  HCG_LAUNCH_CHECK("k_tile_ranges_fields");
  for (int32_t f = 0; f < nf; ++f)
    HCG_HIP(hipMemcpyAsync(h_back + 4 * f, F[f].flags, 16, hipMemcpyDeviceToHost, stream));
  ncand->assign(nf, {});
  for (int32_t f = 0; f < nf; ++f) {
    (*ncand)[f].resize((size_t)F[f].ntx * F[f].nty);
    HCG_HIP(hipMemcpyAsync((*ncand)[f].data(), F[f].ncand, sizeof(uint32_t) * (*ncand)[f].size(),
                           hipMemcpyDeviceToHost, stream));
  }
  HCG_HIP(hipStreamSynchronize(stream));
  for (int32_t f = 0; f < nf; ++f)
    if (h_back[4 * f]) {
      *failed = f;
      return fail(HCG_E_DEVICE, "hcg_plan: candidate-range slots overflowed (internal bound)");
    }

  // ---- the plans
  for (int32_t f = 0; f < nf; ++f) {
    const PlanField& P = F[f];
    auto* p = new hcg_plan_s{};
    p->magic = kPlanMagic;
    (void)hipGetDevice(&p->device);
    p->n = P.n;
    p->nside = P.nside;
    p->pix_base = P.pix_base;
    p->pix_max = pix_max_of[f];
    p->key_bits = key_bits[f];
    p->passes = (key_bits[f] + 7) / 8;
    p->ring_first = P.ring_first;
    p->ring_last = P.ring_last;
    p->grid = P.grid;
    p->centres = 0;
    p->fwhm_deg = fwhm_nom[f];
    p->support_deg = fd[f].support_deg;
    p->sigma_rad = sigma[f];
    p->support_rad = P.support_rad;
    p->kern = kp[f];
    p->ntx = P.ntx;
    p->nty = P.nty;
    p->maxr = P.maxr;
    p->arena_bytes = off[f].bytes;
    p->xyz = P.xyz;
    p->keys = P.keys;
    p->perm = P.perm;
    p->csr = P.csr;
    p->ranges = P.ranges;
    p->nranges = P.nranges;
    p->ncand = P.ncand;
    p->flags = P.flags;
    p->cells = P.cells;
    p->arena = nullptr;  // in the shared arena
    p->batch_owned = 1;
    plan_register(p);
    plans[f] = p;
  }
  *arena_out = arena.release();
  return HCG_OK;
}

}  // namespace hcg

extern "C" hcg_status hcg_plan(hcg_plan_t* out, const double* lon_deg, const double* lat_deg,
                               int64_t n, const hcg_grid_desc* grid, double fwhm_deg,
                               double support_deg, const hcg_opts* opts, void* hip_stream) {
  if (!out) return fail(HCG_E_ARG, "hcg_plan: out is NULL");
  *out = nullptr;
  if (!lon_deg || !lat_deg || !grid) return fail(HCG_E_ARG, "hcg_plan: NULL pointer");
  hcg_status st = check_grid(grid, "hcg_plan");
  if (st != HCG_OK) return st;
  hcg_kernel k{};
  k.type = HCG_KERNEL_GAUSS;
  k.fwhm_deg = fwhm_deg;
  const PlanTarget tg{grid, nullptr, nullptr, grid->nx, grid->ny};
  return plan_build(out, lon_deg, lat_deg, n, tg, &k, support_deg, opts, hip_stream, "hcg_plan");
}

extern "C" hcg_status hcg_plan_ex(hcg_plan_t* out, const double* lon_deg, const double* lat_deg,
                                  int64_t n, const hcg_grid_desc* grid,
                                  const hcg_cell_centres* centres, const hcg_kernel* kernel,
                                  double support_deg, const hcg_opts* opts, void* hip_stream) {
  if (!out) return fail(HCG_E_ARG, "hcg_plan_ex: out is NULL");
  *out = nullptr;
  if (!lon_deg || !lat_deg || !kernel) return fail(HCG_E_ARG, "hcg_plan_ex: NULL pointer");
  if ((grid == nullptr) == (centres == nullptr))
    return fail(HCG_E_ARG, "hcg_plan_ex: give exactly one of grid and centres");
  PlanTarget tg{grid, nullptr, nullptr, 0, 0};
  if (grid) {
    const hcg_status st = check_grid(grid, "hcg_plan_ex");
    if (st != HCG_OK) return st;
    tg.nx = grid->nx;
    tg.ny = grid->ny;
  } else {
    if (!centres->lon_deg || !centres->lat_deg)
      return fail(HCG_E_ARG, "hcg_plan_ex: NULL centre array");
    if (centres->nx < 1 || centres->ny < 1 || (int64_t)centres->nx * centres->ny > INT32_MAX)
      return fail(HCG_E_ARG, "hcg_plan_ex: centres nx, ny out of range");
    tg.clon = centres->lon_deg;
    tg.clat = centres->lat_deg;
    tg.nx = centres->nx;
    tg.ny = centres->ny;
  }
  return plan_build(out, lon_deg, lat_deg, n, tg, kernel, support_deg, opts, hip_stream,
                    "hcg_plan_ex");
}
