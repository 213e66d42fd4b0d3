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

// Linear lon/lat grid: the box of the tile's cell centres.
__global__ void __launch_bounds__(256) k_tile_ranges(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ csr, int ns, int ring_first,
    int ring_last, uint32_t pix_base, GridGeom g, int ntx, int nty, double support_rad, int maxr,
    uint2* __restrict__ ranges, uint32_t* __restrict__ nranges, uint32_t* __restrict__ ncand,
    uint32_t* __restrict__ flags) {
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
  tile_ranges_wave(keys, csr, ns, ring_first, ring_last, pix_base, lon_a, lon_b, lat_a, lat_b, Rs,
                   maxr, ranges + (int64_t)tile * maxr, &nranges[tile], &ncand[tile], flags);
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
    const hipError_t e = hipMallocAsync(&p, bytes, stream);
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
    if (hipMalloc(&arena.p, arena_bytes) != hipSuccess) {
      (void)hipGetLastError();
      arena.p = nullptr;
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
  uint32_t host[16] = {0};
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

// Plans of many fields on linear grids (the batch): each build step runs for
// every field, field f on streams[f % nstreams], with one synchronisation of
// the streams per step.  On failure *failed is the first failing field and
// nothing is left allocated.
hcg_status plan_build_many(int32_t nfields, const hcg_field_desc* fields, const hcg_opts* opts,
                           const hipStream_t* streams, int nstreams, hcg_plan_t* plans,
                           int32_t* failed) {
  *failed = -1;
  for (int32_t f = 0; f < nfields; ++f) plans[f] = nullptr;
  uint32_t* host = nullptr;
  if (hipHostMalloc((void**)&host, sizeof(uint32_t) * 16 * (size_t)nfields) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "cannot allocate page-locked host memory for %d plans", nfields);
  }
  struct HostFree {
    uint32_t* h;
    ~HostFree() { (void)hipHostFree(h); }
  } hf{host};
  std::vector<PlanBuilder> b(nfields);
  auto sync_all = [&]() -> hcg_status {
    for (int k = 0; k < std::min<int>(nstreams, nfields); ++k)
      HCG_HIP(hipStreamSynchronize(streams[k]));
    return HCG_OK;
  };
  hcg_kernel k{};
  k.type = HCG_KERNEL_GAUSS;
  for (int32_t f = 0; f < nfields; ++f) {
    const hcg_field_desc& d = fields[f];
    hcg_status st = HCG_OK;
    if (!d.lon_deg || !d.lat_deg) st = fail(HCG_E_ARG, "hcg_plan: NULL pointer");
    if (st == HCG_OK) st = check_grid(&d.grid, "hcg_plan");
    if (st == HCG_OK) {
      k.fwhm_deg = d.fwhm_deg;
      const PlanTarget tg{&d.grid, nullptr, nullptr, d.grid.nx, d.grid.ny};
      st = b[f].begin(d.lon_deg, d.lat_deg, d.n, tg, &k, d.support_deg, opts,
                      streams[f % nstreams], host + 16 * (size_t)f, "hcg_plan");
    }
    if (st != HCG_OK) {
      *failed = f;
      (void)sync_all();
      return st;
    }
  }
  hcg_status st = sync_all();
  if (st != HCG_OK) return st;
  for (int32_t f = 0; f < nfields; ++f) {
    st = b[f].middle();
    if (st != HCG_OK) {
      *failed = f;
      (void)sync_all();
      return st;
    }
  }
  st = sync_all();
  if (st != HCG_OK) return st;
  for (int32_t f = 0; f < nfields; ++f) {
    st = b[f].finish(&plans[f]);
    if (st != HCG_OK) {
      *failed = f;
      for (int32_t g = 0; g < f; ++g) {
        (void)hcg_destroy(plans[g]);
        plans[g] = nullptr;
      }
      return st;
    }
  }
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
