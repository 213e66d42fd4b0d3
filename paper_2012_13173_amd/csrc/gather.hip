// Data stage of the gridding library: Eq. (1) of HCGrid (Section 2.1) for
// every output cell and channel, gather-side (Section 2.2: each cell pulls
// the samples within its support, so no two workgroups write the same cell).
//
// Work decomposition: one workgroup per 8 x 8 tile of output cells (and per
// 256-channel slab for many channels).  The tile's candidate samples come
// from the plan's sorted-sample ranges and are staged in blocks of 64:
//   1. weights: FP64 haversine distance of every (cell, candidate) pair of
//      the block, exact support test, FP64 Gaussian weight; FP64 sums of the
//      weights per cell;
//   2. accumulation: for many channels the block is a dense contraction
//      U[cells x channels] += Wt[cells x 64] . S[64 x channels] done on the
//      matrix cores (v_mfma_f32_16x16x4_f32: 16 cells x 4 samples x 16
//      channels per instruction, FP32 products and accumulation), skipping
//      every 16-cell x 4-sample sub-block whose weights are all zero; for a
//      few channels each lane owns one cell and accumulates in FP64;
//   3. epilogue: V = U / W~ (W~ the sum of the weights actually multiplied),
//      NaN where no sample is within the support; W map = FP64 sum.
#include <cmath>
#include <vector>

#include "hcg_internal.h"

namespace hcg {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kKB = 64;             // candidates staged per block
constexpr int kSteps = kKB / 4;     // MFMA k-steps (4 samples each) per block
constexpr int kMfmaWaves = 4;
constexpr int kChanPerWave = 64;
constexpr int kChanPerWG = kMfmaWaves * kChanPerWave;

// Squared great-circle distance from the haversine h = sin^2(d/2):
// d^2 = 4 asin^2(sqrt h) = 4h (1 + h/3 + 8h^2/45 + 4h^3/35 + ...).
__device__ __forceinline__ double dist2_from_hav(double h) {
  if (h < 1e-4) return 4.0 * h * (1.0 + h * (1.0 / 3.0 + h * (8.0 / 45.0 + h * (4.0 / 35.0))));
  const double d = 2.0 * asin(sqrt(fmin(h, 1.0)));
  return d * d;
}

// Cell-centre half-angle trigonometry; invalid cells get NaN (never within R).
struct CellTrig {
  double sd, cd, sa, ca, cosd;
};

__device__ __forceinline__ CellTrig cell_trig(const GridGeom& g, int ix, int iy) {
  CellTrig c;
  if (ix >= g.nx || iy >= g.ny) {
    const double nan = __builtin_nan("");
    c.sd = c.cd = c.sa = c.ca = c.cosd = nan;
    return c;
  }
  sincos(0.5 * cell_lat_deg(g, iy) * kDeg2Rad, &c.sd, &c.cd);
  sincos(0.5 * cell_lon_deg(g, ix) * kDeg2Rad, &c.sa, &c.ca);
  c.cosd = (c.cd - c.sd) * (c.cd + c.sd);
  return c;
}

// Haversine of the pair; t = (sin(lat/2), cos(lat/2), sin(lon/2), cos(lon/2))
// of the sample.  sin((a-b)/2) is expanded through the half-angle products.
__device__ __forceinline__ double pair_hav(const CellTrig& c, const double4& t) {
  const double a = c.sd * t.y - c.cd * t.x;
  const double b = c.sa * t.w - c.ca * t.z;
  const double cn = (t.y - t.x) * (t.y + t.x);
  return a * a + c.cosd * cn * (b * b);
}

// Loads the tile's candidate ranges into LDS with exclusive prefix sums;
// returns the total candidate count.  blockDim.x threads take part.
__device__ uint32_t stage_ranges(const uint2* __restrict__ ranges, uint32_t nr, uint2* s_rng,
                                 uint32_t* s_pre) {
  const int nt = blockDim.x;
  for (uint32_t r = threadIdx.x; r < nr; r += nt) s_rng[r] = ranges[r];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t r = 0; r < nr; ++r) {
      s_pre[r] = acc;
      acc += s_rng[r].y - s_rng[r].x;
    }
    s_pre[nr] = acc;
  }
  __syncthreads();
  return s_pre[nr];
}

// Sorted position of candidate q; *cur is a monotone cursor over ranges.
__device__ __forceinline__ uint32_t cand_pos(uint32_t q, const uint2* s_rng, const uint32_t* s_pre,
                                             uint32_t* cur) {
  uint32_t r = *cur;
  while (q >= s_pre[r + 1]) ++r;
  *cur = r;
  return s_rng[r].x + (q - s_pre[r]);
}

// ---------------------------------------------------------------------------
// Many channels, FP32: matrix-core contraction per staged block.
// Workgroup = 4 waves.  Wave w computes the weights of cell block w (16 cells:
// a 4 x 4 patch of the tile) for the block's 64 candidates, one cell per
// lane, 16 candidates per lane, directly in the A-operand layout of
// v_mfma_f32_16x16x4_f32 (lane l holds cell l%16, sample l/16 of each
// 4-sample step).  In the contraction wave w owns channels
// [slab + 64w, slab + 64w + 64) for all four cell blocks; lane l streams
// channels 4(l%16) .. 4(l%16)+3 of sample l/16 of each step (B operand,
// column j of MFMA q is channel 4j + q of the wave's 64).
// ---------------------------------------------------------------------------
template <bool kVec4>
__global__ void __launch_bounds__(256, 2) k_gather_mfma_f32(
    const double4* __restrict__ trig, const uint32_t* __restrict__ perm,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ nranges, int maxr,
    const float* __restrict__ spectra, int64_t C, GridGeom g, int ntx, double hR,
    double inv_two_sig2, float* __restrict__ cube, float* __restrict__ wmap) {
  __shared__ uint2 s_rng[kMaxRangesLimit];
  __shared__ uint32_t s_pre[kMaxRangesLimit + 1];
  __shared__ double4 s_trig[kKB];
  __shared__ uint32_t s_row[kKB];
  __shared__ float s_A[4][kSteps][64];
  __shared__ uint32_t s_nz[4];
  __shared__ double s_Wt[kTileCells];

  const int tile = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx = tile % ntx, ty = tile / ntx;
  const int64_t G = (int64_t)g.nx * g.ny;

  // this lane's cell in the weight phase: block `wave`, cell lane % 16
  const int ci = lane & 15;
  const int my_x = tx * kTileX + (wave & 1) * 4 + (ci & 3);
  const int my_y = ty * kTileY + (wave >> 1) * 4 + (ci >> 2);
  const CellTrig cell = cell_trig(g, my_x, my_y);

  const uint32_t total = stage_ranges(ranges + (int64_t)tile * maxr, nranges[tile], s_rng, s_pre);

  floatx4 acc[4][4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[cb][q] = floatx4{0.f, 0.f, 0.f, 0.f};
  double wsum = 0.0;   // FP64 sum of unrounded weights (this lane's share)
  double wtsum = 0.0;  // FP64 sum of the FP32-rounded weights used in the products
  uint32_t cur = 0;
  const int64_t c_w = (int64_t)blockIdx.y * kChanPerWG + wave * kChanPerWave;
  const int64_t my_ch = c_w + 4 * (lane & 15);

  for (uint32_t q0 = 0; q0 < total; q0 += kKB) {
    // stage the block's candidates
    if (tid < kKB) {
      const uint32_t q = q0 + tid;
      if (q < total) {
        const uint32_t pos = cand_pos(q, s_rng, s_pre, &cur);
        s_trig[tid] = trig[pos];
        s_row[tid] = perm[pos];
      } else {
        const double nan = __builtin_nan("");
        s_trig[tid] = make_double4(nan, nan, nan, nan);
        s_row[tid] = 0u;
      }
    }
    __syncthreads();
    // weights of cell block `wave`
    uint32_t nzbits = 0;
#pragma unroll
    for (int ks = 0; ks < kSteps; ++ks) {
      const double4 t = s_trig[4 * ks + (lane >> 4)];
      const double h = pair_hav(cell, t);
      float wf = 0.f;
      if (h <= hR) {
        const double w = exp(-dist2_from_hav(h) * inv_two_sig2);
        wf = (float)w;
        wsum += w;
        wtsum += (double)wf;
      }
      s_A[wave][ks][lane] = wf;
      if (__ballot(wf != 0.f)) nzbits |= 1u << ks;
    }
    if (lane == 0) s_nz[wave] = nzbits;
    __syncthreads();

    // contraction over the block: B operands for all 16 steps, then MFMAs
    const uint32_t nz0 = s_nz[0], nz1 = s_nz[1], nz2 = s_nz[2], nz3 = s_nz[3];
    floatx4 b[kSteps];
#pragma unroll
    for (int ks = 0; ks < kSteps; ++ks) {
      const int64_t row = s_row[4 * ks + (lane >> 4)];
      const float* src = spectra + row * C + my_ch;
      if (kVec4) {
        if (my_ch + 3 < C) {
          b[ks] = *(const floatx4*)src;
        } else {
          b[ks] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
      } else {
        b[ks].x = (my_ch + 0 < C) ? src[0] : 0.f;
        b[ks].y = (my_ch + 1 < C) ? src[1] : 0.f;
        b[ks].z = (my_ch + 2 < C) ? src[2] : 0.f;
        b[ks].w = (my_ch + 3 < C) ? src[3] : 0.f;
      }
    }
#pragma unroll
    for (int ks = 0; ks < kSteps; ++ks) {
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const uint32_t nz = (cb == 0) ? nz0 : (cb == 1) ? nz1 : (cb == 2) ? nz2 : nz3;
        if ((nz >> ks) & 1u) {
          const float a = s_A[cb][ks][lane];
          acc[cb][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks].x, acc[cb][0], 0, 0, 0);
          acc[cb][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks].y, acc[cb][1], 0, 0, 0);
          acc[cb][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks].z, acc[cb][2], 0, 0, 0);
          acc[cb][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ks].w, acc[cb][3], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // weight sums of cell block `wave`: reduce the four lanes sharing a cell
  wsum += __shfl_xor(wsum, 16);
  wsum += __shfl_xor(wsum, 32);
  wtsum += __shfl_xor(wtsum, 16);
  wtsum += __shfl_xor(wtsum, 32);
  if (lane < 16) {
    s_Wt[wave * 16 + lane] = wtsum;
    if (wmap && blockIdx.y == 0 && my_x < g.nx && my_y < g.ny)
      wmap[(int64_t)my_y * g.nx + my_x] = (float)wsum;
  }
  __syncthreads();

  // epilogue: D[i][j] of block cb sits in lane l, register r with
  // i = 4 (l / 16) + r (cell: x = r, y = l / 16 inside the 4 x 4 block) and
  // j = l % 16 (channel c_w + 4 j + q of MFMA q)
  const float qnan = __builtin_nanf("");
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int y = ty * kTileY + (cb >> 1) * 4 + (lane >> 4);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = tx * kTileX + (cb & 1) * 4 + r;
      if (x >= g.nx || y >= g.ny) continue;
      const double wt = s_Wt[cb * 16 + 4 * (lane >> 4) + r];
      const float inv = (wt > 0.0) ? (float)(1.0 / wt) : 0.f;
      const int64_t cell = (int64_t)y * g.nx + x;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t ch = my_ch + q;
        if (ch < C) cube[ch * G + cell] = (wt > 0.0) ? acc[cb][q][r] * inv : qnan;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Few channels (C <= 8) and pair counting: one lane per cell of the 8 x 8
// tile, candidates staged 64 at a time, FP64 accumulation.
// ---------------------------------------------------------------------------
template <int kCM, bool kCount>
__global__ void __launch_bounds__(64) k_gather_cells(
    const double4* __restrict__ trig, const uint32_t* __restrict__ perm,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ nranges, int maxr,
    const float* __restrict__ spectra, int C, GridGeom g, int ntx, double hR,
    double inv_two_sig2, float* __restrict__ cube, float* __restrict__ wmap,
    unsigned long long* __restrict__ pair_count) {
  __shared__ uint2 s_rng[kMaxRangesLimit];
  __shared__ uint32_t s_pre[kMaxRangesLimit + 1];
  __shared__ double4 s_trig[kKB];
  __shared__ float s_spec[kKB][kCM > 0 ? kCM : 1];

  const int tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int tx = tile % ntx, ty = tile / ntx;
  const int ix = tx * kTileX + (lane & 7), iy = ty * kTileY + (lane >> 3);
  const CellTrig cell = cell_trig(g, ix, iy);
  const uint32_t total = stage_ranges(ranges + (int64_t)tile * maxr, nranges[tile], s_rng, s_pre);

  double accv[kCM > 0 ? kCM : 1];
#pragma unroll
  for (int c = 0; c < (kCM > 0 ? kCM : 1); ++c) accv[c] = 0.0;
  double wsum = 0.0;
  unsigned long long npair = 0;
  uint32_t cur = 0;
  for (uint32_t q0 = 0; q0 < total; q0 += kKB) {
    const uint32_t q = q0 + lane;
    if (q < total) {
      const uint32_t pos = cand_pos(q, s_rng, s_pre, &cur);
      s_trig[lane] = trig[pos];
      if (!kCount) {
        const int64_t row = perm[pos];
#pragma unroll
        for (int c = 0; c < kCM; ++c) s_spec[lane][c] = (c < C) ? spectra[row * C + c] : 0.f;
      }
    } else {
      const double nan = __builtin_nan("");
      s_trig[lane] = make_double4(nan, nan, nan, nan);
    }
    __syncthreads();
    const int kmax = (int)min<uint32_t>(kKB, total - q0);
    for (int k = 0; k < kmax; ++k) {
      const double h = pair_hav(cell, s_trig[k]);
      if (h <= hR) {
        if (kCount) {
          ++npair;
        } else {
          const double w = exp(-dist2_from_hav(h) * inv_two_sig2);
          wsum += w;
#pragma unroll
          for (int c = 0; c < kCM; ++c) accv[c] += w * (double)s_spec[k][c];
        }
      }
    }
    __syncthreads();
  }
  if (kCount) {
    for (int off = 32; off > 0; off >>= 1) npair += __shfl_xor(npair, off);
    if (lane == 0) atomicAdd(pair_count, npair);
    return;
  }
  if (ix >= g.nx || iy >= g.ny) return;
  const int64_t G = (int64_t)g.nx * g.ny;
  const int64_t cellidx = (int64_t)iy * g.nx + ix;
  if (wmap) wmap[cellidx] = (float)wsum;
#pragma unroll
  for (int c = 0; c < kCM; ++c)
    if (c < C) cube[c * G + cellidx] = (wsum > 0.0) ? (float)(accv[c] / wsum) : __builtin_nanf("");
}

}  // namespace hcg

using namespace hcg;

static hcg_status launch_cells(const hcg_plan_s* p, const float* spec, int C, float* cube,
                               float* wmap, hipStream_t stream) {
  const double hR = std::pow(std::sin(0.5 * p->support_rad), 2);
  const double inv2 = 1.0 / (2.0 * p->sigma_rad * p->sigma_rad);
  const unsigned ntiles = (unsigned)(p->ntx * p->nty);
#define HCG_CELLS(CM)                                                                       \
  k_gather_cells<CM, false><<<ntiles, 64, 0, stream>>>(p->trig, p->perm, p->ranges,         \
                                                       p->nranges, p->maxr, spec, C, p->grid, \
                                                       p->ntx, hR, inv2, cube, wmap, nullptr)
  if (C == 1) HCG_CELLS(1);
  else if (C == 2) HCG_CELLS(2);
  else if (C <= 4) HCG_CELLS(4);
  else HCG_CELLS(8);
#undef HCG_CELLS
  HCG_LAUNCH_CHECK("k_gather_cells");
  return HCG_OK;
}

extern "C" hcg_status hcg_grid(hcg_plan_t plan, const void* spectra, int64_t nchan,
                               hcg_dtype dtype, const float* chan_scale, float* cube,
                               float* weights, void* hip_stream) {
  if (!plan) return fail(HCG_E_ARG, "hcg_grid: plan is NULL");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_grid: not a live plan");
  if (!spectra || !cube) return fail(HCG_E_ARG, "hcg_grid: spectra and cube must not be NULL");
  if (nchan < 1) return fail(HCG_E_ARG, "hcg_grid: nchan must be >= 1");
  if (dtype != HCG_F32) return fail(HCG_E_UNSUPPORTED, "hcg_grid: dtype %d is not built", (int)dtype);
  if (chan_scale) return fail(HCG_E_ARG, "hcg_grid: chan_scale must be NULL for HCG_F32");
  const hcg_plan_s* p = plan;
  hipStream_t stream = (hipStream_t)hip_stream;
  const float* spec = (const float*)spectra;
  if (nchan <= 8) return launch_cells(p, spec, (int)nchan, cube, weights, stream);

  // the W map (if asked for) is written by the workgroups of the first slab
  const double hR = std::pow(std::sin(0.5 * p->support_rad), 2);
  const double inv2 = 1.0 / (2.0 * p->sigma_rad * p->sigma_rad);
  const int64_t slabs = (nchan + kChanPerWG - 1) / kChanPerWG;
  if (slabs > 65535) return fail(HCG_E_UNSUPPORTED, "hcg_grid: too many channels");
  dim3 grid((unsigned)(p->ntx * p->nty), (unsigned)slabs);
  const bool vec4 = (nchan % 4 == 0) && (((uintptr_t)spec & 15) == 0);
  float* wmap = weights;
  if (vec4)
    k_gather_mfma_f32<true><<<grid, 256, 0, stream>>>(p->trig, p->perm, p->ranges, p->nranges,
                                                      p->maxr, spec, nchan, p->grid, p->ntx, hR,
                                                      inv2, cube, wmap);
  else
    k_gather_mfma_f32<false><<<grid, 256, 0, stream>>>(p->trig, p->perm, p->ranges, p->nranges,
                                                       p->maxr, spec, nchan, p->grid, p->ntx, hR,
                                                       inv2, cube, wmap);
  HCG_LAUNCH_CHECK("k_gather_mfma_f32");
  return HCG_OK;
}

extern "C" hcg_status hcg_get_plan_stats(hcg_plan_t plan, hcg_plan_stats* stats,
                                         void* hip_stream) {
  if (!plan || !stats) return fail(HCG_E_ARG, "hcg_get_plan_stats: NULL pointer");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_get_plan_stats: not a live plan");
  const hcg_plan_s* p = plan;
  hipStream_t stream = (hipStream_t)hip_stream;
  const double hR = std::pow(std::sin(0.5 * p->support_rad), 2);
  const unsigned ntiles = (unsigned)(p->ntx * p->nty);
  unsigned long long* dcount = nullptr;
  HCG_HIP(hipMalloc(&dcount, sizeof(unsigned long long)));
  struct Free {
    void* q;
    ~Free() { (void)hipFree(q); }
  } fr{dcount};
  HCG_HIP(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), stream));
  k_gather_cells<0, true><<<ntiles, 64, 0, stream>>>(p->trig, p->perm, p->ranges, p->nranges,
                                                     p->maxr, nullptr, 0, p->grid, p->ntx, hR, 0.0,
                                                     nullptr, nullptr, dcount);
  HCG_LAUNCH_CHECK("k_gather_cells<count>");
  unsigned long long pairs = 0;
  HCG_HIP(hipMemcpyAsync(&pairs, dcount, sizeof(pairs), hipMemcpyDeviceToHost, stream));
  std::vector<uint32_t> nc(ntiles);
  HCG_HIP(hipMemcpyAsync(nc.data(), p->ncand, sizeof(uint32_t) * ntiles, hipMemcpyDeviceToHost,
                         stream));
  HCG_HIP(hipStreamSynchronize(stream));
  int64_t cand = 0;
  for (uint32_t v : nc) cand += v;
  stats->pairs = (int64_t)pairs;
  stats->candidates = cand;
  stats->cells = (int64_t)p->grid.nx * p->grid.ny;
  return HCG_OK;
}
