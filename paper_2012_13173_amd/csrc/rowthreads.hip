// The paper's own GPU gather scheme, kept beside the tile kernels as the
// prior-art baseline they are measured against (one channel, as the paper
// grids).
//
// Thread organisation and coarsening (Section 3.5 I): a one-dimensional
// grid of one-dimensional blocks; each thread takes gamma consecutive cells
// of one latitude row of the map.  Each thread searches its own candidates
// (Section 3.4 steps i-iv): the rings within R of its row, in each ring the
// pixel range that its cells' longitude span plus the support can reach, the
// sorted positions of those pixels by binary search in the ring's part of the
// sorted keys; it then walks the samples and accumulates, for its gamma
// cells, the weights and weighted values in registers (step v).  The
// distance and weight are those of the tile kernels' one-lane-per-cell
// path (FP64 chord series, pair_weight64, FP64 sums), so the two differ only
// in how work and candidates are organised.
#include "hcg_internal.h"
#include "sphere.h"

namespace hcg {
namespace {

template <int kGamma>
__global__ void __launch_bounds__(512) k_gather_rowthreads(
    const double4* __restrict__ xyz, const uint32_t* __restrict__ keys,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ csr, int ns, int ring_first,
    int ring_last, uint32_t pix_base, GridGeom g, double support_rad, double c2R, double wscale,
    const float* __restrict__ spectra, float* __restrict__ map, float* __restrict__ wmap) {
  const int per_row = (g.nx + kGamma - 1) / kGamma;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)per_row * g.ny) return;
  const int iy = (int)(t / per_row);
  const int ix0 = (int)(t % per_row) * kGamma;
  const int ncell = min(kGamma, g.nx - ix0);

  CellVec cell[kGamma];
  double acc[kGamma], wsum[kGamma];
#pragma unroll
  for (int j = 0; j < kGamma; ++j) {
    cell[j] = cell_vec(g, ix0 + j, iy);  // NaN past the row's end: never within R
    acc[j] = 0.0;
    wsum[j] = 0.0;
  }
  // step i: the span of the thread's cells and the rings within R of it
  double lon_a = cell_lon_deg(g, ix0) * kDeg2Rad;
  double lon_b = cell_lon_deg(g, ix0 + ncell - 1) * kDeg2Rad;
  if (lon_a > lon_b) { const double s = lon_a; lon_a = lon_b; lon_b = s; }
  const double half_pi = 0.5 * kPi;
  const double lat = fmax(-half_pi, fmin(half_pi, cell_lat_deg(g, iy) * kDeg2Rad));
  const double Rs = support_rad * (1.0 + 1e-9) + 1e-12;  // absorbs rounding of the bounds
  const double sR = sin(0.5 * Rs);
  const double hR = sR * sR;
  const double cos_g = cos(fabs(lat));
  const double z_top = sin(fmin(half_pi, lat + Rs));
  const double z_bot = sin(fmax(-half_pi, lat - Rs));
  const int i_lo = max(ring_first, (int)floor(hpx_ring_of_z(ns, z_top)) - 2);
  const int i_hi = min(ring_last, (int)ceil(hpx_ring_of_z(ns, z_bot)) + 2);

  for (int i = i_lo; i <= i_hi; ++i) {
    // steps ii-iii: the sorted positions of the ring's reachable pixels
    const RingRanges rr = ring_ranges(i, keys, csr, ns, ring_first, pix_base, lon_a, lon_b, lat,
                                      lat, Rs, hR, cos_g);
    // steps iv-v: walk the samples of each piece
    for (int piece = 0; piece < 2; ++piece) {
      const uint32_t a = piece ? rr.a1 : rr.a0, b = piece ? rr.b1 : rr.b0;
      for (uint32_t q = a; q < b; ++q) {
        const double4 v = xyz[q];
        const double s = (double)spectra[perm[q]];
#pragma unroll
        for (int j = 0; j < kGamma; ++j) {
          const double c2 = chord2(cell[j], v);
          if (c2 <= c2R) {
            const double w = pair_weight64(c2, wscale);
            wsum[j] += w;
            acc[j] += w * s;
          }
        }
      }
    }
  }
  const int64_t row = (int64_t)iy * g.nx;
#pragma unroll
  for (int j = 0; j < kGamma; ++j) {
    if (j < ncell) {
      const int64_t c = row + ix0 + j;
      map[c] = (wsum[j] > 0.0) ? (float)(acc[j] / wsum[j]) : __builtin_nanf("");
      if (wmap) wmap[c] = (float)wsum[j];
    }
  }
}

}  // namespace
}  // namespace hcg

using namespace hcg;

extern "C" hcg_status hcg_grid_rowthreads(hcg_plan_t plan, const float* spectra, int gamma,
                                          int block, float* map, float* weights,
                                          void* hip_stream) {
  if (!plan) return fail(HCG_E_ARG, "hcg_grid_rowthreads: plan is NULL");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_grid_rowthreads: not a live plan");
  if (!spectra || !map) return fail(HCG_E_ARG, "hcg_grid_rowthreads: NULL pointer");
  if (gamma < 1 || gamma > 4)
    return fail(HCG_E_ARG, "hcg_grid_rowthreads: gamma must be 1 .. 4 (got %d)", gamma);
  if (block < 64 || block > 512 || block % 64 != 0)
    return fail(HCG_E_ARG, "hcg_grid_rowthreads: block must be a multiple of 64 in 64 .. 512");
  const hcg_plan_s* p = plan;
  // the scheme walks latitude rows of a linear grid with the Gaussian kernel
  if (p->centres || p->kern.type != kGauss)
    return fail(HCG_E_UNSUPPORTED,
                "hcg_grid_rowthreads: needs a plan on a linear grid with the Gaussian kernel");
  const GridGeom g = p->grid;
  const int64_t threads = (int64_t)((g.nx + gamma - 1) / gamma) * g.ny;
  const int64_t blocks = (threads + block - 1) / block;
  const double c2R = support_chord2(p), wscale = weight_scale(p);
  hipStream_t st = (hipStream_t)hip_stream;
#define HCG_ROWS(G)                                                                         \
  k_gather_rowthreads<G><<<(unsigned)blocks, block, 0, st>>>(                               \
      p->xyz, p->keys, p->perm, p->csr, p->nside, p->ring_first, p->ring_last, p->pix_base, \
      g, p->support_rad, c2R, wscale, spectra, map, weights)
  switch (gamma) {
    case 1: HCG_ROWS(1); break;
    case 2: HCG_ROWS(2); break;
    case 3: HCG_ROWS(3); break;
    default: HCG_ROWS(4); break;
  }
#undef HCG_ROWS
  HCG_LAUNCH_CHECK("k_gather_rowthreads");
  return HCG_OK;
}
