// Device geometry shared by the gather kernels and the plan: unit vectors of
// cells, chord and great-circle distances, and the per-ring candidate search
// of Section 3.4 (steps i-iv).
#pragma once

#include <cmath>

#include "hcg_internal.h"

namespace hcg {

// Unit vector of cell (ix, iy); NaN outside the grid (never within R).
struct CellVec {
  double x, y, z;
};

__device__ __forceinline__ CellVec cell_vec(const GridGeom& g, int ix, int iy) {
  CellVec c;
  if (ix >= g.nx || iy >= g.ny) {
    c.x = c.y = c.z = __builtin_nan("");
    return c;
  }
  double sb, cb, sl, cl;
  sincos(cell_lat_deg(g, iy) * kDeg2Rad, &sb, &cb);
  sincos(cell_lon_deg(g, ix) * kDeg2Rad, &sl, &cl);
  c.x = cb * cl;
  c.y = cb * sl;
  c.z = sb;
  return c;
}

// Unit vector of cell (ix, iy) from the plan's array of cell vectors; NaN
// outside the grid (never within R).  A cell whose centre the caller gave as
// non-finite holds NaN in the array.
__device__ __forceinline__ CellVec cell_at(const double4* __restrict__ cells, const GridGeom& g,
                                           int ix, int iy) {
  CellVec c;
  if (ix >= g.nx || iy >= g.ny) {
    c.x = c.y = c.z = __builtin_nan("");
    return c;
  }
  const double4 v = cells[(int64_t)iy * g.nx + ix];
  c.x = v.x;
  c.y = v.y;
  c.z = v.z;
  return c;
}

// Squared chord |u - v|^2 = 4 sin^2(d/2) between a cell and a sample.
__device__ __forceinline__ double chord2(const CellVec& c, const double4& v) {
  const double dx = v.x - c.x, dy = v.y - c.y, dz = v.z - c.z;
  return dx * dx + dy * dy + dz * dz;
}

// Squared great-circle distance from the squared chord c2:
// d^2 = 4 asin^2(chord / 2) = 2 sum_n c2^n / (n^2 binom(2n, n))
//     = c2 (1 + c2/12 + c2^2/90 + c2^3/560 + c2^4/3150 + c2^5/16632 + ...);
// six terms leave a relative error below 2e-17 for c2 < 1e-2 (d < 5.7 deg),
// the arcsine beyond; three terms leave one below 2e-15 for c2 < 1e-4
// (d < 0.57 deg).
// kWide = false: the caller guarantees c2 < 1e-4 (a support radius below
// 0.57 deg, every configuration here), which keeps the longer series, the
// arcsine and their registers out of the kernel.
template <bool kWide = true>
__device__ __forceinline__ double dist2_from_chord2(double c2) {
  if (!kWide) return c2 * (1.0 + c2 * (1.0 / 12.0 + c2 * (1.0 / 90.0)));
  if (c2 < 1e-2)
    return c2 * (1.0 + c2 * (1.0 / 12.0 + c2 * (1.0 / 90.0 + c2 * (1.0 / 560.0 +
           c2 * (1.0 / 3150.0 + c2 * (1.0 / 16632.0))))));
  const double d = 2.0 * asin(fmin(0.5 * sqrt(c2), 1.0));
  return d * d;
}

// FP64 weight of a pair inside the support for the one-lane-per-cell paths
// (FP64 sums): the exponent -d^2 log2(e) / (2 sigma^2) is formed in FP64 and
// evaluated with the hardware base-2 exponential (v_exp_f32, relative error
// about 1e-7) while the result is a normal float, with the FP64 exp2 below
// that (supports wider than about 13 sigma).
__device__ __forceinline__ double pair_weight64(double c2, double wscale) {
  const double e = dist2_from_chord2(c2) * wscale;
  return (e > -126.0) ? (double)__builtin_amdgcn_exp2f((float)e) : exp2(e);
}

// East and north unit vectors of the tangent plane at a cell (east = (-y, x,
// 0) / rho, north = (-z x, -z y, rho^2) / rho, rho = |(x, y)|); at a pole, the
// frame of longitude 0.
struct CellFrame {
  double ex, ey;      // east (ex, ey, 0)
  double nx, ny, nz;  // north
};

__device__ __forceinline__ CellFrame cell_frame(const CellVec& c) {
  const double rho = sqrt(c.x * c.x + c.y * c.y);
  if (!(rho > 0.0)) return CellFrame{0.0, 1.0, c.z > 0.0 ? -1.0 : 1.0, 0.0, 0.0};
  const double r = 1.0 / rho;
  return CellFrame{-c.y * r, c.x * r, -c.z * c.x * r, -c.z * c.y * r, rho};
}

// FP64 weight of a pair inside the support for the kernel shapes other than
// the circular Gaussian (and that one too), evaluated with the FP64 library
// exponential and sine: the elliptical Gaussian takes the sample's offset
// (v - c) in the cell's tangent plane, whose direction is the bearing of the
// great circle from the cell to the sample; the tapered sinc takes d alone.
__device__ __forceinline__ double pair_weight_gen(const KernelParams& k, double c2,
                                                  const double4& v, const CellVec& c,
                                                  const CellFrame& f) {
  const double d2 = dist2_from_chord2<true>(c2);
  if (k.type == kElliptic) {
    const double dx = v.x - c.x, dy = v.y - c.y, dz = v.z - c.z;
    const double xe = dx * f.ex + dy * f.ey;
    const double xn = dx * f.nx + dy * f.ny + dz * f.nz;
    const double a = xn * k.cpa + xe * k.spa, b = xe * k.cpa - xn * k.spa;
    const double s = a * a + b * b;
    if (!(s > 0.0)) return 1.0;  // the sample sits on the cell
    return exp2(d2 * (a * a * k.kmaj + b * b * k.kmin) / s);
  }
  if (k.type == kSinc) {
    const double x = sqrt(d2) * k.sinc_k;
    const double sinc = (x > 0.0) ? sin(x) / x : 1.0;
    return sinc * exp2(d2 * k.taper_k);
  }
  return exp2(d2 * k.wscale);
}

// Candidate search in one ring for cells spanning [lon_a, lon_b] x
// [lat_a, lat_b] (radians): for ring i whose sample band (between the
// latitudes of its two neighbouring rings) comes within R of that span, the
// longitude half-width that a pair within R can have is bounded from the
// haversine,
//   sin^2(dlon/2) <= (sin^2(R/2) - sin^2(dlat_min/2)) / (cos lat_g,min cos lat_n,min),
// widened by half a pixel of that ring (every sample lies within half a
// pixel spacing of its pixel centre in longitude), turned into a pixel range
// and then into a range of sorted positions by binary search inside the
// ring's part of the sorted keys (csr).  Rs is the support radius, hR =
// sin^2(Rs / 2), cos_g = cos of the span's largest |latitude|.
// Ranges of ring i for the tile: up to two [a, b) pieces, in key order.
struct RingRanges {
  uint32_t a0, b0, a1, b1;
};

__device__ inline RingRanges ring_ranges(int i, const uint32_t* __restrict__ keys,
                                  const uint32_t* __restrict__ csr, int ns, int ring_first,
                                  uint32_t pix_base, double lon_a, double lon_b, double lat_a,
                                  double lat_b, double Rs, double hR, double cos_g) {
  RingRanges out{0u, 0u, 0u, 0u};
  const double zt = hpx_ring_z(ns, i - 1), zb = hpx_ring_z(ns, i + 1);
  const double d_hi = asin(fmin(1.0, zt)), d_lo = asin(fmax(-1.0, zb));
  const double dmin = fmax(0.0, fmax(d_lo - lat_b, lat_a - d_hi));
  if (dmin > Rs) return out;
  const double sd = sin(0.5 * dmin);
  const double hrem = hR - sd * sd;
  if (hrem < 0.0) return out;
  const uint32_t ra = csr[i - ring_first], rb = csr[i - ring_first + 1];
  if (rb <= ra) return out;
  const double cos_n = cos(fmax(fabs(d_lo), fabs(d_hi)));
  const double denom = cos_g * cos_n;
  bool whole = !(denom > 1e-300) || hrem >= denom;
  double dal = 0.0;
  if (!whole) {
    dal = 2.0 * asin(sqrt(hrem / denom));
    whole = (lon_b - lon_a) + 2.0 * dal >= 2.0 * kPi;
  }
  const int64_t npix = hpx_ring_npix(ns, i);
  const int64_t start = hpx_ring_start(ns, i);
  int64_t j_lo = 0, j_hi = 0;
  if (!whole) {
    const double shift = (i < ns || i > 3 * ns) ? 0.5 : 0.5 * (double)((i - ns + 1) & 1);
    const double width = 2.0 * kPi / (double)npix;
    const double x_lo = (lon_a - dal - 0.5 * width) / width - shift;
    const double x_hi = (lon_b + dal + 0.5 * width) / width - shift;
    j_lo = (int64_t)ceil(x_lo - 1e-7);
    j_hi = (int64_t)floor(x_hi + 1e-7);
    whole = (j_hi - j_lo + 1) >= npix;
  }
  if (whole) {
    out.a0 = ra;
    out.b0 = rb;
    return out;
  }
  if (j_hi < j_lo) return out;
  int64_t jl = j_lo % npix;
  if (jl < 0) jl += npix;
  int64_t jh = j_hi % npix;
  if (jh < 0) jh += npix;
  const int64_t base = (int64_t)pix_base;
  if (jl <= jh) {
    out.a0 = lower_bound_u32(keys, ra, rb, start + jl - base);
    out.b0 = lower_bound_u32(keys, out.a0, rb, start + jh + 1 - base);
  } else {  // wraps through longitude 0 of this ring: two pieces, in key order
    out.a0 = ra;
    out.b0 = lower_bound_u32(keys, ra, rb, start + jh + 1 - base);
    out.a1 = lower_bound_u32(keys, out.b0, rb, start + jl - base);
    out.b1 = rb;
  }
  return out;
}

// Squared chord of the support radius, 4 sin^2(R / 2), and the exponent
// scale -log2(e) / (2 sigma^2) of the weights.
inline double support_chord2(const hcg_plan_s* p) {
  const double s = std::sin(0.5 * p->support_rad);
  return 4.0 * s * s;
}
inline double weight_scale(const hcg_plan_s* p) { return p->kern.wscale; }

}  // namespace hcg
