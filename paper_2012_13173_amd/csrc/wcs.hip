// World coordinates of the pixel centres of a projected map, for targets
// given by their cell centres (hcg_plan_ex).  The paper grids in the space of
// the FITS world coordinate system (Section 2.1, after Calabretta & Greisen
// 2002, "Paper II"); four of its projections are built here, with a diagonal
// CDELT scaling (no PC matrix):
//   CAR (plate carree) and SFL (Sanson-Flamsteed): cylindrical, reference
//   point on the native equator (phi_0, theta_0) = (0, 0);
//   SIN (orthographic, without the xi/eta terms) and TAN (gnomonic):
//   zenithal, reference point at the native pole (0, 90).
// Steps per pixel (ix, iy), FITS pixel p = (ix + 1, iy + 1):
//   1. intermediate world coordinates x = CDELT1 (p1 - CRPIX1),
//      y = CDELT2 (p2 - CRPIX2), degrees;
//   2. native spherical (phi, theta) from the projection's inverse
//      (Paper II sections 5.1 and 5.2);
//   3. celestial (alpha, delta) by the spherical rotation of Paper II
//      eq. (2), the celestial pole (alpha_p, delta_p) and the native longitude
//      of the celestial pole phi_p = LONPOLE found on the host from the
//      reference point (eqs. (8) to (10); LONPOLE defaults to 0 when
//      delta_0 >= theta_0, else 180; LATPOLE picks between the two solutions
//      of eq. (8)).
#include <cmath>

#include "hcg_internal.h"

namespace hcg {
namespace {

constexpr double kR2D = 57.29577951308232;

struct WcsDev {
  int proj, nx, ny;
  double crpix1, crpix2, cdelt1, cdelt2;
  double alpha_p, delta_p, phi_p;  // degrees
};

__global__ void __launch_bounds__(256) k_wcs_centres(WcsDev w, double* __restrict__ lon,
                                                     double* __restrict__ lat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)w.nx * w.ny) return;
  const double p1 = (double)(i % w.nx) + 1.0, p2 = (double)(i / w.nx) + 1.0;
  const double x = w.cdelt1 * (p1 - w.crpix1), y = w.cdelt2 * (p2 - w.crpix2);
  const double nan = __builtin_nan("");
  double phi, theta;  // native, degrees
  if (w.proj == HCG_PROJ_CAR) {
    phi = x;
    theta = y;
  } else if (w.proj == HCG_PROJ_SFL) {
    theta = y;
    const double c = cos(theta * kDeg2Rad);
    phi = (fabs(theta) < 90.0 && c > 0.0) ? x / c : nan;
  } else {
    const double r = sqrt(x * x + y * y);
    phi = atan2(x, -y) * kR2D;
    if (w.proj == HCG_PROJ_TAN) {
      theta = atan2(kR2D, r) * kR2D;
    } else {  // SIN: r = (180 / pi) cos(theta)
      const double s = r * kDeg2Rad;
      theta = (s <= 1.0) ? acos(s) * kR2D : nan;
    }
  }
  if (!(fabs(theta) <= 90.0) || !isfinite(phi)) {
    lon[i] = nan;
    lat[i] = nan;
    return;
  }
  double st, ct, sdp, cdp, sdl, cdl;
  sincos(theta * kDeg2Rad, &st, &ct);
  sincos(w.delta_p * kDeg2Rad, &sdp, &cdp);
  sincos((phi - w.phi_p) * kDeg2Rad, &sdl, &cdl);
  double alpha = w.alpha_p + atan2(-ct * sdl, st * cdp - ct * sdp * cdl) * kR2D;
  const double sd = fmax(-1.0, fmin(1.0, st * sdp + ct * cdp * cdl));
  alpha = fmod(alpha, 360.0);
  if (alpha < 0.0) alpha += 360.0;
  if (alpha >= 360.0) alpha -= 360.0;
  lon[i] = alpha;
  lat[i] = asin(sd) * kR2D;
}

// Celestial pole of the map (Paper II eqs. (8) to (10)), degrees.
hcg_status celestial_pole(const hcg_wcs& w, double* alpha_p, double* delta_p, double* phi_p) {
  const bool zenithal = (w.proj == HCG_PROJ_SIN || w.proj == HCG_PROJ_TAN);
  const double phi0 = 0.0, theta0 = zenithal ? 90.0 : 0.0;
  const double a0 = w.crval1, d0 = w.crval2;
  *phi_p = w.lonpole_set ? w.lonpole : (d0 >= theta0 ? 0.0 : 180.0);
  if (zenithal) {  // the reference point is the native pole
    *alpha_p = a0;
    *delta_p = d0;
    return HCG_OK;
  }
  // cylindrical, theta0 = 0: delta_p = arg(cos(phi_p - phi0), 0) +- acos(sin d0 / |cos(phi_p - phi0)|)
  const double dphi = (*phi_p - phi0) * kDeg2Rad;
  const double st0 = std::sin(theta0 * kDeg2Rad), ct0 = std::cos(theta0 * kDeg2Rad);
  const double base = std::atan2(st0, ct0 * std::cos(dphi)) * kR2D;
  const double den = std::sqrt(std::max(0.0, 1.0 - std::pow(ct0 * std::sin(dphi), 2)));
  const double ratio = (den > 0.0) ? std::sin(d0 * kDeg2Rad) / den : 2.0;
  if (std::fabs(ratio) > 1.0 + 1e-12)
    return fail(HCG_E_ARG, "hcg_wcs_centres: no celestial pole for this reference point and LONPOLE");
  const double half = std::acos(std::max(-1.0, std::min(1.0, ratio))) * kR2D;
  bool found = false;
  double best = 0.0;
  for (double c : {base + half, base - half}) {
    double v = std::fmod(c + 180.0, 360.0);
    if (v < 0.0) v += 360.0;
    v -= 180.0;  // [-180, 180)
    if (v < -90.0 - 1e-12 || v > 90.0 + 1e-12) continue;
    if (!found || std::fabs(v - w.latpole) < std::fabs(best - w.latpole)) best = v;
    found = true;
  }
  if (!found)
    return fail(HCG_E_ARG, "hcg_wcs_centres: LONPOLE puts no celestial pole in reach");
  const double dp = std::max(-90.0, std::min(90.0, best));
  *delta_p = dp;
  if (std::fabs(std::fabs(dp) - 90.0) < 1e-12) {
    // eq. (2) at a celestial pole: alpha = alpha_p + phi - phi_p + 180 (north)
    // or alpha_p - phi + phi_p (south), at the reference point
    *alpha_p = (dp > 0.0) ? a0 - (phi0 - *phi_p + 180.0) : a0 + (phi0 - *phi_p);
  } else if (std::fabs(std::fabs(d0) - 90.0) < 1e-12) {
    *alpha_p = a0;
  } else {
    const double sdp = std::sin(dp * kDeg2Rad), cdp = std::cos(dp * kDeg2Rad);
    const double sd0 = std::sin(d0 * kDeg2Rad), cd0 = std::cos(d0 * kDeg2Rad);
    *alpha_p = a0 - std::atan2(std::sin(dphi) * ct0 / cd0, (st0 - sdp * sd0) / (cd0 * cdp)) * kR2D;
  }
  return HCG_OK;
}

}  // namespace
}  // namespace hcg

using namespace hcg;

extern "C" hcg_status hcg_wcs_centres(const hcg_wcs* wcs, double* lon_deg, double* lat_deg,
                                      void* hip_stream) {
  if (!wcs || !lon_deg || !lat_deg) return fail(HCG_E_ARG, "hcg_wcs_centres: NULL pointer");
  const hcg_wcs& w = *wcs;
  if (w.proj < HCG_PROJ_CAR || w.proj > HCG_PROJ_TAN)
    return fail(HCG_E_UNSUPPORTED, "hcg_wcs_centres: unknown projection %d", (int)w.proj);
  if (w.nx < 1 || w.ny < 1 || (int64_t)w.nx * w.ny > INT32_MAX)
    return fail(HCG_E_ARG, "hcg_wcs_centres: nx, ny out of range");
  const double vals[] = {w.crpix1, w.crpix2, w.cdelt1, w.cdelt2, w.crval1, w.crval2, w.latpole,
                         w.lonpole_set ? w.lonpole : 0.0};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(HCG_E_ARG, "hcg_wcs_centres: non-finite parameter");
  if (w.cdelt1 == 0.0 || w.cdelt2 == 0.0 || std::fabs(w.crval2) > 90.0)
    return fail(HCG_E_ARG, "hcg_wcs_centres: zero CDELT or |CRVAL2| > 90");
  hcg_status st = check_device_arch();
  if (st != HCG_OK) return st;
  WcsDev d{w.proj, w.nx, w.ny, w.crpix1, w.crpix2, w.cdelt1, w.cdelt2, 0.0, 0.0, 0.0};
  st = celestial_pole(w, &d.alpha_p, &d.delta_p, &d.phi_p);
  if (st != HCG_OK) return st;
  const int64_t ncell = (int64_t)w.nx * w.ny;
  k_wcs_centres<<<(unsigned)((ncell + 255) / 256), 256, 0, (hipStream_t)hip_stream>>>(
      d, lon_deg, lat_deg);
  HCG_LAUNCH_CHECK("k_wcs_centres");
  return HCG_OK;
}
