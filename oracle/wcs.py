"""FP64 pixel <-> sky transforms of FITS world coordinates -- TEST INFRASTRUCTURE.

Only ``tests/`` may import this module (the oracle's rule).  It is the
reference for target grids in projected coordinates: the paper grids in the
space of the FITS world coordinate system (Section 2.1, citing Calabretta &
Greisen 2002, A&A 395, 1077, "Paper II", for it) and exports FITS products
(Section 3.1).
Implemented: CAR (plate carree), SFL (Sanson-Flamsteed), SIN (orthographic,
without the xi/eta extension) and TAN (gnomonic), with a diagonal CDELT
scaling (no PC matrix), LONPOLE and LATPOLE as in Paper II section 2.4.

All angles are degrees.  Steps, each with the Paper II equation it follows:

1. intermediate world coordinates  x = CDELT1 (p1 - CRPIX1), y = CDELT2 (p2 - CRPIX2);
2. projection plane -> native spherical (phi, theta)  (sections 5.1 and 5.2);
3. native -> celestial (alpha, delta) by the spherical rotation of eq. (2),
   with the celestial pole (alpha_p, delta_p) from eqs. (8)-(10) and the
   native longitude of the celestial pole phi_p = LONPOLE (default 0 if
   delta_0 >= theta_0 else 180 deg).
The inverse path (celestial -> pixel) uses eq. (5) and the forward projections.
"""
from __future__ import annotations

import math

import numpy as np

D2R = math.pi / 180.0
R2D = 180.0 / math.pi

# native coordinates (phi_0, theta_0) of the reference point (Paper II, Table 13)
_REF = {"CAR": (0.0, 0.0), "SFL": (0.0, 0.0), "SIN": (0.0, 90.0), "TAN": (0.0, 90.0)}


def _arg(a, b):
    """Paper II's arg(x, y): the angle of the point (x, y), degrees."""
    return np.degrees(np.arctan2(b, a))


def celestial_pole(proj, crval, lonpole=None, latpole=90.0):
    """(alpha_p, delta_p, phi_p) of the celestial pole in native coordinates,
    Paper II eqs. (8)-(10); LATPOLE picks between the two solutions of eq. (8)."""
    phi0, theta0 = _REF[proj]
    a0, d0 = float(crval[0]), float(crval[1])
    phi_p = (0.0 if d0 >= theta0 else 180.0) if lonpole is None else float(lonpole)
    if theta0 == 90.0:  # zenithal: the reference point is the native pole
        return a0, d0, phi_p
    ct0, st0 = math.cos(theta0 * D2R), math.sin(theta0 * D2R)
    dphi = (phi_p - phi0) * D2R
    base = math.degrees(math.atan2(st0, ct0 * math.cos(dphi)))
    den = math.sqrt(1.0 - (ct0 * math.sin(dphi)) ** 2)
    ratio = math.sin(d0 * D2R) / den
    if abs(ratio) > 1.0 + 1e-12:
        raise ValueError("no celestial pole for this reference point and LONPOLE")
    dd = math.degrees(math.acos(max(-1.0, min(1.0, ratio))))
    # the two solutions of eq. (8), as latitudes in [-180, 180); only those in
    # [-90, 90] place a pole
    cands = [((c + 180.0) % 360.0) - 180.0 for c in (base + dd, base - dd)]
    cands = [c for c in cands if -90.0 - 1e-12 <= c <= 90.0 + 1e-12]
    if not cands:
        raise ValueError("LONPOLE puts no celestial pole in reach of this reference point")
    delta_p = min(cands, key=lambda c: abs(c - latpole))
    delta_p = max(-90.0, min(90.0, delta_p))
    if abs(abs(delta_p) - 90.0) < 1e-12:
        # eq. (2) at the pole: alpha = alpha_p + phi - phi_p + 180 (north) or
        # alpha_p - phi + phi_p (south); the reference point fixes alpha_p
        alpha_p = a0 - (phi0 - phi_p + 180.0) if delta_p > 0 else a0 + (phi0 - phi_p)
    elif abs(abs(d0) - 90.0) < 1e-12:
        alpha_p = a0
    else:
        sdp, cdp = math.sin(delta_p * D2R), math.cos(delta_p * D2R)
        sd0, cd0 = math.sin(d0 * D2R), math.cos(d0 * D2R)
        alpha_p = a0 - math.degrees(math.atan2(math.sin(dphi) * ct0 / cd0,
                                               (st0 - sdp * sd0) / (cd0 * cdp)))
    return alpha_p, delta_p, phi_p


def _native_from_plane(proj, x, y):
    """Projection plane (x, y) -> native (phi, theta), Paper II sections 5.1-5.2."""
    if proj == "CAR":
        return x, y
    if proj == "SFL":
        return x / np.cos(y * D2R), y
    r = np.hypot(x, y)
    phi = _arg(-y, x)
    if proj == "TAN":
        theta = np.degrees(np.arctan2(R2D, r))
    else:  # SIN
        s = r * D2R
        if np.any(s > 1.0 + 1e-15):
            raise ValueError("SIN: point outside the projection's disc")
        theta = np.degrees(np.arccos(np.clip(s, -1.0, 1.0)))
    return phi, theta


def _plane_from_native(proj, phi, theta):
    """Native (phi, theta) -> projection plane (x, y): the forward projections."""
    if proj == "CAR":
        return phi, theta
    if proj == "SFL":
        return phi * np.cos(theta * D2R), theta
    if proj == "TAN":
        r = R2D / np.tan(theta * D2R)
    else:  # SIN
        r = R2D * np.cos(theta * D2R)
    return r * np.sin(phi * D2R), -r * np.cos(phi * D2R)


def native_to_celestial(phi, theta, alpha_p, delta_p, phi_p):
    """Paper II eq. (2)."""
    st, ct = np.sin(theta * D2R), np.cos(theta * D2R)
    sdp, cdp = math.sin(delta_p * D2R), math.cos(delta_p * D2R)
    dphi = (phi - phi_p) * D2R
    alpha = alpha_p + _arg(st * cdp - ct * sdp * np.cos(dphi), -ct * np.sin(dphi))
    delta = np.degrees(np.arcsin(np.clip(st * sdp + ct * cdp * np.cos(dphi), -1.0, 1.0)))
    return np.mod(alpha, 360.0), delta


def celestial_to_native(alpha, delta, alpha_p, delta_p, phi_p):
    """Paper II eq. (5)."""
    sd, cd = np.sin(delta * D2R), np.cos(delta * D2R)
    sdp, cdp = math.sin(delta_p * D2R), math.cos(delta_p * D2R)
    da = (alpha - alpha_p) * D2R
    phi = phi_p + _arg(sd * cdp - cd * sdp * np.cos(da), -cd * np.sin(da))
    theta = np.degrees(np.arcsin(np.clip(sd * sdp + cd * cdp * np.cos(da), -1.0, 1.0)))
    return np.mod(phi + 180.0, 360.0) - 180.0, theta


def pix2world(proj, p1, p2, crpix, cdelt, crval, lonpole=None, latpole=90.0):
    """Pixel coordinates -> (alpha, delta) in degrees, alpha in [0, 360)."""
    proj = proj.upper()
    x = cdelt[0] * (np.asarray(p1, dtype=np.float64) - crpix[0])
    y = cdelt[1] * (np.asarray(p2, dtype=np.float64) - crpix[1])
    phi, theta = _native_from_plane(proj, x, y)
    ap, dp, pp = celestial_pole(proj, crval, lonpole, latpole)
    return native_to_celestial(phi, theta, ap, dp, pp)


def world2pix(proj, alpha, delta, crpix, cdelt, crval, lonpole=None, latpole=90.0):
    """(alpha, delta) in degrees -> pixel coordinates (the inverse of pix2world)."""
    proj = proj.upper()
    ap, dp, pp = celestial_pole(proj, crval, lonpole, latpole)
    phi, theta = celestial_to_native(np.asarray(alpha, dtype=np.float64),
                                     np.asarray(delta, dtype=np.float64), ap, dp, pp)
    x, y = _plane_from_native(proj, phi, theta)
    return x / cdelt[0] + crpix[0], y / cdelt[1] + crpix[1]


def cell_centres(proj, nx, ny, crpix, cdelt, crval, lonpole=None, latpole=90.0):
    """(lon, lat) [ny, nx] of the centres of an nx x ny map, pixel (ix, iy)
    at p = (ix + 1, iy + 1) (FITS pixels count from 1)."""
    iy, ix = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                         indexing="ij")
    return pix2world(proj, ix + 1.0, iy + 1.0, crpix, cdelt, crval, lonpole, latpole)
