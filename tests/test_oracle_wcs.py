"""Pins of the WCS oracle (oracle/wcs.py; Calabretta & Greisen 2002, which the
paper cites for its world coordinates in Section 2.1) against facts that do
not depend on its formulas:

* the reference pixel maps to CRVAL, for every projection and reference point;
* CAR and SFL with the reference point on the equator are the closed forms
  alpha = alpha_0 + x, delta = y and alpha = alpha_0 + x / cos y, delta = y
  (and CAR then is the linear lon/lat grid the gather kernels take);
* zenithal radial laws: the great-circle distance (haversine, written here)
  from the reference point is atan(R) for TAN and asin(R) for SIN, R the
  radius in the projection plane in radians, for any reference point;
* orientation: +y runs along the meridian of the reference point towards
  the north, +x towards increasing right ascension;
* oblique cylindrical maps: the pixel column through the reference pixel is
  the meridian of CRVAL, the pixel row the great circle at right angles to
  it (distance |x| from CRVAL);
* world2pix inverts pix2world to 1e-8 pixel.
"""
import math

import numpy as np
import pytest

from oracle import wcs

CRVALS = [(180.0, 30.0), (10.0, 0.0), (300.0, -60.0), (45.0, 89.0), (0.0, 90.0), (0.0, -90.0)]
PROJS = ["CAR", "SFL", "SIN", "TAN"]


def hav_deg(a1, d1, a2, d2):
    """Great-circle distance in degrees (haversine)."""
    a1, d1, a2, d2 = (np.radians(np.asarray(v, dtype=np.float64)) for v in (a1, d1, a2, d2))
    h = np.sin((d2 - d1) / 2) ** 2 + np.cos(d1) * np.cos(d2) * np.sin((a2 - a1) / 2) ** 2
    return np.degrees(2 * np.arcsin(np.sqrt(np.minimum(1.0, h))))


def wrap180(x):
    return (np.asarray(x) + 180.0) % 360.0 - 180.0


@pytest.mark.parametrize("proj", PROJS)
@pytest.mark.parametrize("crval", CRVALS)
def test_reference_pixel_is_crval(proj, crval):
    a, d = wcs.pix2world(proj, 61.0, 45.0, (61.0, 45.0), (-0.01, 0.02), crval)
    assert abs(float(d) - crval[1]) < 1e-9
    if abs(crval[1]) < 90.0:
        assert abs(float(wrap180(a - crval[0]))) < 1e-9


def test_car_on_equator_is_linear_lonlat_grid():
    nx, ny, dl, db, l0 = 40, 30, -0.05, 0.04, 123.0
    lon, lat = wcs.cell_centres("CAR", nx, ny, ((nx + 1) / 2, (ny + 1) / 2), (dl, db), (l0, 0.0))
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    # the linear grid of the gather kernels: lon0 + (ix - (nx-1)/2) dlon, (iy - (ny-1)/2) dlat
    np.testing.assert_allclose(wrap180(lon - (l0 + (ix - (nx - 1) / 2) * dl)), 0.0, atol=1e-10)
    np.testing.assert_allclose(lat, (iy - (ny - 1) / 2) * db, atol=1e-10)


def test_sfl_on_equator_closed_form():
    p1 = np.array([1.0, 20.0, 57.0, 100.0])
    p2 = np.array([3.0, 77.0, 140.0, 160.0])
    a, d = wcs.pix2world("SFL", p1, p2, (50.0, 80.0), (0.1, 0.25), (200.0, 0.0))
    x, y = 0.1 * (p1 - 50.0), 0.25 * (p2 - 80.0)
    np.testing.assert_allclose(d, y, atol=1e-10)
    np.testing.assert_allclose(wrap180(a - 200.0 - x / np.cos(np.radians(y))), 0.0, atol=1e-9)


@pytest.mark.parametrize("proj,law", [("TAN", np.arctan), ("SIN", np.arcsin)])
@pytest.mark.parametrize("crval", CRVALS)
def test_zenithal_radial_law(proj, law, crval):
    rng = np.random.default_rng(11)
    p1 = rng.uniform(-300, 300, 200)
    p2 = rng.uniform(-300, 300, 200)
    cd = (-0.1, 0.1)
    a, d = wcs.pix2world(proj, p1, p2, (0.0, 0.0), cd, crval)
    R = np.radians(np.hypot(cd[0] * p1, cd[1] * p2))
    np.testing.assert_allclose(hav_deg(a, d, *crval), np.degrees(law(R)), atol=1e-9)


@pytest.mark.parametrize("proj", PROJS)
def test_orientation(proj):
    crval = (150.0, 20.0)
    # +y: north along the reference meridian
    a, d = wcs.pix2world(proj, 0.0, 30.0, (0.0, 0.0), (0.1, 0.1), crval)
    assert abs(float(wrap180(a - 150.0))) < 1e-9 and float(d) > 20.0
    # +x: towards increasing right ascension
    a, d = wcs.pix2world(proj, 30.0, 0.0, (0.0, 0.0), (0.1, 0.1), crval)
    assert 0.0 < float(wrap180(a - 150.0)) < 10.0


@pytest.mark.parametrize("proj", ["CAR", "SFL"])
@pytest.mark.parametrize("d0", [30.0, -45.0, 75.0])
def test_oblique_cylindrical_axes(proj, d0):
    cd = (0.2, 0.2)
    # the column through the reference pixel: the meridian of CRVAL
    y = np.arange(-50, 51) * cd[1]
    keep = np.abs(d0 + y) < 89.0
    a, d = wcs.pix2world(proj, np.zeros(101)[keep], np.arange(-50, 51)[keep].astype(float),
                         (0.0, 0.0), cd, (40.0, d0))
    np.testing.assert_allclose(wrap180(a - 40.0), 0.0, atol=1e-9)
    np.testing.assert_allclose(d, d0 + y[keep], atol=1e-9)
    # the row through the reference pixel: distance |x| along a great circle
    x = np.arange(-80, 81) * cd[0]
    a, d = wcs.pix2world(proj, np.arange(-80, 81).astype(float), np.zeros(161), (0.0, 0.0), cd,
                         (40.0, d0))
    np.testing.assert_allclose(hav_deg(a, d, 40.0, d0), np.abs(x), atol=1e-9)


@pytest.mark.parametrize("proj", PROJS)
@pytest.mark.parametrize("crval", [(180.0, 30.0), (10.0, 0.0), (300.0, -60.0), (45.0, 85.0)])
def test_round_trip(proj, crval):
    p1, p2 = np.meshgrid(np.linspace(1, 200, 23), np.linspace(1, 150, 17))
    crpix, cd = (100.5, 75.5), (-0.05, 0.05)
    a, d = wcs.pix2world(proj, p1, p2, crpix, cd, crval)
    q1, q2 = wcs.world2pix(proj, a, d, crpix, cd, crval)
    np.testing.assert_allclose(q1, p1, atol=1e-8)
    np.testing.assert_allclose(q2, p2, atol=1e-8)


def test_sin_outside_disc_raises():
    with pytest.raises(ValueError):
        wcs.pix2world("SIN", 1000.0, 0.0, (0.0, 0.0), (0.1, 0.1), (0.0, 0.0))


def test_unreachable_pole_raises():
    # a cylindrical reference point at delta 30 with LONPOLE 150: the pole would
    # need cos(theta_p) < 0 (60 deg from the reference point, 150 deg round)
    with pytest.raises(ValueError):
        wcs.pix2world("CAR", 0.0, 0.0, (0.0, 0.0), (0.1, 0.1), (40.0, 30.0), lonpole=150.0)


@pytest.mark.parametrize("proj,lonpole", [("CAR", 30.0), ("SFL", 30.0), ("SIN", 150.0),
                                          ("TAN", 150.0)])
def test_non_default_lonpole(proj, lonpole):
    # LONPOLE other than 0 / 180 deg: the reference pixel still maps to CRVAL,
    # the zenithal radial laws still hold, and world2pix inverts pix2world
    crval, cd, crpix = (40.0, 30.0), (-0.1, 0.1), (10.0, 20.0)
    a, d = wcs.pix2world(proj, crpix[0], crpix[1], crpix, cd, crval, lonpole=lonpole)
    assert abs(float(wrap180(a - crval[0]))) < 1e-9 and abs(float(d) - crval[1]) < 1e-9
    p1, p2 = np.meshgrid(np.linspace(-40, 60, 11), np.linspace(-30, 70, 9))
    a, d = wcs.pix2world(proj, p1, p2, crpix, cd, crval, lonpole=lonpole)
    if proj in ("TAN", "SIN"):
        R = np.radians(np.hypot(cd[0] * (p1 - crpix[0]), cd[1] * (p2 - crpix[1])))
        law = np.arctan if proj == "TAN" else np.arcsin
        np.testing.assert_allclose(hav_deg(a, d, *crval), np.degrees(law(R)), atol=1e-9)
    q1, q2 = wcs.world2pix(proj, a, d, crpix, cd, crval, lonpole=lonpole)
    np.testing.assert_allclose(q1, p1, atol=1e-8)
    np.testing.assert_allclose(q2, p2, atol=1e-8)
