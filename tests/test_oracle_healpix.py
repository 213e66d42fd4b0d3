"""Pins for the oracle's HEALPix ring scheme (Section 3.2; Gorski et al. 2005).

Each check rests on a property of the pixelisation itself rather than on the
oracle's own formulas: the ring tables must tile 12 Ns^2 pixels; every pixel
centre (from the ring tables) must map back to its pixel; belt pixels are
diamonds of half-width 1/(2Ns) in t = 2 phi/pi and half-height 2/(3Ns) in z
around their centre; every point lies between the latitudes of the rings
adjacent to its own; all pixels have equal area.
"""
import math

import numpy as np
import pytest

import oracle

NSIDES = [1, 2, 4, 8, 16, 4096, 8192, 16384]


@pytest.mark.parametrize("ns", NSIDES)
def test_ring_tables_tile_the_sphere(ns):
    assert oracle.npix(ns) == 12 * ns * ns
    if ns <= 16:
        rings = list(range(1, 4 * ns))
        total = 0
        for i in rings:
            assert oracle.ring_start(ns, i) == total
            total += oracle.ring_npix(ns, i)
        assert total == 12 * ns * ns
    else:
        rings = sorted(set(list(range(1, 40)) + list(range(ns - 3, ns + 4))
                           + list(range(2 * ns - 3, 2 * ns + 4))
                           + list(range(3 * ns - 3, 3 * ns + 4)) + list(range(4 * ns - 40, 4 * ns))))
    for i in rings:
        if i < 4 * ns - 1:
            assert oracle.ring_start(ns, i + 1) - oracle.ring_start(ns, i) == oracle.ring_npix(ns, i)
        # pixels per ring: 4i in the caps, 4 Ns in the belt, symmetric about the equator
        assert oracle.ring_npix(ns, i) == oracle.ring_npix(ns, 4 * ns - i)
        assert oracle.ring_npix(ns, i) == 4 * min(i, ns, 4 * ns - i)
        # ring latitudes are symmetric about the equator
        assert abs(oracle.ring_z(ns, i) + oracle.ring_z(ns, 4 * ns - i)) < 1e-15
    last = 4 * ns - 1
    assert oracle.ring_start(ns, last) + oracle.ring_npix(ns, last) == 12 * ns * ns
    assert oracle.ring_z(ns, ns) == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert oracle.ring_z(ns, 2 * ns) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("ns", [1, 2, 4, 8, 16, 32])
def test_every_centre_maps_back(ns):
    for p in range(12 * ns * ns):
        lon, lat = oracle.pix2ang(ns, p)
        assert oracle.ang2pix(ns, [lon], [lat])[0] == p


@pytest.mark.parametrize("ns", [4096, 8192, 16384])
def test_sampled_centres_map_back(ns):
    rng = np.random.default_rng(ns)
    pix = np.concatenate([rng.integers(0, 12 * ns * ns, 3000),
                          [0, 1, 12 * ns * ns - 1, 2 * ns * (ns - 1), 2 * ns * (ns + 1) - 1]])
    lonlat = np.array([oracle.pix2ang(ns, int(p)) for p in pix])
    assert np.array_equal(oracle.ang2pix(ns, lonlat[:, 0], lonlat[:, 1]), pix)


def _t_z(lon, lat):
    return (np.mod(lon, 360.0) / 90.0), np.sin(np.radians(lat))


@pytest.mark.parametrize("ns", [1, 4, 64, 8192])
def test_belt_points_lie_in_their_diamond(ns):
    rng = np.random.default_rng(7 + ns)
    n = 20000
    lon = rng.uniform(0, 360, n)
    lat = np.degrees(np.arcsin(rng.uniform(-0.66, 0.66, n)))
    pix = oracle.ang2pix(ns, lon, lat)
    t, z = _t_z(lon, lat)
    for k in range(n):
        clon, clat = oracle.pix2ang(ns, int(pix[k]))
        tc, zc = _t_z(clon, clat)
        dt = (t[k] - tc + 2.0) % 4.0 - 2.0
        assert abs(dt) * 2 * ns + abs(z[k] - zc) * 1.5 * ns <= 1.0 + 1e-9, (lon[k], lat[k])


@pytest.mark.parametrize("ns", [1, 2, 8, 512, 8192])
def test_points_lie_between_adjacent_ring_latitudes(ns):
    rng = np.random.default_rng(11 + ns)
    n = 20000
    lon = rng.uniform(-720, 720, n)
    lat = np.degrees(np.arcsin(rng.uniform(-1, 1, n)))
    pix = oracle.ang2pix(ns, lon, lat)
    z = np.sin(np.radians(lat))
    for k in range(0, n, 7):
        i = oracle.pix2ring(ns, int(pix[k]))
        z_above = 1.0 if i == 1 else oracle.ring_z(ns, i - 1)
        z_below = -1.0 if i == 4 * ns - 1 else oracle.ring_z(ns, i + 1)
        assert z_below - 1e-12 <= z[k] <= z_above + 1e-12


@pytest.mark.parametrize("ns", [2, 4, 8])
def test_equal_area(ns):
    # uniform points on the sphere fill every pixel equally (chi-square)
    rng = np.random.default_rng(1234 + ns)
    n = 1_500_000
    lon = rng.uniform(0, 360, n)
    lat = np.degrees(np.arcsin(rng.uniform(-1, 1, n)))
    counts = np.bincount(oracle.ang2pix(ns, lon, lat), minlength=12 * ns * ns)
    assert counts.shape[0] == 12 * ns * ns
    expected = n / (12 * ns * ns)
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    dof = 12 * ns * ns - 1
    # 6-sigma band of the chi-square distribution
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof), (chi2, dof)


def test_base_pixels_and_poles():
    # Ns = 1: north cap pixels 0..3 centred at lon 45, 135, ..; belt 4..7 at
    # lon 0, 90, ..; south cap 8..11 at 45, 135, ..
    assert list(oracle.ang2pix(1, [10, 100, 190, 280], [60, 60, 60, 60])) == [0, 1, 2, 3]
    assert list(oracle.ang2pix(1, [10, 80, 170, 260], [0, 0, 0, 0])) == [4, 5, 6, 7]
    assert list(oracle.ang2pix(1, [10, 100, 190, 280], [-60] * 4)) == [8, 9, 10, 11]
    for ns in (1, 4, 8192):
        north = oracle.ang2pix(ns, [0, 123], [90, 90])
        assert all(0 <= p <= 3 for p in north)
        south = oracle.ang2pix(ns, [0, 123], [-90, -90])
        assert all(12 * ns * ns - 4 <= p < 12 * ns * ns for p in south)
        # longitude is periodic
        a = oracle.ang2pix(ns, [12.5, 12.5 + 360, 12.5 - 720], [33.3] * 3)
        assert a[0] == a[1] == a[2]
