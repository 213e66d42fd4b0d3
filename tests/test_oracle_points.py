"""Pins for the oracle's neighbour sets and for Eq. (1) at arbitrary cell
centres with the kernel shapes of Section 3.6 (iii) and per-channel flags
(``oracle.neighbours``, ``oracle.grid_points``).

Each oracle function is checked against something other than itself: the
NumPy implementation with chord distances and tangent-plane bearings
(tests/ref_numpy.py), the pinned Gaussian gridder on a linear grid, closed
forms at special distances and bearings, and the brute-force equivalence of a
flag with the removal of that sample.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Kernel
from synth import GridDesc
from tests import ref_numpy

ARCMIN = 1.0 / 60.0
K_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))
FWHM = 3 * ARCMIN
SIG = FWHM / K_SIGMA


def _destination(lon0, lat0, bearing_deg, dist_deg):
    """The point at great-circle distance dist along the given bearing (east
    of north) from (lon0, lat0): a rotation of the pole-centred offset."""
    u = ref_numpy.unit(lon0, lat0)
    l0, b0 = math.radians(lon0), math.radians(lat0)
    east = np.array([-math.sin(l0), math.cos(l0), 0.0])
    north = np.array([-math.sin(b0) * math.cos(l0), -math.sin(b0) * math.sin(l0), math.cos(b0)])
    t, d = math.radians(bearing_deg), math.radians(dist_deg)
    v = math.cos(d) * u + math.sin(d) * (math.sin(t) * east + math.cos(t) * north)
    return math.degrees(math.atan2(v[1], v[0])) % 360.0, math.degrees(math.asin(v[2]))


def _field(seed, n, lon_c, lat_c, nx, ny, cell, edge_samples=True):
    rng = np.random.default_rng(seed)
    g = GridDesc(nx, ny, lon_c, lat_c, cell, cell)
    R = 3 * SIG
    cosl = max(math.cos(math.radians(min(89.9, abs(lat_c) + ny * cell))), 0.05)
    w = (nx + 10) * cell / cosl
    h = (ny + 10) * cell
    lon = (lon_c + rng.uniform(-w / 2, w / 2, n)) % 360.0
    lat = np.clip(lat_c + rng.uniform(-h / 2, h / 2, n), -90.0, 90.0)
    if edge_samples:
        # samples 1e-9 R inside and outside the support of some cells
        cl, cb = ref_numpy.cell_centres(g)
        extra = []
        for q in rng.choice(g.ncells, 12, replace=False):
            for f in (1 - 1e-9, 1 + 1e-9):
                extra.append(_destination(cl[q], cb[q], rng.uniform(0, 360), f * R))
        extra = np.array(extra)
        lon = np.concatenate([lon, extra[:, 0]])
        lat = np.concatenate([lat, extra[:, 1]])
    return lon, lat, g, R


@pytest.mark.parametrize("lon_c,lat_c", [(180.0, 30.0), (0.01, -15.0), (60.0, 89.9)])
def test_neighbours_equal_the_chord_distance_sets(lon_c, lat_c):
    lon, lat, g, R = _field(5, 1500, lon_c, lat_c, 9, 8, 0.7 * ARCMIN)
    cells = np.arange(g.ncells)
    nb = oracle.neighbours(lon, lat, g, R, cells)
    w, d = ref_numpy.weights(g, lon, lat, FWHM, R)
    for q in cells:
        expect = np.nonzero(d[q] <= math.radians(R))[0]
        assert np.array_equal(nb[q], expect), f"cell {q}"
        assert np.array_equal(nb[q], np.nonzero(w[q] > 0)[0])
    # the planted pairs sit 1e-9 R from the edge; both sides are represented
    dd = np.abs(d / math.radians(R) - 1.0)
    assert (dd < 2e-9).sum() >= 12


def test_points_on_a_linear_grid_equal_the_grid_oracle():
    lon, lat, g, R = _field(7, 900, 180.0, 30.0, 11, 9, 0.8 * ARCMIN, edge_samples=False)
    spec = np.random.default_rng(1).standard_normal((lon.shape[0], 3)).astype(np.float32)
    V, W, npairs = oracle.grid_allpairs(lon, lat, spec, g, FWHM, R)
    cl, cb = ref_numpy.cell_centres(g)
    Vp, Wp, npp = oracle.grid_points(lon, lat, spec, cl, cb, R, Kernel.gauss(FWHM),
                                     allpairs=True)
    assert npp.sum() == npairs
    assert np.array_equal(Wp, W.ravel())
    assert np.array_equal(Vp, V.reshape(3, -1).T, equal_nan=True)


KERNELS = [Kernel.gauss(FWHM),
           Kernel.elliptic(FWHM * 1.6, FWHM * 0.8, 35.0),
           Kernel.tapered_sinc(FWHM * 0.9, FWHM * 1.2)]


@pytest.mark.parametrize("kern", KERNELS, ids=["gauss", "elliptic", "sinc"])
@pytest.mark.parametrize("lon_c,lat_c", [(180.0, 30.0), (359.99, 5.0), (20.0, -89.8)])
def test_points_match_numpy_and_bucketed_equals_all_pairs(kern, lon_c, lat_c):
    rng = np.random.default_rng(11)
    R = 3 * SIG * (1.6 if kern.type == 1 else 1.0)
    n = 1200
    lon = (lon_c + rng.uniform(-0.2, 0.2, n) / max(0.05, math.cos(math.radians(lat_c)))) % 360
    lat = np.clip(lat_c + rng.uniform(-0.2, 0.2, n), -90, 90)
    cl = (lon_c + rng.uniform(-0.1, 0.1, 60) / max(0.05, math.cos(math.radians(lat_c)))) % 360
    cb = np.clip(lat_c + rng.uniform(-0.1, 0.1, 60), -90, 90)
    spec = rng.standard_normal((n, 2)).astype(np.float32)
    V, W, np1 = oracle.grid_points(lon, lat, spec, cl, cb, R, kern, allpairs=True)
    Vb, Wb, np2 = oracle.grid_points(lon, lat, spec, cl, cb, R, kern)
    assert np.array_equal(np1, np2) and np1.sum() > 0
    np.testing.assert_allclose(Wb, W, rtol=1e-13, atol=1e-15)
    assert np.array_equal(np.isnan(V), np.isnan(Vb))
    ok = ~np.isnan(V)
    np.testing.assert_allclose(Vb[ok], V[ok], rtol=1e-11, atol=1e-12)
    Vn, Wn = ref_numpy.grid_points(lon, lat, spec, cl, cb, kern, R)
    np.testing.assert_allclose(W, Wn, rtol=1e-11, atol=1e-13)
    assert np.array_equal(np.isnan(V), np.isnan(Vn))
    np.testing.assert_allclose(V[ok], Vn[ok], rtol=1e-9, atol=1e-10)


def test_elliptic_closed_forms():
    sa, sb = 1.7 * SIG, 0.9 * SIG
    k0 = Kernel.elliptic(sa * K_SIGMA, sb * K_SIGMA, 0.0)
    R = 4 * sa
    for lat0 in (0.0, 40.0, -70.0):
        for bearing, pa, sig in ((0.0, 0.0, sa), (180.0, 0.0, sa), (90.0, 0.0, sb),
                                 (0.0, 90.0, sb), (90.0, 90.0, sa), (270.0, 90.0, sa)):
            dist = 1.3 * sig
            slon, slat = _destination(100.0, lat0, bearing, dist)
            k = Kernel.elliptic(sa * K_SIGMA, sb * K_SIGMA, pa)
            _, W, _ = oracle.grid_points([slon], [slat], [[1.0]], [100.0], [lat0], R, k)
            assert W[0] == pytest.approx(math.exp(-1.3 ** 2 / 2), rel=1e-9), (lat0, bearing, pa)
    # a circular ellipse is the Gaussian
    rng = np.random.default_rng(3)
    lon = 50 + rng.uniform(-0.1, 0.1, 300)
    lat = -20 + rng.uniform(-0.1, 0.1, 300)
    spec = rng.standard_normal((300, 1)).astype(np.float32)
    cl, cb = 50 + rng.uniform(-0.05, 0.05, 30), -20 + rng.uniform(-0.05, 0.05, 30)
    Vc, Wc, _ = oracle.grid_points(lon, lat, spec, cl, cb, 3 * SIG,
                                   Kernel.elliptic(FWHM, FWHM, 77.0))
    Vg, Wg, _ = oracle.grid_points(lon, lat, spec, cl, cb, 3 * SIG, Kernel.gauss(FWHM))
    np.testing.assert_allclose(Wc, Wg, rtol=1e-13)
    np.testing.assert_allclose(Vc, Vg, rtol=1e-12, atol=1e-13)
    # the position angle is an axis: pa and pa + 180 give the same map
    V1, W1, _ = oracle.grid_points(lon, lat, spec, cl, cb, 4 * sa, Kernel.elliptic(
        sa * K_SIGMA, sb * K_SIGMA, 20.0))
    V2, W2, _ = oracle.grid_points(lon, lat, spec, cl, cb, 4 * sa, Kernel.elliptic(
        sa * K_SIGMA, sb * K_SIGMA, 200.0))
    np.testing.assert_allclose(W1, W2, rtol=1e-12)
    np.testing.assert_allclose(V1, V2, rtol=1e-11, atol=1e-12)
    # a sample exactly on the cell has weight 1 (bearing undefined)
    _, W0, _ = oracle.grid_points([100.0], [10.0], [[1.0]], [100.0], [10.0], R, k0)
    assert W0[0] == 1.0


def test_tapered_sinc_special_points_and_gaussian_limit():
    b, a = 2.0 * ARCMIN, 3.0 * ARCMIN
    k = Kernel.tapered_sinc(b, a)
    R = 1.5 * b
    lat0 = 25.0
    # d = b: first zero of the sinc; d = b / 2: sinc = 2 / pi
    for f, expect in ((1.0, 0.0), (0.5, 2.0 / math.pi * math.exp(-(0.5 * b / a) ** 2))):
        slon, slat = lat0 * 0 + 10.0, lat0 + f * b
        _, W, _ = oracle.grid_points([slon], [slat], [[1.0]], [10.0], [lat0], R, k)
        assert W[0] == pytest.approx(expect, abs=1e-12, rel=1e-12)  # d carries ~1e-13 rounding
    # b -> infinity: a Gaussian exp(-(d / a)^2), i.e. sigma = a / sqrt(2)
    rng = np.random.default_rng(9)
    lon = 10 + rng.uniform(-0.1, 0.1, 400)
    lat = lat0 + rng.uniform(-0.1, 0.1, 400)
    spec = rng.standard_normal((400, 2)).astype(np.float32)
    cl, cb = 10 + rng.uniform(-0.05, 0.05, 25), lat0 + rng.uniform(-0.05, 0.05, 25)
    Vs, Ws, _ = oracle.grid_points(lon, lat, spec, cl, cb, R, Kernel.tapered_sinc(1e6, a))
    Vg, Wg, _ = oracle.grid_points(lon, lat, spec, cl, cb, R,
                                   Kernel.gauss(a / math.sqrt(2.0) * K_SIGMA))
    np.testing.assert_allclose(Ws, Wg, rtol=1e-9)
    np.testing.assert_allclose(Vs, Vg, rtol=1e-8, atol=1e-9)


def test_flags_equal_sample_removal_per_channel():
    rng = np.random.default_rng(21)
    n = 700
    lon = 180 + rng.uniform(-0.12, 0.12, n)
    lat = 30 + rng.uniform(-0.1, 0.1, n)
    spec = rng.standard_normal((n, 4)).astype(np.float32)
    cl, cb = ref_numpy.cell_centres(GridDesc(8, 7, 180.0, 30.0, ARCMIN, ARCMIN))
    R = 3 * SIG
    kern = Kernel.gauss(FWHM)
    # without flags the masked form is the plain one, W the same in every channel
    V0, W0, _ = oracle.grid_points(lon, lat, spec, cl, cb, R, kern)
    Vm, Wm, _ = oracle.grid_points(lon, lat, spec, cl, cb, R, kern, masked=True)
    assert np.array_equal(Vm, V0, equal_nan=True)
    assert np.array_equal(Wm, np.repeat(W0[:, None], 4, 1))
    # flags (NaN, +-inf) in some rows of channels 1 and 2; channel 3 all flagged
    flagged = spec.copy()
    rows1 = rng.choice(n, 60, replace=False)
    rows2 = rng.choice(n, 200, replace=False)
    flagged[rows1, 1] = np.nan
    flagged[rows2[:100], 2] = np.inf
    flagged[rows2[100:], 2] = -np.inf
    flagged[:, 3] = np.nan
    Vf, Wf, _ = oracle.grid_points(lon, lat, flagged, cl, cb, R, kern, masked=True)
    for c, rows in ((0, []), (1, rows1), (2, rows2)):
        keep = np.setdiff1d(np.arange(n), rows)
        Vr, Wr, _ = oracle.grid_points(lon[keep], lat[keep], spec[keep, c:c + 1], cl, cb, R, kern)
        np.testing.assert_allclose(Wf[:, c], Wr, rtol=1e-13, atol=0)
        assert np.array_equal(np.isnan(Vf[:, c]), np.isnan(Vr[:, 0]))
        ok = ~np.isnan(Vr[:, 0])
        np.testing.assert_allclose(Vf[ok, c], Vr[ok, 0], rtol=1e-12, atol=1e-13)
    assert np.all(Wf[:, 3] == 0) and np.all(np.isnan(Vf[:, 3]))
    # a constant input stays constant wherever its channel has weight
    const = np.where(np.isfinite(flagged), 2.5, flagged).astype(np.float32)
    Vc, Wc, _ = oracle.grid_points(lon, lat, const, cl, cb, R, kern, masked=True)
    ok = Wc > 0
    np.testing.assert_allclose(Vc[ok], 2.5, rtol=1e-14)
    # the NumPy reference agrees
    Vn, Wn = ref_numpy.grid_points(lon, lat, flagged, cl, cb, kern, R, masked=True)
    np.testing.assert_allclose(Wf, Wn, rtol=1e-11, atol=1e-13)
    ok = ~np.isnan(Vf)
    assert np.array_equal(ok, ~np.isnan(Vn))
    np.testing.assert_allclose(Vf[ok], Vn[ok], rtol=1e-9, atol=1e-10)


def test_non_finite_cell_centres_have_no_samples():
    V, W, npair = oracle.grid_points([10.0, 10.01], [5.0, 5.0], [[1.0], [2.0]],
                                     [10.0, np.nan, 10.0], [5.0, 5.0, np.inf], 0.1,
                                     Kernel.gauss(FWHM))
    assert npair.tolist() == [2, 0, 0]
    assert W[0] > 0 and W[1] == 0 and W[2] == 0
    assert np.isnan(V[1, 0]) and np.isnan(V[2, 0]) and np.isfinite(V[0, 0])
