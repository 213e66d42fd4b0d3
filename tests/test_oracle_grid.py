"""Pins for the oracle gridder (Eq. (1), Section 2.1; Gaussian kernel of
Section 3.6 (iii)).

The oracle is checked against: closed-form weights for samples at known
great-circle distances, a third implementation with a different distance
formula (tests/ref_numpy.py), and the invariants that Eq. (1) implies
(constant in -> constant out, a delta reproduces the kernel, linearity, flux,
permutation, channel independence, empty cells, and the resolution of a
densely sampled source).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import GridDesc
from tests import ref_numpy

ARCMIN = 1.0 / 60.0
K_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))


def _one_cell(lon0=180.0, lat0=30.0):
    return GridDesc(1, 1, lon0, lat0, ARCMIN, ARCMIN)


def test_sample_on_cell_centre():
    g = _one_cell()
    V, W, npairs = oracle.grid_allpairs([180.0], [30.0], [[2.5, -1.0]], g, 3 * ARCMIN, 4 * ARCMIN)
    assert npairs == 1 and W[0, 0] == 1.0
    assert V[0, 0, 0] == 2.5 and V[1, 0, 0] == -1.0


@pytest.mark.parametrize("lat0", [0.0, 30.0, -61.0])
def test_closed_form_meridian_weights(lat0):
    # two samples on the cell's meridian at k sigma and m sigma: d is exactly
    # the latitude offset, so w = exp(-k^2/2) and V is their weighted mean
    fwhm = 3 * ARCMIN
    sig = fwhm / K_SIGMA
    k, m = 1.3, 2.2
    g = _one_cell(180.0, lat0)
    V, W, _ = oracle.grid_allpairs([180.0, 180.0], [lat0 + k * sig, lat0 - m * sig], [7.0, -3.0],
                                   g, fwhm, 3 * sig)
    wk, wm = math.exp(-k * k / 2), math.exp(-m * m / 2)
    assert W[0, 0] == pytest.approx(wk + wm, rel=1e-12)
    assert V[0, 0, 0] == pytest.approx((7.0 * wk - 3.0 * wm) / (wk + wm), rel=1e-12)
    assert oracle.sigma_rad(fwhm) == pytest.approx(math.radians(sig), rel=1e-15)


def test_closed_form_equator_and_parallel():
    fwhm = 4 * ARCMIN
    sig = fwhm / K_SIGMA
    # at the equator an RA offset of k sigma is a great-circle distance of k sigma
    V, W, _ = oracle.grid_allpairs([10.0 + 1.7 * sig], [0.0], [1.0], _one_cell(10.0, 0.0), fwhm,
                                   3 * sig)
    assert W[0, 0] == pytest.approx(math.exp(-1.7 ** 2 / 2), rel=1e-12)
    # at Dec 60 an RA offset dA subtends 2 asin(cos(60) sin(dA/2))
    dA = math.radians(2.0 * sig)
    d = 2 * math.asin(math.cos(math.radians(60.0)) * math.sin(dA / 2))
    V, W, _ = oracle.grid_allpairs([10.0 + 2.0 * sig], [60.0], [1.0], _one_cell(10.0, 60.0), fwhm,
                                   3 * sig)
    assert W[0, 0] == pytest.approx(math.exp(-(d / math.radians(sig)) ** 2 / 2), rel=1e-12)


def test_support_is_closed_and_sharp():
    fwhm = 3 * ARCMIN
    R = 3 * fwhm / K_SIGMA
    g = _one_cell(45.0, 10.0)
    inside = oracle.grid_allpairs([45.0], [10.0 + R * (1 - 1e-9)], [1.0], g, fwhm, R)
    outside = oracle.grid_allpairs([45.0], [10.0 + R * (1 + 1e-9)], [1.0], g, fwhm, R)
    assert inside[2] == 1 and inside[1][0, 0] == pytest.approx(math.exp(-4.5), rel=1e-7)
    assert outside[2] == 0 and outside[1][0, 0] == 0.0 and np.isnan(outside[0][0, 0, 0])


def _random_case(seed, n=600, nchan=3, lon_c=180.0, lat_c=30.0, nx=9, ny=7):
    rng = np.random.default_rng(seed)
    cell = 0.8 * ARCMIN
    w = (nx + 8) * cell
    h = (ny + 8) * cell
    lon = lon_c + rng.uniform(-w / 2, w / 2, n)
    lat = lat_c + rng.uniform(-h / 2, h / 2, n)
    spec = rng.standard_normal((n, nchan)).astype(np.float32)
    g = GridDesc(nx, ny, lon_c, lat_c, cell, cell)
    return lon, lat, spec, g, 3 * ARCMIN, 3 * 3 * ARCMIN / K_SIGMA


@pytest.mark.parametrize("lon_c,lat_c", [(180.0, 30.0), (0.0, -20.0), (359.95, 45.0),
                                         (90.0, 89.5)])
def test_matches_independent_numpy_implementation(lon_c, lat_c):
    lon, lat, spec, g, fwhm, R = _random_case(17, lon_c=lon_c, lat_c=lat_c)
    V, W, _ = oracle.grid_allpairs(lon, lat, spec, g, fwhm, R)
    Vn, Wn = ref_numpy.grid(lon, lat, spec, g, fwhm, R)
    _, d = ref_numpy.weights(g, lon, lat, fwhm, R)
    assert np.min(np.abs(d - math.radians(R))) > 1e-12  # no pair sits on the support edge
    assert np.array_equal(np.isnan(V), np.isnan(Vn))
    ok = ~np.isnan(V)
    np.testing.assert_allclose(W, Wn, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(V[ok], Vn[ok], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("lon_c,lat_c", [(180.0, 30.0), (0.02, 10.0), (200.0, 88.0),
                                         (10.0, -89.7)])
def test_bucketed_equals_all_pairs(lon_c, lat_c):
    lon, lat, spec, g, fwhm, R = _random_case(23, n=3000, lon_c=lon_c, lat_c=lat_c, nx=13, ny=11)
    V, W, npairs = oracle.grid_allpairs(lon, lat, spec, g, fwhm, R)
    cells = np.arange(g.ncells)
    Vb, Wb, npb = oracle.grid_cells(lon, lat, spec, g, fwhm, R, cells)
    assert npb.sum() == npairs
    np.testing.assert_allclose(Wb, W.ravel(), rtol=1e-14, atol=0)
    Va = V.reshape(spec.shape[1], -1).T
    assert np.array_equal(np.isnan(Va), np.isnan(Vb))
    ok = ~np.isnan(Va)
    np.testing.assert_allclose(Vb[ok], Va[ok], rtol=1e-13, atol=1e-15)


def test_invariants_constant_delta_linearity_flux():
    lon, lat, spec, g, fwhm, R = _random_case(31, n=800, nchan=2)
    n = lon.shape[0]
    # I1: a constant input gives the same constant wherever W > 0
    V, W, _ = oracle.grid_allpairs(lon, lat, np.full((n, 1), 3.25, np.float32), g, fwhm, R)
    ok = W > 0
    assert ok.sum() > 0.9 * g.ncells
    np.testing.assert_allclose(V[0][ok], 3.25, rtol=1e-14)
    # I2: a delta at sample m gives U_g = V_g W_g = w(d(g, m))
    m = 123
    delta = np.zeros((n, 1), np.float32)
    delta[m] = 1.0
    V, W, _ = oracle.grid_allpairs(lon, lat, delta, g, fwhm, R)
    wmat, _ = ref_numpy.weights(g, lon, lat, fwhm, R)
    U = np.nan_to_num(V[0]) * W
    np.testing.assert_allclose(U.ravel(), wmat[:, m], rtol=1e-12, atol=1e-300)
    # I3: linearity
    a, b = 2.0, -0.5
    s1, s2 = spec[:, :1], spec[:, 1:2]
    V1, _, _ = oracle.grid_allpairs(lon, lat, s1, g, fwhm, R)
    V2, _, _ = oracle.grid_allpairs(lon, lat, s2, g, fwhm, R)
    V12, _, _ = oracle.grid_allpairs(lon, lat, (a * s1 + b * s2).astype(np.float32), g, fwhm, R)
    ok = ~np.isnan(V1)
    np.testing.assert_allclose(V12[ok], (a * V1 + b * V2)[ok], rtol=1e-5, atol=1e-6)
    # I4: flux -- sum_g V_g W_g = sum_n s_n kappa_n with kappa_n = sum_g w_gn
    V, W, _ = oracle.grid_allpairs(lon, lat, s1, g, fwhm, R)
    lhs = float((np.nan_to_num(V[0]) * W).sum())
    rhs = float((wmat.sum(0) * s1[:, 0].astype(np.float64)).sum())
    assert lhs == pytest.approx(rhs, rel=1e-11)


def test_flux_kernel_integral_on_dense_grid():
    # I4 continuum limit: a sample far from the grid edges is counted with
    # kappa = 2 pi sigma^2 (1 - exp(-R^2/2 sigma^2)) / cell_area
    fwhm = 3 * ARCMIN
    sig = fwhm / K_SIGMA
    R = 3 * sig
    cell = sig / 4
    g = GridDesc(121, 121, 0.0, 0.0, cell, cell)
    V, W, _ = oracle.grid_allpairs([0.013 * ARCMIN], [-0.021 * ARCMIN], [1.0], g, fwhm, R)
    kappa = float(W.sum())
    expect = 2 * math.pi * sig * sig * (1 - math.exp(-R * R / (2 * sig * sig))) / (cell * cell)
    assert kappa == pytest.approx(expect, rel=2e-3)


def test_permutation_channels_and_empty_cells():
    lon, lat, spec, g, fwhm, R = _random_case(41, n=500, nchan=4)
    V, W, _ = oracle.grid_allpairs(lon, lat, spec, g, fwhm, R)
    # I5: input order does not matter
    p = np.random.default_rng(0).permutation(lon.shape[0])
    Vp, Wp, _ = oracle.grid_allpairs(lon[p], lat[p], spec[p], g, fwhm, R)
    ok = ~np.isnan(V)
    np.testing.assert_allclose(Vp[ok], V[ok], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Wp, W, rtol=1e-14)
    # I6: channel c of a multi-channel run equals a one-channel run
    V2, _, _ = oracle.grid_allpairs(lon, lat, spec[:, 2:3], g, fwhm, R)
    assert np.array_equal(V2[0], V[2], equal_nan=True)
    # I7: W = 0 exactly where no sample is within R, and V is NaN there
    far = GridDesc(5, 5, 100.0, -40.0, ARCMIN, ARCMIN)
    Vf, Wf, npf = oracle.grid_allpairs(lon, lat, spec, far, fwhm, R)
    assert npf == 0 and np.all(Wf == 0) and np.all(np.isnan(Vf))
    nb = oracle.neighbours(lon, lat, g, R, np.arange(g.ncells))
    empty = np.array([len(x) == 0 for x in nb]).reshape(g.ny, g.nx)
    assert np.array_equal(empty, W == 0)
    assert np.array_equal(np.isnan(V[0]), empty)


def test_resolution_of_dense_gaussian_source():
    # I8: a source of FWHM F_s sampled densely and gridded with a kernel of
    # FWHM F_k (support 3 sigma) has a map variance per axis of
    # sigma_s^2 + c sigma_k^2, c the second moment of the truncated kernel
    fk = 3 * ARCMIN
    fs = 3 * ARCMIN
    sk, ss = fk / K_SIGMA, fs / K_SIGMA
    step = sk / 6
    xs = np.arange(-60, 61) * step
    LON, LAT = np.meshgrid(xs, xs)
    lon, lat = LON.ravel(), LAT.ravel()
    vals = np.exp(-(lon ** 2 + lat ** 2) / (2 * ss * ss)).astype(np.float32)
    cell = sk / 3
    g = GridDesc(61, 61, 0.0, 0.0, cell, cell)
    V, W, _ = oracle.grid_allpairs(lon, lat, vals, g, fk, 3 * sk)
    m = V[0]
    cx = (np.arange(61) - 30) * cell
    X, Y = np.meshgrid(cx, cx)
    var_x = float((m * X * X).sum() / m.sum())
    u = 4.5
    c = 1 - u * math.exp(-u) / (1 - math.exp(-u))
    expect = ss * ss + c * sk * sk
    assert var_x == pytest.approx(expect, rel=0.02)
    # map FWHM is close to sqrt(F_s^2 + F_k^2), ~1.3 % below it after truncation
    fwhm_map = math.sqrt(var_x) * K_SIGMA
    assert fwhm_map == pytest.approx(math.hypot(fs, fk), rel=0.03)


def test_point_source_field_config():
    w = synth.point_source_field()
    lon, lat, spec = w.lon.numpy(), w.lat.numpy(), w.spectra.numpy()
    V, W, npairs = oracle.grid_allpairs(lon, lat, spec, w.grid, w.fwhm_deg, w.support_deg)
    assert w.n == 10_000 and w.grid.nx == 60 and w.nside == 4096
    assert 4.0e5 < npairs < 6.0e5
    assert np.all(W > 0)
    # every injected source shows up as a local excess in the map
    for (sl, sb, amp, _) in w.sources:
        ix = int(round((sl - w.grid.lon0) / w.grid.dlon + (w.grid.nx - 1) / 2))
        iy = int(round((sb - w.grid.lat0) / w.grid.dlat + (w.grid.ny - 1) / 2))
        assert V[0, iy, ix] > 3.0
