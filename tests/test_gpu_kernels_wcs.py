"""GPU parity of the kernel shapes (Section 3.6 (iii)), of projected target
maps given by their cell centres (WCS-space gridding, Section 2.1) and of the
flagged form, through the C ABI, against the FP64 oracle's ``grid_points``.

* ``hcg_wcs_centres`` against the WCS oracle (CAR, SFL, SIN, TAN): 1e-9 deg.
* ``hcg_plan_ex`` on cell centres: every projection, few and many channels,
  1e-5 per channel (and per cell, through the shared check) and W to 1e-6.
* elliptical Gaussian and Gaussian-tapered sinc kernels in the FP32 form
  (both accumulation kernels) and the low-precision forms at their budgets.
* ``hcg_grid_masked``: non-finite values leave their sample out of that
  channel; V to 1e-5, each channel's W to 1e-6 (FP64 sums, C <= 8) or 1e-5
  (FP32 matrix-core sums).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2012_13173_amd as hcg
import synth
from oracle import wcs as owcs
from synth import GridDesc
from tests.gridcheck import assert_cube_close

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
ARCMIN = 1.0 / 60.0
K_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))
TOL_F32 = 1e-5

LOWP = {
    "f16_scaled": (hcg.HCG_F16_SCALED, 1e-3),
    "bf16_split": (hcg.HCG_BF16_SPLIT, 5e-5),
    "fp8e4m3_split": (hcg.HCG_FP8E4M3_SPLIT, 1e-2),
}

MAPS = [  # proj, nx, ny, crpix, cdelt (deg), crval
    ("CAR", 41, 33, (20.0, 17.0), (-0.6 * ARCMIN, 0.6 * ARCMIN), (180.0, 30.0)),
    ("SFL", 37, 29, (19.0, 15.5), (-0.6 * ARCMIN, 0.6 * ARCMIN), (359.9, -35.0)),
    ("SIN", 40, 40, (20.5, 20.5), (-0.6 * ARCMIN, 0.6 * ARCMIN), (120.0, 62.0)),
    ("TAN", 36, 44, (18.0, 22.0), (-0.6 * ARCMIN, 0.6 * ARCMIN), (10.0, 80.0)),
    ("TAN", 30, 30, (15.5, 15.5), (-0.6 * ARCMIN, 0.6 * ARCMIN), (300.0, -89.5)),
]


def _wcs_args(m):
    proj, nx, ny, crpix, cdelt, crval = m
    return proj, nx, ny, crpix, cdelt, crval


def _angdist_deg(l1, b1, l2, b2):
    l1, b1, l2, b2 = (np.radians(np.asarray(x, dtype=np.float64)) for x in (l1, b1, l2, b2))
    h = np.sin((b2 - b1) / 2) ** 2 + np.cos(b1) * np.cos(b2) * np.sin((l2 - l1) / 2) ** 2
    return np.degrees(2 * np.arcsin(np.sqrt(np.clip(h, 0, 1))))


@pytest.mark.parametrize("m", MAPS + [("SIN", 50, 50, (25.5, 25.5), (-3.0, 3.0), (40.0, 10.0))],
                         ids=lambda m: f"{m[0]}_{m[5][1]}")
def test_wcs_centres_match_the_wcs_oracle(m):
    proj, nx, ny, crpix, cdelt, crval = _wcs_args(m)
    lon, lat = hcg.hcg_wcs_centres(proj, nx, ny, crpix, cdelt, crval)
    torch.cuda.synchronize()
    lon, lat = lon.cpu().numpy(), lat.cpu().numpy()
    with np.errstate(invalid="ignore"):
        try:
            olon, olat = owcs.cell_centres(proj, nx, ny, crpix, cdelt, crval)
        except ValueError:  # SIN: pixels outside the disc
            olon = np.full((ny, nx), np.nan)
            olat = np.full((ny, nx), np.nan)
            iy, ix = np.mgrid[0:ny, 0:nx]
            x = cdelt[0] * (ix + 1 - crpix[0])
            y = cdelt[1] * (iy + 1 - crpix[1])
            inside = np.hypot(x, y) * math.pi / 180 <= 1.0
            a, b = owcs.pix2world(proj, ix[inside] + 1.0, iy[inside] + 1.0, crpix, cdelt, crval)
            olon[inside], olat[inside] = a, b
    assert np.array_equal(np.isnan(lon), np.isnan(olon))
    ok = ~np.isnan(olon)
    assert ok.sum() > 0
    assert np.all((lon[ok] >= 0) & (lon[ok] < 360))
    d = _angdist_deg(lon[ok], lat[ok], olon[ok], olat[ok])
    assert d.max() < 1e-9, d.max()


def _field_for(lon_c, lat_c, cl, cb, R, n, nchan, seed):
    """Coordinate-uniform samples over the cells' lon/lat box plus 2R."""
    ok = np.isfinite(cl)
    lonr = np.unwrap(np.radians(cl[ok]))
    lo, hi = np.degrees(lonr.min()), np.degrees(lonr.max())
    bmin, bmax = cb[ok].min(), cb[ok].max()
    pad = 2 * R
    coslat = max(math.cos(math.radians(min(89.9, max(abs(bmin), abs(bmax)) + pad))), 0.02)
    w = min(360.0, (hi - lo) + 2 * pad / coslat)
    h = (bmax - bmin) + 2 * pad
    lon, lat = synth.uniform_positions(n, (lo + hi) / 2, (bmin + bmax) / 2, w, h, seed)
    lat = lat.clamp(-90.0, 90.0)
    g = torch.Generator().manual_seed(seed + 1)
    spec = torch.randn((n, nchan), generator=g, dtype=torch.float32)
    return lon.double(), lat.double(), spec


def _oracle_points(lon, lat, spec, cl, cb, R, okern, masked=False):
    V, W, _ = oracle.grid_points(lon.numpy(), lat.numpy(), spec.numpy(), cl.ravel(), cb.ravel(), R,
                                 okern, masked=masked)
    ny, nx = cl.shape
    C = spec.shape[1]
    Vr = V.T.reshape(C, ny, nx)
    Wr = W.T.reshape(C, ny, nx) if masked else W.reshape(ny, nx)
    return Vr, Wr


def _grid(plan, spec, form=hcg.HCG_F32, weights=True):
    g = plan.grid
    C = int(spec.shape[1])
    cube = torch.empty((C, g.ny, g.nx), dtype=torch.float32, device=DEV)
    W = torch.empty((g.ny, g.nx), dtype=torch.float32, device=DEV) if weights else None
    s = spec.to(DEV).contiguous()
    if form == hcg.HCG_F32:
        hcg.hcg_grid(plan, s, cube, W)
    else:
        enc, scale = hcg.hcg_quantize(s, form)
        hcg.hcg_grid(plan, enc, cube, W, dtype=form, chan_scale=scale)
    torch.cuda.synchronize()
    return cube.cpu().numpy(), (W.cpu().numpy() if weights else None)


def _assert_w(W, Wr, rtol=1e-6):
    W = np.asarray(W, dtype=np.float64)
    Wr = np.asarray(Wr, dtype=np.float64)
    assert np.array_equal(W == 0, Wr == 0)
    scale = np.abs(Wr).max()
    np.testing.assert_allclose(W, Wr, rtol=rtol, atol=rtol * scale)


@pytest.mark.parametrize("m", MAPS, ids=lambda m: f"{m[0]}_{m[5][1]}")
@pytest.mark.parametrize("nchan", [1, 40])
def test_projected_maps_against_oracle(m, nchan):
    proj, nx, ny, crpix, cdelt, crval = _wcs_args(m)
    fwhm = 3 * ARCMIN
    R = 3 * fwhm / K_SIGMA
    cl_d, cb_d = hcg.hcg_wcs_centres(proj, nx, ny, crpix, cdelt, crval)
    cl, cb = owcs.cell_centres(proj, nx, ny, crpix, cdelt, crval)  # the oracle's own centres
    lon, lat, spec = _field_for(crval[0], crval[1], cl, cb, R, 25_000, nchan, 600 + nx)
    plan = hcg.hcg_plan_ex(lon.to(DEV), lat.to(DEV), hcg.Kernel.gauss(fwhm), R,
                           cell_lon=cl_d, cell_lat=cb_d)
    V, W = _grid(plan, spec)
    Vr, Wr = _oracle_points(lon, lat, spec, cl, cb, R, oracle.Kernel.gauss(fwhm))
    assert_cube_close(V, Vr, TOL_F32, f"{proj} C={nchan}")
    _assert_w(W, Wr)
    plan.destroy()


def test_centres_of_a_linear_grid_give_the_linear_plan_map():
    w = synth.small_cube(n=20_000, nchan=30, nx=37, ny=29, seed=620)
    g = w.grid
    ix = np.arange(g.nx)
    iy = np.arange(g.ny)
    cl = np.broadcast_to(g.lon0 + (ix - (g.nx - 1) / 2) * g.dlon, (g.ny, g.nx)).copy()
    cb = np.broadcast_to((g.lat0 + (iy - (g.ny - 1) / 2) * g.dlat)[:, None], (g.ny, g.nx)).copy()
    lin = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), g, w.fwhm_deg, w.support_deg)
    cen = hcg.hcg_plan_ex(w.lon.to(DEV), w.lat.to(DEV), hcg.Kernel.gauss(w.fwhm_deg),
                          w.support_deg, cell_lon=torch.from_numpy(cl).to(DEV),
                          cell_lat=torch.from_numpy(cb).to(DEV))
    V1, W1 = _grid(lin, w.spectra)
    V2, W2 = _grid(cen, w.spectra)
    np.testing.assert_allclose(W2, W1, rtol=1e-6)
    np.testing.assert_allclose(V2, V1, rtol=1e-5, atol=1e-5)
    lin.destroy()
    cen.destroy()


KERNELS = {
    "elliptic": (hcg.Kernel.elliptic(4.5 * ARCMIN, 2.5 * ARCMIN, 35.0),
                 oracle.Kernel.elliptic(4.5 * ARCMIN, 2.5 * ARCMIN, 35.0), 3 * 4.5 / K_SIGMA),
    "sinc": (hcg.Kernel.tapered_sinc(2.5 * ARCMIN, 3.5 * ARCMIN),
             oracle.Kernel.tapered_sinc(2.5 * ARCMIN, 3.5 * ARCMIN), 2.5 * 1.5),
}


@pytest.mark.parametrize("kname", list(KERNELS))
@pytest.mark.parametrize("nchan", [1, 5, 67, 300])
def test_kernel_shapes_on_a_linear_grid(kname, nchan):
    hk, ok_, R_arcmin = KERNELS[kname]
    R = R_arcmin * ARCMIN
    w = synth.small_cube(n=20_000, nchan=nchan, nx=29, ny=23, seed=640 + nchan)
    plan = hcg.hcg_plan_ex(w.lon.to(DEV), w.lat.to(DEV), hk, R, grid=w.grid)
    g = w.grid
    ix = np.arange(g.nx)
    iy = np.arange(g.ny)
    cl = np.broadcast_to(g.lon0 + (ix - (g.nx - 1) / 2) * g.dlon, (g.ny, g.nx))
    cb = np.broadcast_to((g.lat0 + (iy - (g.ny - 1) / 2) * g.dlat)[:, None], (g.ny, g.nx))
    Vr, Wr = _oracle_points(w.lon, w.lat, w.spectra, cl, cb, R, ok_)
    V, W = _grid(plan, w.spectra)
    e = assert_cube_close(V, Vr, TOL_F32, f"{kname} f32 C={nchan}")
    print(f"{kname} f32 C={nchan}: {e.max():.2e}", flush=True)
    _assert_w(W, Wr)
    if nchan > 8:
        for name, (form, tol) in LOWP.items():
            V, W = _grid(plan, w.spectra, form)
            e = assert_cube_close(V, Vr, tol, f"{kname} {name} C={nchan}")
            print(f"{kname} {name} C={nchan}: {e.max():.2e}", flush=True)
            _assert_w(W, Wr)
    plan.destroy()


def test_elliptic_kernel_on_a_projected_map():
    proj, nx, ny, crpix, cdelt, crval = MAPS[2]
    hk, ok_, R_arcmin = KERNELS["elliptic"]
    R = R_arcmin * ARCMIN
    cl_d, cb_d = hcg.hcg_wcs_centres(proj, nx, ny, crpix, cdelt, crval)
    cl, cb = owcs.cell_centres(proj, nx, ny, crpix, cdelt, crval)
    lon, lat, spec = _field_for(crval[0], crval[1], cl, cb, R, 25_000, 20, 660)
    plan = hcg.hcg_plan_ex(lon.to(DEV), lat.to(DEV), hk, R, cell_lon=cl_d, cell_lat=cb_d)
    V, W = _grid(plan, spec)
    Vr, Wr = _oracle_points(lon, lat, spec, cl, cb, R, ok_)
    assert_cube_close(V, Vr, TOL_F32, "SIN elliptic")
    _assert_w(W, Wr)
    plan.destroy()


def _flag(spec, frac, seed):
    g = np.random.default_rng(seed)
    s = spec.numpy().copy()
    m = g.random(s.shape) < frac
    vals = g.choice([np.nan, np.inf, -np.inf], size=int(m.sum()))
    s[m] = vals
    if s.shape[1] > 2:
        s[:, 2] = np.nan  # one channel flagged everywhere
    return torch.from_numpy(s)


@pytest.mark.parametrize("nchan", [1, 3, 8, 20, 67, 300])
@pytest.mark.parametrize("many_tiles", [False, True])
def test_masked_form_against_oracle(nchan, many_tiles):
    if many_tiles and nchan > 8:
        pytest.skip("the tile count only selects the few-channel kernel's variant")
    nx, ny = (264, 256) if many_tiles else (29, 23)
    n = 160_000 if many_tiles else 15_000
    w = synth.small_cube(n=n, nchan=nchan, nx=nx, ny=ny, seed=700 + nchan, cell_arcmin=0.6)
    spec = _flag(w.spectra, 0.05, 701 + nchan)
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg)
    C = nchan
    cube = torch.empty((C, ny, nx), dtype=torch.float32, device=DEV)
    Wc = torch.empty((C, ny, nx), dtype=torch.float32, device=DEV)
    hcg.hcg_grid_masked(plan, spec.to(DEV), cube, Wc)
    torch.cuda.synchronize()
    g = w.grid
    if many_tiles:
        rng = np.random.default_rng(5)
        cells = rng.choice(nx * ny, 1500, replace=False)
    else:
        cells = np.arange(nx * ny)
    iy, ix = np.divmod(cells, nx)
    cl = g.lon0 + (ix - (nx - 1) / 2) * g.dlon
    cb = g.lat0 + (iy - (ny - 1) / 2) * g.dlat
    V, W, _ = oracle.grid_points(w.lon.numpy(), w.lat.numpy(), spec.numpy(), cl, cb,
                                 w.support_deg, oracle.Kernel.gauss(w.fwhm_deg), masked=True)
    Vg = cube.reshape(C, -1)[:, torch.from_numpy(cells).to(DEV)].cpu().numpy()
    Wg = Wc.reshape(C, -1)[:, torch.from_numpy(cells).to(DEV)].cpu().numpy()
    assert_cube_close(Vg, V.T, TOL_F32, f"masked C={C}")
    if C > 2:
        assert np.all(np.isnan(Vg[2])) and np.all(Wg[2] == 0)
    _assert_w(Wg, W.T, rtol=1e-6 if C <= 8 else 1e-5)
    # without flags the masked form is the plain one, W the same in every channel
    cube2 = torch.empty_like(cube)
    Wc2 = torch.empty_like(Wc)
    hcg.hcg_grid_masked(plan, w.spectra.to(DEV), cube2, Wc2)
    cube3 = torch.empty_like(cube)
    W3 = torch.empty((ny, nx), dtype=torch.float32, device=DEV)
    hcg.hcg_grid(plan, w.spectra.to(DEV), cube3, W3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(cube2.cpu().numpy(), cube3.cpu().numpy(), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(Wc2.cpu().numpy(), np.broadcast_to(W3.cpu().numpy(), (C, ny, nx)),
                               rtol=1e-5)
    plan.destroy()


def test_masked_form_with_a_kernel_shape():
    hk, ok_, R_arcmin = KERNELS["sinc"]
    R = R_arcmin * ARCMIN
    w = synth.small_cube(n=15_000, nchan=40, nx=25, ny=21, seed=720)
    spec = _flag(w.spectra, 0.1, 721)
    plan = hcg.hcg_plan_ex(w.lon.to(DEV), w.lat.to(DEV), hk, R, grid=w.grid)
    cube = torch.empty((40, 21, 25), dtype=torch.float32, device=DEV)
    Wc = torch.empty_like(cube)
    hcg.hcg_grid_masked(plan, spec.to(DEV), cube, Wc)
    torch.cuda.synchronize()
    g = w.grid
    ix = np.arange(g.nx)
    iy = np.arange(g.ny)
    cl = np.broadcast_to(g.lon0 + (ix - (g.nx - 1) / 2) * g.dlon, (g.ny, g.nx))
    cb = np.broadcast_to((g.lat0 + (iy - (g.ny - 1) / 2) * g.dlat)[:, None], (g.ny, g.nx))
    Vr, Wr = _oracle_points(w.lon, w.lat, spec, cl, cb, R, ok_, masked=True)
    assert_cube_close(cube.cpu().numpy(), Vr, TOL_F32, "masked sinc")
    _assert_w(Wc.cpu().numpy(), Wr, rtol=1e-5)
    plan.destroy()


def test_plan_ex_and_wcs_errors():
    import ctypes
    w = synth.small_cube(n=2000, nchan=4, nx=8, ny=8, seed=730)
    lib = hcg.load()
    lon, lat = w.lon.to(DEV), w.lat.to(DEV)
    vp = ctypes.c_void_p
    h = vp()
    g = hcg.grid_desc(w.grid)
    k = hcg.Kernel.gauss(w.fwhm_deg).c
    cl = torch.zeros((8, 8), dtype=torch.float64, device=DEV)
    cc = hcg.CellCentresC(8, 8, vp(cl.data_ptr()), vp(cl.data_ptr()))
    args = (vp(lon.data_ptr()), vp(lat.data_ptr()), w.n)
    # both and neither of grid and centres
    assert lib.hcg_plan_ex(ctypes.byref(h), *args, ctypes.byref(g), ctypes.byref(cc),
                           ctypes.byref(k), w.support_deg, None, None) == hcg.HCG_E_ARG
    assert lib.hcg_plan_ex(ctypes.byref(h), *args, None, None, ctypes.byref(k), w.support_deg,
                           None, None) == hcg.HCG_E_ARG
    for bad in (hcg.Kernel.gauss(0.0), hcg.Kernel.elliptic(0.05, -1.0, 0.0),
                hcg.Kernel.tapered_sinc(0.05, 0.0)):
        assert lib.hcg_plan_ex(ctypes.byref(h), *args, ctypes.byref(g), None, ctypes.byref(bad.c),
                               w.support_deg, None, None) == hcg.HCG_E_ARG
    assert lib.hcg_plan_ex(ctypes.byref(h), *args, ctypes.byref(g), None,
                           ctypes.byref(hcg.Kernel(7, fwhm=0.05).c), w.support_deg, None,
                           None) == hcg.HCG_E_UNSUPPORTED
    assert h.value is None
    # the paper-scheme gather serves only linear Gaussian plans
    plan = hcg.hcg_plan_ex(lon, lat, hcg.Kernel.tapered_sinc(0.05, 0.06), 0.07, grid=w.grid)
    out = torch.empty((8, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(hcg.HcgError) as ei:
        hcg.hcg_grid_rowthreads(plan, w.spectra[:, 0].contiguous().to(DEV), out)
    assert ei.value.status == hcg.HCG_E_UNSUPPORTED
    plan.destroy()
    with pytest.raises(hcg.HcgError) as ei:
        hcg.hcg_wcs_centres(9, 4, 4, (1, 1), (0.1, 0.1), (0, 0))
    assert ei.value.status == hcg.HCG_E_UNSUPPORTED
    with pytest.raises(hcg.HcgError) as ei:
        hcg.hcg_wcs_centres("TAN", 4, 4, (1, 1), (0.0, 0.1), (0, 0))
    assert ei.value.status == hcg.HCG_E_ARG
