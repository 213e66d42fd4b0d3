"""GPU parity of hcg_grid_rowthreads, the paper's own gather scheme (one
thread per gamma cells of a row, per-thread candidate search; Sections 3.4
and 3.5), against the FP64 oracle and against hcg_grid on one channel.

Both kernels sum in FP64 and differ only in the order of the sums, so the
maps must agree to 1e-6 relative per cell (W too) and with the oracle to the
FP32 bound of 1e-5; NaN patterns identical.  Cases: every gamma with ragged
row ends, block sizes 64 .. 512, longitude wrap, polar cap, south, a wide
support, empty cells, and the 5 deg x 5 deg, 90 x 90 field of the paper's
experiments at 10^7 samples with sampled cells."""
import numpy as np
import pytest
import torch

import paper_2012_13173_amd as hcg
import synth
from tests.gridcheck import (assert_cube_close, assert_weights_close, gather_cells, run_oracle,
                             sample_cells, sampled_oracle)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL_F32 = 1e-5


def _both(w, gamma, block):
    """(rowthreads V, W), (hcg_grid V, W) for channel 0 of w, as numpy."""
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)
    g = w.grid
    spec = w.spectra[:, 0].contiguous().to(DEV)
    V = torch.full((g.ny, g.nx), -7.0, dtype=torch.float32, device=DEV)
    W = torch.full((g.ny, g.nx), -7.0, dtype=torch.float32, device=DEV)
    hcg.hcg_grid_rowthreads(plan, spec, V, W, gamma=gamma, block=block)
    Vt = torch.empty((1, g.ny, g.nx), dtype=torch.float32, device=DEV)
    Wt = torch.empty((g.ny, g.nx), dtype=torch.float32, device=DEV)
    hcg.hcg_grid(plan, spec[:, None].contiguous(), Vt, Wt)
    torch.cuda.synchronize()
    plan.destroy()
    return (V.cpu().numpy(), W.cpu().numpy()), (Vt[0].cpu().numpy(), Wt.cpu().numpy())


def _one_channel(w):
    return synth.Workload(w.name, w.lon, w.lat, w.spectra[:, :1].contiguous(), w.grid,
                          w.fwhm_deg, w.support_deg, w.nside, w.sources)


def _check(w, gamma, block, what):
    (V, W), (Vt, Wt) = _both(w, gamma, block)
    assert np.array_equal(np.isnan(V), np.isnan(Vt)), f"{what}: NaN pattern differs from hcg_grid"
    ok = ~np.isnan(Vt)
    np.testing.assert_allclose(V[ok], Vt[ok], rtol=1e-6, atol=1e-6 * np.abs(Vt[ok]).max())
    np.testing.assert_allclose(W, Wt, rtol=1e-6, atol=0)
    Vr, Wr, _ = run_oracle(_one_channel(w))
    assert_cube_close(V[None], Vr, TOL_F32, what)
    assert_weights_close(W, Wr)


@pytest.mark.parametrize("gamma", [1, 2, 3, 4])
@pytest.mark.parametrize("block", [64, 256, 512])
def test_gamma_and_block(gamma, block):
    w = synth.small_cube(n=15_000, nchan=1, nx=29, ny=19)  # 29 cells: ragged for gamma 2, 3, 4
    _check(w, gamma, block, f"gamma {gamma} block {block}")


@pytest.mark.parametrize("kw", [
    dict(lon_c=0.05, nx=40, ny=21, name="ra_wrap"),
    dict(lon_c=359.9, nx=33, ny=17, name="ra_wrap_high"),
    dict(lat_c=75.0, lon_c=300.0, nx=24, ny=24, name="polar_cap"),
    dict(lat_c=-60.0, nx=24, ny=9, name="south"),
    dict(fwhm_arcmin=300.0, cell_arcmin=60.0, nx=20, ny=20, pad_arcmin=400.0,
         name="wide_support"),
    dict(nx=50, ny=44, pad_arcmin=-6.0, name="empty_cells"),
])
def test_geometry_cases(kw):
    w = synth.small_cube(n=20_000, nchan=1, **kw)
    _check(w, 3, 64, kw["name"])


@pytest.mark.parametrize("nx,ny,n", [(1, 1, 500), (2, 3, 800), (5, 1, 1)])
def test_tiny_maps(nx, ny, n):
    # rows narrower than gamma, a single cell, a single sample
    w = synth.small_cube(n=n, nchan=1, nx=nx, ny=ny, pad_arcmin=1.0)
    for gamma in (1, 3, 4):
        _check(w, gamma, 64, f"{nx}x{ny} n={n} gamma {gamma}")


def test_argument_errors():
    w = synth.small_cube(n=2000, nchan=1, nx=8, ny=8)
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)
    spec = w.spectra[:, 0].contiguous().to(DEV)
    V = torch.empty((8, 8), dtype=torch.float32, device=DEV)
    for gamma, block in [(0, 64), (5, 64), (1, 32), (1, 100), (1, 1024)]:
        with pytest.raises(hcg.HcgError):
            hcg.hcg_grid_rowthreads(plan, spec, V, gamma=gamma, block=block)
    with pytest.raises(ValueError):
        hcg.hcg_grid_rowthreads(plan, spec[:100].contiguous(), V)
    plan.destroy()


def test_paper_field_sampled():
    """5 deg x 5 deg at 200" (90 x 90 cells), FWHM 300", 10^7 samples: about
    14,000 samples within R of each cell."""
    w = synth.paper_field(10_000_000, device=DEV)
    g = w.grid
    print(f"{w.name}: {w.n} samples -> {g.nx} x {g.ny}", flush=True)
    (V, W), (Vt, Wt) = _both(w, 2, 64)
    ok = ~np.isnan(Vt)
    assert np.array_equal(np.isnan(V), ~ok)
    np.testing.assert_allclose(V[ok], Vt[ok], rtol=1e-6, atol=1e-6 * np.abs(Vt[ok]).max())
    np.testing.assert_allclose(W, Wt, rtol=1e-6, atol=0)
    groups = sample_cells(g, seed=5, patches=2, patch=4)
    cells = np.concatenate(groups)
    ref = [sampled_oracle(w, c) for c in groups]
    Vr = np.concatenate([v for v, _ in ref])
    Wr = np.concatenate([x for _, x in ref])
    Vg, Wg = gather_cells(torch.from_numpy(V)[None], torch.from_numpy(W), cells)
    assert_cube_close(Vg.T, Vr.T, TOL_F32, "paper field, sampled")
    assert_weights_close(Wg, Wr)
