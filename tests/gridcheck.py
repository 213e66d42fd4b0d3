"""Helpers shared by the GPU parity tests: run the HIP path on a workload,
compute the oracle on the same inputs, and compare them."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2012_13173_amd as hcg


def run_gpu(w, nside=None, want_plan=False, stream=None):
    """Plan + grid on cuda:0.  Returns (cube [C, ny, nx] np.float32, W np.float32[, plan])."""
    dev = torch.device("cuda:0")
    lon, lat = w.lon.to(dev), w.lat.to(dev)
    spec = w.spectra.to(dev).contiguous()
    plan = hcg.hcg_plan(lon, lat, w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside if nside is None else nside, stream=stream)
    cube = torch.empty((w.nchan, w.grid.ny, w.grid.nx), dtype=torch.float32, device=dev)
    W = torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=dev)
    hcg.hcg_grid(plan, spec, cube, W, stream=stream)
    torch.cuda.synchronize()
    out = (cube.cpu().numpy(), W.cpu().numpy())
    if want_plan:
        return out + (plan,)
    plan.destroy()
    return out


def run_oracle(w):
    lon, lat, spec = w.lon.cpu().numpy(), w.lat.cpu().numpy(), w.spectra.cpu().numpy()
    V, W, npairs = oracle.grid_allpairs(lon, lat, spec, w.grid, w.fwhm_deg, w.support_deg)
    return V, W, npairs


def channel_errors(V_gpu, V_ref):
    """Per-channel relative L2 error over cells where the reference is finite
    (the primary norm), after checking that the NaN patterns agree."""
    V_gpu = np.asarray(V_gpu, dtype=np.float64).reshape(V_gpu.shape[0], -1)
    V_ref = np.asarray(V_ref, dtype=np.float64).reshape(V_ref.shape[0], -1)
    nan_g, nan_r = np.isnan(V_gpu), np.isnan(V_ref)
    assert np.array_equal(nan_g, nan_r), f"NaN patterns differ in {int((nan_g != nan_r).sum())} places"
    ok = ~nan_r
    d = np.where(ok, V_gpu - V_ref, 0.0)
    r = np.where(ok, V_ref, 0.0)
    num = np.sqrt((d * d).sum(1))
    den = np.sqrt((r * r).sum(1))
    return np.where(den > 0, num / np.maximum(den, 1e-300), num)


def cell_errors(V_gpu, V_ref):
    """Per-cell error of every channel in units of that channel's RMS over the
    cells where the reference is finite: |V - V_ref| / rms_c(V_ref)."""
    V_gpu = np.asarray(V_gpu, dtype=np.float64).reshape(V_gpu.shape[0], -1)
    V_ref = np.asarray(V_ref, dtype=np.float64).reshape(V_ref.shape[0], -1)
    ok = ~np.isnan(V_ref)
    r = np.where(ok, V_ref, 0.0)
    rms = np.sqrt((r * r).sum(1) / np.maximum(ok.sum(1), 1))
    d = np.where(ok, np.abs(V_gpu - V_ref), 0.0)
    return d / np.maximum(rms, 1e-300)[:, None]


def assert_cube_close(V_gpu, V_ref, tol, what=""):
    """Per-channel relative L2 <= tol, and every single cell within
    10 tol of its channel's RMS (so one bad cell cannot hide in a norm)."""
    e = channel_errors(V_gpu, V_ref)
    assert float(e.max()) <= tol, f"{what}: max per-channel rel L2 {e.max():.3e} > {tol:.1e}"
    ce = cell_errors(V_gpu, V_ref)
    worst = np.unravel_index(int(np.argmax(ce)), ce.shape)
    assert float(ce.max()) <= 10.0 * tol, (
        f"{what}: cell {worst[1]} channel {worst[0]} off by {ce.max():.3e} x the channel RMS "
        f"(bound {10 * tol:.1e})")
    return e


def assert_weights_close(W_gpu, W_ref, rtol=1e-6):
    W_gpu = np.asarray(W_gpu, dtype=np.float64)
    W_ref = np.asarray(W_ref, dtype=np.float64)
    assert np.array_equal(W_gpu == 0, W_ref == 0)
    np.testing.assert_allclose(W_gpu, W_ref, rtol=rtol, atol=0)



def sample_cells(grid, seed, patches=4, patch=16):
    """Groups of flat cell indices sampling a full-size map: seeded
    patch x patch patches, the four corners and the ends of the centre row.
    Each group is small enough in the sky for the oracle to grid alone."""
    rng = np.random.default_rng(seed)
    groups = []
    for _ in range(patches):
        x0 = int(rng.integers(0, grid.nx - patch + 1))
        y0 = int(rng.integers(0, grid.ny - patch + 1))
        ix, iy = np.meshgrid(np.arange(x0, x0 + patch), np.arange(y0, y0 + patch))
        groups.append((iy * grid.nx + ix).ravel())
    ny, nx = grid.ny, grid.nx
    for c in (0, nx - 1, (ny - 1) * nx, ny * nx - 1, (ny // 2) * nx, (ny // 2) * nx + nx - 1):
        groups.append(np.array([c]))
    return groups


def sampled_oracle(w, cells):
    """FP64 oracle values (V [ncells, C], W [ncells]) of a compact group of
    cells, from the samples in a box around it that holds every sample within
    the support radius (box margins twice the radius, widened by 1/cos(lat)
    in longitude)."""
    import math
    g = w.grid
    lon = w.lon.cpu().numpy()
    lat = w.lat.cpu().numpy()
    iy, ix = np.divmod(cells, g.nx)
    clon = g.lon0 + (ix - (g.nx - 1) / 2) * g.dlon
    clat = g.lat0 + (iy - (g.ny - 1) / 2) * g.dlat
    m = 2.0 * w.support_deg
    coslat = math.cos(math.radians(min(89.0, max(abs(clat.min()), abs(clat.max())) + m)))
    sel = np.nonzero((lat >= clat.min() - m) & (lat <= clat.max() + m)
                     & (lon >= clon.min() - m / coslat) & (lon <= clon.max() + m / coslat))[0]
    rows = w.spectra.index_select(0, torch.from_numpy(sel).to(w.spectra.device)).cpu().numpy()
    V, W, _ = oracle.grid_cells(lon[sel], lat[sel], rows, g, w.fwhm_deg, w.support_deg, cells)
    return V, W


def gather_cells(cube, W, cells):
    """Values of a device cube [C, ny, nx] and W map at flat cell indices:
    (V [ncells, C], W [ncells]) as float64 numpy arrays."""
    idx = torch.from_numpy(np.ascontiguousarray(cells, dtype=np.int64)).to(cube.device)
    V = cube.reshape(cube.shape[0], -1).index_select(1, idx).T.cpu().numpy().astype(np.float64)
    return V, W.reshape(-1).index_select(0, idx).cpu().numpy().astype(np.float64)
