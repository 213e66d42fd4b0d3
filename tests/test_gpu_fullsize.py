"""GPU parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (hcg_plan + hcg_grid on the whole map, and the
plan-ordered encodings through hcg_quantize_packed + hcg_grid_packed), checked
on sampled cells that the FP64 oracle computes one by one: seeded 16 x 16-cell
patches, the corners and the ends of the centre row.

* drift scan, 9,120,000 samples x 1,024 channels, 600 x 600 cells: FP32 and
  every low-precision form;
* drift scan, 1,976,000 samples x 8,192 channels, 400 x 400 cells: FP32,
  BF16, FP16 x scale, BF16 hi+lo;
* large cube, 20,064,000 samples x 1,024 channels, 3000 x 3000 cells: FP32,
  FP8 E4M3 x scale and FP8 E4M3 hi+lo x scale;
* the 64-field batch (one persistent launch), every field.

Per-channel relative L2 over the sampled cells, tolerances as in
test_gpu_precision.py (FP32 1e-5); W map elementwise 1e-6."""
import numpy as np
import pytest
import torch

import paper_2012_13173_amd as hcg
import synth
from tests.gridcheck import (assert_cube_close, assert_weights_close, gather_cells,
                             sample_cells, sampled_oracle)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {hcg.HCG_F32: 1e-5, hcg.HCG_F16_SCALED: 1e-3, hcg.HCG_BF16_SPLIT: 5e-5,
       hcg.HCG_BF16: 1e-2, hcg.HCG_FP8E4M3_SCALED: 1e-1, hcg.HCG_FP8E4M3_SPLIT: 1e-2}
NAME = {hcg.HCG_F32: "f32", hcg.HCG_F16_SCALED: "f16_scaled", hcg.HCG_BF16_SPLIT: "bf16_split",
        hcg.HCG_BF16: "bf16", hcg.HCG_FP8E4M3_SCALED: "fp8e4m3_scaled",
        hcg.HCG_FP8E4M3_SPLIT: "fp8e4m3_split"}


def _check(w, forms, seed, packed=()):
    g = w.grid
    print(f"{w.name}: {w.n} samples x {w.nchan} channels", flush=True)
    groups = sample_cells(g, seed)
    cells = np.concatenate(groups)
    ref = [sampled_oracle(w, c) for c in groups]
    Vr = np.concatenate([v for v, _ in ref])
    Wr = np.concatenate([x for _, x in ref])
    plan = hcg.hcg_plan(w.lon, w.lat, g, w.fwhm_deg, w.support_deg, nside=w.nside)
    cube = torch.empty((w.nchan, g.ny, g.nx), dtype=torch.float32, device=DEV)
    W = torch.empty((g.ny, g.nx), dtype=torch.float32, device=DEV)
    for form in forms:
        if form == hcg.HCG_F32:
            hcg.hcg_grid(plan, w.spectra, cube, W)
        else:
            enc, scale = hcg.hcg_quantize(w.spectra, form)
            hcg.hcg_grid(plan, enc, cube, W, dtype=form, chan_scale=scale)
            del enc
        torch.cuda.synchronize()
        V, Wg = gather_cells(cube, W, cells)
        e = assert_cube_close(V.T, Vr.T, TOL[form], f"{w.name} {NAME[form]}")
        assert_weights_close(Wg, Wr)
        print(f"  {NAME[form]:>15s}: {cells.size} cells, max {e.max():.2e} "
              f"median {np.median(e):.2e}", flush=True)
    for form in packed:  # plan-ordered encodings, as bench.py times them
        enc, scale = hcg.hcg_quantize_packed(plan, w.spectra, form)
        hcg.hcg_grid_packed(plan, enc, cube, W, dtype=form, chan_scale=scale)
        del enc
        torch.cuda.synchronize()
        V, Wg = gather_cells(cube, W, cells)
        e = assert_cube_close(V.T, Vr.T, TOL[form], f"{w.name} packed {NAME[form]}")
        assert_weights_close(Wg, Wr)
        print(f"  packed {NAME[form]:>15s}: {cells.size} cells, max {e.max():.2e} "
              f"median {np.median(e):.2e}", flush=True)
    plan.destroy()
    del cube, W
    torch.cuda.empty_cache()


def test_drift_scan_1024_full_size():
    w = synth.drift_scan_1024(device=DEV)
    _check(w, [hcg.HCG_F32, hcg.HCG_BF16, hcg.HCG_F16_SCALED, hcg.HCG_BF16_SPLIT,
               hcg.HCG_FP8E4M3_SCALED, hcg.HCG_FP8E4M3_SPLIT], seed=11,
           packed=[hcg.HCG_F16_SCALED, hcg.HCG_BF16, hcg.HCG_BF16_SPLIT,
                   hcg.HCG_FP8E4M3_SCALED, hcg.HCG_FP8E4M3_SPLIT])
    del w
    torch.cuda.empty_cache()


def test_drift_scan_8192_full_size():
    w = synth.drift_scan_8192(device=DEV)
    _check(w, [hcg.HCG_F32, hcg.HCG_BF16, hcg.HCG_F16_SCALED, hcg.HCG_BF16_SPLIT], seed=12,
           packed=[hcg.HCG_F16_SCALED, hcg.HCG_BF16_SPLIT])
    del w
    torch.cuda.empty_cache()


def test_large_cube_full_size():
    w = synth.drift_scan_large(device=DEV)
    _check(w, [hcg.HCG_F32, hcg.HCG_FP8E4M3_SCALED, hcg.HCG_FP8E4M3_SPLIT], seed=14,
           packed=[hcg.HCG_FP8E4M3_SPLIT, hcg.HCG_F16_SCALED])
    del w
    torch.cuda.empty_cache()


def test_batch_64_fields_full_size():
    """The 64-field batch as bench.py runs it (one persistent launch, tuned
    and graph-captured), every field checked on a sampled patch and its
    corners."""
    ws = synth.batch_fields(device=DEV)
    print(f"batch: {len(ws)} fields, {sum(w.n * w.nchan for w in ws):.4g} sample*channels",
          flush=True)
    b = hcg.hcg_plan_batch([(w.lon, w.lat, w.grid, w.fwhm_deg, w.support_deg) for w in ws])
    cubes = [torch.empty((w.nchan, w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
             for w in ws]
    wts = [torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV) for w in ws]
    hcg.hcg_grid_batch(b, [w.spectra for w in ws], cubes, wts)
    torch.cuda.synchronize()
    worst = 0.0
    for f, w in enumerate(ws):
        groups = sample_cells(w.grid, seed=100 + f, patches=1, patch=6)
        cells = np.concatenate(groups)
        ref = [sampled_oracle(w, c) for c in groups]
        Vr = np.concatenate([v for v, _ in ref])
        Wr = np.concatenate([x for _, x in ref])
        V, Wg = gather_cells(cubes[f], wts[f], cells)
        e = assert_cube_close(V.T, Vr.T, TOL[hcg.HCG_F32], f"batch {w.name}")
        assert_weights_close(Wg, Wr)
        worst = max(worst, float(e.max()))
    print(f"  all fields: max per-channel rel L2 {worst:.2e}", flush=True)
    b.destroy()
    del cubes, wts, ws
    torch.cuda.empty_cache()
