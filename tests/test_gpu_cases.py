"""GPU parity cases beyond the basic grid tests, through the C ABI:

* few channels (C <= 8) on maps of >= 1024 tiles, where the one-lane-per-cell
  gather writes the map directly (no split of the candidate lists);
* supports of 5 sigma (Section 3.6 (iii) allows 3 to 5 sigma) in the FP32 form
  and every low-precision form, input order and plan-ordered;
* a non-finite spectrum value stays near its sample: padding of a tile's
  candidate list never multiplies it, so it reaches only tiles that list the
  sample as a candidate -- cells within R + the 8 x 8 tile's diagonal + a
  HEALPix pixel (exactly the cells within R for C <= 8);
* the binding refuses spectra whose row count is not the plan's sample count,
  before any launch;
* tiles with more candidate ranges than the phase-rotated staging holds (a
  wide support at longitude 0, two ranges per ring) next to tiles that are
  rotated, in the FP32 form and two matrix-core forms;
* input-order BF16, FP16 x scale and FP8 x scale spectra whose rows are read
  eight elements at a time (512-channel slabs, C a multiple of 8, aligned)
  against the same spectra read four at a time (256-channel slabs), bit for
  bit, and against the oracle;
* channels stay apart: with channel 0 non-finite in every sample, no other
  channel of any form holds a NaN where the map has samples (lanes whose
  channels lie past the last one read their row's first channels, whose
  products go to accumulators that are never stored).
"""
import math

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

FORMS = {
    "f16_scaled": (hcg.HCG_F16_SCALED, 1e-3),
    "bf16_split": (hcg.HCG_BF16_SPLIT, 5e-5),
    "fp8e4m3_split": (hcg.HCG_FP8E4M3_SPLIT, 1e-2),
    "bf16": (hcg.HCG_BF16, 1e-2),
    "fp8e4m3_scaled": (hcg.HCG_FP8E4M3_SCALED, 1e-1),
}


def _plan(w):
    return hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)


def _grid(w, plan, form=hcg.HCG_F32, packed=False, spectra=None):
    spec = (w.spectra if spectra is None else spectra).to(DEV).contiguous()
    cube = torch.empty((w.nchan, w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
    W = torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
    if form == hcg.HCG_F32:
        hcg.hcg_grid(plan, spec, cube, W)
    elif packed:
        enc, scale = hcg.hcg_quantize_packed(plan, spec, form)
        hcg.hcg_grid_packed(plan, enc, cube, W, dtype=form, chan_scale=scale)
    else:
        enc, scale = hcg.hcg_quantize(spec, form)
        hcg.hcg_grid(plan, enc, cube, W, dtype=form, chan_scale=scale)
    torch.cuda.synchronize()
    return cube, W


@pytest.mark.parametrize("nchan", [1, 5])
def test_few_channels_on_many_tiles(nchan):
    # 264 x 256 cells = 33 x 32 = 1056 tiles: the direct-write gather
    w = synth.small_cube(n=250_000, nchan=nchan, nx=264, ny=256, cell_arcmin=0.5, seed=410 + nchan)
    plan = _plan(w)
    info = plan.info()
    assert info["ntiles_x"] * info["ntiles_y"] >= 1024
    print(f"C={nchan}: {info['ntiles_x'] * info['ntiles_y']} tiles", flush=True)
    cube, W = _grid(w, plan)
    plan.destroy()
    groups = sample_cells(w.grid, seed=7 + nchan, patches=4, patch=12)
    cells = np.concatenate(groups)
    ref = [sampled_oracle(w, c) for c in groups]
    Vr = np.concatenate([v for v, _ in ref])
    Wr = np.concatenate([x for _, x in ref])
    V, Wg = gather_cells(cube, W, cells)
    assert_cube_close(V.T, Vr.T, TOL_F32, f"C={nchan}, 1056 tiles")
    assert_weights_close(Wg, Wr)


@pytest.mark.parametrize("nchan", [1, 67, 300])
def test_five_sigma_support_every_form(nchan):
    w = synth.small_cube(n=15_000, nchan=nchan, nx=29, ny=19, support_sigma=5.0, seed=430)
    Vr, Wr, _ = run_oracle(w)
    plan = _plan(w)
    cube, W = _grid(w, plan)
    e = assert_cube_close(cube.cpu().numpy(), Vr, TOL_F32, f"f32 5 sigma C={nchan}")
    print(f"{'f32':>15s} C={nchan:4d} 5 sigma: max {e.max():.2e}", flush=True)
    assert_weights_close(W.cpu().numpy(), Wr)
    for name, (form, tol) in FORMS.items():
        for packed in (False, True):
            cube, W = _grid(w, plan, form, packed)
            what = f"{'packed ' if packed else ''}{name} 5 sigma C={nchan}"
            e = assert_cube_close(cube.cpu().numpy(), Vr, tol, what)
            print(f"{what}: max {e.max():.2e}", flush=True)
            assert_weights_close(W.cpu().numpy(), Wr)
    plan.destroy()


def _dist_to(w, lon0, lat0):
    """[ny, nx] great-circle distance (degrees) of every cell centre to a point."""
    g = w.grid
    ix = np.arange(g.nx)
    iy = np.arange(g.ny)
    cl = np.radians(g.lon0 + (ix - (g.nx - 1) / 2) * g.dlon)[None, :]
    cb = np.radians(g.lat0 + (iy - (g.ny - 1) / 2) * g.dlat)[:, None]
    l0, b0 = math.radians(lon0), math.radians(lat0)
    h = np.sin((cb - b0) / 2) ** 2 + np.cos(cb) * math.cos(b0) * np.sin((cl - l0) / 2) ** 2
    return np.degrees(2 * np.arcsin(np.sqrt(np.minimum(h, 1.0))))


@pytest.mark.parametrize("nchan", [1, 40])
def test_non_finite_value_stays_near_its_sample(nchan):
    # sample 0 sits near a corner; its value is NaN in every channel
    w = synth.small_cube(n=20_000, nchan=nchan, nx=48, ny=40, seed=450)
    g = w.grid
    w.lon[0] = g.lon0 - 0.4 * g.nx * g.dlon
    w.lat[0] = g.lat0 - 0.4 * g.ny * g.dlat
    spec = w.spectra.clone()
    spec[0] = float("nan")
    plan = _plan(w)
    dist = _dist_to(w, float(w.lon[0]), float(w.lat[0]))
    R = w.support_deg
    # matrix-core forms: a tile that lists sample 0 as a candidate has its
    # cells within R + its diagonal (7 sqrt(2) cells) + a pixel of sample 0
    pix = math.degrees(math.sqrt(4 * math.pi / (12.0 * w.nside ** 2)))
    reach = R + 7 * math.sqrt(2) * g.dlat + 2 * pix
    empty = np.isnan(_grid(w, plan)[0].cpu().numpy()[0])  # cells without samples
    forms = [("f32", hcg.HCG_F32)] + ([] if nchan <= 8 else
                                      [(k, v[0]) for k, v in FORMS.items()])
    for name, form in forms:
        cube, _ = _grid(w, plan, form, spectra=spec)
        V = cube.cpu().numpy()
        bad = np.isnan(V).any(0) & ~empty
        if nchan <= 8:
            # one lane per cell in FP64: exactly the cells within R
            assert np.array_equal(bad, dist <= R), name
        else:
            assert bad.any(), name
            assert dist[bad].max() <= reach, f"{name}: NaN at {dist[bad].max():.4f} deg > {reach:.4f}"
        print(f"{name}: {int(bad.sum())} cells reached, farthest {dist[bad].max():.4f} deg "
              f"(R {R:.4f})", flush=True)
    plan.destroy()


def test_spectra_row_count_is_checked_before_any_launch():
    w = synth.small_cube(n=3000, nchan=12, nx=10, ny=10, seed=470)
    plan = _plan(w)
    cube = torch.empty((12, 10, 10), dtype=torch.float32, device=DEV)
    short = w.spectra[:-1].to(DEV).contiguous()
    with pytest.raises(ValueError):
        hcg.hcg_grid(plan, short, cube)
    enc, scale = hcg.hcg_quantize(short, hcg.HCG_BF16_SPLIT)
    with pytest.raises(ValueError):
        hcg.hcg_grid(plan, enc, cube, dtype=hcg.HCG_BF16_SPLIT)
    plan.destroy()
    b = hcg.hcg_plan_batch([(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg)])
    with pytest.raises(ValueError):
        hcg.hcg_grid_batch(b, [short], [cube])
    with pytest.raises(ValueError):
        hcg.hcg_grid_batch(b, [w.spectra.to(DEV)], [cube],
                           [torch.empty((9, 10), dtype=torch.float32, device=DEV)])
    b.destroy()


def test_batch_with_a_wide_support_field():
    # one field of support 0.64 deg (FWHM 30', 3 sigma) makes the persistent
    # kernel take the long distance series; the narrow fields must not change
    ws = [synth.small_cube(n=6000, nchan=24, nx=20, ny=16, seed=481, name="narrow24"),
          synth.small_cube(n=9000, nchan=1, nx=18, ny=18, seed=482, fwhm_arcmin=30.0,
                           cell_arcmin=10.0, pad_arcmin=40.0, name="wide1"),
          synth.small_cube(n=9000, nchan=96, nx=16, ny=14, seed=483, fwhm_arcmin=30.0,
                           cell_arcmin=10.0, pad_arcmin=40.0, lat_c=-50.0, name="wide96"),
          synth.small_cube(n=5000, nchan=3, nx=9, ny=11, seed=484, name="narrow3")]
    assert ws[1].support_deg >= 0.57 and ws[2].support_deg >= 0.57
    b = hcg.hcg_plan_batch([(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg)
                            for w in ws])
    cubes = [torch.empty((w.nchan, w.grid.ny, w.grid.nx), device=DEV) for w in ws]
    wts = [torch.empty((w.grid.ny, w.grid.nx), device=DEV) for w in ws]
    hcg.hcg_grid_batch(b, [w.spectra.to(DEV) for w in ws], cubes, wts)
    torch.cuda.synchronize()
    for w, c, x in zip(ws, cubes, wts):
        Vr, Wr, _ = run_oracle(w)
        assert_cube_close(c.cpu().numpy(), Vr, TOL_F32, w.name)
        assert_weights_close(x.cpu().numpy(), Wr)
    b.destroy()


def test_tiles_of_more_ranges_than_a_rotation_holds():
    # centred on longitude 0 with a 38' support and nside 8192 (rings 0.28'
    # apart): tiles that straddle longitude 0 reach every ring on both sides
    # of it, two ranges per ring, more than half the staging room, and are
    # read in the plan's order; the other tiles are read phase-rotated
    # (40 x 16 cells of 5': the outer tile columns do not reach longitude 0)
    w = synth.small_cube(n=50_000, nchan=16, nx=40, ny=16, cell_arcmin=5.0, fwhm_arcmin=30.0,
                         pad_arcmin=40.0, lon_c=0.0, lat_c=10.0, nside=8192, seed=490)
    plan = _plan(w)
    nr = hcg.u32(plan.export(hcg.HCG_ARR_TILE_NRANGES))
    print(f"ranges per tile: {sorted(set(nr.tolist()))}", flush=True)
    assert nr.max() > 512 and nr.min() <= 512
    Vr, Wr, _ = run_oracle(w)
    cube, W = _grid(w, plan)
    assert_cube_close(cube.cpu().numpy(), Vr, TOL_F32, "f32, > 512 ranges")
    assert_weights_close(W.cpu().numpy(), Wr)
    for name in ("f16_scaled", "bf16_split"):
        form, tol = FORMS[name]
        for packed in (False, True):
            cube, W = _grid(w, plan, form, packed)
            assert_cube_close(cube.cpu().numpy(), Vr, tol, f"{name} packed={packed}, > 512 ranges")
            assert_weights_close(W.cpu().numpy(), Wr)
    plan.destroy()


@pytest.mark.parametrize("nchan", [520, 516])
def test_rows_read_eight_channels_at_a_time(nchan):
    """A map of 576 8 x 8 tiles takes 512-channel slabs above 256 channels.
    C = 520: the input-order BF16, FP16 x scale and FP8 x scale gathers read a
    lane's eight channels of a row in one load (the second slab holds 8
    channels); the same encoding placed four elements off an eight-element
    boundary is read four channels at a time in 256-channel slabs, and both
    give the same cube bit for bit (the
    same weights and the same products in the same order per channel).
    C = 516 (not a multiple of 8) takes the four-channel reads for both.  Each
    cube matches the oracle on sampled cells at the form's budget."""
    w = synth.small_cube(n=120_000, nchan=nchan, nx=192, ny=192, cell_arcmin=0.5,
                         seed=470 + nchan)
    plan = _plan(w)
    info = plan.info()
    assert info["ntiles_x"] * info["ntiles_y"] >= 512
    groups = sample_cells(w.grid, seed=9, patches=3, patch=10)
    cells = np.concatenate(groups)
    ref = [sampled_oracle(w, c) for c in groups]
    Vr = np.concatenate([v for v, _ in ref])
    Wr = np.concatenate([x for _, x in ref])
    spec = w.spectra.to(DEV).contiguous()
    g = w.grid
    for form, tol in [(hcg.HCG_BF16, 1e-2), (hcg.HCG_F16_SCALED, 1e-3),
                      (hcg.HCG_FP8E4M3_SCALED, 1e-1)]:
        print(f"C={nchan} form {form}", flush=True)
        enc, scale = hcg.hcg_quantize(spec, form)
        cube = torch.empty((nchan, g.ny, g.nx), dtype=torch.float32, device=DEV)
        W = torch.empty((g.ny, g.nx), dtype=torch.float32, device=DEV)
        hcg.hcg_grid(plan, enc, cube, W, dtype=form, chan_scale=scale)
        flat = torch.empty(enc.numel() + 4, dtype=enc.dtype, device=DEV)
        off = flat[4:].view(enc.shape)
        off.copy_(enc)
        esz = enc.element_size()
        assert off.data_ptr() % (8 * esz) == 4 * esz  # four elements off
        cube_off = torch.empty_like(cube)
        hcg.hcg_grid(plan, off, cube_off, None, dtype=form, chan_scale=scale)
        torch.cuda.synchronize()
        assert torch.equal(cube.view(torch.int32), cube_off.view(torch.int32)), (
            f"C={nchan} form {form}: eight- and four-channel reads differ")
        V, Wg = gather_cells(cube, W, cells)
        assert_cube_close(V.T, Vr.T, tol, f"C={nchan} form {form}, 576 tiles")
        assert_weights_close(Wg, Wr)
        del enc, flat, off, cube, cube_off
    plan.destroy()


@pytest.mark.parametrize("nchan", [40, 300, 520])
def test_a_non_finite_channel_stays_in_its_channel(nchan):
    # C = 40: one 64-channel group per wave, partly past the last channel;
    # C = 300: 256-channel slabs, the second holding 44; C = 520 on 576
    # tiles: eight channels per lane, the second 512-channel slab holding 8
    w = synth.small_cube(n=120_000, nchan=nchan, nx=192, ny=192, cell_arcmin=0.5,
                         seed=480 + nchan)
    spec = w.spectra.clone()
    spec[:, 0] = float("nan")
    plan = _plan(w)
    empty = np.isnan(_grid(w, plan)[0].cpu().numpy()[1])  # cells without samples
    assert (~empty).sum() > 0.9 * empty.size
    forms = [("f32", hcg.HCG_F32)] + [(k, v[0]) for k, v in FORMS.items()]
    for name, form in forms:
        print(f"C={nchan} {name}", flush=True)
        cube, _ = _grid(w, plan, form, spectra=spec)
        V = cube.cpu().numpy()
        leaked = np.isnan(V[1:]) & ~empty[None]
        assert not leaked.any(), (
            f"C={nchan} {name}: NaN in {int(leaked.sum())} values of channels 1..{nchan - 1}")
        if form == hcg.HCG_F32:
            assert np.isnan(V[0]).all(), f"C={nchan}: channel 0 should be NaN everywhere"
        del cube
    plan.destroy()
