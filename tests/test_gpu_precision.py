"""GPU parity of the low-precision matrix-core forms of hcg_grid against the
FP64 oracle on the FP32 master spectra, and exactness of hcg_quantize.

Error budgets follow from the element precision (unit roundoff u, error of a
weighted mean ~ u/sqrt(3) per rounded factor, two rounded factors per term):
FP16 x FP16 (u = 2^-11) ~ 4e-4 -> 1e-3; BF16 hi+lo (u ~ 2^-16) ~ 1e-5 ->
5e-5; FP8 E4M3 hi+lo (u ~ 2^-8, plus the dropped lo.lo product) ~ 2e-3 ->
1e-2; plain BF16 (u = 2^-8) ~ 3e-3 and FP8 E4M3 (u = 2^-4) ~ 4e-2 are
reported against looser bounds (1e-2, 1e-1): on noise channels they cannot
meet 1e-3 / 1e-2."""
import numpy as np
import pytest
import torch

import paper_2012_13173_amd as hcg
import synth
from tests.gridcheck import assert_cube_close, assert_weights_close, channel_errors, run_oracle

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

FORMS = {
    "f32": (hcg.HCG_F32, 1e-5),
    "f16_scaled": (hcg.HCG_F16_SCALED, 1e-3),
    "bf16_split": (hcg.HCG_BF16_SPLIT, 5e-5),
    "bf16": (hcg.HCG_BF16, 1e-2),
    "fp8e4m3_scaled": (hcg.HCG_FP8E4M3_SCALED, 1e-1),
    "fp8e4m3_split": (hcg.HCG_FP8E4M3_SPLIT, 1e-2),
}


def _grid_form(w, plan, form):
    spec = w.spectra.to(DEV).contiguous()
    cube = torch.empty((w.nchan, w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
    W = torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
    if form == hcg.HCG_F32:
        hcg.hcg_grid(plan, spec, cube, W)
    else:
        enc, scale = hcg.hcg_quantize(spec, form)
        hcg.hcg_grid(plan, enc, cube, W, dtype=form, chan_scale=scale)
    torch.cuda.synchronize()
    return cube.cpu().numpy(), W.cpu().numpy()


@pytest.mark.parametrize("nchan", [300, 67, 1024, 5, 1])
def test_forms_against_oracle(nchan):
    w = synth.small_cube(n=15_000, nchan=nchan, nx=29, ny=19)
    Vr, Wr, _ = run_oracle(w)
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg)
    for name, (form, tol) in FORMS.items():
        V, W = _grid_form(w, plan, form)
        e = assert_cube_close(V, Vr, tol, f"{name} C={nchan}")
        print(f"{name:>15s} C={nchan:5d}: max {e.max():.2e} median {np.median(e):.2e}")
        assert_weights_close(W, Wr)
    plan.destroy()


def test_constant_input_is_exact_in_every_form():
    w = synth.small_cube(n=12_000, nchan=64, nx=21, ny=13)
    w.spectra[:] = 2.5  # exactly representable in every form and scale
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg)
    for name, (form, _) in FORMS.items():
        V, W = _grid_form(w, plan, form)
        assert (W > 0).all()
        np.testing.assert_allclose(V, 2.5, rtol=1e-5, err_msg=name)
    plan.destroy()


@pytest.mark.parametrize("C", [97, 96])  # element-wise kernel, and rows read 4 channels at a time
def test_quantize_matches_reference_roundings(C):
    g = torch.Generator(device=DEV).manual_seed(3)
    n = 5000
    x = torch.randn((n, C), generator=g, device=DEV) * torch.logspace(-3, 3, C, device=DEV)
    x[:, 5] = 0.0  # an all-zero channel gets scale 1
    x[17, 9] = 1e-30  # deep underflow in every narrow form
    bf, _ = hcg.hcg_quantize(x, hcg.HCG_BF16)
    assert torch.equal(bf.view(torch.int16), x.to(torch.bfloat16).view(torch.int16))
    sp, _ = hcg.hcg_quantize(x, hcg.HCG_BF16_SPLIT)
    hi = x.to(torch.bfloat16)
    lo = (x - hi.float()).to(torch.bfloat16)
    assert torch.equal(sp[0].view(torch.int16), hi.view(torch.int16))
    assert torch.equal(sp[1].view(torch.int16), lo.view(torch.int16))
    amax = x.abs().amax(0).double().cpu().numpy()
    for form, top, tdt in ((hcg.HCG_F16_SCALED, 2.0 ** 14, torch.float16),
                           (hcg.HCG_FP8E4M3_SCALED, 448.0, torch.float8_e4m3fn)):
        q, scale = hcg.hcg_quantize(x, form)
        want = np.where(amax > 0, 2.0 ** np.ceil(np.log2(np.maximum(amax, 1e-300) / top)), 1.0)
        assert np.array_equal(scale.double().cpu().numpy(), want)
        ref = (x / scale).to(tdt)
        if tdt == torch.float16:
            assert torch.equal(q.view(torch.int16), ref.view(torch.int16))
        else:
            assert torch.equal(q, ref.view(torch.uint8))
        # every channel uses its range: the largest |x|/scale is within a factor 2 of top
        scaled_max = (x / scale).abs().amax(0)
        nz = torch.from_numpy(amax > 0).to(DEV)
        assert bool(((scaled_max[nz] <= top) & (scaled_max[nz] > top / 2)).all())
    # FP8 hi + lo: the scale of the single FP8 form, hi its encoding, lo the
    # encoding of the remainder
    q8, s8 = hcg.hcg_quantize(x, hcg.HCG_FP8E4M3_SCALED)
    sp8, ss8 = hcg.hcg_quantize(x, hcg.HCG_FP8E4M3_SPLIT)
    assert torch.equal(ss8, s8) and tuple(sp8.shape) == (2, n, C)
    assert torch.equal(sp8[0], q8)
    y = x / ss8
    lo = (y - y.to(torch.float8_e4m3fn).float()).to(torch.float8_e4m3fn)
    assert torch.equal(sp8[1], lo.view(torch.uint8))


def test_grid_rejects_scale_mismatch():
    w = synth.small_cube(n=2000, nchan=16, nx=8, ny=8)
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg)
    spec = w.spectra.to(DEV)
    cube = torch.empty((16, 8, 8), dtype=torch.float32, device=DEV)
    enc, scale = hcg.hcg_quantize(spec, hcg.HCG_F16_SCALED)
    with pytest.raises(hcg.HcgError):
        hcg.hcg_grid(plan, enc, cube, dtype=hcg.HCG_F16_SCALED, chan_scale=None)
    bf, _ = hcg.hcg_quantize(spec, hcg.HCG_BF16)
    with pytest.raises(hcg.HcgError):
        hcg.hcg_grid(plan, bf, cube, dtype=hcg.HCG_BF16, chan_scale=scale)
    plan.destroy()
