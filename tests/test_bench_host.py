"""Host-side checks of bench.py (no GPU needed): the one-GPU contract and the
CPU-baseline leg (the oracle on sampled patches, the error against a cube)."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_oracle_sample_and_errors():
    w = synth.small_cube(n=6000, nchan=7, nx=40, ny=36)
    samp = bench.oracle_sample(w, budget_s=0.5, patch=8, max_patches=3, seed=1)
    assert samp["cells"].size == samp["V"].shape[0] == 8 * 8 * samp["patches"]
    assert samp["pairs"] > 0
    cb = bench.cpu_baseline(w, samp, 10 * samp["pairs"])
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    # extrapolated by pair work: ten times the pairs take ten times the time
    assert cb["value"] == pytest.approx(w.n * w.nchan / (10 * samp["t"]), rel=1e-12)
    # a cube that equals the oracle on the sampled cells has zero error; a
    # scaled one has exactly the scale's relative error in every channel
    cube = torch.full((w.nchan, w.grid.ny * w.grid.nx), float("nan"), dtype=torch.float64)
    cube[:, torch.from_numpy(samp["cells"])] = torch.from_numpy(samp["V"].T.copy())
    cube = cube.reshape(w.nchan, w.grid.ny, w.grid.nx)
    assert np.allclose(bench.sampled_errors(cube, samp), 0.0)
    e = bench.sampled_errors(cube * 1.01, samp)
    np.testing.assert_allclose(e, 0.01, rtol=1e-6)


def test_error_records_and_budgets():
    errs = {"f32": np.array([2e-6, 9e-6]), "packed_f16_scaled": np.array([3e-4, 1.2e-3]),
            "fp8e4m3_split": np.array([1e-3, 2e-3])}
    forms = {"packed_f16_scaled": {"grid_ms": 1.0}}
    bench.add_errors(forms, errs)
    assert forms["f32"]["meets_budget"] and forms["fp8e4m3_split"]["meets_budget"]
    assert not forms["packed_f16_scaled"]["meets_budget"]
    assert forms["packed_f16_scaled"]["budget"] == 1e-3
    assert forms["packed_f16_scaled"]["rel_l2_max_over_channels"] == 1.2e-3
    # the paper's ~21 CPU-hours per TB of FP32 values, as updates per second
    assert bench.PAPER_CONTEXT["sample_channel_updates_per_s"] == pytest.approx(3.3e6, rel=0.01)
