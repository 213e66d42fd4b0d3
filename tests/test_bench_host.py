"""Host-side checks of bench.py (no GPU needed): the one-GPU contract and the
CPU-baseline leg (the oracle on sampled patches, the error against a cube)."""
import os
import subprocess
import sys

import numpy as np
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
    cb = bench.cpu_baseline(w, samp)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    # a cube that equals the oracle on the sampled cells has zero error; a
    # scaled one has exactly the scale's relative error in every channel
    cube = torch.full((w.nchan, w.grid.ny * w.grid.nx), float("nan"), dtype=torch.float64)
    cube[:, torch.from_numpy(samp["cells"])] = torch.from_numpy(samp["V"].T.copy())
    cube = cube.reshape(w.nchan, w.grid.ny, w.grid.nx)
    assert np.allclose(bench.sampled_errors(cube, samp), 0.0)
    e = bench.sampled_errors(cube * 1.01, samp)
    np.testing.assert_allclose(e, 0.01, rtol=1e-6)
