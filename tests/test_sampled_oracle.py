"""The sampled-cell oracle used by the full-size GPU parity tests: the sample
box it cuts around a group of cells must hold every sample within the support
radius, so its values equal the all-pairs oracle's at those cells."""
import numpy as np

import synth
from tests.gridcheck import run_oracle, sample_cells, sampled_oracle


def test_sampled_cells_equal_all_pairs():
    w = synth.small_cube(n=12_000, nchan=5, nx=45, ny=37)
    Vr, Wr, _ = run_oracle(w)
    groups = sample_cells(w.grid, seed=3, patches=3, patch=8)
    assert len(groups) == 9
    for cells in groups:
        V, W = sampled_oracle(w, cells)
        np.testing.assert_array_equal(W, Wr.reshape(-1)[cells])
        np.testing.assert_array_equal(V, Vr.reshape(Vr.shape[0], -1)[:, cells].T)


def test_sampled_cells_near_the_pole():
    w = synth.small_cube(n=12_000, nchan=3, nx=31, ny=21, lat_c=84.0)
    Vr, Wr, _ = run_oracle(w)
    for cells in sample_cells(w.grid, seed=5, patches=2, patch=6):
        V, W = sampled_oracle(w, cells)
        np.testing.assert_array_equal(W, Wr.reshape(-1)[cells])
        np.testing.assert_array_equal(V, Vr.reshape(Vr.shape[0], -1)[:, cells].T)
