"""Pins for the oracle's pre-ordering (Section 3.3 step I) and ring lookup
table (Section 3.3 step III, Fig. 3)."""
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    vals = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            vals[k] = [int(x) for x in v]
    return vals


def test_sort_is_the_order_of_key_index_pairs():
    rng = np.random.default_rng(5)
    for n in (1, 2, 17, 1000, 50_000):
        keys = rng.integers(0, max(2, n // 10), n).astype(np.uint32)  # many ties
        sk, perm = oracle.sort_keys(keys)
        brute = sorted(range(n), key=lambda i: (int(keys[i]), i))
        assert np.array_equal(perm, np.array(brute))
        assert np.array_equal(sk, keys[perm])
        assert np.all(np.diff(sk.astype(np.int64)) >= 0)


def test_fig3_ring_table():
    g = _golden("fig3_ring_lut.txt")
    ns = 8
    # 9 pixels on 4 consecutive belt rings holding 6, 3, 7, 1 samples
    rings = [10, 11, 12, 13]
    layout = {10: [(0, 2), (1, 2), (2, 2)], 11: [(5, 1), (6, 2)], 12: [(3, 3), (4, 2), (9, 2)],
              13: [(7, 1)]}
    lon, lat = [], []
    for r in rings:
        for j, m in layout[r]:
            c_lon, c_lat = oracle.pix2ang(ns, oracle.ring_start(ns, r) + j)
            for q in range(m):
                lon.append(c_lon + 0.3 * (q - 0.5 * (m - 1)))  # small offsets inside the pixel
                lat.append(c_lat + 0.1 * (q - 0.5 * (m - 1)))
    lon, lat = np.array(lon), np.array(lat)
    assert lon.shape[0] == g["n_samples"][0]
    order = np.random.default_rng(3).permutation(lon.shape[0])
    pix = oracle.ang2pix(ns, lon[order], lat[order])
    assert len(set(pix.tolist())) == g["n_pixels"][0]
    sk, _ = oracle.sort_keys(pix)
    csr = oracle.ring_csr(ns, sk, rings[0], rings[-1])
    assert csr.tolist() == g["csr_0based"]
    assert (csr[:-1] + 1).tolist() == g["r_start_1based"]
