"""The seeded input generators: exact species counts, positions in the box,
clustered fraction, reproducibility."""
import numpy as np

import synth


def test_species_counts_exact_and_seeded():
    rng = np.random.default_rng(1)
    s = synth.exact_species(2 ** 21, [0.5, 0.3, 0.2], np.random.default_rng(2))
    assert np.array_equal(np.bincount(s), [1048576, 629146, 419430])
    s6 = synth.exact_species(2 ** 24 // 64, np.ones(6), rng)
    c = np.bincount(s6)
    assert c.sum() == 2 ** 24 // 64 and c.max() - c.min() <= 1


def test_positions_in_box_and_reproducible():
    a = synth.clustered_positions(50000, 2.0, np.random.default_rng(5), halos=50)
    b = synth.clustered_positions(50000, 2.0, np.random.default_rng(5), halos=50)
    assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() < 2.0
    u = synth.uniform_positions(1000, 3.0, np.random.default_rng(6))
    assert u.min() >= 0.0 and u.max() < 3.0


def test_clustered_is_clustered():
    n = 200000
    p = synth.clustered_positions(n, 1.0, np.random.default_rng(7), halos=200, f_cl=0.7)
    h, _ = np.histogramdd(p.T, bins=32, range=[(0, 1)] * 3)
    # a uniform box would have ~6 per cell with tiny spread; halos give heavy cells
    assert h.max() > 50 * h.mean()


def test_tables_and_params():
    r_s, r_cut, eps = synth.scaled_params(2 ** 24)
    assert abs(r_s - 1.25 / 1024) < 1e-15 and abs(eps - 1 / 10240) < 1e-15 and r_cut == 4.5 * r_s
    t = synth.sample_table(lambda r: synth.newtonian_treepm_factor(r, r_s), 2048, r_cut, synth.GRID_R2)
    assert t[0] == 1.0 and 0.0175 < t[-1] < 0.0176
    p = synth.uniform_4096(1)
    assert p.n == 4096 and p.D == 2 and p.tables.shape == (2, 2, 1024) and p.lattice.dtype == np.uint64
