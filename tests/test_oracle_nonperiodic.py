"""The non-periodic reading (section 2: isolated runs use the tree alone):
the oracle run on a lattice four times the box gives the plain sum over
pairs with no periodic image, pinned against a numpy brute force; its tree
stays within the paper's tree tolerance of that sum."""
import numpy as np

import oracle
import synth


def plain_direct(pos, species, mass, G, eps):
    """sum_j G[a_i, b_j] m_j d / (r^2 + eps^2)^(3/2) with d = x_j - x_i, no images."""
    d = pos[:, None, :] - pos[:, :, None]                # d[:, i, j] = x_j - x_i
    r2 = np.sum(d * d, axis=0) + eps * eps
    np.fill_diagonal(r2, np.inf)
    k = G[species[:, None], species[None, :]] * mass[None, :] / r2 ** 1.5
    return np.einsum("ij,xij->xi", k, d)


def test_padded_lattice_is_the_plain_sum():
    p = synth.isolated_problem(600, 2, 3, ntab=64)
    assert oracle.box_of(p) == 4 * p.box and np.array_equal(oracle.lattice_of(p), oracle.lattice(p.pos, 4 * p.box))
    p.tables[:] = 1.0                                     # bare Newton with G: no table interpolation
    X = oracle.lattice(p.pos, 4 * p.box)
    law = oracle.make_law(p.G, p.tables, p.grid, p.r_cut, p.eps, p.theta)
    acc, _ = oracle.direct(X, p.species, p.mass, p.D, 4 * p.box, law)
    # the lattice rounds positions to 2^-64 of the padded box; compare with those positions
    pos = X.astype(np.float64) * (4 * p.box) * 2.0 ** -64
    ref = plain_direct(pos, p.species.astype(np.int64), p.mass, p.G, p.eps)
    rms = np.sqrt(np.mean(np.sum(ref ** 2, axis=0)))
    assert np.max(np.abs(acc - ref)) < 1e-12 * rms


def test_tree_within_tolerance_of_plain_sum():
    p = synth.isolated_problem(4000, 3, 4, ntab=512)
    X = oracle.lattice(p.pos, 4 * p.box)
    law = oracle.make_law(p.G, p.tables, p.grid, p.r_cut, p.eps, p.theta)
    T = oracle.Tree(X, p.species, p.mass, p.D, 4 * p.box, p.leaf_size)
    T.monopoles()
    T.groups(64)
    acc, _, cnt, _ = T.force(law)
    ref, _ = oracle.direct(X, p.species, p.mass, p.D, 4 * p.box, law)
    rel = np.linalg.norm(acc - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert cnt["pn"] > 0
    assert np.percentile(rel, 99) < 0.005
