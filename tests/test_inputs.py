"""The seeded input generators (no method arithmetic in them); properties
checked with the oracle where the method is involved."""
import numpy as np
from scipy import ndimage

from paper_1705_06149_amd import inputs


def test_obstacle_mask_properties():
    for n, seed in [(64, 1), (32, 2)]:
        m = inputs.obstacle_mask(n, seed)
        assert m.shape == (n, n, n) and m.dtype == np.uint8
        assert 0.05 <= m.mean() < 0.2
        # margin: nothing touches the walls, the row under the lid is fluid
        assert m[:, n - 1, :].sum() == 0 and m[0].sum() == 0 and m[:, :, 0].sum() == 0
        lab, k = ndimage.label(m == 0, structure=ndimage.generate_binary_structure(3, 1))
        assert k == 1
        assert np.array_equal(m, inputs.obstacle_mask(n, seed))
    assert not np.array_equal(inputs.obstacle_mask(32, 1), inputs.obstacle_mask(32, 2))


def test_obstacle_sizes_in_range():
    n = 64
    rng_mask = inputs.obstacle_mask(n, 3, frac=0.01)
    lab, k = ndimage.label(rng_mask)
    for sl in ndimage.find_objects(lab):
        ext = [s.stop - s.start for s in sl]
        assert min(ext) >= 4


def test_div_free_perturbation(oracle):
    n = 16
    u, v, w = inputs.div_free_perturbation(n, n, n, seed=5, sigma=1e-2)
    g = oracle.Grid(n, n, n)
    d = oracle.divergence(g, u, v, w)
    assert np.max(np.abs(d)) <= 1e-12 * np.max(np.abs(u)) * n
    assert np.all(u[:, :, [0, -1]] == 0) and np.all(v[:, [0, -1], :] == 0) and np.all(w[[0, -1]] == 0)
    allv = np.concatenate([u[:, :, 1:-1].ravel(), v[:, 1:-1, :].ravel(), w[1:-1].ravel()])
    assert abs(allv.std() - 1e-2) < 1e-12


def test_lid_basis_vanishes_on_side_walls():
    B = inputs.lid_profile_basis(12, 10, nmodes=4)
    assert B.shape == (4, 4, 10, 13)
    assert np.max(np.abs(B[:, :, :, 0])) < 1e-15 and np.max(np.abs(B[:, :, :, -1])) < 1e-14
