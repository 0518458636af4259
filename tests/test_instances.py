"""The synthetic instance recipes: deterministic, symmetric, positive off the
diagonal (the problem statement of Sec. 2.1), with the stated spatial layout."""
import numpy as np

from paper_2003_11902_amd import instances as I


def test_deterministic_and_valid():
    for kind in ("uniform", "clustered"):
        xy1, d1 = I.make_instance(kind, 300, seed=17)
        xy2, d2 = I.make_instance(kind, 300, seed=17)
        assert np.array_equal(d1, d2) and np.array_equal(xy1, xy2)
        assert d1.dtype == np.int32 and np.array_equal(d1, d1.T)
        assert np.all(np.diag(d1) == 0)
        off = ~np.eye(300, dtype=bool)
        assert d1[off].min() >= 1


def test_rounding_is_nearest_integer():
    xy = np.array([[0.0, 0.0], [3.0, 4.0], [0.0, 1.49], [0.0, 2.5]])
    d = I.distance_matrix(xy)
    assert d[0, 1] == 5 and d[0, 2] == 1 and d[0, 3] == 3


def test_coincident_cities_redrawn():
    # side 3 with 40 cities forces coincident rounded positions to be redrawn
    xy, d = I.make_instance("uniform", 40, seed=1, side=30.0)
    off = ~np.eye(40, dtype=bool)
    assert d[off].min() >= 1


def test_batch_recipe_sizes():
    rng = np.random.default_rng(10000)
    sizes = rng.integers(100, 2001, size=256)
    assert sizes.min() >= 100 and sizes.max() <= 2000
