"""Pins of the oracle's soft obstacle costs (Sec. VI-VII: the slowness near
obstacles is a function of the distance to the nearest hard obstacle,
found by a distance transform): brute force over all hard pixels on small
images, scipy's exact Euclidean distance transform on larger ones, and the
distance ramp the workload generator builds on the host."""
import itertools

import numpy as np
import pytest
from scipy.ndimage import distance_transform_edt

import oracle
from paper_2306_01301_amd import scenes

HARD = 255


def _table_identity(n):
    # code = min(d^2, 254): exposes the squared distance itself
    return np.minimum(np.arange(2 * n * n + 2), 254).astype(np.uint8)


@pytest.mark.parametrize("seed,n,frac", [(1, 8, 0.1), (2, 12, 0.3), (3, 16, 0.02), (4, 9, 0.0)])
def test_brute_force(seed, n, frac):
    rng = np.random.default_rng(seed)
    img = np.where(rng.random((n, n)) < frac, HARD, rng.integers(0, 200, (n, n))).astype(np.uint8)
    tab = _table_identity(n)
    got = oracle.soft_costs(img, tab)
    hard = np.argwhere(img == HARD)
    for j, i in itertools.product(range(n), range(n)):
        if img[j, i] == HARD:
            assert got[j, i] == HARD
            continue
        d2 = min(((hard[:, 0] - j) ** 2 + (hard[:, 1] - i) ** 2).tolist(), default=None)
        want = tab[-1] if d2 is None else tab[min(d2, len(tab) - 1)]
        assert got[j, i] == want, (j, i)


def test_scipy_distance_transform():
    rng = np.random.default_rng(5)
    img = scenes.mixed_clutter(rng, 128, 0.15)
    d2 = np.rint(distance_transform_edt(img != HARD) ** 2).astype(np.int64)
    tab = np.arange(65536) % 251
    tab = tab.astype(np.uint8)
    got = oracle.soft_costs(img, tab)
    want = np.where(img == HARD, HARD, tab[np.minimum(d2, len(tab) - 1)])
    assert np.array_equal(got, want)


def test_equals_the_ramp_of_the_workload_generator():
    rng = np.random.default_rng(6)
    img = scenes.maze(rng, 4, 32, 4)
    width, peak = 4.0, 64
    q = np.arange(int(width * width) + 1)
    tab = np.where(q < width * width, np.rint(peak * (width - np.sqrt(q)) / width), 0)
    tab = np.clip(tab, 0, 254).astype(np.uint8)
    assert np.array_equal(oracle.soft_costs(img, tab), scenes.soft_ramp(img, width, peak))
