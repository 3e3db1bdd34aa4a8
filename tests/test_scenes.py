"""Scene construction (seeded inputs shared by the oracle and the GPU path):
particles per cell given per axis, as the hinge at the paper's resolution
uses them (4 per cell in 3D, 2 x 2 x 1)."""
import math

import numpy as np
import pytest

from paper_2605_09097_amd import scenes


def test_per_axis_counts_and_volumes():
    sc = scenes.hinge_scene(cells_B=1, cells_S=3, length=0.03, width=0.012, hinge=0.006, margin=0.002,
                            band=0.002, ppc1d=(2, 2, 1), n_frames=40)
    for D in (sc.B, sc.S):
        # one particle volume is a quarter cell, and every cell of the
        # sampled region holds four sub-cell centres: on a cell's lattice
        # the unjittered positions take 2, 2 and 1 distinct offsets per axis
        assert np.allclose(D.vol, D.dx ** 3 / 4)
        assert np.allclose(D.mass, 1000.0 * D.vol)
        frac = np.mod(D.x / D.dx, 1.0)
        for a, k in enumerate((2, 2, 1)):
            centre = (np.floor(frac[:, a] * k) + 0.5) / k
            assert np.all(np.abs(frac[:, a] - centre) <= 0.1 + 1e-9)  # jitter 0.1 dx
    # the regions are cut along the length only, where both layouts place
    # two particles per cell: the same volume as 2 x 2 x 2 per cell
    ref = scenes.hinge_scene(cells_B=1, cells_S=3, length=0.03, width=0.012, hinge=0.006, margin=0.002,
                             band=0.002, ppc1d=2, n_frames=40)
    for D, R in ((sc.B, ref.B), (sc.S, ref.S)):
        assert math.isclose(D.vol.sum(), R.vol.sum(), rel_tol=1e-12)
        assert D.n_particles * 2 == R.n_particles


def test_uniform_count_equals_the_same_count_per_axis():
    a = scenes.hinge_scene(cells_B=1, cells_S=2, length=0.03, width=0.012, hinge=0.006, margin=0.002,
                           band=0.002, ppc1d=2, n_frames=40)
    b = scenes.hinge_scene(cells_B=1, cells_S=2, length=0.03, width=0.012, hinge=0.006, margin=0.002,
                           band=0.002, ppc1d=(2, 2, 2), n_frames=40)
    for da, db in ((a.B, b.B), (a.S, b.S)):
        assert np.array_equal(da.x, db.x)
        assert np.array_equal(da.vol, db.vol)
        assert np.array_equal(da.flags, db.flags)


def test_per_axis_counts_are_validated():
    with pytest.raises(ValueError):
        scenes.hinge_scene(cells_B=1, cells_S=2, length=0.03, width=0.012, hinge=0.006, margin=0.002,
                           band=0.002, ppc1d=(2, 2), n_frames=40)
    with pytest.raises(ValueError):
        scenes.hinge_scene(cells_B=1, cells_S=2, length=0.03, width=0.012, hinge=0.006, margin=0.002,
                           band=0.002, ppc1d=(2, 0, 2), n_frames=40)
