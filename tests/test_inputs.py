"""Seeded synthetic inputs: determinism, shapes and ranges (not gpu)."""
import numpy as np

import heat_inputs


def test_bumps_deterministic_and_shaped():
    times = np.linspace(0, 1, 12).reshape(4, 3)
    a = heat_inputs.bump_source(np.random.default_rng(1), 20, 2, times)
    b = heat_inputs.bump_source(np.random.default_rng(1), 20, 2, times)
    assert a.shape == (4, 3, 400) and np.array_equal(a, b)


def test_smooth_initial_vanishes_near_boundary():
    u = heat_inputs.smooth_initial(np.random.default_rng(2), 63, 2).reshape(63, 63)
    assert np.abs(u[0]).max() < 0.2 * np.abs(u).max()
    u3 = heat_inputs.smooth_initial(np.random.default_rng(2), 15, 3)
    assert u3.shape == (15 ** 3,)


def test_kappa_patches_and_range():
    k = heat_inputs.lognormal_kappa(np.random.default_rng(3), 64, 2).reshape(64, 64)
    assert k.min() >= 0.1 and k.max() <= 10.0
    assert len(np.unique(k)) <= 64
    assert np.all(k[0:7, 0:7] == k[0, 0])          # nodes 1..7 of 64 share a patch


def test_batch_specs_are_seeded():
    a = heat_inputs.batch_problem_specs(8)
    assert a == heat_inputs.batch_problem_specs(8)
    assert all(p["n"] in (64, 128, 192, 256, 384) and 1 <= p["s"] <= 3 and 8 <= p["nt"] <= 64
               for p in a)
