"""The seeded input recipe (synth): masks, outliers, noise and core layouts have the
shapes and statistics the workloads state, and the same seed gives the same inputs."""
import math

import numpy as np
import pytest

import synth
from oracle import tr


def test_same_seed_same_inputs():
    w = synth.scaled(synth.WORKLOADS["tr4_100_r5"], (12, 10, 9, 8))
    a = synth.make_workload(w, 3, tr.reconstruct)
    b = synth.make_workload(w, 3, tr.reconstruct)
    c = synth.make_workload(w, 4, tr.reconstruct)
    for u, v in zip(a[1:], b[1:]):
        np.testing.assert_array_equal(u, v)
    assert not np.array_equal(a[3], c[3])


def test_bernoulli_mask_density():
    m = synth.bernoulli_mask((40, 50, 60), 0.1, 0)
    assert m.dtype == np.uint8 and set(np.unique(m)) <= {0, 1}
    n = m.size
    assert abs(m.mean() - 0.1) < 4 * math.sqrt(0.1 * 0.9 / n)


def test_block_mask_is_blockwise_and_shared_by_channels():
    dims = (40, 50, 3, 7)
    m = synth.block_mask(dims, 16, 0.8, 1)
    # every 16x16 tile of a frame is all observed or all missing, the same in every channel
    for f in range(dims[3]):
        for c in range(dims[2]):
            np.testing.assert_array_equal(m[:, :, c, f], m[:, :, 0, f])
        for bi in range(0, dims[0], 16):
            for bj in range(0, dims[1], 16):
                tile = m[bi:bi + 16, bj:bj + 16, 0, f]
                assert tile.min() == tile.max()
    # tiles missing with probability 0.8 (3 x 4 tiles per frame, 7 frames: 84 tiles)
    frac_obs_tiles = np.mean([m[bi, bj, 0, f] for f in range(7) for bi in range(0, 40, 16)
                              for bj in range(0, 50, 16)])
    assert abs(frac_obs_tiles - 0.2) < 4 * math.sqrt(0.2 * 0.8 / 84)


@pytest.mark.parametrize("law", ["uniform_std", "saltpepper", "uniform01"])
def test_outliers_replace_only_observed_entries(law):
    dims = (30, 20, 25)
    w = synth.Workload("t", dims, (2, 2, 2), 0.3, 0.2, law, 10.0)
    g = np.random.default_rng(5)
    xstar = g.standard_normal(dims)
    mask = synth.bernoulli_mask(dims, w.rho, 5)
    X = synth.assemble(w, xstar, mask, 5)
    changed = X != xstar
    obs = mask.astype(bool)
    assert not np.any(changed & ~obs)                 # unobserved entries keep X*
    frac = changed[obs].mean()                        # about 20 % of the observed ones
    assert abs(frac - 0.2) < 4 * math.sqrt(0.2 * 0.8 / obs.sum())
    vals = X[changed]
    if law == "uniform_std":
        lim = 10.0 * np.std(xstar)
        assert np.all(np.abs(vals) <= lim)
        assert np.abs(vals).max() > 0.9 * lim         # spread over the whole range
    elif law == "saltpepper":
        mx = np.max(np.abs(xstar))
        assert set(np.unique(vals)) == {-mx, mx}
    else:
        assert np.all((vals >= 0.0) & (vals < 1.0))


def test_noise_variance():
    dims = (50, 40, 30)
    w = synth.Workload("t", dims, (2, 2, 2), 1.0, 0.0, "uniform_std", noise_var=1e-3)
    xstar = np.zeros(dims)
    X = synth.assemble(w, xstar, np.ones(dims, dtype=np.uint8), 2)
    n = X.size
    assert abs(X.var() - 1e-3) < 5 * 1e-3 * math.sqrt(2.0 / n)


def test_flat_core_layout_roundtrip():
    dims, ranks = (5, 4, 6), (2, 3, 4)
    Z = synth.gaussian_cores(dims, ranks, 0)
    flat = synth.cores_to_flat(Z)
    assert [f.size for f in flat] == [ranks[j] * dims[j] * ranks[(j + 1) % 3] for j in range(3)]
    back = synth.flat_to_cores(flat, dims, ranks)
    for a, b in zip(Z, back):
        np.testing.assert_array_equal(a, b)


def test_normalised_workload_keeps_exact_tr_rank():
    w = synth.scaled(synth.WORKLOADS["video_240x320x3x200_r8"], (32, 24, 3, 5))
    cores, xstar, mask, X = synth.make_workload(w, 0, tr.reconstruct)
    assert np.max(np.abs(xstar)) == pytest.approx(1.0)
    np.testing.assert_allclose(tr.reconstruct(cores), xstar, rtol=1e-12, atol=1e-12)
