"""The host recomputation of the full-size inputs (tests/_inputs.py) on small shapes of the
same recipes: its reconstruction, standard deviation and maximum against the oracle's
whole-tensor reconstruction, and its values against the recipe applied to whole arrays."""
import math

import numpy as np
import pytest

from oracle import rng as orng
from oracle import tr
from _inputs import OracleInputs, _noise_seed


@pytest.mark.parametrize("name,dims", [("tr5_60_r8", (5, 4, 3, 4, 2)), ("tr4_100_r5", (6, 5, 4, 3)),
                                       ("video_240x320x3x200_r8", (20, 18, 3, 4)),
                                       ("tr4_200_r10", (4, 3, 5, 2))])
def test_host_inputs_match_the_recipe_on_whole_arrays(name, dims):
    o = OracleInputs(name, 3, dims)
    X = tr.reconstruct(o.cores) * o.scale
    n = X.size
    lin = np.arange(n, dtype=np.int64)
    idx = np.stack(np.unravel_index(lin, dims, order="F"), axis=1)
    np.testing.assert_allclose(o.clean_at(idx), X.ravel(order="F"), rtol=1e-12, atol=1e-14)
    assert o.std_clean() == pytest.approx(float(np.std(X)), rel=1e-9)
    assert o.max_abs_clean() * o.scale == pytest.approx(float(np.max(np.abs(X))), rel=1e-12)
    if o.w.normalise_max:
        assert float(np.max(np.abs(X))) == pytest.approx(1.0, rel=1e-12)
    # the recipe on whole arrays: noise, then outliers on the selected observed entries
    w = o.w
    obs, sel, u = orng.sample_mask_at(3, dims, w.rho, o.block, w.outlier_frac, lin)
    x = X.ravel(order="F").copy()
    if w.noise_var > 0:
        u1 = orng.sample_mask(_noise_seed(3, 1), dims, 1.0)[2]
        u2 = orng.sample_mask(_noise_seed(3, 2), dims, 1.0)[2]
        x += np.sqrt(-2 * np.log1p(-u1)) * np.cos(2 * math.pi * u2) * math.sqrt(w.noise_var)
    p = sel.astype(bool)
    if w.outlier_law == "uniform_std":
        x[p] = (2 * u[p] - 1) * w.outlier_scale * np.std(X)
    elif w.outlier_law == "saltpepper":
        x[p] = np.where(u[p] < 0.5, -1.0, 1.0) * np.max(np.abs(X))
    else:
        x[p] = u[p]
    got_obs, got = o.entries(idx)
    np.testing.assert_array_equal(got_obs, obs)
    np.testing.assert_allclose(got, x, rtol=1e-9, atol=1e-12)
    # the observed entries of a slice, in column-major order
    for k in range(len(dims)):
        sl = o.mask_of_slice(k, 1)
        want = idx[(obs == 1) & (idx[:, k] == 1)]
        np.testing.assert_array_equal(sl, want)
