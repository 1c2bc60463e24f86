"""Parity at the workloads' full sizes, in the configurations bench.py times.

The oracle cannot unfold these tensors, so it computes sampled outputs one at a time.  The
device problem is built exactly as bench.py builds it; the oracle's inputs are recomputed
on the host from the seed alone (tests/_inputs.py: its own reconstruction and its own
counter generator), never read back from the device, and the two are checked against each
other at sampled entries (mask bit for bit, values to FP32 rounding).  Outputs compared:
  * reconstructed entries (Def. 1) at a uniform sample of positions;
  * whole gradient rows of eq. (9) from the observed entries of a slice (gradient_row);
  * the FGMC Gram matrix (eq. 13, cheap at any size) against the explicit sum of
    Kronecker factors;
  * RStS index sets (bit-exact) and the complete sketched gradient (eq. 15), whose
    subtensor the oracle can hold.
Bars: reconstruction 1e-5 relative; FP32 gradient rows 1e-4 relative Frobenius (a row sums
about 1e6 FP32 products, so its rounding grows like sqrt(n) 2^-24 ~ 6e-5); the BF16 forms
as in test_gpu_bf16 (2e-2); Gram 1e-12; index sets exact."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import bench  # noqa: E402
import synth  # noqa: E402
from oracle import awrtrd as aw  # noqa: E402
from oracle import rng as orng  # noqa: E402
from oracle import tr  # noqa: E402
from _helpers import rel  # noqa: E402
from _inputs import OracleInputs  # noqa: E402

import paper_2305_09044_amd as trd  # noqa: E402


class Full:
    """One workload at full size: device problem plus host copies for the oracle."""

    def __init__(self, name, seed=0, perturbed=False):
        w, dims, Xd, Pd, xs, cores_t = bench.build_inputs(name, seed)
        self.w, self.dims, self.seed = w, tuple(dims), seed
        self.prob = trd.Problem(Xd, Pd, dims, w.ranks)
        self.Xd, self.Pd, self.xs = Xd, Pd, xs
        self.n = int(np.prod(dims))
        self.oin = OracleInputs(name, seed)
        # the start of a fit, or (the differentiation form) the true cores perturbed
        Z = (synth.perturbed_cores(self.oin.cores, seed, rel=0.1) if perturbed
             else synth.init_cores(dims, w.ranks, seed))
        self.Z = [z.astype(np.float32).astype(np.float64) for z in Z]
        self.cores = [torch.from_numpy(f).cuda() for f in synth.cores_to_flat(self.Z, np.float32)]
        self.strides = np.cumprod((1,) + self.dims[:-1])
        self._rows = {}

    def oracle_row(self, k, i, sigma):
        key = (k, i, sigma)
        if key not in self._rows:
            idx, vals = self.slice_entries(k, i)
            self._rows[key] = aw.gradient_row(self.Z, k, idx, vals, sigma)
        return self._rows[key]

    def slice_entries(self, k, i):
        """Indices (n, N) and values of the observed entries with i_k = i (host recipe)."""
        idx = self.oin.mask_of_slice(k, i)
        _, vals = self.oin.entries(idx)
        return idx, vals

    def check_inputs(self, n=1 << 16, seed=3):
        """device mask == host mask bit for bit, device X == host X to FP32 rounding, at a
        uniform sample of entries"""
        lin = np.random.default_rng(seed).integers(0, self.n, n)
        idx = np.stack(np.unravel_index(lin, self.dims, order="F"), axis=1)
        obs, vals = self.oin.entries(idx)
        li = torch.from_numpy(lin).cuda()
        np.testing.assert_array_equal(self.Pd[li].cpu().numpy(), obs)
        got = self.Xd[li].cpu().numpy().astype(np.float64)
        scale = float(np.max(np.abs(vals)))
        err = float(np.max(np.abs(got - vals))) / scale
        assert err <= 1e-6, err
        return obs, vals

    def close(self):
        self.prob.close()
        del self.prob, self.Xd, self.Pd, self.xs, self.cores, self.oin
        torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def cfg_prec():
    f = Full("tr5_60_r8")
    f.check_inputs()
    yield f
    f.close()


def _grad_rows(f, k, rows, sigma, prec):
    f.prob.set_precision(prec)
    d, stats = f.prob.grad(f.cores, k, sigma)
    f.prob.set_precision("native")
    r, r2 = f.w.ranks[k], f.w.ranks[(k + 1) % len(f.dims)]
    D = d.cpu().numpy().astype(np.float64).reshape(f.dims[k], r2 * r)
    return [(D[i], f.oracle_row(k, i, sigma)) for i in rows], stats


@pytest.mark.parametrize("prec,bar", [("native", 1e-4), ("bf16x3", 2e-2), ("bf16", 2e-2)])
def test_precision_workload_gradient_rows(cfg_prec, prec, bar):
    # 60^5, rank 8, 10% observed: rows of d for a first and a middle core
    f = cfg_prec
    sigma = 1.0
    worst = 0.0
    for k, rows in ((0, (0, 37)), (1, (59,)), (2, (59,)), (3, (11,)), (4, (30,))):
        pairs, stats = _grad_rows(f, k, rows, sigma, prec)
        for got, ref in pairs:
            e = rel(got, ref)
            worst = max(worst, e)
            assert e <= bar, (prec, k, e)
    print(f"{prec}: worst gradient-row error {worst:.2e}")


def test_precision_workload_reconstruction_and_gram(cfg_prec):
    f = cfg_prec
    g = np.random.default_rng(7)
    n = int(np.prod(f.dims))
    lin = np.sort(g.choice(n, 4096, replace=False)).astype(np.int64)
    got = f.prob.reconstruct(f.cores, torch.from_numpy(lin).cuda()).cpu().numpy()
    ref = tr.reconstruct_at(f.Z, lin)
    assert rel(got, ref) <= 1e-5
    for k in (0, 3):
        G = f.prob.fgmc_gram(f.cores, k).cpu().numpy()
        assert rel(G, aw.gram_fgmc(f.Z, k)) <= 1e-12


@pytest.mark.parametrize("prec,bar", [("native", 1e-3), ("bf16x3", 2e-2), ("bf16", 2e-2)])
def test_precision_workload_step_rows_follow_the_scaled_direction(cfg_prec, prec, bar):
    # one full-size step on core 1: the change of a sampled row is eta times that row of the
    # oracle's scaled direction h = d (G + lambda I)^{-1} (eq. 10), with d the oracle's
    # gradient row and G its FGMC Gram; the common factor is the step's eta (eq. 11)
    f = cfg_prec
    sigma, k, lam_rel = 1.0, 1, 1e-9
    G = aw.gram_fgmc(f.Z, k)
    C = G + lam_rel * np.trace(G) / G.shape[0] * np.eye(G.shape[0])
    cores = [c.clone() for c in f.cores]
    f.prob.set_precision(prec)
    eta, flags = f.prob.step(cores, k, sigma, lam_rel)
    f.prob.set_precision("native")
    assert int(flags) == 0
    r, r2 = f.w.ranks[k], f.w.ranks[(k + 1) % len(f.dims)]
    new = cores[k].cpu().numpy().astype(np.float64).reshape(f.dims[k], r2 * r)
    old = f.cores[k].cpu().numpy().astype(np.float64).reshape(f.dims[k], r2 * r)
    for i in (59,):
        h = np.linalg.solve(C, f.oracle_row(k, i, sigma))   # C symmetric: d C^{-1} row-wise
        delta = new[i] - old[i]
        est = float(delta @ h / (h @ h))
        assert rel(delta, est * h) <= bar, (prec, i, rel(delta, est * h))
        assert est == pytest.approx(float(eta), rel=bar), (prec, est, float(eta))


def test_precision_workload_step_decreases_loss(cfg_prec):
    # at full size the line search is checked by what it guarantees: a positive step that
    # lowers the frozen-weight objective, in each timed precision
    f = cfg_prec
    sigma = 1.0
    for prec in ("native", "bf16x3", "bf16"):
        cores = [c.clone() for c in f.cores]
        f.prob.set_precision("native")
        before = float(f.prob.loss_fwd(cores, sigma))
        f.prob.set_precision(prec)
        eta, flags = f.prob.step(cores, 1, sigma)
        f.prob.set_precision("native")
        after = float(f.prob.loss_fwd(cores, sigma))
        assert int(flags) == 0 and float(eta) > 0.0, prec
        assert after < before, (prec, before, after)


@pytest.mark.parametrize("name", ["tr4_100_r5", "video_240x320x3x200_r8"])
def test_sketch_workloads_full_size(name):
    # RStS at the workloads' sketch sizes: index sets bit-exact, sketched gradient complete
    f = Full(name)
    try:
        f.check_inputs()
        sizes = list(f.w.sketch)
        sigma = 0.5
        for t, k in ((0, 0), (3, len(f.dims) - 1)):
            got = trd.trd_sample_sketch(11, t, k, f.dims, sizes)
            ref = orng.sketch_indices(11, t, k, f.dims, sizes)
            for j in range(len(f.dims)):
                assert got[j].cpu().numpy().tolist() == ref[j]
            sk, _ = trd.make_sketch(sizes, 11, t)
            d, stats = f.prob.grad(f.cores, k, sigma, sketch=sk)
            # the sketched subtensor from the host recipe (column-major over the sketch)
            grid = np.meshgrid(*[np.asarray(s, dtype=np.int64) for s in ref], indexing="ij")
            idx = np.stack([g.ravel(order="F") for g in grid], axis=1)
            obs, vals = f.oin.entries(idx)
            shape = [len(s) for s in ref]
            Xs = vals.reshape(shape, order="F")
            Ps = obs.reshape(shape, order="F")
            cs = [z[:, np.asarray(s), :] for z, s in zip(f.Z, ref)]
            _, info = aw.core_update(Xs, Ps, cs, k, sigma)
            r, r2 = f.w.ranks[k], f.w.ranks[(k + 1) % len(f.dims)]
            D = d.cpu().numpy().astype(np.float64).reshape(f.dims[k], r2 * r)
            assert rel(D, info.d) <= 1e-4, (name, t, k)
            assert int(stats[2].item()) == int(Ps.sum())
    finally:
        f.close()


@pytest.fixture(scope="module")
def cfg_diff():
    f = Full("tr4_200_r10", perturbed=True)
    f.check_inputs()
    yield f
    f.close()


def test_differentiation_workload_pattern_bit_exact(cfg_diff):
    # 200^4 mask and outlier selection from the device sampler, against the oracle's
    # generator at a uniform sample of entries (and the observed count it implies)
    f = cfg_diff
    w = f.w
    g = np.random.default_rng(3)
    lin = g.integers(0, f.n, 1 << 16)
    m, sel, u = orng.sample_mask_at(f.seed, f.dims, w.rho, 0, w.outlier_frac, lin)
    li = torch.from_numpy(lin).cuda()
    np.testing.assert_array_equal(f.Pd[li].cpu().numpy(), m)
    # where an observed entry was not selected as an outlier it keeps its clean value
    keep = (m == 1) & (sel == 0)
    np.testing.assert_array_equal(f.Xd[li].cpu().numpy()[keep], f.xs[li].cpu().numpy()[keep])
    assert abs(f.prob.info()["n_obs"] / f.n - w.rho) < 1e-4


@pytest.mark.parametrize("prec,bar", [("native", 1e-4), ("bf16", 2e-2)])
def test_differentiation_workload_backward_rows(cfg_diff, prec, bar):
    # the all-core backward at 200^4, rank 10 (r_k r_{k+1} = 100, K = 128): rows of dL/dZ_k
    # for every core against minus the oracle's gradient row at the same point
    f = cfg_diff
    sigma = 0.8
    f.prob.set_precision(prec)
    grads = f.prob.loss_bwd(f.cores, sigma)
    f.prob.set_precision("native")
    worst = 0.0
    for k, i in ((0, 0), (1, 117), (2, 199), (3, 64)):
        r, r2 = f.w.ranks[k], f.w.ranks[(k + 1) % 4]
        G = grads[k].cpu().numpy().astype(np.float64).reshape(f.dims[k], r2 * r)
        e = rel(-G[i], f.oracle_row(k, i, sigma))
        worst = max(worst, e)
        assert e <= bar, (prec, k, i, e)
    print(f"{prec}: 200^4 rank-10 backward, worst row error {worst:.2e}")
