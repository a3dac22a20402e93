"""Pins of the oracle's filter steps (Fig. 1: update, estimation, resampling,
prediction) and of the whole SMC (CPU only): invariants, exact integer
properties of systematic resampling, Box-Muller statistics, brute force over
a small transform grid, a one-parameter filter against its posterior by
quadrature, and recovery of known synthetic transforms."""

import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import synth


def _params(**kw):
    lim = kw.pop("limit", list(np.deg2rad([15.0] * 3)) + [8.0] * 3)
    p = dict(n_particles=64, n_iters=5, seed=7, score="dice", limit=lim, sigma_score=0.02,
             sigma0=list(0.15 * np.asarray(lim)), anneal=0.85)
    p.update(kw)
    return p


def geodesic_deg(p, q, orc):
    R1, R2 = orc.euler_R(p[:3]), orc.euler_R(q[:3])
    return float(np.degrees(np.arccos(np.clip((np.trace(R1.T @ R2) - 1) / 2, -1, 1))))


# ------------------------------------------------------------------ update / normalise

def test_loglik_shape(orc):
    assert orc.loglik(1.0, "dice", 0.02) == 0.0
    assert orc.loglik(0.0, "ssd", 0.1) == 0.0
    assert orc.loglik(-np.inf, "ncc", 0.02) == -np.inf
    zs = np.linspace(0, 1, 11)
    ll = [orc.loglik(z, "ncc", 0.05) for z in zs]
    assert np.all(np.diff(ll) > 0)
    # a Gaussian in the deficit: doubling the deficit quadruples the log-likelihood
    assert abs(orc.loglik(0.8, "dice", 0.05) / orc.loglik(0.9, "dice", 0.05) - 4.0) < 1e-12


def test_normalise_invariants(orc):
    rng = np.random.default_rng(0)
    lw = rng.normal(-50, 10, 300)
    x = rng.normal(size=(300, 6))
    a = orc.normalise(lw, x)
    assert a["w"].max() == 1.0 and not a["degenerate"]
    wn = a["w"] / a["w"].sum()
    assert abs(wn.sum() - 1.0) < 1e-15
    assert np.allclose(a["est"], np.average(x, axis=0, weights=a["w"]), rtol=0, atol=1e-13)
    assert abs(a["ess"] - 1.0 / np.sum(wn * wn)) < 1e-10
    b = orc.normalise(lw + 123.25, x)  # shift invariance
    assert np.allclose(b["w"], a["w"], rtol=1e-13, atol=0) and np.allclose(b["est"], a["est"], atol=1e-13)
    eq = orc.normalise(np.zeros(50), x[:50])
    assert abs(eq["ess"] - 50) < 1e-12
    one = np.full(50, -np.inf)
    one[17] = -3.0
    o = orc.normalise(one, x[:50])
    assert o["ess"] == 1.0 and np.array_equal(o["est"], x[17])
    d = orc.normalise(np.full(10, -np.inf), x[:10])
    assert d["degenerate"] and np.allclose(d["est"], x[:10].mean(0), atol=1e-15)


# ------------------------------------------------------------------ resampling

def _resample_bigint(w, u32):
    n = len(w)
    q = [int(np.floor(v * 2.0 ** 48)) for v in w]
    Q = sum(q)
    C = list(itertools.accumulate(q))
    out = []
    for j in range(n):
        pointer = (Fraction(j) + Fraction(u32, 2 ** 32)) * Fraction(Q, n)
        out.append(next(i for i, c in enumerate(C) if c > pointer))
    return out, q, Q


def test_systematic_resampling_exact(orc):
    rng = np.random.default_rng(1)
    for n in (1, 2, 7, 64, 257):
        for _ in range(5):
            w = np.exp(rng.normal(0, 3, n))
            w /= w.max()
            w[rng.random(n) < 0.2] = 0.0
            w[int(rng.integers(n))] = 1.0
            u = int(rng.integers(0, 2 ** 32))
            anc = orc.resample(w, u)
            ref, q, Q = _resample_bigint(w, u)
            assert list(anc) == ref
            counts = np.bincount(anc, minlength=n)
            assert counts.sum() == n and np.all(np.diff(anc) >= 0)
            for i in range(n):
                lo = (n * q[i]) // Q
                assert counts[i] in (lo, lo + 1) if (n * q[i]) % Q else counts[i] == lo


def test_equal_weights_resample_to_identity(orc):
    for u in (0, 1, 2 ** 31, 2 ** 32 - 1):
        assert np.array_equal(orc.resample(np.ones(33), u), np.arange(33))


def test_resampling_at_the_particle_limit(orc):
    """Flat weights (every particle scored alike, e.g. no overlap anywhere) at
    the largest particle count still give every particle one copy: the CDF
    total, N 2^48, stays below 2^64.  One particle more would wrap it, so the
    oracle (like the library) refuses N = 65536."""
    n = orc.MAX_PARTICLES
    assert n == 2 ** 16 - 1
    for u in (0, 2 ** 32 - 1):
        assert np.array_equal(orc.resample(np.ones(n), u), np.arange(n))
    with pytest.raises(ValueError):
        orc.resample(np.ones(n + 1), 0)
    with pytest.raises(ValueError):
        orc.filter_update(dict(n_particles=n + 1, n_iters=2, limit=[0.1] * 6, sigma_score=0.01, sigma0=[0.0] * 6),
                          1, np.zeros((n + 1, 6)), np.zeros(n + 1))


# ------------------------------------------------------------------ random draws

def test_box_muller_normals(orc):
    g = np.array([orc.gauss6(11, 0, j, 3) for j in range(20000)])
    assert np.all(np.abs(g.mean(0)) < 0.03) and np.all(np.abs(g.var(0) - 1) < 0.04)
    assert stats.kstest(g.ravel(), "norm").pvalue > 0.01
    c = np.corrcoef(g.T)
    assert np.max(np.abs(c - np.eye(6))) < 0.03
    assert not np.array_equal(orc.gauss6(11, 0, 5, 3), orc.gauss6(11, 1, 5, 3))  # pair id in counter
    assert not np.array_equal(orc.gauss6(11, 0, 5, 3), orc.gauss6(11, 0, 5, 4))  # iteration in counter


def test_box_muller_ten_million_draws(orc):
    """10^7 normals through the prediction step itself (unit width, no
    annealing, limits far away, zero parents): pooled mean and variance
    within 1e-3, normal by Kolmogorov-Smirnov, axes uncorrelated."""
    n = 10_000_000 // 6 + 1
    prm = dict(n_particles=n, n_iters=2, seed=2024, limit=[1e6] * 6, sigma0=[1.0] * 6, anneal=1.0,
               sigma_score=0.1)
    g = orc.perturb(prm, 1, np.zeros((n, 6)), np.arange(n, dtype=np.int32))
    x = g.ravel()
    assert abs(x.mean()) < 1e-3 and abs(x.var() - 1.0) < 1e-3
    assert stats.kstest(x, "norm").pvalue > 0.01
    assert np.abs(np.corrcoef(g.T) - np.eye(6)).max() < 5e-3


def test_init_uniform_in_limits(orc):
    p = _params(n_particles=20000, x0=[0.1, -0.1, 0.0, 1.0, 2.0, -3.0])
    x = orc.init_particles(p)
    lo = np.asarray(p["x0"]) - np.asarray(p["limit"])
    u = (x - lo) / (2 * np.asarray(p["limit"]))
    assert np.all((u > 0) & (u <= 1))
    for d in range(6):
        assert stats.kstest(u[:, d], "uniform").pvalue > 0.01


def test_perturb_reflects_and_anneals(orc):
    p = _params(n_particles=4000, sigma0=[0.0] * 6)
    x = orc.init_particles(p)
    anc = np.arange(4000, dtype=np.int32)[::-1].copy()
    assert np.array_equal(orc.perturb(p, 2, x, anc), x[anc])
    p = _params(n_particles=4000)
    xm = np.tile(np.asarray(p.get("x0", [0] * 6), float), (4000, 1))
    k = 3
    d = orc.perturb(p, k, xm, np.zeros(4000, np.int32)) - xm
    sig = np.asarray(p["sigma0"]) * p["anneal"] ** (k - 1)
    assert np.allclose(d.std(0) / sig, 1.0, atol=0.05)
    big = _params(n_particles=4000, sigma0=[1.0] * 3 + [30.0] * 3)
    y = orc.perturb(big, 1, xm, np.zeros(4000, np.int32))
    assert np.all(np.abs(y) <= np.asarray(big["limit"]) + 1e-12)


def test_last_iteration_does_not_resample(orc):
    p = _params(n_particles=16, n_iters=3)
    x = orc.init_particles(p)
    z = np.linspace(0.1, 0.9, 16)
    r = orc.filter_update(p, 3, x, z)
    assert np.all(r["anc"] == -1)
    r = orc.filter_update(p, 2, x, z)
    assert np.all(r["anc"] >= 0)


# ------------------------------------------------------------------ whole SMC

def test_smc_deterministic(orc):
    pair = synth.shell_pair(seed=2, side=32)
    p = _params(n_particles=64, n_iters=4, limit=list(np.deg2rad([15.0] * 3)) + [4.0] * 3)
    a = orc.smc_run(pair["src"], pair["tgt"], p)
    b = orc.smc_run(pair["src"], pair["tgt"], p)
    assert np.array_equal(a["est"], b["est"]) and np.array_equal(a["states"], b["states"])
    assert np.array_equal(a["trace_score"], b["trace_score"])


def _toy_pair(shift):
    """24^3 smooth asymmetric blobs; the source is the target moved by
    +shift voxels along x, so only t_x matters and its true value is shift."""
    g = np.arange(24, dtype=float)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")

    def blob(xx):
        return (40 + 150 * np.exp(-((xx - 11) ** 2 / 18.0 + (Y - 12) ** 2 / 32.0 + (Z - 12) ** 2 / 50.0))
                + 30 * np.exp(-((xx - 16) ** 2 + (Y - 9) ** 2 + (Z - 14) ** 2) / 8.0))
    return np.round(blob(X - shift)).astype(np.uint8), np.round(blob(X)).astype(np.uint8)


def test_one_parameter_filter_matches_quadrature(orc):
    """Only t_x free (limit 3 voxels, truth 2.4, so the prior box truncates
    the posterior).  After one iteration the estimate is the self-normalised
    importance-sampling mean of the posterior prior x likelihood; after two
    it is the mean of likelihood x (reflected Gaussian prediction of the
    first posterior).  Both are computed by quadrature on 2401 nodes from the
    oracle's own scores and must agree within four Monte Carlo standard
    errors; a likelihood with sigma^2 for 2 sigma^2 or without the square
    moves the mean by more than ten."""
    from scipy.stats import norm
    src, tgt = _toy_pair(2.4)
    L, s0, ss = 3.0, 0.5, 0.05
    prm = dict(n_particles=16384, n_iters=1, seed=0, score="ncc", interp="trilinear", sigma_score=ss,
               limit=[0, 0, 0, L, 0, 0], sigma0=[0, 0, 0, s0, 0, 0], anneal=0.9)
    xs = np.linspace(-L, L, 2401)
    st = np.zeros((len(xs), 6))
    st[:, 3] = xs
    z = orc.Problem(orc.Volume(src), orc.Volume(tgt)).score(prm, st)
    ll = np.array([orc.loglik(v, "ncc", ss) for v in z])
    lik = np.exp(ll - ll.max())

    def mean_of(dens):
        return np.trapezoid(xs * dens, xs) / np.trapezoid(dens, xs)
    m1 = mean_of(lik)
    p1 = lik / np.trapezoid(lik, xs)
    ker = (norm.pdf(xs[:, None] - xs[None, :], scale=s0) + norm.pdf(2 * L - xs[:, None] - xs[None, :], scale=s0)
           + norm.pdf(-2 * L - xs[:, None] - xs[None, :], scale=s0))
    m2 = mean_of(lik * np.trapezoid(ker * p1[None, :], xs, axis=1))
    for K, want in ((1, m1), (2, m2)):
        for seed in (0, 1):
            r = orc.smc_run(src, tgt, dict(prm, n_iters=K, seed=seed))
            w = np.exp(r["logw"] - r["logw"].max())
            w /= w.sum()
            tx = r["states"][:, 3]
            assert np.all(r["states"][:, [0, 1, 2, 4, 5]] == 0.0)
            assert abs(np.sum(w * tx) - r["est"][3]) < 1e-12
            se = np.sqrt(np.sum(w ** 2 * (tx - r["est"][3]) ** 2))
            assert abs(r["est"][3] - want) < 4 * se, (K, seed, r["est"][3], want, se)
    for wrong in (2 * ll, -(1 - z) / (2 * ss ** 2)):
        assert abs(mean_of(np.exp(wrong - wrong.max())) - m1) > 10 * 0.007


def test_smc_brute_force_grid(orc):
    """Small exhaustive search: 24^3 filled ellipsoid (semi-axes 10/7/4.5), grid
    {-10,-5,0,5,10} deg x {-2..2} voxels (5^6 points).  The brute-force argmax sits at the truth and the SMC
    estimate lies within one grid step of it."""
    ang = np.deg2rad([-10, -5, 0, 5, 10])
    tr = np.arange(-2, 3, dtype=float)
    gt = np.array([np.deg2rad(5), np.deg2rad(-5), 0.0, 1.0, -1.0, 2.0])
    pair = synth.mask_pair((24, 24, 24), outer=(10.0, 7.0, 4.5), inner=None, gt=gt)
    grid = np.array(list(itertools.product(ang, ang, ang, tr, tr, tr)))
    pb = orc.Problem(pair["src"], pair["tgt"])
    lim = list(np.deg2rad([12.5] * 3)) + [2.5] * 3
    p = _params(limit=lim)
    z = pb.score(p, grid)
    best = grid[np.argmax(z)]
    assert np.allclose(best, gt) and np.sum(z == z.max()) == 1
    r = orc.smc_run(pair["src"], pair["tgt"], _params(limit=lim, n_particles=256, n_iters=12))
    est = r["est"]
    assert np.all(np.abs(est[:3] - best[:3]) <= np.deg2rad(5)) and np.all(np.abs(est[3:] - best[3:]) <= 1.0)


def test_smc_recovers_mask_transforms(orc):
    """Recovery of known transforms of filled ellipsoids: median over ten
    seeds within 1 degree and 1 voxel."""
    errs = []
    for seed in range(1, 11):
        pair = synth.mask_pair((64, 64, 64), outer=(24, 16, 10), inner=None, seed=seed)
        r = orc.smc_run(pair["src"], pair["tgt"], _params(n_particles=256, n_iters=15, seed=seed,
                                                             sigma_score=0.01))
        errs.append((geodesic_deg(r["est"], pair["gt"], orc), np.linalg.norm(r["est"][3:] - pair["gt"][3:])))
        assert r["trace_score"][-1] > r["trace_score"][0]
    errs = np.array(errs)
    assert np.median(errs[:, 0]) <= 1.0 and np.median(errs[:, 1]) <= 1.0, errs


def test_smc_recovers_image_transform_ncc(orc):
    """Recovery of known transforms of speckle images through the cone FOV
    with NCC: median over ten seeds within 1 degree and 1 voxel."""
    errs = []
    for seed in range(1, 11):
        pair = synth.speckle_pair(side=48, seed=seed, trans=12 * 48 / 160)
        src = orc.Volume(pair["src"], fov=pair["src_fov"])
        lim = list(np.deg2rad([20.0] * 3)) + [12 * 48 / 160] * 3
        r = orc.smc_run(src, pair["tgt"], _params(n_particles=384, n_iters=15, seed=seed, score="ncc",
                                                   limit=lim))
        errs.append((geodesic_deg(r["est"], pair["gt"], orc), np.linalg.norm(r["est"][3:] - pair["gt"][3:])))
    errs = np.array(errs)
    assert np.median(errs[:, 0]) <= 1.0 and np.median(errs[:, 1]) <= 1.0, errs


def test_proposal_draw_and_importance_correction(orc):
    """Truncated-Gaussian prior draw: inside the box, Gaussian away from the
    walls; and exp(lq) are importance weights from q to the uniform prior
    (self-normalised IS mean of x equals the box centre)."""
    lim = np.array([0.3, 0.3, 0.3, 8.0, 8.0, 8.0])
    x0 = np.array([0.05, -0.02, 0.0, 1.0, -2.0, 0.5])
    mu = x0 + np.array([0.1, -0.05, 0.0, 2.0, 1.0, -1.5])
    sd = np.array([0.02, 0.02, 0.02, 0.5, 0.5, 0.5])
    p = _params(n_particles=20000, x0=list(x0), limit=list(lim),
                proposal=dict(mean=list(mu), logvar=list(2 * np.log(sd))))
    x, lq = orc.init_proposal(p)
    assert np.all(np.abs(x - x0) <= lim + 1e-12)
    for d in range(6):
        assert stats.kstest((x[:, d] - mu[d]) / sd[d], "norm").pvalue > 0.01
    assert np.allclose(lq, 0.5 * np.sum(((x - mu) / sd) ** 2, axis=1), rtol=1e-12)
    wide = _params(n_particles=40000, x0=list(x0), limit=list(lim),
                   proposal=dict(mean=list(mu), logvar=list(2 * np.log(lim * 0.8))))
    xw, lqw = orc.init_proposal(wide)
    w = np.exp(lqw - lqw.max())
    est = (w[:, None] * xw).sum(0) / w.sum()
    ess = w.sum() ** 2 / (w * w).sum()
    assert np.all(np.abs(est - x0) < 4 * lim / np.sqrt(3 * ess)), (est, x0)


# ------------------------------------------------------------------ learned-proposal label and map

def test_cloud_moments_against_numpy(orc):
    """The label of the learned proposal: numpy's weighted average and
    weighted variance under the softmax of the log-weights, in units of the
    limits about x0; invariant to a shift of every log-weight; uniform when
    every weight is -inf; floored variance."""
    rng = np.random.default_rng(21)
    n = 300
    x0 = np.array([0.1, -0.05, 0.02, 3.0, -2.0, 1.0])
    L = np.array([0.3, 0.25, 0.2, 12.0, 10.0, 8.0])
    x = x0 + L * rng.uniform(-1, 1, (n, 6))
    lw = rng.normal(0, 4, n)
    lw[rng.random(n) < 0.1] = -np.inf
    w = np.exp(lw - lw.max())
    m = np.average(x, axis=0, weights=w)
    v = np.average((x - m) ** 2, axis=0, weights=w)
    mean, var = orc.cloud_moments(lw, x, x0, L)
    assert np.allclose(mean, (m - x0) / L, rtol=1e-12, atol=1e-14)
    assert np.allclose(var, v / L ** 2, rtol=1e-11, atol=0)
    mean2, var2 = orc.cloud_moments(lw + 123.5, x, x0, L)
    assert np.allclose(mean2, mean, rtol=1e-12, atol=1e-14) and np.allclose(var2, var, rtol=1e-11)
    mu, vu = orc.cloud_moments(np.full(n, -np.inf), x, x0, L)
    assert np.allclose(mu, (x.mean(0) - x0) / L, atol=1e-13) and np.allclose(vu, x.var(0) / L ** 2, rtol=1e-11)
    one = np.full(n, -np.inf)
    one[17] = 0.0
    m1, v1 = orc.cloud_moments(one, x, x0, L, var_floor=1e-4)
    assert np.allclose(m1, (x[17] - x0) / L, atol=1e-14) and np.all(v1 == 1e-4)


def test_proposal_from_network_closed_forms(orc):
    """Zero outputs give the box centre and the variance var_scale L^2;
    outputs are clipped (means to the box, log-variances to [-20, 2]); and
    the network's own label format maps back to the cloud it summarises."""
    x0 = np.array([0.1, -0.05, 0.02, 3.0, -2.0, 1.0])
    L = np.array([0.3, 0.25, 0.2, 12.0, 10.0, 8.0])
    m, lv = orc.proposal_from_network(np.zeros(12), x0, L, 4.0)
    assert np.allclose(m, x0, atol=1e-15) and np.allclose(np.exp(lv), 4.0 * L ** 2, rtol=1e-14)
    out = np.array([2.0, -3.0, 0.5, -0.25, 1.0, -1.0, 5.0, -30.0, 0.0, -1.0, 2.0, -20.0], np.float32)
    m, lv = orc.proposal_from_network(out, x0, L, 1.0)
    assert np.allclose(m, x0 + L * np.array([1.0, -1.0, 0.5, -0.25, 1.0, -1.0]), atol=1e-15)
    assert np.allclose(lv - 2 * np.log(L), [2.0, -20.0, 0.0, -1.0, 2.0, -20.0], atol=1e-14)
    rng = np.random.default_rng(5)
    x = x0 + L * rng.uniform(-0.3, 0.3, (64, 6))
    lw = rng.normal(0, 1, 64)
    mean, var = orc.cloud_moments(lw, x, x0, L)
    label = np.concatenate([mean, np.log(var)]).astype(np.float32)
    m, lv = orc.proposal_from_network(label, x0, L, 1.0)
    w = np.exp(lw - lw.max())
    xm = np.average(x, axis=0, weights=w)
    assert np.allclose(m, xm, rtol=1e-6, atol=1e-6 * L)
    assert np.allclose(np.exp(lv), np.average((x - xm) ** 2, axis=0, weights=w), rtol=1e-6)
