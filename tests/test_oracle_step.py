"""Pins of the oracle's FCIQMC step [Sec. 3] against closed forms and the
paper's printed numbers."""
import math

import numpy as np
import pytest

from oracle import stats


def _dense_T(orc, h, addrs, vals, S, dtau):
    """Deterministic T c = (1 + dtau (S - H)) c over the ranked basis."""
    H = orc.csr_matrix(h)
    D = H.shape[0]
    c = np.zeros(D)
    for a, v in zip(addrs, vals):
        c[orc.rank(a, h.M, h.N)] += v
    return c + dtau * (S * c - H @ c), H


def _to_dense(orc, h, addrs, vals):
    D = orc.dimension(h.M, h.N)
    c = np.zeros(D)
    for a, v in zip(addrs, vals):
        c[orc.rank((int(a[0]), int(a[1])), h.M, h.N)] += v
    return c


@pytest.mark.parametrize("model,M,N,u,dtau,early", [(0, 5, 5, 6.0, 0.01, False), (1, 5, 4, 3.0, 0.01, False),
                                                    (0, 2, 3, 2.0, 0.02, False), (0, 5, 5, 6.0, 0.01, True),
                                                    (1, 5, 4, 3.0, 0.01, True)])
def test_step_unbiased(orc, model, M, N, u, dtau, early):
    """E[T~ c] = T c (Sec. 3.2): average over seeds of the full stochastic
    step (matrix compression + late vector compression, or early
    compression of every contribution, Sec. 7.1) equals the deterministic
    product, checked within 5 standard errors per entry."""
    rng = np.random.default_rng(17)
    D = orc.dimension(M, N)
    idx = rng.choice(D, size=min(D, 12), replace=False)
    addrs = [orc.unrank(int(i), M, N) for i in idx]
    vals = rng.choice([-1, 1], len(idx)) * rng.uniform(0.2, 40.0, len(idx))
    S = -1.3
    h = orc.ham(model, M, N, 1.0, u)
    Tc, _ = _dense_T(orc, h, addrs, vals, S, dtau)
    nseed = 3000
    acc = np.zeros(D)
    acc2 = np.zeros(D)
    ref = addrs[0]
    for s in range(nseed):
        P = orc.params(model, M, N, 1.0, u, dtau=dtau, target=100.0, seed=1000 + s, early=early)
        out = orc.step(P, addrs, vals, S, 7, ref, 1.0)
        x = _to_dense(orc, h, out["addr"], out["val"])
        acc += x
        acc2 += x * x
    mean = acc / nseed
    sd = np.sqrt(np.maximum(acc2 / nseed - mean ** 2, 0.0) / nseed)
    z = np.abs(mean - Tc) / np.maximum(sd, 1e-9)
    assert np.all((np.abs(mean - Tc) < 1e-9) | (z < 5.0)), z.max()


@pytest.mark.parametrize("model", [0, 1])
def test_exact_columns_give_deterministic_product(orc, model):
    """Every |c| >= t_rel m and every resulting |w| >= theta: the step is the
    deterministic power-method step (Sec. 3.1) up to rounding."""
    M, N = (6, 4) if model == 0 else (5, 4)
    h = orc.ham(model, M, N, 1.0, 2.0)
    D = orc.dimension(M, N)
    addrs = [orc.unrank(i, M, N) for i in range(D)]
    vals = np.full(D, 1000.0) + np.arange(D)
    S, dtau = -2.0, 1e-3
    P = orc.params(model, M, N, 1.0, 2.0, dtau=dtau, target=1e5, seed=1)
    out = orc.step(P, addrs, vals, S, 3, addrs[0], 1.0)
    Tc, H = _dense_T(orc, h, addrs, vals, S, dtau)
    got = _to_dense(orc, h, out["addr"], out["val"])
    assert np.allclose(got, Tc, rtol=1e-13, atol=0)
    assert out["stats"]["exact_steps"] == D and out["stats"]["inexact_steps"] == 0
    # the projected energy numerator is y^T H c, the denominator y^T c
    c = got
    y = np.zeros(D)
    y[0] = 1.0
    assert math.isclose(out["stats"]["hproj"], y @ (H @ c), rel_tol=1e-13)
    assert out["stats"]["vproj"] == c[0]


def test_printed_step_two_norm_reconstruction(orc):
    """Sec. 4 printed rows 1-2 (6/6, u = 6, dtau = 0.01): after step 1 the
    vector holds 10 walkers on the uniform state and 1 on a neighbour; the
    printed step-2 norm 12.1052 equals the two diagonal survivors computed
    with S^(1) = -0.0409038, one spawn of weight (m/n)(-dtau H) c merged onto
    the neighbour, and one newly created entry of value 1."""
    M = N = 6
    h = orc.ham(orc.REAL1D, M, N, 1.0, 6.0)
    uni = orc.encode([1] * 6)
    d0, dest, hv = orc.column(h, uni)
    nb = (int(dest[0][0]), int(dest[0][1]))
    d1, _, _ = orc.column(h, nb)
    S1 = orc.shift_update(0.0, 11.0, 10.0, 1000.0, 0.08, 0.0016, 0.01)
    P = orc.params(orc.REAL1D, M, N, 1.0, 6.0, dtau=0.01, target=1000.0, seed=0)
    out = orc.step(P, [uni, nb], [10.0, 1.0], S1, 2, uni, 10.0, events=True)
    ev = out["events"]
    big = ev[ev["parent"] == 0]["value"]
    assert len(big) == 10 and np.all(big == big[0])          # ceil(10) picks
    spawn = big[0]
    assert spawn == (-(0.01 * hv[0])) * 10.0 * (12.0 / 10.0)
    recon = 10.0 * (1 + 0.01 * (S1 - d0)) + 1.0 * (1 + 0.01 * (S1 - d1)) + spawn + 1.0
    assert round(recon, 4) == 12.1052


def test_compression_probability(orc):
    """Vector compression (Eq. vec-compression): an isolated merged value
    |w| < theta survives as sign(w) theta with probability |w| / theta."""
    M = N = 8
    h = orc.ham(orc.REAL1D, M, N, 1.0, 1.0)
    rng = np.random.default_rng(4)
    D = orc.dimension(M, N)
    idx = rng.choice(D, 400, replace=False)
    addrs = [orc.unrank(int(i), M, N) for i in idx]
    theta = 0.5
    kept = 0
    trials = 0
    for s in range(10):
        # dtau tiny: survivors ~ c, spawns ~ 1e-9 and die
        P = orc.params(orc.REAL1D, M, N, 1.0, 1.0, dtau=1e-12, target=1.0, theta=theta, seed=s)
        out = orc.step(P, addrs, np.full(400, 0.2), 0.0, 1, addrs[0], 1.0)
        v = out["val"]
        assert np.all(np.abs(v) >= theta)
        big = np.abs(v) >= 0.49
        kept += int(np.sum(big))
        trials += 400
    p = kept / trials
    assert abs(p - 0.4) < 5 * math.sqrt(0.4 * 0.6 / trials)


def test_exact_branch_threshold(orc):
    """|c| >= t_rel m selects the exact column; smaller t_rel gives more
    exact columns, t_rel = inf none (Sec. 7.1)."""
    M = N = 6
    uni = orc.encode([1] * 6)                              # m = 12
    for c, trel, exact in [(12.0, 1.0, 1), (11.99, 1.0, 0), (6.0, 0.5, 1), (5.9, 0.5, 0),
                           (1e9, float("inf"), 0)]:
        P = orc.params(orc.REAL1D, M, N, 1.0, 6.0, dtau=1e-3, t_rel=trel, seed=2)
        if c > 1e6:
            continue
        out = orc.step(P, [uni], [c], 0.0, 1, uni, 1.0)
        assert out["stats"]["exact_steps"] == exact


def test_blocking_ar1_closed_form():
    """Variance of the mean of an AR(1) series, sigma^2/(1-phi)^2/n for
    large n (Eq. VarianceCorrelationFunctions)."""
    rng = np.random.default_rng(8)
    phi, n = 0.9, 1 << 17
    errs = []
    for rep in range(6):
        e = rng.standard_normal(n)
        x = np.empty(n)
        x[0] = e[0] / math.sqrt(1 - phi * phi)
        for i in range(1, n):
            x[i] = phi * x[i - 1] + e[i]
        r = stats.blocking_analysis(x)
        assert r.success
        errs.append(r.err)
    expect = 1.0 / (1 - phi) / math.sqrt(n)
    assert abs(np.mean(errs) / expect - 1.0) < 0.12


def test_blocking_uncorrelated_and_invariance():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(1 << 14)
    r = stats.blocking_analysis(x)
    assert r.k <= 3
    assert abs(r.err - 1 / math.sqrt(len(x))) < 0.1 / math.sqrt(len(x)) * 3
    # the blocking transformation keeps the sample mean
    assert math.isclose(stats._blocked(x, 5).mean(), x.mean(), rel_tol=1e-12)


def test_ratio_of_means_linear_propagation():
    rng = np.random.default_rng(10)
    n = 1 << 14
    X = 2.0 + rng.standard_normal(n) * 0.1
    Y = 1.0 + rng.standard_normal(n) * 0.05
    r = stats.ratio_of_means(X, Y)
    ref = np.sqrt((0.1 / 2.0) ** 2 + 0.05 ** 2) * 2.0 / math.sqrt(n)
    assert math.isclose(r.ratio, X.mean() / Y.mean())
    assert abs(r.err / ref - 1) < 0.15


def test_c1_oracle_energies_within_3_sigma_of_ed(orc):
    """The 6/6 ring: u = 6, dtau 1e-3, target 1e3, 1e4 steps, seed 0."""
    P = orc.params(orc.REAL1D, 6, 6, 1.0, 6.0, dtau=1e-3, target=1e3, seed=0)
    a = orc.start_address(orc.REAL1D, 6, 6)
    st, _, _ = orc.run(P, [a], [10.0], 0.0, 1, 10000, a, 10.0)
    E0 = orc.eigs_sparse(orc.ham(orc.REAL1D, 6, 6, 1.0, 6.0), 1)[0]
    se = stats.shift_estimator(st["shift"], skip=2000)
    pe = stats.projected_energy(st["hproj"], st["vproj"], skip=2000)
    assert abs(se.mean - E0) < 3 * se.err
    assert abs(pe.ratio - E0) < 3 * pe.err
    # bookkeeping invariants of the time series (Sec. 4, row semantics)
    assert np.all(st["exact_steps"][1:] + st["inexact_steps"][1:] == st["len"][:-1])
    assert st["step"][0] == 1 and st["step"][-1] == 10000


@pytest.mark.parametrize("M,N", [(5, 4), (8, 8), (16, 16), (7, 12)])
def test_sampled_pair_order_is_a_bijection(orc, M, N):
    """The stochastic removal-pair choice (Sec. 6.3) maps the P sampling
    indices one to one onto the valid pairs {p <= q occupied, n_p >= 2 when
    p = q}, so the uniform index gives each pair probability 1/P.  Checked
    for random parents against the pair set built from the occupations."""
    rng = np.random.default_rng(5)
    h = orc.ham(orc.MOM1D, M, N, 1.0, 2.0)
    for _ in range(25):
        occ = np.zeros(M, int)
        for x in rng.integers(0, M, N):
            occ[x] += 1
        a = orc.encode(list(occ))
        want = {(p, q) for p in range(M) for q in range(p, M)
                if occ[p] > 0 and occ[q] > 0 and (p != q or occ[p] >= 2)}
        got = [orc.sampled_pair(h, a, i) for i in range(len(want))]
        assert len(set(got)) == len(got) == len(want)
        assert set(got) == want
        with pytest.raises(Exception):
            orc.sampled_pair(h, a, len(want))


@pytest.mark.parametrize("model", [0, 1])
def test_early_compression_contributions(orc, model):
    """Early compression (Sec. 7.1): every spawn that survives has |v| >= theta
    or |v| = theta exactly; the late step keeps small spawns; both steps see
    the same parents, so early keeps at most as many spawn events."""
    rng = np.random.default_rng(23)
    M, N = (6, 6) if model == 0 else (6, 5)
    D = orc.dimension(M, N)
    idx = rng.choice(D, size=min(D, 40), replace=False)
    addrs = [orc.unrank(int(i), M, N) for i in idx]
    vals = rng.choice([-1, 1], len(idx)) * rng.uniform(0.5, 30.0, len(idx))
    theta = 0.7
    late = orc.step(orc.params(model, M, N, 1.0, 4.0, dtau=0.01, theta=theta, seed=3), addrs, vals,
                    -1.0, 5, addrs[0], 1.0, events=True)
    early = orc.step(orc.params(model, M, N, 1.0, 4.0, dtau=0.01, theta=theta, seed=3, early=True),
                     addrs, vals, -1.0, 5, addrs[0], 1.0, events=True)
    lv = np.abs(late["events"]["value"])
    ev = np.abs(early["events"]["value"])
    assert np.any(lv < theta)
    assert np.all(ev >= theta)
    assert len(ev) < len(lv) and early["stats"]["spawns"] == len(ev)
