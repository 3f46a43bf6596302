"""Pins of the oracle's Gram-Schmidt orthogonalisation for excited states
[Sec. 2.2]: the projected vector is orthogonal to the one projected out
(to rounding), projecting a vector out of itself leaves nothing, disjoint
vectors are unchanged, the union is handled entry by entry as on a dense
vector over the ranked basis, and two step-synchronised runs of the 6/6 ring
give the first excited energy of exact diagonalisation within 3 sigma.
"""
import numpy as np
import pytest

from oracle import stats


def _sparse(orc, rng, M, N, n):
    D = orc.dimension(M, N)
    idx = rng.choice(D, size=n, replace=False)
    addrs = np.array([orc.unrank(int(i), M, N) for i in idx], np.uint64)
    vals = rng.standard_normal(n) * rng.uniform(0.5, 50.0, n)
    return idx, addrs, vals


def test_projection_is_orthogonal(orc):
    rng = np.random.default_rng(11)
    for trial in range(10):
        _, ak, vk = _sparse(orc, rng, 7, 7, 300)
        _, aj, vj = _sparse(orc, rng, 7, 7, 250)
        a, v, alpha = orc.orthogonalise(ak, vk, aj, vj)
        d = orc.overlap(a, v, aj, vj)
        assert abs(d) <= 1e-12 * np.linalg.norm(vj) * np.linalg.norm(v)


def test_projection_matches_dense_update(orc):
    """Entry by entry, the result is v_k - (alpha v_j) over the union of the
    two supports (0 where a vector has no entry), written out densely."""
    M = N = 6
    rng = np.random.default_rng(12)
    D = orc.dimension(M, N)
    for trial in range(5):
        ik, ak, vk = _sparse(orc, rng, M, N, 200)
        ij, aj, vj = _sparse(orc, rng, M, N, 150)
        a, v, alpha = orc.orthogonalise(ak, vk, aj, vj)
        dk = np.zeros(D)
        dj = np.zeros(D)
        dk[ik] = vk
        dj[ij] = vj
        want = dk - alpha * dj
        got = np.zeros(D)
        for row, x in zip(a, v):
            got[orc.rank((int(row[0]), int(row[1])), M, N)] = x
        assert np.array_equal(got, want)
        assert np.count_nonzero(want) == len(v)


def test_self_projection_and_disjoint_vectors(orc):
    rng = np.random.default_rng(13)
    _, a, v = _sparse(orc, rng, 6, 6, 100)
    out, vals, alpha = orc.orthogonalise(a, v, a, v)
    assert alpha == 1.0 and len(vals) == 0
    out, vals, alpha = orc.orthogonalise(a[:50], v[:50], a[50:], v[50:])
    assert alpha == 0.0
    assert np.array_equal(out, a[:50]) and np.array_equal(vals, v[:50])


@pytest.mark.slow
def test_first_excited_state_of_the_6_6_ring(orc):
    """Two step-synchronised runs of the 6/6 ring at u = 6 (N_t = 1e3, 1e4
    steps; the second starts one hop from the uniform state): the shift of
    the orthogonalised run estimates E1 within 3 sigma, the first run E0."""
    h = orc.ham(orc.REAL1D, 6, 6, 1.0, 6.0)
    E = np.linalg.eigvalsh(orc.dense_matrix(h))
    Ps = [orc.params(orc.REAL1D, 6, 6, 1.0, 6.0, dtau=1e-3, target=1e3, seed=s) for s in (0, 1)]
    a = orc.start_address(orc.REAL1D, 6, 6)
    b = orc.column(h, a)[1][0]
    rows, _ = orc.spectral_run(Ps, [a, b], a, 10000)
    s0 = stats.shift_estimator(np.array([x["shift"] for x in rows[0]]), skip=3000)
    s1 = stats.shift_estimator(np.array([x["shift"] for x in rows[1]]), skip=3000)
    assert abs(s0.mean - E[0]) < 3 * s0.err
    assert abs(s1.mean - E[1]) < 3 * s1.err
