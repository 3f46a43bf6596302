"""Pins of the oracle's replica overlap and variational energy [Sec. 4.3].

The overlap c_A . c_B is checked against routes that share nothing with
its implementation (Python integers over the ranked dense basis, exact
rationals over a dict join) and against the exactness it promises; the
variational-energy estimator against a closed form and, end to end, against
exact diagonalisation on the 6/6 ring that the paper uses for its printed
replica result.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import stats


def test_overlap_is_exactly_rounded_under_cancellation(orc):
    a = np.array([3, 5, 9], np.uint64)
    # naive left-to-right summation of the products loses the 1.0
    assert orc.overlap(a, [1e16, 1.0, -1e16], a, [1.0, 1.0, 1.0]) == 1.0
    assert orc.overlap(a, [1e16, 1.0, -1e16], a[::-1], [1.0, 1.0, 1.0][::-1]) == 1.0


def test_overlap_integer_amplitudes_on_dense_basis(orc):
    """Integer amplitudes make every product and sum exact: the overlap is
    the integer dot product of the two vectors written out densely over the
    combinatorially ranked basis of the 6/6 space."""
    M = N = 6
    D = orc.dimension(M, N)
    rng = random.Random(7)
    for trial in range(5):
        ra = rng.sample(range(D), 200)
        rb = rng.sample(range(D), 150)
        xa = [rng.randint(-2 ** 20, 2 ** 20) for _ in ra]
        xb = [rng.randint(-2 ** 20, 2 ** 20) for _ in rb]
        da, db = [0] * D, [0] * D
        for r, x in zip(ra, xa):
            da[r] = x
        for r, x in zip(rb, xb):
            db[r] = x
        want = sum(p * q for p, q in zip(da, db))
        aa = np.array([orc.unrank(r, M, N)[0] for r in ra], np.uint64)
        ab = np.array([orc.unrank(r, M, N)[0] for r in rb], np.uint64)
        got = orc.overlap(aa, np.array(xa, float), ab, np.array(xb, float))
        assert got == float(want)


def test_overlap_brute_force_rationals(orc):
    """Random doubles over a wide exponent range: the result is the exact
    rational sum of the rounded products, rounded once."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        keys = rng.choice(1 << 40, size=300, replace=False).astype(np.uint64)
        ka, kb = keys[:200], keys[100:]
        va = rng.standard_normal(200) * np.exp2(rng.integers(-30, 30, 200))
        vb = rng.standard_normal(200) * np.exp2(rng.integers(-30, 30, 200))
        da = {int(k): float(v) for k, v in zip(ka, va)}
        exact = Fraction(0)
        for k, v in zip(kb, vb):
            if int(k) in da:
                exact += Fraction(da[int(k)] * float(v))
        got = orc.overlap(ka, va, kb, vb)
        assert got == float(exact)
        assert got == orc.overlap(kb, vb, ka, va)


def test_overlap_two_word_addresses_match_both_words(orc):
    a = np.array([[1, 0], [1, 7], [2, 7]], np.uint64)
    b = np.array([[1, 7], [2, 0], [2, 7]], np.uint64)
    assert orc.overlap(a, [2.0, 3.0, 5.0], b, [7.0, 11.0, 13.0]) == 3.0 * 7.0 + 5.0 * 13.0
    assert orc.overlap(a[:1], [2.0], b[1:2], [3.0]) == 0.0
    with pytest.raises(ValueError):
        orc.overlap(np.array([4, 4], np.uint64), [1.0, 1.0], a[:, 0], [1.0, 1.0, 1.0])


def test_replica_pair_order(orc):
    assert orc.replica_pairs(2) == [(0, 1)]
    assert orc.replica_pairs(4) == [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def test_variational_energy_constant_shift_closed_form():
    """With every shift equal to E the numerator is E times the denominator
    at every step, so the estimator is E whatever the overlaps."""
    rng = np.random.default_rng(1)
    n = 4096
    O = rng.uniform(1.0, 3.0, size=(3, n))
    r = stats.variational_energy(np.full((3, n), -2.5), O)
    assert abs(r.ratio + 2.5) < 1e-12
    with pytest.raises(ValueError):
        stats.variational_energy(np.zeros((3, n)), O[:2])


def replica_trajectories(orc, R, steps, seeds, M=6, N=6, u=6.0, dtau=1e-3, target=1e3):
    """R oracle replicas stepped together from 10 walkers on the uniform
    state; returns shifts (R, steps), overlaps (P, steps), stats rows."""
    a0 = orc.start_address(orc.REAL1D, M, N)
    Ps = [orc.params(orc.REAL1D, M, N, 1.0, u, dtau=dtau, target=target, seed=s) for s in seeds]
    st = [(np.asarray([a0], np.uint64), np.array([10.0]), 0.0) for _ in range(R)]
    pairs = orc.replica_pairs(R)
    shifts = np.zeros((R, steps))
    ovl = np.zeros((len(pairs), steps))
    rows = [[] for _ in range(R)]
    for n in range(steps):
        for r in range(R):
            addrs, vals, S = st[r]
            o = orc.step(Ps[r], addrs, vals, S, n + 1, a0, 10.0)
            st[r] = (o["addr"], o["val"], o["stats"]["shift"])
            shifts[r, n] = o["stats"]["shift"]
            rows[r].append(o["stats"])
        for k, (A, B) in enumerate(pairs):
            ovl[k, n] = orc.overlap(st[A][0], st[A][1], st[B][0], st[B][1])
    return shifts, ovl, rows, st


@pytest.mark.slow
def test_c1_variational_energy_within_3_sigma_of_ed(orc):
    """Two replicas of the 6/6 ring at u = 6 (seeds 0 and 1, 1e4 steps): the
    variational energy agrees with exact diagonalisation within three
    standard errors.  For this system and two replicas the paper prints
    -4.02149 with an error of 0.0025."""
    shifts, ovl, _, _ = replica_trajectories(orc, 2, 10000, [0, 1])
    E0 = orc.eigs_sparse(orc.ham(orc.REAL1D, 6, 6, 1.0, 6.0), 1)[0]
    r = stats.variational_energy(shifts, ovl, skip=2000)
    assert np.all(ovl[:, 2000:] > 0)
    assert abs(r.ratio - E0) < 3 * r.err
    assert abs(r.ratio - (-4.02149)) < 3 * math.hypot(r.err, 0.0025)
