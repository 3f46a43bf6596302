"""Pins of the oracle's initiator rule (the initiator approximation the paper
names in Sec. 1 and in the sign-problem paragraph of Sec. 3.2; reading:
entry i is an initiator when |c_i| > n_a, and a spawn of a non-initiator
counts only onto an address occupied in c^(n)).

Pinned against the plain step (n_a = 0), against the plain step's own event
list filtered by the rule, and against a dense closed form of the
deterministic step."""
import math

import numpy as np
import pytest


def _key(a):
    return (int(a[0]), int(a[1]))


def _table(out, name="addr", val="val"):
    return {_key(a): float(v) for a, v in zip(out[name], out[val])}


def _state(orc, M, N, n, seed, lo=0.2, hi=30.0):
    rng = np.random.default_rng(seed)
    D = orc.dimension(M, N)
    idx = rng.choice(D, size=min(D, n), replace=False)
    addrs = [orc.unrank(int(i), M, N) for i in idx]
    vals = rng.choice([-1, 1], len(idx)) * rng.uniform(lo, hi, len(idx))
    return addrs, vals


CASES = [(0, 7, 7, 0, 0.0, False), (1, 7, 6, 0, 0.0, False), (2, 9, 5, 3, 0.0, False),
         (2, 9, 5, 3, 0.5, False), (0, 7, 7, 0, 0.0, True), (1, 7, 6, 0, 0.0, True)]


@pytest.mark.parametrize("model,M,N,lx,g,early", CASES)
def test_zero_threshold_is_the_plain_step(orc, model, M, N, lx, g, early):
    """n_a = 0: every nonzero entry is an initiator, so the step, its
    statistics and its events are the plain step's; the merged dump may add
    input addresses whose survivor is exactly 0 (value 0)."""
    addrs, vals = _state(orc, M, N, 60, 5)
    kw = dict(dtau=0.01, theta=0.6, seed=9, early=early, lx=lx, g=g, t_rel=2.0)
    plain = orc.step(orc.params(model, M, N, 1.0, 3.0, **kw), addrs, vals, -1.0, 4, addrs[0], 1.0,
                     events=True, merged=True)
    init = orc.step(orc.params(model, M, N, 1.0, 3.0, initiator=0.0, **kw), addrs, vals, -1.0, 4, addrs[0],
                    1.0, events=True, merged=True)
    assert np.array_equal(plain["addr"], init["addr"]) and np.array_equal(plain["val"], init["val"])
    assert plain["stats"] == init["stats"]
    assert np.array_equal(plain["events"], init["events"])
    pm, im = _table(plain, "merged_addr", "merged_val"), _table(init, "merged_addr", "merged_val")
    inputs = {_key(a) for a in addrs}
    assert all(im[k] == v for k, v in pm.items())
    assert all(k in inputs and v == 0.0 for k, v in im.items() if k not in pm)


@pytest.mark.parametrize("model,M,N,lx,g,early", CASES)
@pytest.mark.parametrize("n_a", [3.0, 12.5, math.inf])
def test_rule_filters_the_plain_events(orc, model, M, N, lx, g, early, n_a):
    """Any n_a: the events are the plain step's; the merged value of an input
    address is the plain step's (every spawn onto it counts); an address
    outside the input gets the exact sum of the events of initiator parents
    (|c| > n_a) that reach it, and is absent when there are none.  Where the
    merged value equals the plain one, so does the compressed output."""
    addrs, vals = _state(orc, M, N, 60, 11)
    # one parent exactly at the threshold: not an initiator
    if math.isfinite(n_a):
        vals[1] = -n_a
    kw = dict(dtau=0.01, theta=0.6, seed=13, early=early, lx=lx, g=g, t_rel=2.0)
    plain = orc.step(orc.params(model, M, N, 1.0, 3.0, **kw), addrs, vals, -1.0, 6, addrs[0], 1.0,
                     events=True, merged=True)
    init = orc.step(orc.params(model, M, N, 1.0, 3.0, initiator=n_a, **kw), addrs, vals, -1.0, 6, addrs[0],
                    1.0, events=True, merged=True)
    assert np.array_equal(plain["events"], init["events"])
    assert plain["stats"]["spawns"] == init["stats"]["spawns"]
    assert plain["stats"]["exact_steps"] == init["stats"]["exact_steps"]
    inputs = {_key(a) for a in addrs}
    pm, im = _table(plain, "merged_addr", "merged_val"), _table(init, "merged_addr", "merged_val")
    kept = {}
    for e in plain["events"]:
        d = _key(e["dest"])
        if d not in inputs and abs(vals[e["parent"]]) > n_a:
            kept.setdefault(d, []).append(float(e["value"]))
    want = {k: pm.get(k, 0.0) for k in inputs}
    want.update({k: math.fsum(v) for k, v in kept.items()})
    assert im == want
    dropped = sum(1 for e in plain["events"]
                  if _key(e["dest"]) not in inputs and not abs(vals[e["parent"]]) > n_a)
    assert dropped > 0
    po, io = _table(plain), _table(init)
    for k, v in io.items():
        if k in pm and pm[k] == im[k]:
            assert po[k] == v
    if n_a == math.inf:
        assert set(io) <= inputs


@pytest.mark.parametrize("model,M,N", [(0, 6, 5), (1, 6, 5)])
def test_deterministic_step_closed_form(orc, model, M, N):
    """All parents spawn exactly and theta is below every value: the step is
    c' = P_occ (T c) + (1 - P_occ) T (P_init c) with T = 1 + dtau (S - H),
    P_occ the projector on the occupied addresses and P_init the one on the
    initiators (dense linear algebra over the ranked basis)."""
    h = orc.ham(model, M, N, 1.0, 2.0)
    D = orc.dimension(M, N)
    rng = np.random.default_rng(31)
    idx = rng.choice(D, size=D // 2, replace=False)
    addrs = [orc.unrank(int(i), M, N) for i in idx]
    vals = rng.choice([-1, 1], len(idx)) * rng.uniform(200.0, 2000.0, len(idx))
    n_a = 1000.0
    vals[0] = n_a
    S, dtau = -1.5, 1e-3
    P = orc.params(model, M, N, 1.0, 2.0, dtau=dtau, target=1e6, theta=1e-9, t_rel=1.0, seed=2,
                   initiator=n_a)
    out = orc.step(P, addrs, vals, S, 3, addrs[0], 1.0)
    assert out["stats"]["inexact_steps"] == 0
    H = orc.csr_matrix(h).toarray()
    c = np.zeros(D)
    for i, v in zip(idx, vals):
        c[i] = v
    occ = c != 0.0
    init = np.abs(c) > n_a
    T = np.eye(D) + dtau * (S * np.eye(D) - H)
    want = np.where(occ, T @ c, T @ np.where(init, c, 0.0))
    got = np.zeros(D)
    for a, v in zip(out["addr"], out["val"]):
        got[orc.rank(_key(a), M, N)] = v
    assert np.allclose(got, want, rtol=1e-12, atol=1e-9)
    # the rule removed something: the plain step grows the support further
    plain = orc.step(orc.params(model, M, N, 1.0, 2.0, dtau=dtau, target=1e6, theta=1e-9, t_rel=1.0, seed=2),
                     addrs, vals, S, 3, addrs[0], 1.0)
    assert len(plain["addr"]) > len(out["addr"])


def test_threshold_must_be_non_negative(orc):
    addrs, vals = _state(orc, 5, 5, 10, 1)
    with pytest.raises(Exception):
        orc.step(orc.params(0, 5, 5, initiator=-1.0), addrs, vals, 0.0, 1, addrs[0], 1.0)
    with pytest.raises(Exception):
        orc.step(orc.params(0, 5, 5, initiator=math.nan), addrs, vals, 0.0, 1, addrs[0], 1.0)


def test_occupied_address_with_a_zero_survivor(orc):
    """An input address whose diagonal survivor is exactly 0 (here
    1 + dtau (S - H_aa) = 0 with dtau = 1/16 and S = H_aa - 16) is still
    occupied in c^(n): non-initiator spawns onto it count, and its merged
    value is the plain step's."""
    M, N = 7, 7
    addrs, vals = _state(orc, M, N, 600, 4, lo=0.5, hi=20.0)
    # H_aa = (u/2) sum_i n_i (n_i - 1) on the ring (Sec. 2.5), u = 2
    diag = [sum(n * (n - 1) for n in orc.decode(a, M, N)) for a in addrs]
    h0 = max(set(diag), key=diag.count)
    n_a = 8.0
    kw = dict(dtau=1.0 / 16.0, theta=0.01, seed=5, t_rel=0.0)
    S = float(h0) - 16.0
    plain = orc.step(orc.params(0, M, N, 1.0, 2.0, **kw), addrs, vals, S, 2, addrs[0], 1.0,
                     events=True, merged=True)
    init = orc.step(orc.params(0, M, N, 1.0, 2.0, initiator=n_a, **kw), addrs, vals, S, 2, addrs[0], 1.0,
                    events=True, merged=True)
    inputs = {_key(a) for a in addrs}
    zero = {_key(a) for a, d in zip(addrs, diag) if d == h0}
    pm, im = _table(plain, "merged_addr", "merged_val"), _table(init, "merged_addr", "merged_val")
    reached = {_key(e["dest"]) for e in plain["events"] if not abs(vals[e["parent"]]) > n_a}
    cases = zero & reached
    assert len(cases) >= 5
    assert all(im[k] == pm[k] for k in cases)
    assert all(im[k] == pm.get(k, 0.0) for k in inputs)


def test_bias_shrinks_as_the_walker_number_grows(orc):
    """The 6/6 ring at u = 6 with n_a = 3: at N_t = 50 few entries exceed n_a
    and the truncated spawning leaves a large positive energy bias; at
    N_t = 1000 most of the weight sits on initiators and the bias falls by
    more than a factor of ten (the plain step has none at either size)."""
    from oracle import stats
    M = N = 6
    E0 = orc.eigs_sparse(orc.ham(0, M, N, 1.0, 6.0), 1)[0]
    a = orc.start_address(0, M, N)
    bias = {}
    for Nt in (50.0, 1000.0):
        P = orc.params(0, M, N, 1.0, 6.0, dtau=0.01, target=Nt, seed=7, initiator=3.0)
        st, _, _ = orc.run(P, [a], [10.0], 0.0, 1, 12000, a, 10.0)
        pe = stats.projected_energy(st["hproj"], st["vproj"], skip=3000)
        bias[Nt] = (pe.ratio - E0, pe.err)
    (b0, e0), (b1, e1) = bias[50.0], bias[1000.0]
    assert b0 > 20 * e0 and b0 > 0.5
    assert abs(b1) < 0.1 * b0
