"""Parity at the full benchmark sizes, in the launch configuration bench.py
times, on sampled outputs the oracle computes one by one.

The vector is grown to its target (1e8 walkers for the momentum-space
benchmark, 1e7 for the 20/20 real-space ring with two address words and for
the 6 x 6 lattice of Sec. 7.2 with importance sampling), then two single
steps run with sampled dumps: the dumps keep the spawn events into, and the
merged sums of, a fixed sample of about 2^-k of all addresses (the library's
sampling rule: bits 24 .. 24+k-1 of its address hash are zero).

The expected values come from the oracle, not from the dumps.  Every parent
that can spawn into a sampled address lies in that address's column (the
connectivity of the Hamiltonian is symmetric, also under importance
sampling), so the test collects, for every sampled merged address, the
entries of the state that lie in its column, regenerates all their spawn
events with the oracle and checks, bit for bit:

* the spawn events into sampled addresses (parent, attempt, destination,
  value) equal the oracle's events of those parents into sampled addresses;
  a parent whose events were lost, or an event sent elsewhere, fails;
* each sampled merged amplitude equals the diagonal survivor plus the
  oracle's events into it, summed exactly;
* every entry of the state in the sample is among the merged addresses, and
  the oracle events of a random sample of parents into sampled addresses
  all land on merged addresses (no sampled destination is missing);
* the compressed value follows the compression rule with the oracle's draw;

and for the whole new state: len, ||c||_1 (exact sum), y.c and y.Hc, with
every sum of the step exactly rounded (no inexact flag).
"""
import sys

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


def _flush(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pad2(a):
    a = np.asarray(a, dtype=np.uint64).reshape(len(a), -1)
    if a.shape[1] == 2:
        return a
    return np.concatenate([a, np.zeros((len(a), 1), np.uint64)], 1)


def _keys(a):
    """Sortable structured keys (hi, lo) of addresses given as W words."""
    a = _pad2(a)
    k = np.empty(len(a), dtype=[("hi", np.uint64), ("lo", np.uint64)])
    k["hi"], k["lo"] = a[:, 1], a[:, 0]
    return k


class _State:
    """Sorted lookup over a state (addresses as W words, values)."""

    def __init__(self, addrs, vals):
        k = _keys(addrs)
        self.order = np.argsort(k, kind="stable")
        self.k = k[self.order]
        self.v = np.asarray(vals)[self.order]

    def find(self, addrs):
        """Values of `addrs` (0 where absent) and a presence mask."""
        q = _keys(addrs)
        pos = np.searchsorted(self.k, q)
        pos = np.minimum(pos, len(self.k) - 1)
        hit = self.k[pos] == q
        return np.where(hit, self.v[pos], 0.0), hit


def _mix64(x):
    x = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        x = x ^ (x >> np.uint64(30))
        x = x * np.uint64(0xBF58476D1CE4E5B9)
        x = x ^ (x >> np.uint64(27))
        x = x * np.uint64(0x94D049BB133111EB)
        x = x ^ (x >> np.uint64(31))
    return x


def _sampled(addrs, W, k):
    """The library's dump sample: bits 24 .. 24+k-1 of the address hash zero."""
    a = _pad2(addrs)
    if W == 1:
        h = _mix64(a[:, 0])
    else:
        with np.errstate(over="ignore"):
            h = _mix64(a[:, 0] ^ _mix64(a[:, 1] + np.uint64(0x9E3779B97F4A7C15)))
    return ((h >> np.uint64(24)) & np.uint64((1 << k) - 1)) == 0


def _tuple_keys(a):
    a = _pad2(a)
    return list(zip(a[:, 1].tolist(), a[:, 0].tolist()))


@pytest.mark.parametrize("name,k", [("c3", 14), ("c2", 10), ("c2d", 12)])
def test_full_size_sampled_step(orc, name, k):
    import bench
    import paper_2601_19505_amd as fq
    wl = bench.WORKLOADS[name]
    cfg = synthetic.CONFIGS[wl["cfg"]]
    W = cfg["W"]
    flags = fq.FLAG_DUMP_SPAWNS | fq.FLAG_DUMP_MERGED | (k << 8)
    s = bench.make_solver(fq, wl, cfg, flags=flags)
    a0 = fq.encode(synthetic.start_occupation(cfg["model"], cfg["M"], cfg["N"]), W)
    s.set_state([a0], [10.0], 0.0, 0, ref=a0, yref=10.0)
    _flush(f"[full size {name}] ramp to {cfg['target']:.3g} walkers, layout buckets={s.layout.buckets} "
           f"slots={s.layout.lds_slots} block={s.layout.block} spawn_block={s.layout.spawn_block}")
    bench.ramp(s, cfg["target"], 100, f"full size {name}")
    cap = 4 * ((wl["spawn_capacity"] + wl["table_capacity"]) >> k) + 65536
    # step n -> n+1: the spawn dump holds the spawns of c^(n+1) for step n+2
    s.run(1)
    a1, v1, S1, n1 = s.get_state()
    ev = s.spawn_dump(cap)
    # step n+1 -> n+2: the merged dump holds the sums of step n+2
    st2 = s.run(1)
    mg = s.merged_dump(cap)
    a2, v2, S2, n2 = s.get_state()
    s.close()
    _flush(f"[full size {name}] state {len(v1)} entries, {len(ev[0])} sampled events, "
           f"{len(mg[0])} sampled merged amplitudes")
    assert n2 == n1 + 1 and len(ev[0]) > 1000 and len(mg[0]) > 500

    lx, g = cfg.get("lx", 0), cfg.get("g", 0.0)
    P = orc.params(cfg["model"], cfg["M"], cfg["N"], cfg["t"], cfg["u"], dtau=cfg["dtau"],
                   target=cfg["target"], theta=cfg["theta"], seed=cfg["seed"], lx=lx, g=g)
    h = orc.ham(cfg["model"], cfg["M"], cfg["N"], cfg["t"], cfg["u"], lx=lx, g=g)
    state1 = _State(a1, v1)
    mg_a = _pad2(mg[0])
    assert np.all(_sampled(mg_a, W, k))
    merged = set(_tuple_keys(mg_a))
    # every sampled entry of the state has its survivor among the merged addresses
    assert set(_tuple_keys(_pad2(a1)[_sampled(a1, W, k)])) <= merged
    # every parent of a sampled merged address: the entries of c^(n+1) in its
    # column, and the address itself (its diagonal survivor)
    cand = [mg_a]
    diag = np.zeros(len(mg_a))
    for i in range(len(mg_a)):
        d, dests, _ = orc.column(h, mg_a[i], cap=4096)
        diag[i] = d
        cand.append(dests)
    cand = np.unique(_keys(np.concatenate(cand)))
    cand_a = np.stack([cand["lo"], cand["hi"]], 1)
    pv, hit = state1.find(cand_a)
    parents, pvals = cand_a[hit], pv[hit]
    # plus a random sample of parents, for the completeness of the sampled destinations
    rng = np.random.default_rng(7)
    extra = rng.choice(len(v1), size=min(len(v1), 4000), replace=False)
    parents = np.concatenate([parents, _pad2(a1[extra])])
    pvals = np.concatenate([pvals, v1[extra]])
    u = np.unique(_keys(parents), return_index=True)[1]
    parents, pvals = parents[u], pvals[u]
    _flush(f"[full size {name}] oracle events of {len(pvals)} parents")
    ocap = len(pvals) + int(np.ceil(np.abs(pvals)).sum()) + 1024  # records of these parents
    o = orc.step(P, parents, pvals, S1, n1 + 1, parents[0], 10.0, cap=ocap, events=True)
    oe = o["events"]
    odest = _pad2(oe["dest"])
    into_sample = _sampled(odest, W, k)
    okeys = _tuple_keys(odest[into_sample])
    # no sampled destination is missing from the merged dump
    assert set(okeys) <= merged
    pkeys = _tuple_keys(parents)
    want = {}
    for e, d in zip(oe[into_sample], okeys):
        want[(pkeys[int(e["parent"])], int(e["attempt"]))] = (d, float(e["value"]).hex())
    par, att, dst, val = ev
    got = {}
    for p, a_, d, v in zip(_tuple_keys(par), att, _tuple_keys(dst), val):
        got[(p, int(a_))] = (d, float(v).hex())
    assert len(got) == len(par)
    # the oracle's event set covers every parent of the sampled addresses
    # that were merged, so the two sets must agree exactly
    assert got == want
    # merged amplitude = diagonal survivor + the oracle's events, exactly summed
    into = {}
    for (_, (d, vh)) in want.items():
        into.setdefault(d, []).append(float.fromhex(vh))
    surv_c, _ = state1.find(mg_a)
    for i, key in enumerate(_tuple_keys(mg_a)):
        terms = list(into.get(key, []))
        if surv_c[i] != 0.0:
            terms.append(surv_c[i] * (1.0 + cfg["dtau"] * (S1 - diag[i])))
        assert float(orc.fsum(terms)).hex() == float(mg[1][i]).hex(), key
    # compression of the sampled merged amplitudes
    new_c, _ = _State(a2, v2).find(mg_a)
    theta = cfg["theta"]
    for i in range(len(mg_a)):
        w = float(mg[1][i])
        if abs(w) >= theta:
            exp = w
        elif w == 0.0:
            exp = 0.0
        else:
            uu = int(orc.draw(cfg["seed"], mg_a[i], n2, 1, 0)[0]) * 2.0 ** -32
            exp = (theta if w > 0 else -theta) if uu * theta < abs(w) else 0.0
        assert float(new_c[i]).hex() == float(exp).hex()
    # statistics of the whole new state
    row = st2[0]
    assert int(row["flags"]) == 0
    assert int(row["len"]) == len(v2)
    assert float(row["norm"]).hex() == float(orc.fsum(np.abs(v2))).hex()
    ref = _pad2(np.asarray([a0]))[0]
    diag_r = orc.column(h, ref, cap=4096)[0]
    dcol, hcol = orc.row(h, ref, cap=4096)  # y.Hc takes the row of the reference
    state2 = _State(a2, v2)
    cref = state2.find(np.asarray([a0]))[0][0]
    assert float(row["vproj"]).hex() == float(10.0 * cref).hex()
    ccol, _ = state2.find(dcol)
    terms = [10.0 * (hv * cv) for hv, cv in zip(hcol, ccol)] + [10.0 * (diag_r * cref)]
    assert float(row["hproj"]).hex() == float(orc.fsum(terms)).hex()
