"""Parity at the full benchmark sizes, in the launch configuration bench.py
times, on sampled outputs the oracle computes one by one.

The vector is grown to its target (1e8 walkers for the momentum-space
benchmark, 1e7 for the 20/20 real-space ring with two address words and for
the 6 x 6 lattice of Sec. 7.2 with importance sampling), then
two single steps run with sampled dumps (about 2^-k of all addresses).  For
the sampled addresses the test checks, bit for bit:

* every dumped spawn event (parent, attempt, destination, value) equals the
  oracle's event regenerated from that parent, and every oracle event of
  those parents that lands on a sampled address was dumped;
* the merged pre-compression amplitude equals the diagonal survivor plus the
  dumped events, summed exactly;
* the compressed value follows the compression rule with the oracle's draw;

and for the whole new state: len, ||c||_1 (exact sum), y.c and y.Hc.
"""
import sys

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


def _flush(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _key(a):
    a = np.asarray(a, dtype=np.uint64).reshape(len(a), -1)
    hi = a[:, 1] if a.shape[1] > 1 else np.zeros(len(a), np.uint64)
    return hi, a[:, 0]


def _index(addrs):
    hi, lo = _key(addrs)
    order = np.lexsort((lo, hi))
    return hi[order], lo[order], order


def _lookup(idx, vals, addrs):
    """Values of `addrs` in a state (0 where absent)."""
    shi, slo, order = idx
    hi, lo = _key(addrs)
    out = np.zeros(len(hi))
    # combine the two words into one sortable key per word pair
    pos = np.searchsorted(shi, hi, side="left")
    for i in range(len(hi)):
        p, q = pos[i], np.searchsorted(shi, hi[i], side="right")
        j = p + np.searchsorted(slo[p:q], lo[i])
        if j < q and slo[j] == lo[i]:
            out[i] = vals[order[j]]
    return out


def _pad2(a):
    a = np.asarray(a, dtype=np.uint64).reshape(len(a), -1)
    if a.shape[1] == 2:
        return a
    return np.concatenate([a, np.zeros((len(a), 1), np.uint64)], 1)


@pytest.mark.parametrize("name,k", [("c3", 12), ("c2", 10), ("c2d", 10)])
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
    warm = {"c3": 1500, "c2": 3000, "c2d": 2000}[name]
    _flush(f"[full size {name}] warmup {warm} steps, layout buckets={s.layout.buckets} "
           f"slots={s.layout.lds_slots} block={s.layout.block} spawn_block={s.layout.spawn_block}")
    done = 0
    while done < warm:
        s.run(min(500, warm - done))
        done += min(500, warm - done)
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
    par, att, dst, val = ev
    idx1 = _index(a1)
    # oracle events of the dumped parents
    ukeys = {}
    for p in _pad2(par):
        ukeys.setdefault((int(p[1]), int(p[0])), None)
    plist = np.array([[lo, hi] for hi, lo in ukeys], dtype=np.uint64)
    pvals = _lookup(idx1, v1, plist if W == 2 else plist[:, :1])
    assert np.all(pvals != 0.0)
    cap = len(pvals) + int(np.ceil(np.abs(pvals)).sum()) + 1024  # records of these parents
    o = orc.step(P, plist, pvals, S1, n1 + 1, plist[0], 10.0, cap=cap, events=True)
    sampled = set(zip(*(x.tolist() for x in _key(mg[0]))))
    want = {}
    for e in o["events"]:
        d = (int(e["dest"][1]), int(e["dest"][0]))
        if d in sampled:
            pk = (int(plist[e["parent"]][1]), int(plist[e["parent"]][0]))
            want[(pk, int(e["attempt"]))] = (d, float(e["value"]).hex())
    got = {}
    for p, a_, d, v in zip(_pad2(par), att, _pad2(dst), val):
        got[((int(p[1]), int(p[0])), int(a_))] = ((int(d[1]), int(d[0])), float(v).hex())
    assert len(got) == len(par)
    assert got == want
    # merged amplitude = diagonal survivor + events, exactly summed
    into = {}
    for (pk, _), (d, vh) in got.items():
        into.setdefault(d, []).append(float.fromhex(vh))
    mg_a = _pad2(mg[0])
    surv_c = _lookup(idx1, v1, mg[0])
    for i in range(len(mg_a)):
        key = (int(mg_a[i][1]), int(mg_a[i][0]))
        terms = list(into.get(key, []))
        if surv_c[i] != 0.0:
            diag = orc.column(h, mg_a[i], cap=4096)[0]
            terms.append(surv_c[i] * (1.0 + cfg["dtau"] * (S1 - diag)))
        assert float(orc.fsum(terms)).hex() == float(mg[1][i]).hex(), key
    # compression of the sampled merged amplitudes
    new_c = _lookup(_index(a2), v2, mg[0])
    theta = cfg["theta"]
    for i in range(len(mg_a)):
        w = float(mg[1][i])
        if abs(w) >= theta:
            exp = w
        elif w == 0.0:
            exp = 0.0
        else:
            u = int(orc.draw(cfg["seed"], mg_a[i], n2, 1, 0)[0]) * 2.0 ** -32
            exp = (theta if w > 0 else -theta) if u * theta < abs(w) else 0.0
        assert float(new_c[i]).hex() == float(exp).hex()
    # statistics of the whole new state
    row = st2[0]
    assert int(row["len"]) == len(v2)
    assert float(row["norm"]).hex() == float(orc.fsum(np.abs(v2))).hex()
    ref = _pad2(np.asarray([a0]))[0]
    diag_r = orc.column(h, ref, cap=4096)[0]
    dcol, hcol = orc.row(h, ref, cap=4096)  # y.Hc takes the row of the reference
    cref = _lookup(_index(a2), v2, np.asarray([a0]))[0]
    assert float(row["vproj"]).hex() == float(10.0 * cref).hex()
    ccol = _lookup(_index(a2), v2, dcol if W == 2 else dcol[:, :1])
    terms = [10.0 * (hv * cv) for hv, cv in zip(hcol, ccol)] + [10.0 * (diag_r * cref)]
    assert float(row["hproj"]).hex() == float(orc.fsum(terms)).hex()
