"""Batch, server, state copy and autotuning on the GPU, through the C ABI.

Every instance of a batch and every request of the server must produce
exactly the statistics it produces alone (and, for a small instance, exactly
the oracle's): the step is a pure function of (Hamiltonian, parameters,
state, step, seed), all random numbers are counter based and every sum is
exactly rounded, so the comparison is bit for bit.
"""
import sys

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

LAYOUT = dict(lds_slots=1024, block=256, spawn_block=256)


def _fq():
    import paper_2601_19505_amd as fq
    return fq


def _flush(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _spec(model, M, N, u, dtau, target, seed, table, spawn, buckets=0, W=1):
    return dict(model=model, M=M, N=N, t=1.0, u=u, dtau=dtau, target_walkers=target, seed=seed,
                addr_words=W, table_capacity=table, spawn_capacity=spawn, buckets=buckets, **LAYOUT)


def _solo(spec, steps):
    fq = _fq()
    s = fq.Solver(**spec)
    a = fq.start_address(spec["model"], spec["M"], spec["N"], spec["addr_words"])
    s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = s.run(steps)
    s.close()
    return st


def _real_specs():
    # uneven sizes, a u scan, one instance with the two-pass partition
    return [
        _spec(0, 6, 6, 6.0, 1e-3, 1e3, 0, 1024, 8192),
        _spec(0, 8, 8, 1.0, 1e-3, 5e3, 11, 8192, 65536),
        _spec(0, 8, 8, 3.0, 1e-3, 5e3, 12, 8192, 65536),
        _spec(0, 10, 10, 10.0, 5e-4, 2e4, 13, 40000, 200000),
        _spec(0, 12, 12, 6.0, 1e-3, 2e4, 14, 60000, 300000, buckets=128),
        _spec(0, 7, 5, 2.0, 2e-3, 2e3, 15, 4096, 32768),
    ]


def test_batch_equals_solo_bit_exact():
    fq = _fq()
    specs = _real_specs()
    steps = 600
    _flush(f"[batch] {len(specs)} real-space instances, {steps} steps")
    b = fq.Batch(specs)
    for i, sp in enumerate(specs):
        a = fq.start_address(sp["model"], sp["M"], sp["N"])
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = b.run(steps)
    # a second call continues where the first stopped
    st2 = b.run(100)
    b.close()
    for i, sp in enumerate(specs):
        solo = _solo(sp, steps + 100)
        assert st[i].tobytes() == solo[:steps].tobytes(), i
        assert st2[i].tobytes() == solo[steps:].tobytes(), i


def test_batch_instance_equals_oracle(orc):
    fq = _fq()
    specs = _real_specs()[:3]
    steps = 400
    b = fq.Batch(specs)
    for i, sp in enumerate(specs):
        a = fq.start_address(sp["model"], sp["M"], sp["N"])
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = b.run(steps)
    b.close()
    sp = specs[0]
    P = orc.params(0, sp["M"], sp["N"], 1.0, sp["u"], dtau=sp["dtau"], target=sp["target_walkers"],
                   seed=sp["seed"])
    a = orc.start_address(0, sp["M"], sp["N"])
    ost, _, _ = orc.run(P, [a], [10.0], 0.0, 1, steps, a, 10.0)
    for f in ost.dtype.names:
        g, o = st[0][f], ost[f]
        if g.dtype.kind == "f":
            assert np.array_equal(g.view(np.uint64), o.view(np.uint64)), f
        else:
            assert np.array_equal(g, o), f


def test_batch_with_initiator_instances(orc):
    """Instances with and without the initiator rule share one batch (the
    merge launch takes the largest LDS size of its instances): each equals
    its solo run, and the initiator instance equals the oracle's run with
    the same threshold, bit for bit."""
    fq = _fq()
    specs = _real_specs()[:4]
    specs[1] = dict(specs[1], initiator=3.0)
    specs[3] = dict(specs[3], initiator=0.0)
    steps = 400
    _flush(f"[batch initiator] {len(specs)} instances, {steps} steps")
    b = fq.Batch(specs)
    for i, sp in enumerate(specs):
        a = fq.start_address(sp["model"], sp["M"], sp["N"])
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = b.run(steps)
    b.close()
    for i, sp in enumerate(specs):
        assert st[i].tobytes() == _solo(sp, steps).tobytes(), i
    sp = specs[1]
    P = orc.params(0, sp["M"], sp["N"], 1.0, sp["u"], dtau=sp["dtau"], target=sp["target_walkers"],
                   seed=sp["seed"], initiator=3.0)
    a = orc.start_address(0, sp["M"], sp["N"])
    ost, _, _ = orc.run(P, [a], [10.0], 0.0, 1, steps, a, 10.0)
    for f in ost.dtype.names:
        g, o = st[1][f], ost[f]
        if g.dtype.kind == "f":
            assert np.array_equal(g.view(np.uint64), o.view(np.uint64)), f
        else:
            assert np.array_equal(g, o), f


def test_batch_momentum_equals_solo():
    fq = _fq()
    specs = [_spec(1, 8, 8, 4.0, 1e-3, 5e3, 21, 8192, 65536),
             _spec(1, 10, 10, 2.0, 1e-3, 2e4, 22, 60000, 400000, buckets=128),
             _spec(1, 5, 4, 3.0, 1e-2, 500, 23, 1024, 8192)]
    steps = 300
    _flush(f"[batch momentum] {len(specs)} instances")
    b = fq.Batch(specs)
    for i, sp in enumerate(specs):
        a = fq.start_address(1, sp["M"], sp["N"])
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = b.run(steps)
    b.close()
    for i, sp in enumerate(specs):
        assert st[i].tobytes() == _solo(sp, steps).tobytes(), i


def test_batch_rejects_mixed_kinds():
    fq = _fq()
    specs = [_spec(0, 6, 6, 6.0, 1e-3, 1e3, 0, 1024, 8192),
             dict(_spec(0, 6, 6, 6.0, 1e-3, 1e3, 0, 1024, 8192), block=512)]
    with pytest.raises(fq.FqError):
        fq.Batch(specs)


def _mean_loop(x):
    acc = 0.0
    for v in x:
        acc += float(v)
    return acc / len(x)


def test_server_alone_equals_mix(orc):
    """Requests admitted over several ticks under a pool that cannot hold all
    of them at once: every result equals the solo run of that request, and
    the oracle's run of the same request (last statistics row bit for bit,
    the means over the second half of the steps)."""
    fq = _fq()
    rng = np.random.default_rng(3)
    reqs = []
    for k in range(7):
        M = int(rng.integers(6, 11))
        sp = dict(model=0, M=M, N=M, t=1.0, u=float(rng.uniform(1, 10)), dtau=1e-3,
                  target_walkers=float(rng.choice([300.0, 1e3, 3e3])), seed=500 + k,
                  table_capacity=16384, spawn_capacity=131072)
        reqs.append((sp, int(rng.integers(150, 500))))
    one = fq.workspace_size(*fq._ham_params(0, 10, 10), fq._layout(16384, 131072, 0, 1024, 256, 256))[0]
    pool = int(2.5 * one) + (1 << 20)  # the maps plus room for two resident solves
    sv = fq.Server(0, pool, lds_slots=1024, block=256, spawn_block=256, max_active=4,
                   steps_per_tick=64)
    ids = []
    saw_queue = False
    # arrivals: two requests before the first tick, then one per tick
    pending = list(range(len(reqs)))
    for _ in range(2):
        i = pending.pop(0)
        sp, n = reqs[i]
        ids.append(sv.submit(sp, fq.start_address(0, sp["M"], sp["N"]), 10.0, n))
    done = 0
    ticks = 0
    while done < len(reqs):
        if pending:
            i = pending.pop(0)
            sp, n = reqs[i]
            ids.append(sv.submit(sp, fq.start_address(0, sp["M"], sp["N"]), 10.0, n))
        active, queued, fin = sv.tick()
        saw_queue |= queued > 0
        done += fin
        ticks += 1
        assert ticks < 500
    _flush(f"[server] {len(reqs)} requests in {ticks} ticks, queue seen: {saw_queue}")
    assert saw_queue
    infos = [sv.poll(rid) for rid in ids]
    sv.close()
    for info, (sp, n) in zip(infos, reqs):
        assert info["state"] == fq.REQ_DONE and info["steps_done"] == n
        solo = _solo(dict(sp, addr_words=1, **LAYOUT), n)
        P = orc.params(0, sp["M"], sp["N"], 1.0, sp["u"], dtau=sp["dtau"], target=sp["target_walkers"],
                       seed=sp["seed"])
        a = orc.start_address(0, sp["M"], sp["N"])
        ost, _, _ = orc.run(P, [a], [10.0], 0.0, 1, n, a, 10.0)
        for ref in (solo, ost):
            last = ref[-1]
            for f in ("step", "len", "exact_steps", "inexact_steps", "spawns"):
                assert info["last"][f] == int(last[f]), f
            for f in ("shift", "norm", "hproj", "vproj"):
                assert float(info["last"][f]).hex() == float(last[f]).hex(), f
            tail = ref[ref["step"] * 2 > n]
            assert info["n_mean"] == len(tail)
            assert info["mean_shift"] == _mean_loop(tail["shift"])
            assert info["mean_hproj"] == _mean_loop(tail["hproj"])
            assert info["mean_vproj"] == _mean_loop(tail["vproj"])


def test_copy_state_continues_identically():
    fq = _fq()
    c = synthetic.CONFIGS["c1"]
    kw = dict(t=c["t"], u=c["u"], dtau=c["dtau"], target_walkers=c["target"], seed=c["seed"])
    a = fq.Solver(c["model"], c["M"], c["N"], table_capacity=1024, spawn_capacity=8192, **kw)
    s0 = fq.start_address(c["model"], c["M"], c["N"])
    a.set_state([s0], [10.0], 0.0, 0, ref=s0, yref=10.0)
    a.run(500)
    b = fq.Solver(c["model"], c["M"], c["N"], table_capacity=2048, spawn_capacity=16384,
                  buckets=128, lds_slots=1024, block=256, spawn_block=512, **kw)
    b.copy_state_from(a)
    sa = a.run(300)
    sb = b.run(300)
    assert sa.tobytes() == sb.tobytes()
    a.close()
    b.close()


def test_autotune_picks_a_candidate_and_leaves_source_unchanged():
    fq = _fq()
    c = synthetic.CONFIGS["c1"]
    kw = dict(t=c["t"], u=c["u"], dtau=c["dtau"], target_walkers=c["target"], seed=c["seed"],
              table_capacity=1024, spawn_capacity=8192)
    s0 = fq.start_address(c["model"], c["M"], c["N"])
    ref = fq.Solver(c["model"], c["M"], c["N"], **kw)
    ref.set_state([s0], [10.0], 0.0, 0, ref=s0, yref=10.0)
    r1 = ref.run(400)
    r2 = ref.run(200)
    a = fq.Solver(c["model"], c["M"], c["N"], **kw)
    a.set_state([s0], [10.0], 0.0, 0, ref=s0, yref=10.0)
    assert a.run(400).tobytes() == r1.tobytes()
    cands = [dict(buckets=1, lds_slots=1024, block=256, spawn_block=256),
             dict(buckets=8, lds_slots=1024, block=512, spawn_block=256),
             dict(buckets=4, lds_slots=2048, block=1024, spawn_block=1024),
             dict(buckets=4, lds_slots=8192, block=256)]  # invalid: slots > 8 * block
    ms, best = a.autotune(cands, trial_steps=20)
    _flush(f"[autotune] ms/step {ms}, best {best}")
    assert best in (0, 1, 2) and ms[best] > 0 and ms[3] < 0
    assert a.run(200).tobytes() == r2.tobytes()
    a.close()
    ref.close()


def test_batch_autotune_picks_a_layout_and_leaves_batch_unchanged():
    """fq_batch_autotune times shared layouts on device copies: the best
    candidate is a valid one, an invalid candidate reads negative, the batch
    continues exactly as an untouched twin, and a batch re-created with the
    chosen layout from copied states continues identically too."""
    fq = _fq()
    specs = _real_specs()[:4]
    twins = []
    for _ in range(2):
        b = fq.Batch(specs)
        for i, sp in enumerate(specs):
            a = fq.start_address(sp["model"], sp["M"], sp["N"])
            b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
        b.run(300)
        twins.append(b)
    cands = [dict(lds_slots=1024, block=256, spawn_block=256),
             dict(lds_slots=2048, block=512, spawn_block=256),
             dict(lds_slots=4096, block=1024, spawn_block=512),
             dict(lds_slots=8192, block=256)]  # invalid: slots > 8 * block
    ms, best = twins[0].autotune(cands, trial_steps=10)
    _flush(f"[batch autotune] ms/step {ms}, best {best}")
    assert best in (0, 1, 2) and ms[best] > 0 and ms[3] < 0
    tb = fq.Batch([dict(sp, buckets=0, **cands[best]) for sp in specs])
    for i in range(len(specs)):
        tb.instance(i).copy_state_from(twins[0].instance(i))
    ref = twins[1].run(200)
    assert twins[0].run(200).tobytes() == ref.tobytes()
    assert tb.run(200).tobytes() == ref.tobytes()
    for b in twins + [tb]:
        b.close()
