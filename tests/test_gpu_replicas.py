"""Replica overlaps and the variational energy on the GPU [Sec. 4.3].

Replicas are batch instances of one Hamiltonian with different seeds.  Each
replica's trajectory is bit-identical to the oracle's, and the overlap
c_A . c_B after every step is the exactly rounded sum of the rounded
products, so the overlap series is compared with the oracle's bit for bit;
at the full momentum-space size the last overlap is compared with the
oracle's overlap of the two exported states.
"""
import sys

import numpy as np
import pytest

import synthetic
from oracle import stats
from test_oracle_replicas import replica_trajectories

pytestmark = pytest.mark.gpu


def _flush(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _replicas(fq, R, seeds, M=6, N=6, u=6.0, dtau=1e-3, target=1e3, W=1, table=1024, spawn=8192,
              buckets=0, **lay):
    specs = [dict(model=fq.REAL1D, M=M, N=N, t=1.0, u=u, dtau=dtau, target_walkers=target, seed=s,
                  addr_words=W, table_capacity=table, spawn_capacity=spawn, buckets=buckets, **lay)
             for s in seeds[:R]]
    b = fq.Batch(specs)
    a = fq.start_address(fq.REAL1D, M, N, W)
    for i in range(R):
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    return b


@pytest.mark.parametrize("R,W,buckets,M,u,target,steps", [
    (2, 1, 0, 6, 6.0, 1e3, 1000),
    (3, 2, 4, 6, 6.0, 1e3, 400),
    (2, 1, 64, 8, 3.0, 5e3, 400),
    (8, 1, 2, 5, 4.0, 3e2, 200),  # the largest replica set, 28 pairs
])
def test_replica_overlaps_bit_exact(orc, R, W, buckets, M, u, target, steps):
    import paper_2601_19505_amd as fq
    seeds = [0, 1, 5, 6, 7, 8, 9, 10]
    _flush(f"[replicas] R={R} W={W} buckets={buckets} M=N={M} u={u} steps={steps}")
    b = _replicas(fq, R, seeds, M=M, N=M, u=u, target=target, W=W, buckets=buckets,
                  table=16384, spawn=131072)
    st, ov, inexact = b.run_replicas(steps)
    b.close()
    shifts, want, rows, _ = replica_trajectories(orc, R, steps, seeds[:R], M=M, N=M, u=u, target=target)
    assert not inexact
    assert ov.shape == (steps, R * (R - 1) // 2)
    for r in range(R):
        assert np.array_equal(st[r]["shift"], shifts[r])
        assert np.array_equal(st[r]["len"], [x["len"] for x in rows[r]])
    assert ov.T.tobytes() == want.tobytes()
    assert np.all(ov[-1] > 0)


def test_replicas_c1_variational_energy_within_3_sigma_of_ed(orc):
    """Two replicas of the 6/6 ring at u = 6 (N_t = 1e3) for 1e4 steps: the
    overlap series equals the oracle's bit for bit and the variational
    energy agrees with exact diagonalisation within three standard errors."""
    import paper_2601_19505_amd as fq
    b = _replicas(fq, 2, [0, 1])
    st, ov, _ = b.run_replicas(10000)
    b.close()
    shifts, want, _, _ = replica_trajectories(orc, 2, 10000, [0, 1])
    assert ov.T.tobytes() == want.tobytes()
    E0 = orc.eigs_sparse(orc.ham(orc.REAL1D, 6, 6, 1.0, 6.0), 1)[0]
    r = stats.variational_energy(np.stack([st[0]["shift"], st[1]["shift"]]), ov.T, skip=2000)
    _flush(f"[replicas c1] variational energy {r.ratio:.6f} +- {r.err:.6f} (ED {E0:.8f})")
    assert abs(r.ratio - E0) < 3 * r.err


def test_replicas_split_runs_equal_one_run(orc):
    """Chunked calls continue the series exactly (rows do not depend on how
    the steps are split over calls, including the 4096-row chunking)."""
    import paper_2601_19505_amd as fq
    b = _replicas(fq, 2, [3, 4])
    _, ov1, _ = b.run_replicas(5000)
    b.close()
    b = _replicas(fq, 2, [3, 4])
    _, x, _ = b.run_replicas(1234)
    _, y, _ = b.run_replicas(5000 - 1234)
    b.close()
    assert np.concatenate([x, y]).tobytes() == ov1.tobytes()


def test_replica_set_is_validated():
    import paper_2601_19505_amd as fq
    specs = [dict(model=fq.REAL1D, M=6, N=6, t=1.0, u=6.0, dtau=1e-3, target_walkers=1e3, seed=s,
                  table_capacity=1024, spawn_capacity=8192) for s in (0, 1)]
    specs[1]["u"] = 5.0
    b = fq.Batch(specs)
    a = fq.start_address(fq.REAL1D, 6, 6)
    for i in range(2):
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    with pytest.raises(fq.FqError) as ei:
        b.run_replicas(10)
    assert ei.value.status == -1
    b.close()
    one = fq.Batch(specs[:1])
    one.instance(0).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    with pytest.raises(fq.FqError):
        one.run_replicas(10)
    one.close()
    b = _replicas(fq, 2, [0, 1])
    b.instance(1).run(3)  # replicas at different steps
    with pytest.raises(fq.FqError) as ei:
        b.run_replicas(10)
    assert ei.value.status == -1
    b.close()


def test_replicas_full_size_momentum(orc):
    """Two replicas at the full momentum-space size (16/16, u = 4, 1e8
    walkers each): after the growth phase the last overlap equals the
    oracle's overlap of the two exported states, bit for bit."""
    import bench
    import paper_2601_19505_amd as fq
    wl = bench.WORKLOADS["c3"]
    cfg = synthetic.CONFIGS["c3"]
    specs = [dict(model=cfg["model"], M=cfg["M"], N=cfg["N"], t=cfg["t"], u=cfg["u"], dtau=cfg["dtau"],
                  target_walkers=cfg["target"], seed=s, addr_words=cfg["W"], threshold=cfg["theta"],
                  table_capacity=wl["table_capacity"], spawn_capacity=wl["spawn_capacity"],
                  buckets=wl["buckets"], lds_slots=wl["lds_slots"], block=wl["block"],
                  spawn_block=wl["spawn_block"]) for s in (cfg["seed"], cfg["seed"] + 100)]
    b = fq.Batch(specs)
    a = fq.encode(synthetic.start_occupation(cfg["model"], cfg["M"], cfg["N"]), cfg["W"])
    for i in range(2):
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    done = 0
    while done < 1500:
        st, ov, inexact = b.run_replicas(500)
        done += 500
        _flush(f"[replicas c3] step {done} norms {st[0]['norm'][-1]:.4g} {st[1]['norm'][-1]:.4g} "
               f"overlap {ov[-1, 0]:.6g}")
    sa = b.instance(0).get_state()
    sb = b.instance(1).get_state()
    b.close()
    assert not inexact
    assert sa[3] == sb[3] == 1500 and len(sa[1]) > 1_000_000
    want = orc.overlap(sa[0], sa[1], sb[0], sb[1])
    assert float(ov[-1, 0]).hex() == float(want).hex()
