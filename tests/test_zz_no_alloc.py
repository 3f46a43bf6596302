"""The allocation-free replica entry point (fq_batch_run_replicas_static)
against the entry point with a caller scratch buffer (fq_batch_run_replicas),
through the C ABI: two calls in a row, the second with a smaller input (two
replicas of a smaller batch after three replicas of a larger one), must give
bit-identical statistics rows, overlaps and states; a batch whose scratch
exceeds the static array is rejected."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _flush(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _batch(fq, R, M, target, buckets, table, spawn, seeds):
    specs = [dict(model=fq.REAL1D, M=M, N=M, t=1.0, u=4.0, dtau=1e-3, target_walkers=target, seed=s,
                  table_capacity=table, spawn_capacity=spawn, buckets=buckets, lds_slots=2048, block=512)
             for s in seeds[:R]]
    b = fq.Batch(specs)
    a = fq.start_address(fq.REAL1D, M, M)
    for i in range(R):
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    return b


def _state_map(b, R):
    out = []
    for i in range(R):
        a, v, sh, st = b.instance(i).get_state()
        out.append(({int(x): float(y).hex() for x, y in zip(a[:, 0], v)}, float(sh).hex(), st))
    return out


def _compare(fq, R, M, target, buckets, table, spawn, steps):
    seeds = [11, 12, 13]
    _flush(f"[no-alloc] R={R} M=N={M} N_t={target} buckets={buckets} steps={steps}")
    ref = _batch(fq, R, M, target, buckets, table, spawn, seeds)
    st_r, ov_r, inx_r = ref.run_replicas(steps)
    sref = _state_map(ref, R)
    ref.close()
    b = _batch(fq, R, M, target, buckets, table, spawn, seeds)
    st_s, ov_s, inx_s = b.run_replicas_static(steps)
    sst = _state_map(b, R)
    b.close()
    assert st_s.tobytes() == st_r.tobytes()
    assert ov_s.tobytes() == ov_r.tobytes()
    assert inx_s == inx_r
    assert sst == sref
    return ov_s


def test_static_scratch_equals_caller_scratch():
    import paper_2601_19505_amd as fq
    # first call: three replicas, 64 buckets; second call, in a row on the
    # same GPU (the static array still holds the first call's contents): two
    # replicas, 16 buckets
    ov1 = _compare(fq, 3, 10, 2e4, 64, 60000, 400000, 600)
    ov2 = _compare(fq, 2, 8, 3e3, 16, 8192, 65536, 400)
    assert ov1.shape == (600, 3) and ov2.shape == (400, 1)
    assert np.all(np.isfinite(ov1)) and np.all(np.isfinite(ov2))


def test_static_scratch_rejects_too_large_batches():
    import paper_2601_19505_amd as fq
    # eight replicas at 8192 buckets need about 6.4 MB of scratch (> 4 MiB)
    b = _batch(fq, 8, 8, 1e3, 8192, 4096, 16384, list(range(8)))
    with pytest.raises(fq.FqError, match="static scratch"):
        b.run_replicas_static(2)
    b.close()
