"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol the header declares, and its host helpers agree with the oracle."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT

import paper_2601_19505_amd as fq
import synthetic


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(fq_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = fq.lib()
    names = _declared()
    assert "fq_run" in names and "fq_set_state" in names
    for n in names:
        assert hasattr(L, n), n
    assert b"gfx950" in L.fq_version()


def test_encode_matches_oracle(orc):
    rng = np.random.default_rng(3)
    for M, N, W in [(6, 6, 1), (20, 20, 2), (16, 16, 1), (2, 5, 1), (32, 31, 1), (64, 63, 2)]:
        occs = synthetic.random_occupations(rng, M, N, 50)
        for o in occs:
            g = fq.encode(o, W)
            w0, w1 = orc.encode(o)
            assert int(g[0]) == w0
            assert (int(g[1]) if W == 2 else 0) == w1


def test_encode_rejects_overflow():
    with pytest.raises(fq.FqError):
        fq.encode([40, 40], 1)


def _ws(model=0, M=6, N=6, W=1, lx=0, g=0.0, t=1.0, u=6.0, dtau=1e-3, target=1e3, theta=1.0,
        flags=0, n_a=0.0, **kw):
    h = fq.Hamiltonian(model, M, N, lx, t, u, g)
    p = fq.Params(dtau, target, 0.08, 0.0016, theta, 1.0, 0, W, flags, n_a)
    lay = fq.Layout(kw.get("table", 1000), kw.get("spawn", 4000), kw.get("buckets", 0),
                    kw.get("slots", 0), kw.get("block", 0), kw.get("spawn_block", 0))
    return fq.workspace_size(h, p, lay)


def test_workspace_size_and_defaults():
    n, lay = _ws()
    assert n > 0 and lay.buckets >= 1 and lay.lds_slots == 4096 and lay.block == 1024
    assert lay.spawn_block == 256
    n2, lay2 = _ws(table=10_000_000, spawn=40_000_000)
    assert n2 > n and lay2.buckets & (lay2.buckets - 1) == 0 and lay2.buckets > 1000
    n3, lay3 = _ws(model=1, M=16, N=16)
    assert lay3.block == 512


@pytest.mark.parametrize("kw", [dict(M=1), dict(model=1, M=2, N=3), dict(M=40, N=30, W=1),
                                dict(slots=3000), dict(block=128), dict(slots=8192, block=512),
                                dict(buckets=3), dict(spawn_block=128), dict(spawn_block=2048),
                                dict(model=2, M=9, lx=1), dict(model=2, M=10, lx=3),
                                dict(model=2, M=6, lx=6), dict(model=1, M=8, g=0.1),
                                dict(g=float("nan")), dict(model=2, M=36, N=36, lx=6, W=1, u=1.0),
                                dict(target=float("inf")), dict(target=0.0), dict(theta=float("nan")),
                                dict(theta=0.0), dict(dtau=0.0), dict(dtau=float("inf")),
                                dict(flags=128, n_a=-1.0), dict(flags=128, n_a=float("nan")),
                                dict(buckets=65536)])
def test_workspace_size_rejects_invalid(kw):
    with pytest.raises(fq.FqError):
        _ws(**kw)


def test_largest_bucket_count_accepted():
    n, lay = _ws(buckets=32768, slots=1024, block=512, table=10_000_000, spawn=40_000_000)
    assert n > 0 and lay.buckets == 32768


def test_initiator_threshold_accepted():
    """The initiator rule takes any n_a >= 0, infinity included; without
    the flag the threshold is ignored."""
    for n_a in (0.0, 3.0, float("inf")):
        assert _ws(flags=fq.FLAG_INITIATOR, n_a=n_a)[0] > 0
    assert _ws(n_a=-1.0)[0] > 0
    # the flag bit sits above the 31 address bits of the momentum benchmark
    assert _ws(model=1, M=16, N=16, flags=fq.FLAG_INITIATOR, n_a=3.0)[0] > 0


def test_lattice_workspace_sizes():
    """The 6 x 6 lattice with 36 bosons needs two address words (71 bits)."""
    n, lay = _ws(model=2, M=36, N=36, lx=6, W=2, g=1.0, t=0.1, u=1.0, table=1000, spawn=4000)
    assert n > 0
    n1, _ = _ws(model=0, M=6, N=6, g=0.5)
    assert n1 > 0


def test_solver_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        fq.Solver(0, 6, 6)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asking for more exits with a message."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _width_bound(model, N, t, u):
    z = 4.0 if model == 2 else 2.0
    return abs(u) * 0.5 * N * (N - 1) + 2.0 * z * abs(t) * N


@pytest.mark.parametrize("model,M,N,lx,t,u,g", [
    (0, 6, 6, 0, 1.0, 6.0, 0.0),      # the 6/6 ring of the accuracy examples
    (1, 16, 16, 0, 1.0, 4.0, 0.0),    # the momentum-space benchmark
    (2, 36, 36, 6, 0.1, 1.0, 1.0),    # the 6 x 6 lattice of the performance benchmarks
    (0, 12, 12, 0, 1.0, 6.0, 0.0),
    (0, 20, 20, 0, 1.0, -2.0, 0.3),   # attractive interaction, importance sampling
])
def test_dtau_stability_bound(model, M, N, lx, t, u, g):
    """dtau is checked against the stability bound of Sec. 3.1, dtau <
    2 / (E_max - E_0), with E_max - E_0 bounded by |u| N (N-1)/2 + 2 z |t| N:
    just below the bound is accepted, just above rejected, and the unchecked
    flag accepts it."""
    W = 2 if N + M - 1 > 62 else 1
    lim = 2.0 / _width_bound(model, N, t, u)
    kw = dict(model=model, M=M, N=N, lx=lx, t=t, u=u, g=g, W=W)
    assert _ws(dtau=lim * 0.999, **kw)[0] > 0
    with pytest.raises(fq.FqError, match="stability bound"):
        _ws(dtau=lim * 1.001, **kw)
    assert _ws(dtau=lim * 1.001, flags=fq.FLAG_UNCHECKED_DTAU, **kw)[0] > 0


@pytest.mark.parametrize("model,M,N,lx,t,u,g", [
    (0, 6, 6, 0, 1.0, 6.0, 0.0), (0, 5, 7, 0, 1.0, -3.0, 0.0), (0, 2, 5, 0, 1.0, 4.0, 0.0),
    (1, 6, 6, 0, 1.0, 6.0, 0.0), (1, 5, 4, 0, 0.5, 3.0, 0.0),
    (2, 4, 5, 2, 1.0, 2.0, 0.2), (2, 6, 6, 3, 0.1, 1.0, 1.0), (2, 9, 4, 3, 1.0, 0.5, 0.0),
])
def test_width_bound_holds_against_dense_spectrum(orc, model, M, N, lx, t, u, g):
    """The width bound the dtau check uses is an upper bound on the true
    spectral width E_max - E_0 (dense eigenvalues of small systems; the
    similarity transform of importance sampling keeps the spectrum)."""
    h = orc.ham(model, M, N, t, u, lx=lx, g=g)
    ev = np.linalg.eigvals(orc.dense_matrix(h)).real
    assert ev.max() - ev.min() <= _width_bound(model, N, t, u) * (1 + 1e-12)
