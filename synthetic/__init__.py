"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  This module holds none of the method's arithmetic: it produces
occupation-number vectors, amplitudes and parameter sets; each side (the CPU
oracle and the GPU library) encodes and processes them with its own code.

Workloads (all t = 1, threshold 1, 1D periodic Bose-Hubbard):

* `c1`: real space M = N = 6, u = 6, dtau = 1e-3, N_t = 1e3, 1e4 steps, seed 0,
  uniform start with 10 walkers;
* `c2`: real space M = N = 20, u = 6, dtau = 1e-3, N_t = 1e7, 2e4 steps, seed 1,
  128-bit (W = 2) addresses;
* `c3`: momentum space M = N = 16, u = 4, dtau = 5e-4, N_t = 1e8, 5e3 steps,
  seed 2, start from the k = 0 condensate with 10 walkers;
* the batch: 64 real-space instances, M = N uniform in 8..24, u log-uniform in
  [1, 10], N_t log-linear in log D mapped into [1e4, 1e7], seeds 1000 + i;
* the stream: a Poisson stream (rate 50/s) of real-space solves, M = N in 6..20,
  u uniform in [1, 10], 2e3..2e4 steps, N_t log-uniform in [1e3, 1e7];
* the benchmark system of Sec. 7.2: the periodic 6 x 6 square lattice with
  N = 36, u = 1, t = 0.1, Gutzwiller importance sampling (g = 1, reading),
  dtau = 1.5e-3 (reading: half the stability bound 2 / (E_max - E_0) of
  Sec. 3.1, about 3.0e-3 here), N_t = 1e7, 71-bit (W = 2) addresses, seed 3; and a
  3 x 2 lattice with N = 6 and the same couplings at N_t = 1e3, small enough
  for exact diagonalisation.
"""
import math

import numpy as np

REAL1D = 0
MOM1D = 1
REAL2D = 2

CONFIGS = {
    "c1": dict(model=REAL1D, M=6, N=6, t=1.0, u=6.0, dtau=1e-3, target=1e3, steps=10_000,
               seed=0, W=1, theta=1.0),
    "c2": dict(model=REAL1D, M=20, N=20, t=1.0, u=6.0, dtau=1e-3, target=1e7, steps=20_000,
               seed=1, W=2, theta=1.0),
    "c3": dict(model=MOM1D, M=16, N=16, t=1.0, u=4.0, dtau=5e-4, target=1e8, steps=5_000,
               seed=2, W=1, theta=1.0),
    "c2d": dict(model=REAL2D, M=36, N=36, lx=6, t=0.1, u=1.0, g=1.0, dtau=1.5e-3, target=1e7,
                steps=50_000, seed=3, W=2, theta=1.0),
    "c2d_small": dict(model=REAL2D, M=6, N=6, lx=3, t=0.1, u=1.0, g=1.0, dtau=1e-2, target=1e3,
                      steps=10_000, seed=0, W=1, theta=1.0),
}


def start_occupation(model, M, N):
    if model == MOM1D:
        return [N] + [0] * (M - 1)
    return [N // M + (1 if j < N % M else 0) for j in range(M)]


def random_occupations(rng, M, N, n, momentum_sector=None):
    """n distinct random occupation vectors with N bosons in M modes
    (stars and bars: uniform over the Fock basis).  With momentum_sector=K
    only states whose total momentum sum_j j n_j = K (mod M) are kept."""
    seen = set()
    out = []
    tries = 0
    while len(out) < n and tries < 200 * n + 1000:
        tries += 1
        bars = np.sort(rng.choice(N + M - 1, M - 1, replace=False))
        edges = np.concatenate([[-1], bars, [N + M - 1]])
        occ = tuple(int(x) for x in np.diff(edges) - 1)
        if momentum_sector is not None and sum(j * o for j, o in enumerate(occ)) % M != momentum_sector:
            continue
        if occ in seen:
            continue
        seen.add(occ)
        out.append(occ)
    return np.array(out, dtype=np.int32).reshape(-1, M)


def random_amplitudes(rng, n, lo=0.05, hi=300.0, signed=True, heavy=0.1):
    """Amplitudes with a log-uniform magnitude in [lo, hi]; a fraction
    `heavy` of entries is raised into [hi, 10 hi] so that exact columns,
    stochastic columns and sub-threshold values all occur."""
    mag = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    k = rng.random(n) < heavy
    mag[k] *= rng.uniform(1.0, 10.0, k.sum())
    if signed:
        mag *= rng.choice([-1.0, 1.0], n)
    return mag


def batch_instances(n=64, seed=4242):
    """The 64-instance batch: M = N ~ U{8..24}, u = exp(U[ln 1, ln 10]),
    N_t log-linear in log D into [1e4, 1e7], dtau_i = min(1e-3,
    1/(u N(N-1)/2 + 4 t N)), seeds 1000 + i."""
    rng = np.random.default_rng(seed)
    out = []
    Ms = rng.integers(8, 25, n)
    us = np.exp(rng.uniform(0.0, math.log(10.0), n))
    logD = np.array([math.log(math.comb(2 * m - 1, m)) for m in Ms])
    lo, hi = math.log(math.comb(15, 8)), math.log(math.comb(47, 24))
    for i in range(n):
        M = int(Ms[i])
        frac = (logD[i] - lo) / (hi - lo)
        target = float(10 ** (4 + 3 * frac))
        u = float(us[i])
        dtau = min(1e-3, 1.0 / (u * M * (M - 1) / 2 + 4 * M))
        out.append(dict(model=REAL1D, M=M, N=M, t=1.0, u=u, dtau=dtau, target=target,
                        seed=1000 + i, W=1, theta=1.0))
    return out


def poisson_requests(n=1000, rate=50.0, seed=77, steps=(2000, 20000), walkers=(1e3, 1e7),
                     sizes=(6, 20)):
    """Finite Poisson request stream: arrival times and solve parameters."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    reqs = []
    for i in range(n):
        M = int(rng.integers(sizes[0], sizes[1] + 1))
        u = float(rng.uniform(1.0, 10.0))
        dtau = min(1e-3, 1.0 / (u * M * (M - 1) / 2 + 4 * M))
        reqs.append(dict(arrival=float(t[i]), model=REAL1D, M=M, N=M, t=1.0, u=u, dtau=dtau,
                         target=float(math.exp(rng.uniform(math.log(walkers[0]),
                                                           math.log(walkers[1])))),
                         steps=int(rng.integers(steps[0], steps[1] + 1)), seed=5000 + i, W=1,
                         theta=1.0))
    return reqs
