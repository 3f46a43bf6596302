"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Single steps from the same seeded input state must give bit-identical spawn
events (parent, attempt, destination, value), bit-identical merged
pre-compression amplitudes, the identical compressed state and identical
statistics (the merge, norm and projected-energy sums are exactly rounded on
both sides, so agreement is bit for bit; the floating-point tolerance of the
method, 1e-12 relative, is therefore met with margin).
"""
import sys

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


def _fq():
    import paper_2601_19505_amd as fq
    return fq


def _flush(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def one_step(orc, model, M, N, u, dtau, n_entries, seed, W=1, buckets=4, slots=2048, block=512,
             t_rel=1.0, theta=1.0, step=6, shift=-1.3, sector=None, lo=0.05, hi=300.0, t=1.0,
             spawn_block=None, early=False, lx=0, g=0.0, initiator=None):
    fq = _fq()
    spawn_block = block if spawn_block is None else spawn_block
    _flush(f"[one_step] model={model} M={M} N={N} lx={lx} g={g} W={W} n={n_entries} B={buckets} "
           f"slots={slots} block={block} spawn_block={spawn_block} t_rel={t_rel} early={early} "
           f"initiator={initiator}")
    rng = np.random.default_rng(seed)
    occs = synthetic.random_occupations(rng, M, N, n_entries, momentum_sector=sector)
    vals = synthetic.random_amplitudes(rng, len(occs), lo=lo, hi=hi)
    oaddr = np.array([orc.encode(o) for o in occs], dtype=np.uint64)
    gaddr = fq.encode_many(occs, W)
    assert np.array_equal(gaddr[:, 0], oaddr[:, 0])
    ref_o, ref_g = oaddr[0], gaddr[0]
    P = orc.params(model, M, N, t, u, dtau=dtau, target=1e4, theta=theta, t_rel=t_rel,
                   seed=seed + 99, early=early, lx=lx, g=g, initiator=initiator)
    o = orc.step(P, oaddr, vals, shift, step + 1, ref_o, 10.0, events=True, merged=True)
    # room for the input and for the merged table of the step
    cap_t = max(4096, 4 * len(occs), 2 * len(o["merged_addr"]))
    s = fq.Solver(model, M, N, t=t, u=u, dtau=dtau, target_walkers=1e4, threshold=theta,
                  t_rel=t_rel, seed=seed + 99, addr_words=W,
                  flags=3 | (fq.FLAG_EARLY_COMPRESSION if early else 0), table_capacity=cap_t,
                  spawn_capacity=max(8 * len(o["events"]), 65536), buckets=buckets,
                  lds_slots=slots, block=block, spawn_block=spawn_block, lx=lx, g=g, initiator=initiator)
    s.set_state(gaddr, vals, shift, step, ref=ref_g, yref=10.0)
    ev = s.spawn_dump()
    st = s.run(1)
    mg = s.merged_dump()
    ga, gv, gsh, gstep = s.get_state()
    s.close()
    return o, ev, st, mg, (ga, gv, gsh, gstep), oaddr


def _key2(a):
    a = np.asarray(a, dtype=np.uint64)
    if a.ndim == 1 or a.shape[1] == 1:
        a = a.reshape(-1, 1)
        return [(0, int(x)) for x in a[:, 0]]
    return [(int(x[1]), int(x[0])) for x in a]


def check_parity(o, ev, st, mg, state, oaddr):
    # spawn events: identical multisets keyed by (parent, attempt)
    par, att, dst, val = ev
    go = {}
    for p_, a_, d_, v_ in zip(_key2(par), att, _key2(dst), val):
        go[(p_, int(a_))] = (d_, float(v_).hex())
    oe = o["events"]
    oo = {}
    for e in oe:
        pk = (int(oaddr[e["parent"]][1]), int(oaddr[e["parent"]][0]))
        oo[(pk, int(e["attempt"]))] = ((int(e["dest"][1]), int(e["dest"][0])), float(e["value"]).hex())
    assert len(go) == len(par) == len(oe)
    assert go == oo
    # merged amplitudes before compression: bit-identical
    gm = dict(zip(_key2(mg[0]), (float(x).hex() for x in mg[1])))
    om = dict(zip(_key2(o["merged_addr"]), (float(x).hex() for x in o["merged_val"])))
    assert gm == om
    # compressed state
    ga, gv, gsh, gstep = state
    gs = dict(zip(_key2(ga), (float(x).hex() for x in gv)))
    os_ = dict(zip(_key2(o["addr"]), (float(x).hex() for x in o["val"])))
    assert gs == os_
    # statistics row; every sum exactly rounded (no contribution off the fixed-point grid)
    row = st[0]
    assert int(row["flags"]) == 0
    for f in ("step", "len", "exact_steps", "inexact_steps", "spawns"):
        assert int(row[f]) == int(o["stats"][f]), f
    for f in ("shift", "norm", "hproj", "vproj"):
        assert float(row[f]).hex() == float(o["stats"][f]).hex(), (f, row[f], o["stats"][f])
    assert gsh == row["shift"] and gstep == row["step"]


CASES = [
    # model, M, N, u, dtau, n, seed, W, buckets, slots, block, t_rel
    (0, 6, 6, 6.0, 1e-3, 200, 1, 1, 4, 1024, 256, 1.0),
    (0, 8, 5, 2.5, 1e-2, 600, 2, 1, 8, 2048, 512, 0.5),
    (0, 2, 3, 4.0, 1e-2, 4, 3, 1, 1, 1024, 256, 1.0),
    (0, 12, 12, 6.0, 1e-3, 3000, 4, 2, 16, 4096, 1024, 1.0),
    (0, 20, 20, 6.0, 1e-3, 3000, 5, 2, 16, 4096, 512, 1.0),
    (0, 20, 20, 6.0, 1e-3, 3000, 5, 1, 32, 2048, 1024, 1.0),
    (1, 5, 4, 3.0, 1e-2, 56, 6, 1, 2, 1024, 256, 1.0),
    (1, 8, 8, 4.0, 1e-3, 1500, 7, 1, 8, 2048, 512, 1.0),
    (1, 7, 6, 2.0, 1e-3, 400, 8, 2, 4, 2048, 256, 2.0),
    (0, 7, 7, 1.0, 1e-3, 300, 9, 1, 2, 2048, 512, float("inf")),
    (0, 7, 7, 1.0, 1e-3, 300, 10, 1, 2, 2048, 512, 0.0),
    # two-pass spawn partition (B > 64)
    (0, 12, 12, 6.0, 1e-3, 3000, 15, 1, 256, 2048, 512, 1.0),
    (0, 20, 20, 6.0, 1e-3, 3000, 16, 2, 128, 2048, 1024, 1.0),
    (1, 10, 10, 4.0, 1e-3, 2500, 17, 1, 128, 2048, 1024, 1.0),
    # the most buckets: coarse groups of 512 buckets in the second pass
    (0, 20, 20, 6.0, 1e-3, 3000, 18, 2, 32768, 1024, 512, 1.0),
    (1, 10, 10, 4.0, 1e-3, 2500, 19, 1, 32768, 1024, 256, 1.0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"m{c[0]}_M{c[1]}N{c[2]}_W{c[7]}_B{c[8]}")
def test_single_step_bit_exact(orc, case):
    model, M, N, u, dtau, n, seed, W, B, slots, block, t_rel = case
    r = one_step(orc, model, M, N, u, dtau, n, seed, W, B, slots, block, t_rel=t_rel)
    check_parity(*r)


def test_single_step_momentum_c3_sector(orc):
    # the benchmark model (M = N = 16, u = 4, dtau = 5e-4) in the K = 0 sector
    r = one_step(orc, 1, 16, 16, 4.0, 5e-4, 3000, 11, 1, 512, 4096, 512, sector=0)
    check_parity(*r)


def test_single_step_threshold_and_tiny_values(orc):
    # theta = 0.5 and many sub-threshold amplitudes (compression path)
    r = one_step(orc, 0, 9, 9, 3.0, 2e-3, 800, 12, 1, 8, 2048, 512, theta=0.5, lo=0.01, hi=2.0)
    check_parity(*r)


@pytest.mark.parametrize("M,N,W", [(32, 31, 1), (64, 63, 2)])
def test_single_step_largest_addresses(orc, M, N, W):
    # N+M-1 = 62 bits in one word, 126 bits in two words
    r = one_step(orc, 0, M, N, 1.0, 5e-4, 500, 13, W, 8, 2048, 512)
    check_parity(*r)


def test_tiny_contributions_are_flagged(orc):
    """Sums are exact integer sums on a grid of 2^-80 (Sec. 3.2, annihilation).
    With dtau = 1e-12 the spawn values (about 1e-12 |H c|) are not multiples
    of 2^-80: the row carries ROW_INEXACT, fq_last_error names the step, the
    spawn events stay bit-identical, and every merged sum lies within its
    rounding bound (one 2^-81 per term, plus half an ulp of each final
    rounding) of the oracle's exactly rounded sum."""
    fq = _fq()
    o, ev, st, mg, state, oaddr = one_step(orc, 0, 6, 6, 6.0, 1e-12, 300, 21, 1, 4, 1024, 256,
                                           lo=0.05, hi=2.0)
    assert int(st[0]["flags"]) & fq.ROW_INEXACT
    par, att, dst, val = ev
    go = {(p_, int(a_)): (d_, float(v_).hex()) for p_, a_, d_, v_ in zip(_key2(par), att, _key2(dst), val)}
    oo = {((int(oaddr[e["parent"]][1]), int(oaddr[e["parent"]][0])), int(e["attempt"])):
          ((int(e["dest"][1]), int(e["dest"][0])), float(e["value"]).hex()) for e in o["events"]}
    assert go == oo
    nterm = {}
    for e in o["events"]:
        k = (int(e["dest"][1]), int(e["dest"][0]))
        nterm[k] = nterm.get(k, 0) + 1
    for a in oaddr:
        k = (int(a[1]), int(a[0]))
        nterm[k] = nterm.get(k, 0) + 1
    gm = dict(zip(_key2(mg[0]), mg[1]))
    om = dict(zip(_key2(o["merged_addr"]), o["merged_val"]))
    assert set(gm) == set(om)
    worst = 0
    for k, w in om.items():
        tol = nterm[k] * 2.0 ** -81 + np.spacing(abs(w)) + np.spacing(abs(gm[k]))
        assert abs(gm[k] - w) <= tol, (k, gm[k], w)
        worst += gm[k] != w
    assert worst > 0  # some sums did round off the oracle's value


def test_inexact_flag_reported_by_run(orc):
    """A run whose sums leave the exact domain says so in fq_last_error."""
    fq = _fq()
    s = fq.Solver(0, 6, 6, u=6.0, dtau=1e-12, target_walkers=1e3, seed=5, table_capacity=1024,
                  spawn_capacity=8192)
    a = fq.start_address(0, 6, 6)
    s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = s.run(5)
    msg = s.last_error()
    s.close()
    assert np.all(st["flags"] & fq.ROW_INEXACT)
    assert "FQ_ROW_INEXACT" in msg and "step 1" in msg


def test_single_entry_state(orc):
    r = one_step(orc, 0, 6, 6, 6.0, 1e-2, 1, 14, 1, 1, 1024, 256)
    check_parity(*r)


EARLY_CASES = [
    # model, M, N, u, dtau, n, seed, W, buckets, slots, block, t_rel, theta
    (0, 6, 6, 6.0, 1e-3, 200, 31, 1, 4, 1024, 256, 1.0, 1.0),
    (1, 8, 8, 4.0, 1e-3, 1500, 32, 1, 8, 2048, 512, 1.0, 1.0),
    (0, 20, 20, 6.0, 1e-3, 3000, 33, 2, 128, 2048, 1024, 1.0, 0.5),
    (1, 10, 10, 4.0, 1e-3, 2500, 34, 1, 128, 2048, 1024, 0.0, 2.0),
]


@pytest.mark.parametrize("case", EARLY_CASES, ids=lambda c: f"early_m{c[0]}_M{c[1]}_W{c[7]}_B{c[8]}")
def test_single_step_early_compression_bit_exact(orc, case):
    model, M, N, u, dtau, n, seed, W, B, slots, block, t_rel, theta = case
    r = one_step(orc, model, M, N, u, dtau, n, seed, W, B, slots, block, t_rel=t_rel, theta=theta,
                 early=True, lo=0.01, hi=50.0)
    check_parity(*r)


LATTICE_CASES = [
    # model, M, N, lx, g, t, u, dtau, n, seed, W, buckets, slots, block, t_rel, early
    (2, 9, 9, 3, 0.0, 1.0, 2.0, 1e-3, 400, 41, 1, 4, 2048, 512, 1.0, False),
    (2, 9, 9, 3, 0.5, 1.0, 2.0, 1e-3, 400, 42, 1, 4, 2048, 512, 1.0, False),
    (2, 12, 10, 4, 0.3, 1.0, 1.0, 1e-3, 1500, 43, 2, 16, 2048, 1024, 0.5, False),
    (2, 4, 5, 2, 0.2, 1.0, 2.0, 1e-2, 50, 46, 1, 1, 1024, 256, 1.0, False),
    (2, 16, 12, 4, 0.5, 1.0, 1.0, 1e-3, 800, 47, 1, 32, 4096, 1024, 0.0, False),
    (0, 8, 8, 0, 0.4, 1.0, 3.0, 1e-3, 600, 45, 1, 8, 2048, 512, 1.0, False),
    (2, 9, 9, 3, 0.5, 1.0, 2.0, 1e-3, 400, 48, 1, 4, 2048, 512, 1.0, True),
    # the largest two-word address: a 9 x 7 lattice with N = 64 (126 bits)
    (2, 63, 64, 9, 0.3, 1.0, 1.0, 5e-4, 500, 49, 2, 8, 2048, 512, 1.0, False),
    # the benchmark system of Sec. 7.2 (6 x 6, N = 36, 71-bit addresses), two-pass partition
    (2, 36, 36, 6, 1.0, 0.1, 1.0, 1.5e-3, 3000, 44, 2, 128, 4096, 1024, 1.0, False),
]


@pytest.mark.parametrize("case", LATTICE_CASES,
                         ids=lambda c: f"lat_m{c[0]}_M{c[1]}_lx{c[3]}_g{c[4]}_W{c[10]}_B{c[11]}_e{int(c[15])}")
def test_single_step_lattice_bit_exact(orc, case):
    """Square lattice and Gutzwiller importance sampling (Sec. 3.3, Sec.
    7.2): spawn events, merged sums, the compressed state and every
    statistic (the projected energy through the row of the reference)
    bit-identical to the oracle."""
    model, M, N, lx, g, t, u, dtau, n, seed, W, B, slots, block, t_rel, early = case
    r = one_step(orc, model, M, N, u, dtau, n, seed, W, B, slots, block, t_rel=t_rel, t=t, lx=lx, g=g,
                 early=early, lo=0.05 if not early else 0.01, hi=300.0 if not early else 50.0)
    check_parity(*r)


def test_small_lattice_trajectory_and_energies(orc):
    """The 3 x 2 lattice with N = 6 at the couplings of the Sec. 7.2
    benchmark (u = 1, t = 0.1, g = 1, dtau = 0.01, N_t = 1e3): all 1e4
    statistics rows equal the oracle's bit for bit, and the shift and the
    projected energy agree with exact diagonalisation within 3 sigma."""
    from oracle import stats
    fq = _fq()
    c = synthetic.CONFIGS["c2d_small"]
    _flush("[lattice trajectory] 3 x 2, N = 6, 10000 steps")
    s = fq.Solver(c["model"], c["M"], c["N"], t=c["t"], u=c["u"], dtau=c["dtau"],
                  target_walkers=c["target"], seed=c["seed"], addr_words=1, table_capacity=1024,
                  spawn_capacity=8192, lx=c["lx"], g=c["g"])
    a = fq.start_address(c["model"], c["M"], c["N"])
    s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = s.run(c["steps"])
    s.close()
    P = orc.params(c["model"], c["M"], c["N"], c["t"], c["u"], dtau=c["dtau"], target=c["target"],
                   seed=c["seed"], lx=c["lx"], g=c["g"])
    oa = orc.start_address(c["model"], c["M"], c["N"])
    ost, _, _ = orc.run(P, [oa], [10.0], 0.0, 1, c["steps"], oa, 10.0)
    for f in ost.dtype.names:
        assert st[f].tobytes() == ost[f].tobytes(), f
    E0 = np.linalg.eigvalsh(orc.dense_matrix(orc.ham(c["model"], c["M"], c["N"], c["t"], c["u"],
                                                     lx=c["lx"])))[0]
    se = stats.shift_estimator(st["shift"], skip=2000)
    pe = stats.projected_energy(st["hproj"], st["vproj"], skip=2000)
    _flush(f"[lattice energies] shift {se.mean:.6f} +- {se.err:.6f}, projected {pe.ratio:.6f} +- "
           f"{pe.err:.6f}, ED {E0:.8f}")
    assert abs(se.mean - E0) < 3 * se.err
    assert abs(pe.ratio - E0) < 3 * pe.err


def _c1_gpu(steps, buckets=0, slots=0, block=0, spawn_block=0, early=False):
    fq = _fq()
    c = synthetic.CONFIGS["c1"]
    s = fq.Solver(c["model"], c["M"], c["N"], t=c["t"], u=c["u"], dtau=c["dtau"],
                  target_walkers=c["target"], seed=c["seed"], addr_words=1,
                  flags=fq.FLAG_EARLY_COMPRESSION if early else 0, table_capacity=1024,
                  spawn_capacity=8192, buckets=buckets, lds_slots=slots, block=block,
                  spawn_block=spawn_block)
    a = fq.start_address(c["model"], c["M"], c["N"])
    s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = s.run(steps)
    s.close()
    return st


@pytest.mark.parametrize("early", [False, True], ids=["late", "early"])
def test_c1_trajectory_bit_exact_vs_oracle(orc, early):
    """The 6/6 ring at u = 6 (N_t = 1e3) end to end (1e4 steps): every
    statistics row of the GPU run equals the oracle's bit for bit (late and
    early compression)."""
    _flush(f"[c1 trajectory] 10000 steps, early={early}")
    c = synthetic.CONFIGS["c1"]
    st = _c1_gpu(c["steps"], early=early)
    P = orc.params(c["model"], c["M"], c["N"], c["t"], c["u"], dtau=c["dtau"], target=c["target"],
                   seed=c["seed"], early=early)
    a = orc.start_address(c["model"], c["M"], c["N"])
    ost, _, _ = orc.run(P, [a], [10.0], 0.0, 1, c["steps"], a, 10.0)
    for f in ost.dtype.names:
        g, o = st[f], ost[f]
        if g.dtype.kind == "f":
            bad = np.nonzero(g.view(np.uint64) != o.view(np.uint64))[0]
        else:
            bad = np.nonzero(g != o)[0]
        assert len(bad) == 0, (f, bad[:5], g[bad[:5]], o[bad[:5]])


@pytest.mark.parametrize("early", [False, True], ids=["late", "early"])
def test_c1_energy_within_3_sigma_of_ed(orc, early):
    from oracle import stats
    st = _c1_gpu(10_000, early=early)
    E0 = orc.eigs_sparse(orc.ham(0, 6, 6, 1.0, 6.0), 1)[0]
    se = stats.shift_estimator(st["shift"], skip=2000)
    pe = stats.projected_energy(st["hproj"], st["vproj"], skip=2000)
    _flush(f"[c1 energy] shift {se.mean:.5f} +- {se.err:.5f}  proj {pe.ratio:.5f} +- {pe.err:.5f}  "
           f"E0 {E0:.8f}")
    assert abs(se.mean - E0) < 3 * se.err
    assert abs(pe.ratio - E0) < 3 * pe.err


def test_schedule_independence():
    """Bucket count, LDS table size and workgroup size do not change a bit."""
    ref = _c1_gpu(3000)
    for B, slots, block, sb in [(1, 1024, 256, 1024), (8, 1024, 1024, 256), (64, 4096, 512, 512),
                                (2, 2048, 1024, 256), (128, 1024, 256, 256)]:
        st = _c1_gpu(3000, B, slots, block, sb)
        assert st.tobytes() == ref.tobytes(), (B, slots, block, sb)


INITIATOR_CASES = [
    # model, M, N, lx, g, t, u, dtau, n, seed, W, buckets, slots, block, t_rel, early, n_a
    (0, 8, 5, 0, 0.0, 1.0, 2.5, 1e-2, 600, 51, 1, 8, 2048, 512, 0.5, False, 20.0),
    (0, 12, 12, 0, 0.0, 1.0, 6.0, 1e-3, 3000, 52, 2, 16, 4096, 1024, 1.0, False, 20.0),
    # 32 address bits: 16-byte records, the flag in bit 63
    (0, 20, 13, 0, 0.0, 1.0, 4.0, 1e-3, 2000, 53, 1, 16, 2048, 512, 1.0, False, 20.0),
    # the momentum benchmark system (31 bits): 12-byte records, the flag in bit 31
    (1, 16, 16, 0, 0.0, 1.0, 4.0, 5e-4, 3000, 54, 1, 64, 4096, 512, 1.0, False, 20.0),
    (1, 8, 8, 0, 0.0, 1.0, 4.0, 1e-3, 1500, 55, 1, 8, 2048, 512, 1.0, False, 0.0),
    (1, 7, 6, 0, 0.0, 1.0, 2.0, 1e-3, 400, 56, 2, 4, 2048, 256, 2.0, False, float("inf")),
    # two-pass partition
    (1, 10, 10, 0, 0.0, 1.0, 4.0, 1e-3, 2500, 57, 1, 128, 2048, 1024, 1.0, False, 30.0),
    (0, 20, 20, 0, 0.0, 1.0, 6.0, 1e-3, 3000, 58, 2, 128, 2048, 1024, 1.0, False, 50.0),
    # lattice, importance sampling, early compression
    (2, 9, 9, 3, 0.5, 1.0, 2.0, 1e-3, 400, 59, 1, 4, 2048, 512, 1.0, False, 20.0),
    (2, 36, 36, 6, 1.0, 0.1, 1.0, 1.5e-3, 3000, 60, 2, 128, 4096, 1024, 1.0, False, 20.0),
    (0, 8, 8, 0, 0.0, 1.0, 3.0, 1e-3, 600, 61, 1, 8, 2048, 512, 1.0, True, 5.0),
    (2, 9, 9, 3, 0.5, 1.0, 2.0, 1e-3, 400, 62, 1, 4, 2048, 512, 1.0, True, 5.0),
]


@pytest.mark.parametrize("case", INITIATOR_CASES,
                         ids=lambda c: f"init_m{c[0]}_M{c[1]}N{c[2]}_W{c[10]}_B{c[11]}_e{int(c[15])}_na{c[16]}")
def test_single_step_initiator_bit_exact(orc, case):
    """Initiator rule (|c| > n_a; non-initiator spawns count only onto
    addresses of c^(n)): spawn events, merged sums (every input address
    included), the compressed state and the statistics equal the oracle's
    bit for bit."""
    model, M, N, lx, g, t, u, dtau, n, seed, W, B, slots, block, t_rel, early, n_a = case
    r = one_step(orc, model, M, N, u, dtau, n, seed, W, B, slots, block, t_rel=t_rel, t=t, lx=lx, g=g,
                 early=early, lo=0.05 if not early else 0.01, hi=300.0 if not early else 50.0, initiator=n_a)
    check_parity(*r)
    o, mg = r[0], r[3]
    if 0.0 < n_a < float("inf"):
        # the rule acted: some events of non-initiator parents reach an
        # address outside c^(n) and are missing from the merged sums
        merged = set(_key2(mg[0]))
        missed = [e for e in o["events"] if (int(e["dest"][1]), int(e["dest"][0])) not in merged]
        assert missed


def test_initiator_trajectory_bit_exact_vs_oracle(orc):
    """The 6/6 ring at u = 6 with the initiator rule at n_a = 3 for 3000
    steps from one start address: every statistics row of the GPU run equals
    the oracle's bit for bit."""
    fq = _fq()
    c = synthetic.CONFIGS["c1"]
    steps = 3000
    _flush(f"[initiator trajectory] {steps} steps")
    s = fq.Solver(c["model"], c["M"], c["N"], t=c["t"], u=c["u"], dtau=c["dtau"],
                  target_walkers=c["target"], seed=c["seed"], addr_words=1, table_capacity=1024,
                  spawn_capacity=8192, initiator=3.0)
    a = fq.start_address(c["model"], c["M"], c["N"])
    s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    st = s.run(steps)
    s.close()
    P = orc.params(c["model"], c["M"], c["N"], c["t"], c["u"], dtau=c["dtau"], target=c["target"],
                   seed=c["seed"], initiator=3.0)
    oa = orc.start_address(c["model"], c["M"], c["N"])
    ost, _, _ = orc.run(P, [oa], [10.0], 0.0, 1, steps, oa, 10.0)
    for f in ost.dtype.names:
        gv, ov = st[f], ost[f]
        if gv.dtype.kind == "f":
            bad = np.nonzero(gv.view(np.uint64) != ov.view(np.uint64))[0]
        else:
            bad = np.nonzero(gv != ov)[0]
        assert len(bad) == 0, (f, bad[:5], gv[bad[:5]], ov[bad[:5]])
