"""Benchmark of the FCIQMC hot path on one MI355X.

Default workload (the configuration the headline metric is quoted on):
momentum-space 1D Bose-Hubbard, M = N = 16, u = 4, t = 1, dtau = 5e-4,
target 1e8 walkers, FP64 amplitudes, seed 2, start from the k = 0 condensate
with 10 walkers.

Schedule (the paper likewise equilibrates before it times, Sec. 7.2):
  1. ramp, untimed: steps until ||c||_1 first reaches N_t, then 500 more
     steps so that the shift has settled (`ramp_steps` in the output);
  2. `--warmup` untimed steps;
  3. exactly `--steps` steps timed between two torch.cuda.synchronize()
     calls.
No headline value is printed when the mean ||c||_1 of the timed steps is
below 0.9 N_t.

value = walker-steps/s = sum over the timed steps of ||c^(n)||_1 / wall time.
A step is four launches: merge, spawn, spawn partition, shift update.  The
`roofline` object prices the dominant kernel by its algorithmic HBM bytes
(merge of step k: read c^(k-1) and the spawn records of step k, write c^(k);
spawn: read c^(k), write the spawn records of step k+1; 8 W + 8 bytes per
entry or record) over its mean launch time measured with HIP events on the
stream it runs on; `roofline.step` prices the whole step the same way,
(8 W + 8) (L_n + 2 S_n + L_(n+1)) bytes per step over the wall time.  The CPU
oracle is timed on a bounded sample of the same steady-state vector, on one
core and as independent processes on every core the run may use.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthetic  # noqa: E402

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c3": dict(cfg="c3", name="mom1d_M16_N16_u4_dtau5e-4_Nt1e8",
               table_capacity=19_500_000, spawn_capacity=200_000_000, buckets=16384,
               lds_slots=2048, block=512, spawn_block=256, steps=1000),
    "c2": dict(cfg="c2", name="real1d_M20_N20_u6_dtau1e-3_Nt1e7_W2",
               table_capacity=12_000_000, spawn_capacity=40_000_000, buckets=16384,
               lds_slots=2048, block=512, spawn_block=256, steps=1000),
    "c2d": dict(cfg="c2d", name="real2d_6x6_N36_u1_t0.1_g1_dtau1.5e-3_Nt1e7_W2",
                table_capacity=30_000_000, spawn_capacity=60_000_000, buckets=16384,
                lds_slots=2048, block=512, spawn_block=256, steps=2000),
    "c1": dict(cfg="c1", name="real1d_M6_N6_u6_dtau1e-3_Nt1e3",
               table_capacity=1024, spawn_capacity=8192, buckets=0, lds_slots=0, block=0,
               spawn_block=0, steps=10_000),
}


MODEL_NAMES = {0: "real-space 1D Bose-Hubbard ring", 1: "momentum-space 1D Bose-Hubbard",
               2: "real-space Bose-Hubbard on a periodic square lattice, Gutzwiller importance sampling"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "step_kernels_mom1d_M16N16_1e8_hbm_bytes.txt")


def measured_traffic(fq, kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE and
    WRITE_SIZE summary (calibrated against a streaming copy), or None when
    the summary is absent or was taken with other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    digest = [ln.split(":", 1)[1].strip() for ln in lines if ln.startswith("# kernel source sha256:")]
    if not digest or digest[0] != fq.source_digest():
        return None
    total, seen = 0.0, set()
    for i, ln in enumerate(lines):
        if ln.startswith("void " + kernel + "<") and i + 1 < len(lines):
            nxt = lines[i + 1].split()
            if "calibrated" in nxt and nxt[0] in ("FETCH_SIZE", "WRITE_SIZE"):
                total += float(nxt[nxt.index("calibrated") + 1]) * 1e9
                seen.add(nxt[0])
    return total if seen == {"FETCH_SIZE", "WRITE_SIZE"} else None


VALU_PROFILE = os.path.join(ROOT, "profiles", "step_kernels_mom1d_M16N16_1e8_valu_instructions.txt")
# wave64 VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs x
# 2.4 GHz, one instruction per SIMD every 4 cycles
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def measured_valu(fq, kernel):
    """VALU instructions per launch of `kernel` from the committed
    SQ_INSTS_VALU summary, or None when absent or taken with other kernel
    sources."""
    try:
        with open(VALU_PROFILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    digest = [ln.split(":", 1)[1].strip() for ln in lines if ln.startswith("# kernel source sha256:")]
    if not digest or digest[0] != fq.source_digest():
        return None
    for i, ln in enumerate(lines):
        if ln.startswith("void " + kernel + "<"):
            # the counters of this kernel: indented lines up to the next kernel
            for nx in lines[i + 1:]:
                if not nx.startswith(" "):
                    break
                f = nx.split()
                if f and f[0] == "SQ_INSTS_VALU":
                    return float(f[1])
    return None


def make_solver(fq, wl, cfg, **over):
    kw = dict(t=cfg["t"], u=cfg["u"], dtau=cfg["dtau"], target_walkers=cfg["target"],
              seed=cfg["seed"], addr_words=cfg["W"], threshold=cfg["theta"],
              lx=cfg.get("lx", 0), g=cfg.get("g", 0.0),
              table_capacity=wl["table_capacity"], spawn_capacity=wl["spawn_capacity"],
              buckets=wl["buckets"], lds_slots=wl["lds_slots"], block=wl["block"],
              spawn_block=wl["spawn_block"])
    kw.update(over)
    return fq.Solver(cfg["model"], cfg["M"], cfg["N"], **kw)


def _oracle_step_time(cfg, addrs, vals, shift, step_index, order, k):
    """One oracle step over the entries order[:k]: (seconds, walkers, entries)."""
    import oracle
    P = oracle.params(cfg["model"], cfg["M"], cfg["N"], cfg["t"], cfg["u"], dtau=cfg["dtau"],
                      target=cfg["target"], theta=cfg["theta"], seed=cfg["seed"],
                      lx=cfg.get("lx", 0), g=cfg.get("g", 0.0))
    n = len(vals)
    a2 = np.zeros((n, 2), np.uint64)
    a2[:, :addrs.shape[1]] = addrs
    ref = a2[int(np.argmax(np.abs(vals)))]
    idx = order[:k]
    t0 = time.perf_counter()
    oracle.step(P, a2[idx], vals[idx], shift, step_index, ref, 10.0,
                cap=64 * (k + int(np.abs(vals[idx]).sum())) + 1024)
    return time.perf_counter() - t0, float(np.abs(vals[idx]).sum()), k


def _cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return dict(cpu_model=model, nproc=usable, cpu_count=os.cpu_count())


# worker processes of the all-cores figure: at most this many (the CPU share
# of one GPU on a shared node)
CPU_WORKERS_MAX = 16


def cpu_baseline(state, cfg, step_index, shift, budget_s=15.0):
    """Time the oracle's step on a bounded sample of the steady-state vector:
    on one host core, and as independent processes on every usable core
    (each on its own random sample of the same size), summed."""
    import subprocess
    import tempfile
    addrs, vals = state
    n = len(vals)
    order = np.random.default_rng(123).permutation(n)
    k = min(n, 4000)
    t_used = 0.0
    while True:
        dt, walkers, _ = _oracle_step_time(cfg, addrs, vals, shift, step_index, order, k)
        t_used += dt
        if dt > budget_s / 3 or k == n or t_used > budget_s:
            break
        k = min(n, int(k * min(8.0, max(2.0, (budget_s / 2) / max(dt, 1e-3)))))
    info = _cpu_info()
    out = dict(value=walkers / dt, unit="walker-steps/s", cores=1, kind="oracle",
               sample=f"one oracle step over {k} of {n} steady-state entries "
                      f"({walkers:.3g} walkers), {dt:.1f} s, serial C on one host core",
               entries_per_s=k / dt, **info)
    # all cores: independent oracle processes (no GPU use), one per usable core
    nw = max(1, min(CPU_WORKERS_MAX, info["nproc"]))
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "state.npz")
        np.savez(path, addrs=addrs, vals=vals)
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker", path,
                                   cfg_key(cfg), str(step_index), repr(shift), str(1000 + i), str(k)],
                                  stdout=subprocess.PIPE, text=True)
                 for i in range(nw)]
        res = [json.loads(p.communicate()[0].strip().splitlines()[-1]) for p in procs]
    rates = [r["walkers"] / r["seconds"] for r in res]
    out["all_cores"] = dict(value=float(sum(rates)), unit="walker-steps/s", processes=nw,
                            kind="oracle",
                            sample=f"{nw} concurrent oracle processes, each one step over its own "
                                   f"random {k} of the {n} steady-state entries")
    return out


def cfg_key(cfg):
    for k, v in synthetic.CONFIGS.items():
        if v is cfg:
            return k
    raise KeyError("not a named configuration")


def oracle_worker(path, key, step_index, shift, seed, k):
    """Entry of one all-cores worker process: one timed oracle step."""
    z = np.load(path)
    addrs, vals = z["addrs"], z["vals"]
    order = np.random.default_rng(seed).permutation(len(vals))
    dt, walkers, k = _oracle_step_time(synthetic.CONFIGS[key], addrs, vals, shift, step_index, order, k)
    print(json.dumps(dict(seconds=dt, walkers=walkers, entries=k)), flush=True)


def _spec(inst, **lay):
    """Solver keyword arguments of a synthetic instance description."""
    import math
    M, N, tgt = inst["M"], inst["N"], inst["target"]
    dim = math.comb(N + M - 1, N)
    table = int(min(dim, 1.2 * tgt)) + 4096
    spawn = int(2.5 * tgt) + 65536
    return dict(model=inst["model"], M=M, N=N, t=inst["t"], u=inst["u"], dtau=inst["dtau"],
                target_walkers=tgt, seed=inst["seed"], addr_words=inst["W"],
                threshold=inst["theta"], table_capacity=table, spawn_capacity=spawn, **lay)


BATCH_LAYOUT = dict(lds_slots=2048, block=512, spawn_block=256)


# shared layouts the batch autotuner tries (hash and tile shapes)
BATCH_CANDIDATES = [dict(lds_slots=sl, block=bl, spawn_block=sb)
                    for sl in (1024, 2048, 4096) for bl in (256, 512, 1024) for sb in (256, 512)
                    if sl <= 8 * bl]


def bench_batched(fq, torch, n=64, warmup=1500, steps=500, trial_steps=20):
    """The 64-instance batch (real-space, M = N in 8..24, u log-uniform in
    [1, 10], N_t 1e4..1e7) after `warmup` steps: walker-steps/s of the batch
    with the fixed layout, of the batch with the layout the batch autotuner
    picks (fq_batch_autotune over BATCH_CANDIDATES, timed on device copies
    of the states), and of the same instances stepped one at a time (plain
    per-instance launches), all from the same state; the three runs must
    agree bit for bit."""
    specs = [_spec(x, **BATCH_LAYOUT) for x in synthetic.batch_instances(n)]
    b = fq.Batch(specs)
    for i, sp in enumerate(specs):
        a = fq.start_address(sp["model"], sp["M"], sp["N"])
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    t0 = time.perf_counter()
    done = 0
    while done < warmup:
        k = min(500, warmup - done)
        b.run(k)
        done += k
        log(f"[bench] batch warmup {done}/{warmup} ({time.perf_counter() - t0:.1f} s)")
    ms, best = b.autotune(BATCH_CANDIDATES, trial_steps=trial_steps)
    tuned_layout = BATCH_CANDIDATES[best]
    log(f"[bench] batch autotune: best {tuned_layout} {ms[best]:.3f} ms/step over {len(ms)} candidates")
    tspecs = [dict(sp, buckets=0, **tuned_layout) for sp in specs]
    tb = fq.Batch(tspecs)
    for i in range(n):
        tb.instance(i).copy_state_from(b.instance(i))
    plain = []
    for i, sp in enumerate(specs):
        s = fq.Solver(**sp)
        s.copy_state_from(b.instance(i))
        plain.append(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = b.run(steps)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t1
    t1 = time.perf_counter()
    stt = tb.run(steps)
    torch.cuda.synchronize()
    wall_t = time.perf_counter() - t1
    same_t = stt.tobytes() == st.tobytes()
    tb.close()
    wall_p = 0.0
    same = True
    for i, s in enumerate(plain):
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        si = s.run(steps)
        torch.cuda.synchronize()
        wall_p += time.perf_counter() - t2
        same &= si.tobytes() == st[i].tobytes()
        s.close()
    b.close()
    ws = float(st["norm"].sum())
    out = dict(workload=f"batch of {n} real-space 1D Bose-Hubbard instances (M = N in 8..24, "
                        f"u log-uniform in [1, 10], N_t 1e4..1e7)",
               instances=n, warmup=warmup, steps=steps, walkers_total=float(st["norm"][:, -1].sum()),
               layout=dict(BATCH_LAYOUT), walker_steps_per_s=ws / wall_b, ms_per_step=wall_b / steps * 1e3,
               autotuned=dict(layout=tuned_layout, candidates=len(ms), trial_steps=trial_steps,
                              trial_ms_per_step=float(ms[best]),
                              walker_steps_per_s=ws / wall_t, ms_per_step=wall_t / steps * 1e3,
                              identical_to_fixed=bool(same_t)),
               plain_walker_steps_per_s=ws / wall_p, plain_ms_per_step=wall_p / steps * 1e3,
               speedup_vs_plain=wall_p / min(wall_b, wall_t), identical_to_plain=bool(same))
    log(f"[bench] batched {out['walker_steps_per_s']:.4g} walker-steps/s (fixed), "
        f"{out['autotuned']['walker_steps_per_s']:.4g} (autotuned {tuned_layout}), plain "
        f"{out['plain_walker_steps_per_s']:.4g}, identical {same} {same_t}")
    return out


PAPER_2D_STEPS_PER_S = 112.0  # Sec. 7.2: one CPU node, 32 threads, N_t = 1e7


def bench_lattice(fq, torch, warmup=100, steps=2000, settle=500):
    """The benchmark system of Sec. 7.2 (periodic 6 x 6 lattice, N = 36,
    u = 1, t = 0.1, Gutzwiller importance sampling, N_t = 1e7): FCIQMC steps
    per second at steady state, beside the paper's CPU figure (context: a
    different machine; the paper times 5e4 steps after 2.5e4 equilibration
    steps)."""
    wl = WORKLOADS["c2d"]
    cfg = synthetic.CONFIGS[wl["cfg"]]
    s = make_solver(fq, wl, cfg)
    a = fq.encode(synthetic.start_occupation(cfg["model"], cfg["M"], cfg["N"]), cfg["W"])
    s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    ramp_steps, _, _, _ = ramp(s, cfg["target"], settle, "lattice ramp", chunk=500)
    if warmup:
        s.run(warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = s.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    s.close()
    sps = steps / wall
    out = dict(workload=wl["name"], model=MODEL_NAMES[cfg["model"]], ramp_steps=ramp_steps,
               warmup=warmup, steps=steps, steps_per_s=sps, ms_per_step=wall / steps * 1e3,
               walker_steps_per_s=float(st["norm"].sum()) / wall,
               mean_len=float(st["len"].mean()), mean_spawns=float(st["spawns"].mean()),
               shift_mean=float(st["shift"].mean()),
               paper_context=dict(steps_per_s=PAPER_2D_STEPS_PER_S,
                                  hardware="one CPU node, 32 threads, CPU model not stated"),
               ratio_to_paper=sps / PAPER_2D_STEPS_PER_S)
    log(f"[bench] lattice {sps:.1f} steps/s ({out['walker_steps_per_s']:.4g} walker-steps/s); "
        f"paper {PAPER_2D_STEPS_PER_S:.0f} steps/s on 32 CPU threads")
    return out


def bench_replicas(fq, torch, wl, cfg, warmup=100, steps=300, settle=500):
    """Two replicas of the momentum-space workload (seeds differ) in one
    batch with the overlap c_A . c_B computed after every step on the
    device (Sec. 4.3).  The same replicas then run the same number of steps
    without overlaps; the difference per step is the cost of the join."""
    specs = [dict(model=cfg["model"], M=cfg["M"], N=cfg["N"], t=cfg["t"], u=cfg["u"], dtau=cfg["dtau"],
                  target_walkers=cfg["target"], seed=sd, addr_words=cfg["W"], threshold=cfg["theta"],
                  table_capacity=wl["table_capacity"], spawn_capacity=wl["spawn_capacity"],
                  buckets=wl["buckets"], lds_slots=wl["lds_slots"], block=wl["block"],
                  spawn_block=wl["spawn_block"]) for sd in (cfg["seed"], cfg["seed"] + 100)]
    b = fq.Batch(specs)
    a = fq.encode(synthetic.start_occupation(cfg["model"], cfg["M"], cfg["N"]), cfg["W"])
    for i in range(2):
        b.instance(i).set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    ramp_steps, _, _, _ = ramp(b, cfg["target"], settle, "replica ramp", chunk=500)
    if warmup:
        b.run(warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, ov, inexact = b.run_replicas(steps)
    torch.cuda.synchronize()
    wall_o = time.perf_counter() - t1
    t2 = time.perf_counter()
    st2 = b.run(steps)
    torch.cuda.synchronize()
    wall_n = time.perf_counter() - t2
    b.close()
    rec = 8 * cfg["W"] + 8
    join_bytes = float(rec * (st["len"][0] + st["len"][1]).astype(np.float64).mean())
    over_ms = (wall_o - wall_n) / steps * 1e3
    out = dict(workload=f"2 replicas of {wl['name']} (seeds {cfg['seed']}, {cfg['seed'] + 100})",
               replicas=2, ramp_steps=ramp_steps, warmup=warmup, steps=steps,
               walker_steps_per_s=float(st["norm"].sum()) / wall_o, ms_per_step=wall_o / steps * 1e3,
               ms_per_step_without_overlaps=wall_n / steps * 1e3, overlap_ms_per_step=over_ms,
               overlap_algorithmic_bytes_per_step=join_bytes,
               overlap_GBs_from_difference=join_bytes / max(over_ms, 1e-6) / 1e6,
               last_overlap=float(ov[-1, 0]), inexact=bool(inexact),
               mean_walkers=[float(st["norm"][0].mean()), float(st["norm"][1].mean())])
    log(f"[bench] replicas {out['walker_steps_per_s']:.4g} walker-steps/s, {out['ms_per_step']:.3f} ms/step "
        f"({out['ms_per_step_without_overlaps']:.3f} without overlaps)")
    del st2
    return out


def _serve(fq, torch, reqs, pool, tick, max_active, t_arrival, log_every=20):
    """Serve `reqs` (arrival offsets t_arrival, seconds) with continuous
    batching.  Returns per-request (arrival, admission, completion) times,
    walker-steps and the number of ticks."""
    sv = fq.Server(fq.REAL1D, pool, lds_slots=BATCH_LAYOUT["lds_slots"], block=BATCH_LAYOUT["block"],
                   spawn_block=BATCH_LAYOUT["spawn_block"], max_active=max_active, steps_per_tick=tick)
    n = len(reqs)
    ids, adm, comp = [], {}, {}
    t0 = time.perf_counter()
    i, ticks, max_queued = 0, 0, 0
    while len(comp) < n:
        now = time.perf_counter() - t0
        while i < n and t_arrival[i] <= now:
            r = reqs[i]
            sp = _spec(r)
            sp.pop("addr_words")
            ids.append(sv.submit(sp, fq.start_address(r["model"], r["M"], r["N"]), 10.0, r["steps"]))
            i += 1
        active, queued, fin = sv.tick()
        ticks += 1
        max_queued = max(max_queued, queued)
        now = time.perf_counter() - t0
        for k, rid in enumerate(ids):
            if rid in comp:
                continue
            st = sv.poll(rid)["state"]
            if st >= fq.REQ_RUNNING and rid not in adm:
                adm[rid] = now
            if st >= fq.REQ_DONE:
                comp[rid] = now
        if active == 0 and queued == 0 and i < n:
            time.sleep(max(0.0, t_arrival[i] - now))
        if ticks % log_every == 0:
            log(f"[bench] served: {len(comp)}/{n} done, {active} active, {queued} queued, "
                f"{i} arrived ({now:.1f} s)")
    ws, ok = [], True
    for rid in ids:
        info = sv.poll(rid)
        ok &= info["state"] == fq.REQ_DONE
        ws.append(info["walker_steps"])
    sv.close()
    arr = np.asarray(t_arrival[:n])
    return dict(arrival=arr, admit=np.array([adm[r] for r in ids]), done=np.array([comp[r] for r in ids]),
                walker_steps=np.asarray(ws), ticks=ticks, max_queued=max_queued, all_done=bool(ok))


def bench_served(fq, torch, n_req=100, tick=250, budget=200e9, max_active=128, load=0.8, n_calib=16,
                 plain=True):
    """The Poisson request stream of real-space solves (M = N in 6..20, u in
    [1, 10], 2e3..2e4 steps, N_t log-uniform in [1e3, 1e7]) served with
    continuous batching under an HBM budget.

    1. Capacity: a burst of the first n_calib requests gives the served
       throughput; capacity = requests per second the GPU completes for this
       request mix.
    2. Stream: the first n_req requests of the stream, their arrival times
       rescaled to the rate load x capacity (the configured 50/s is far above
       what one GPU completes for requests of about 5e9 walker-steps each).
       Latency = completion - arrival, queue wait = admission - arrival.
    3. Plain: the same requests served one at a time in arrival order by a
       plain solver each (no batching): every request's service time is
       measured alone, and the latencies follow from the same arrival times
       (first come, first served on one GPU)."""
    reqs = synthetic.poisson_requests(1000)
    free = torch.cuda.mem_get_info()[0]
    pool = int(min(budget, 0.85 * free))
    # 1. capacity from a burst
    cal = _serve(fq, torch, reqs[:n_calib], pool, tick, max_active, [0.0] * n_calib, log_every=50)
    cal_make = float(cal["done"].max())
    capacity = n_calib / cal_make
    rate = load * capacity
    log(f"[bench] served capacity {capacity:.2f} requests/s (burst of {n_calib}); stream at {rate:.2f}/s")
    # 2. the stream at rate
    base = np.array([r["arrival"] for r in reqs[:n_req]])
    t_arr = (base - base[0]) * (50.0 / rate)
    sv = _serve(fq, torch, reqs[:n_req], pool, tick, max_active, list(t_arr))
    lat = sv["done"] - sv["arrival"]
    wait = sv["admit"] - sv["arrival"]
    makespan = float(sv["done"].max())
    ws = float(sv["walker_steps"].sum())
    out = dict(workload=f"first {n_req} requests of a Poisson stream of real-space solves (M = N in 6..20, "
                        "u in [1, 10], 2e3..2e4 steps, N_t log-uniform in [1e3, 1e7]), continuous batching, "
                        f"arrivals rescaled to {load} x the measured capacity",
               requests=n_req, pool_bytes=pool, steps_per_tick=tick, max_active=max_active,
               capacity_requests_per_s=capacity, capacity_burst_requests=n_calib, load=load,
               arrival_rate_per_s=rate, ticks=sv["ticks"], max_queued=sv["max_queued"],
               p50_latency_s=float(np.percentile(lat, 50)), p90_latency_s=float(np.percentile(lat, 90)),
               p99_latency_s=float(np.percentile(lat, 99)), mean_queue_wait_s=float(wait.mean()),
               p99_queue_wait_s=float(np.percentile(wait, 99)),
               queued_requests=int(np.sum(wait > 1e-3)),
               walker_steps_per_s=ws / makespan, makespan_s=makespan, all_done=sv["all_done"],
               mean_walker_steps_per_request=ws / n_req)
    log(f"[bench] served p50 {out['p50_latency_s']:.2f} s p99 {out['p99_latency_s']:.2f} s, "
        f"{out['walker_steps_per_s']:.4g} walker-steps/s, {out['queued_requests']} requests queued "
        f"(max {out['max_queued']} at once)")
    if plain:
        # 3. one at a time: measured service times, FIFO on the same arrivals
        svc = np.zeros(n_req)
        t0 = time.perf_counter()
        for k, r in enumerate(reqs[:n_req]):
            sp = _spec(r, **BATCH_LAYOUT)
            s = fq.Solver(**sp)
            a = fq.start_address(r["model"], r["M"], r["N"])
            s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s.run(r["steps"])
            torch.cuda.synchronize()
            svc[k] = time.perf_counter() - t1
            s.close()
            if k % 10 == 9:
                log(f"[bench] plain service {k + 1}/{n_req} ({time.perf_counter() - t0:.1f} s)")
        fin = np.zeros(n_req)
        for k in range(n_req):
            fin[k] = max(t_arr[k], fin[k - 1] if k else 0.0) + svc[k]
        plat = fin - t_arr
        out["plain"] = dict(rule="each request alone on a plain solver, first come first served on the "
                                 "same arrival times; service times measured",
                            p50_latency_s=float(np.percentile(plat, 50)),
                            p99_latency_s=float(np.percentile(plat, 99)),
                            walker_steps_per_s=ws / float(svc.sum()), makespan_s=float(fin.max()),
                            service_s_total=float(svc.sum()))
        out["speedup_vs_plain"] = out["walker_steps_per_s"] / out["plain"]["walker_steps_per_s"]
        log(f"[bench] plain p50 {out['plain']['p50_latency_s']:.2f} s p99 {out['plain']['p99_latency_s']:.2f} s, "
            f"{out['plain']['walker_steps_per_s']:.4g} walker-steps/s")
    return out


def blocked_error(x):
    """Standard error of the mean of a correlated series by blocking
    (Flyvbjerg-Petersen): the largest blocked estimate over levels that keep
    at least 32 blocks."""
    x = np.asarray(x, dtype=np.float64)
    best = 0.0
    while len(x) >= 32:
        best = max(best, math.sqrt(np.var(x) / (len(x) - 1)))
        n = len(x) // 2
        x = 0.5 * (x[:2 * n:2] + x[1:2 * n:2])
    return best


def compression_study(fq, torch, steps=20000, skip=5000):
    """Statistical efficiency f = 1 / (sigma^2 Omega t) of the shift (Sec. 7.1)
    for late and early compression: sigma = blocked error of the mean shift,
    Omega = timed steps, t = GPU time per step from HIP events.  Systems: C1
    (the 6/6 ring, N_t = 1e3), the 12/12 ring of the paper's efficiency
    figure (u = 6, N_t = 1e4) and C2 (the 20/20 ring with two address words,
    N_t = 1e7, timed after the ramp)."""
    c1, c2 = synthetic.CONFIGS["c1"], synthetic.CONFIGS["c2"]
    systems = [
        ("c1", "real-space ring M = N = 6, u = 6, dtau = 1e-3, N_t = 1e3 (C1)",
         dict(model=c1["model"], M=c1["M"], N=c1["N"], u=c1["u"], dtau=c1["dtau"], target_walkers=c1["target"],
              seed=c1["seed"], addr_words=c1["W"], table_capacity=4096, spawn_capacity=32768), None),
        ("ring12", "real-space ring M = N = 12, u = 6, dtau = 1e-3, N_t = 1e4",
         dict(model=fq.REAL1D, M=12, N=12, u=6.0, dtau=1e-3, target_walkers=1e4, seed=7,
              table_capacity=40000, spawn_capacity=200000), None),
        ("c2", "real-space ring M = N = 20, u = 6, dtau = 1e-3, N_t = 1e7, two address words (C2)",
         dict(model=c2["model"], M=c2["M"], N=c2["N"], u=c2["u"], dtau=c2["dtau"], target_walkers=c2["target"],
              seed=c2["seed"], addr_words=c2["W"], table_capacity=WORKLOADS["c2"]["table_capacity"],
              spawn_capacity=WORKLOADS["c2"]["spawn_capacity"], buckets=WORKLOADS["c2"]["buckets"],
              lds_slots=WORKLOADS["c2"]["lds_slots"], block=WORKLOADS["c2"]["block"],
              spawn_block=WORKLOADS["c2"]["spawn_block"]), c2["target"]),
    ]
    res = {}
    for key, desc, kw, ramp_to in systems:
        out = {"workload": desc}
        for name, flag in (("late", 0), ("early", fq.FLAG_EARLY_COMPRESSION)):
            kw2 = dict(kw)
            model, M, N = kw2.pop("model"), kw2.pop("M"), kw2.pop("N")
            s = fq.Solver(model, M, N, flags=flag, **kw2)
            a = fq.start_address(model, M, N, kw2.get("addr_words", 1))
            s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
            if ramp_to is not None:
                ramp(s, ramp_to, skip, f"compression {key} {name} ramp", chunk=500)
            else:
                s.run(skip)
            s.set_timing(True)
            s.kernel_time(reset=True)
            st = s.run(steps)
            kms, nl = s.kernel_time()
            s.close()
            t = sum(kms.values()) / 1e3 / max(nl, 1)
            sig = blocked_error(st["shift"])
            out[name] = dict(mean_shift=float(st["shift"].mean()), sigma=sig, steps=steps, s_per_step=t,
                             f=1.0 / (sig * sig * steps * t), mean_len=float(st["len"].mean()),
                             mean_norm=float(st["norm"].mean()), mean_spawns=float(st["spawns"].mean()))
            log(f"[bench] compression {key} {name}: shift {out[name]['mean_shift']:.5f} +- {sig:.5f}, "
                f"{t * 1e3:.4f} ms/step, f {out[name]['f']:.4g}")
        res[key] = out
    return res


def ramp(s, target, settle, what, chunk=250, limit=60000):
    """Untimed ramp of a solver or batch `s`: steps until ||c||_1 first
    reaches the target (every instance of a batch), then `settle` more steps.
    Returns (steps run, step count at which the target was first reached,
    seconds, last statistics row; a batch's rows hold one entry per
    instance)."""
    t0 = time.perf_counter()
    done, reached, last = 0, None, None
    while reached is None:
        if done >= limit:
            raise RuntimeError(f"{what}: ||c||_1 did not reach {target:.3g} in {limit} steps")
        st = s.run(chunk)
        norm = st["norm"] if st.ndim == 1 else st["norm"].min(axis=0)
        hit = np.nonzero(norm >= target)[0]
        if len(hit):
            reached = done + int(hit[0]) + 1
        done += chunk
        last = st[..., -1]
        log(f"[bench] {what} {done}: norm {np.min(last['norm']):.4g} len {np.max(last['len'])} "
            f"({time.perf_counter() - t0:.1f} s)")
    rest = reached + settle - done
    while rest > 0:
        k = min(chunk, rest)
        last = s.run(k)[..., -1]
        done += k
        rest -= k
    log(f"[bench] {what}: target reached at step {reached}, {done} ramp steps "
        f"({time.perf_counter() - t0:.1f} s)")
    return done, reached, time.perf_counter() - t0, last


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--oracle-worker":
        p, key, stp, shift, seed, k = sys.argv[2:8]
        oracle_worker(p, key, int(stp), float(shift), int(seed), int(k))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps after the ramp (default 100)")
    ap.add_argument("--settle", type=int, default=500,
                    help="ramp steps after ||c||_1 first reaches N_t")
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--diag", action="store_true", help="per-phase kernel timers (diagnostics)")
    ap.add_argument("--buckets", type=int, default=None)
    ap.add_argument("--slots", type=int, default=None)
    ap.add_argument("--block", type=int, default=None)
    ap.add_argument("--spawn-block", type=int, default=None)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the served measurement")
    ap.add_argument("--no-replicas", action="store_true", help="skip the replica-overlap measurement")
    ap.add_argument("--no-lattice", action="store_true",
                    help="skip the 6 x 6 lattice measurement (the paper's benchmark system)")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--batch-warmup", type=int, default=1500)
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--no-serve-plain", action="store_true",
                    help="skip the one-at-a-time comparison of the served stream")
    ap.add_argument("--compression-study", action="store_true",
                    help="only compare late and early compression by statistical efficiency")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a streaming negation over this many MiB (reads and writes "
                         "that many bytes): the reference kernel for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; sharding over several "
                                   "GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2601_19505_amd as fq

    if args.compression_study:
        torch.cuda.set_device(0)
        print(json.dumps({"compression_study": compression_study(fq, torch)}), flush=True)
        return
    wl = dict(WORKLOADS[args.workload])
    for k_arg, k_wl in (("buckets", "buckets"), ("slots", "lds_slots"), ("block", "block"),
                        ("spawn_block", "spawn_block")):
        if getattr(args, k_arg) is not None:
            wl[k_wl] = getattr(args, k_arg)
    cfg = synthetic.CONFIGS[wl["cfg"]]
    steps = wl["steps"] if args.steps is None else args.steps
    warmup = 100 if args.warmup is None else args.warmup
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * 2**20 // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
        torch.cuda.empty_cache()
    s = make_solver(fq, wl, cfg, **({"flags": fq.FLAG_PHASE_TIMING} if args.diag else {}))
    occ = synthetic.start_occupation(cfg["model"], cfg["M"], cfg["N"])
    a = fq.encode(occ, cfg["W"])
    s.set_state([a], [10.0], 0.0, 0, ref=a, yref=10.0)
    log(f"[bench] workload {wl['name']}: layout buckets={s.layout.buckets} "
        f"slots={s.layout.lds_slots} block={s.layout.block} spawn_block={s.layout.spawn_block} "
        f"workspace={s.nbytes / 2**30:.2f} GiB")
    ramp_steps, first_reach, ramp_s, prev = ramp(s, cfg["target"], args.settle, "ramp")
    if warmup:
        prev = s.run(warmup)[-1]
    log(f"[bench] warmup {warmup} steps after the ramp: norm {prev['norm']:.4g} len {prev['len']}")
    torch.cuda.synchronize()
    s.set_timing(True)
    s.kernel_time(reset=True)
    if args.diag:
        s.debug_counters(reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = s.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    kms, nl = s.kernel_time()
    s.set_timing(False)
    if args.diag:
        d = s.debug_counters()
        log("[bench] diag " + json.dumps({k: round(v, 3) for k, v in d.items()}))
    log(f"[bench] timed {steps} steps in {wall:.3f} s; norm {st['norm'][-1]:.4g} len {st['len'][-1]}; "
        f"kernel ms/step " + ", ".join(f"{k} {v / max(nl, 1):.3f}" for k, v in kms.items()))
    walker_steps = float(st["norm"].sum())
    mean_norm = float(st["norm"].mean())
    valid = mean_norm >= 0.9 * cfg["target"]
    value = walker_steps / wall
    # spawns of the step after the timed region (written by the last timed spawn launch)
    nxt_last = float(s.run(1)["spawns"][-1])
    # algorithmic HBM bytes per launch: merge k reads c^(k-1) and the spawn
    # records of step k and writes c^(k); spawn k reads c^(k) and writes the
    # spawn records of step k+1
    rec = 8 * cfg["W"] + 8
    lens = np.concatenate([[prev["len"]], st["len"]]).astype(np.float64)
    spw = st["spawns"].astype(np.float64)
    nxt = np.concatenate([spw[1:], [nxt_last]])
    per_kernel = {
        "merge": float((rec * (lens[:-1] + spw + lens[1:])).mean()),
        "spawn": float((rec * (lens[1:] + nxt)).mean()),
    }
    kern = {}
    for k, b in per_kernel.items():
        t_s = kms[k] / 1e3 / max(nl, 1)
        kern[k] = {"mean_ms": t_s * 1e3, "algorithmic_bytes": b, "achieved_GBs": b / t_s / 1e9,
                   "frac": b / t_s / 1e9 / HBM_PEAK_GBS}
    kern["partition"] = {"mean_ms": kms["partition"] / max(nl, 1),
                         "algorithmic_bytes": float(2 * rec * nxt.mean())}
    kern["partition"]["achieved_GBs"] = (kern["partition"]["algorithmic_bytes"] /
                                         max(kern["partition"]["mean_ms"], 1e-9) / 1e6)
    kern["finalize"] = {"mean_ms": kms["finalize"] / max(nl, 1)}
    for k in ("merge", "spawn", "partition"):
        tr = measured_traffic(fq, "k_" + ("part" if k == "partition" else k)) if args.workload == "c3" else None
        kern[k]["traffic"] = tr
        if k in ("merge", "spawn") and args.workload == "c3":
            vi = measured_valu(fq, "k_" + k)
            if vi is not None:
                kern[k]["valu_insts_per_launch"] = vi
                kern[k]["valu_issue_frac"] = vi / (kern[k]["mean_ms"] * 1e-3) / VALU_ISSUE_PEAK
    dom = max(per_kernel, key=lambda k: kern[k]["mean_ms"])
    achieved = kern[dom]["achieved_GBs"]
    # the whole step: (8 W + 8) (L_n + 2 S_n + L_(n+1)) bytes over the wall time
    step_bytes = rec * (lens[:-1] + 2.0 * spw + lens[1:])
    step_gbs = float(step_bytes.sum()) / wall / 1e9
    traffic_step = None
    if all(kern[k].get("traffic") is not None for k in ("merge", "spawn", "partition")):
        traffic_step = sum(kern[k]["traffic"] for k in ("merge", "spawn", "partition"))
    out = {
        "metric": "FCIQMC walker-steps/s at 1e8 walkers",
        "value": value if valid else None,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "model": MODEL_NAMES[cfg["model"]],
                   "M": cfg["M"], "N": cfg["N"], "u": cfg["u"], "dtau": cfg["dtau"],
                   "target_walkers": cfg["target"], "seed": cfg["seed"],
                   "addr_words": cfg["W"], "buckets": s.layout.buckets,
                   "lds_slots": s.layout.lds_slots, "block": s.layout.block,
                   "spawn_block": s.layout.spawn_block,
                   "mean_norm": mean_norm, "mean_len": float(st["len"].mean()),
                   "mean_spawns": float(st["spawns"].mean())},
        "ramp": {"steps": ramp_steps, "first_reach_step": first_reach, "settle_steps": args.settle,
                 "seconds": ramp_s,
                 "rule": "untimed: steps until ||c||_1 first reaches N_t, then the settle steps; "
                         "--warmup and --steps count after it"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": kern[dom]["traffic"],
                     "kernel": "k_" + dom, "mean_kernel_ms": kern[dom]["mean_ms"],
                     "algorithmic_bytes_per_launch": kern[dom]["algorithmic_bytes"],
                     "step": {"achieved": step_gbs, "frac": step_gbs / HBM_PEAK_GBS,
                              "algorithmic_bytes_per_step": float(step_bytes.mean()),
                              "traffic_per_step": traffic_step}},
        "kernels": kern,
        "entry_steps_per_s": float(st["len"].sum()) / wall,
        "spawns_per_s": float(st["spawns"].sum()) / wall,
        "shift_mean": float(st["shift"].mean()),
    }
    if not valid:
        out["error"] = (f"timed mean ||c||_1 {mean_norm:.4g} is below 0.9 N_t: not the stated "
                        f"configuration, no headline value")
    state = s.get_state() if not args.no_cpu_baseline else None
    s.close()
    del s
    torch.cuda.empty_cache()
    if not args.no_lattice and args.workload == "c3":
        out["lattice_2d"] = bench_lattice(fq, torch)
        torch.cuda.empty_cache()
    if not args.no_replicas and args.workload == "c3":
        out["replicas"] = bench_replicas(fq, torch, wl, cfg)
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched"] = bench_batched(fq, torch, warmup=args.batch_warmup, steps=args.batch_steps)
        torch.cuda.empty_cache()
    if not args.no_serve:
        out["served"] = bench_served(fq, torch, n_req=args.serve_requests, plain=not args.no_serve_plain)
        torch.cuda.empty_cache()
    if state is not None:
        addrs, vals, shift, step = state
        log(f"[bench] cpu baseline on {len(vals)} entries (budget {args.cpu_budget} s)")
        out["cpu_baseline"] = cpu_baseline((addrs, vals), cfg, step + 1, shift, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
