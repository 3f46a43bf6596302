"""MI355X-native FCIQMC hot path (Rimu.jl, arXiv 2601.19505), Python binding.

Thin ctypes marshalling over the C ABI of ``include/fciqmc.h``
(``libfciqmc.so``, built for gfx950).  Every step of the method runs in the
HIP kernels of that library; PyTorch is used only to allocate the device
workspace and to supply the current stream.  Importing this package does not
need a GPU; creating a solver does, and fails loudly if the library is
missing.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfciqmc.so")

REAL1D = 0
MOM1D = 1
REAL2D = 2

FLAG_DUMP_SPAWNS = 1
FLAG_DUMP_MERGED = 2
FLAG_PHASE_TIMING = 4
FLAG_EARLY_COMPRESSION = 32
FLAG_UNCHECKED_DTAU = 64
FLAG_INITIATOR = 128

STATUS = {0: "OK", -1: "EINVAL", -2: "ECAPACITY", -3: "EHIP", -4: "ENOMEM", -5: "EBUSY",
          -6: "EDIVERGED", -7: "ENOTFOUND"}


class FqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Hamiltonian(C.Structure):
    _fields_ = [("model", C.c_int32), ("M", C.c_int32), ("N", C.c_int32), ("lx", C.c_int32),
                ("t", C.c_double), ("u", C.c_double), ("g", C.c_double)]


class Params(C.Structure):
    _fields_ = [("dtau", C.c_double), ("target_walkers", C.c_double), ("zeta", C.c_double),
                ("xi", C.c_double), ("threshold", C.c_double), ("t_rel", C.c_double),
                ("seed", C.c_uint64), ("addr_words", C.c_int32), ("flags", C.c_int32),
                ("initiator_threshold", C.c_double)]


class Layout(C.Structure):
    _fields_ = [("table_capacity", C.c_int64), ("spawn_capacity", C.c_int64),
                ("buckets", C.c_int32), ("lds_slots", C.c_int32), ("block", C.c_int32),
                ("spawn_block", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("step", C.c_int64), ("len", C.c_int64), ("exact_steps", C.c_int64),
                ("inexact_steps", C.c_int64), ("spawns", C.c_int64), ("shift", C.c_double),
                ("norm", C.c_double), ("hproj", C.c_double), ("vproj", C.c_double),
                ("flags", C.c_int64)]


class ServerConfig(C.Structure):
    _fields_ = [("model", C.c_int32), ("addr_words", C.c_int32), ("lds_slots", C.c_int32),
                ("block", C.c_int32), ("spawn_block", C.c_int32), ("max_active", C.c_int32),
                ("steps_per_tick", C.c_int64)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("steps_done", C.c_int64),
                ("last", StepStats), ("mean_shift", C.c_double), ("mean_hproj", C.c_double),
                ("mean_vproj", C.c_double), ("n_mean", C.c_int64), ("workspace_bytes", C.c_int64),
                ("walker_steps", C.c_double)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3

STATS_DTYPE = np.dtype([("step", np.int64), ("len", np.int64), ("exact_steps", np.int64),
                        ("inexact_steps", np.int64), ("spawns", np.int64), ("shift", np.float64),
                        ("norm", np.float64), ("hproj", np.float64), ("vproj", np.float64),
                        ("flags", np.int64)])
ROW_INEXACT = 1  # FQ_ROW_INEXACT: some sum of the row's step was not exactly rounded
assert STATS_DTYPE.itemsize == C.sizeof(StepStats)

_lib = None


def lib():
    """Load libfciqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2601_19505_amd.build` (hipcc, gfx950)")
        # PyTorch ships its own HIP runtime under the same soname; load it
        # first so the library binds to it and the process has one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, vp = C.POINTER, C.c_void_p
        u64p, f64p, i64p, i32p = P(C.c_uint64), P(C.c_double), P(C.c_int64), P(C.c_int32)
        sig = {
            "fq_version": (C.c_char_p, []),
            "fq_encode": (C.c_int, [i32p, C.c_int32, C.c_int32, u64p]),
            "fq_workspace_size": (C.c_int, [P(Hamiltonian), P(Params), P(Layout), P(C.c_size_t),
                                            P(Layout)]),
            "fq_create": (C.c_int, [P(Hamiltonian), P(Params), P(Layout), vp, C.c_size_t, P(vp)]),
            "fq_set_state": (C.c_int, [vp, u64p, f64p, C.c_int64, C.c_double, C.c_int64, u64p,
                                       C.c_double, vp]),
            "fq_run": (C.c_int, [vp, C.c_int64, vp, vp]),
            "fq_get_state": (C.c_int, [vp, u64p, f64p, C.c_int64, i64p, f64p, i64p, vp]),
            "fq_read_spawn_dump": (C.c_int, [vp, u64p, i64p, u64p, f64p, C.c_int64, i64p, vp]),
            "fq_read_merged_dump": (C.c_int, [vp, u64p, f64p, C.c_int64, i64p, vp]),
            "fq_set_timing": (C.c_int, [vp, C.c_int32]),
            "fq_kernel_time": (C.c_int, [vp, f64p, C.c_int32, i64p, C.c_int32]),
            "fq_get_layout": (C.c_int, [vp, P(Layout)]),
            "fq_debug_counters": (C.c_int, [vp, f64p, C.c_int32, C.c_int32, vp]),
            "fq_destroy": (C.c_int, [vp]),
            "fq_last_error": (C.c_char_p, [vp]),
            "fq_copy_state": (C.c_int, [vp, vp, vp]),
            "fq_autotune": (C.c_int, [vp, P(Layout), C.c_int32, C.c_int32, vp, C.c_size_t, f64p,
                                      i32p, vp]),
            "fq_batch_workspace_size": (C.c_int, [C.c_int32, P(Hamiltonian), P(Params), P(Layout),
                                                  P(C.c_size_t)]),
            "fq_batch_create": (C.c_int, [C.c_int32, P(Hamiltonian), P(Params), P(Layout), vp,
                                          C.c_size_t, P(vp)]),
            "fq_batch_instance": (C.c_int, [vp, C.c_int32, P(vp)]),
            "fq_batch_run": (C.c_int, [vp, C.c_int64, vp, vp]),
            "fq_batch_failed": (C.c_int32, [vp]),
            "fq_batch_autotune": (C.c_int, [vp, P(Layout), C.c_int32, C.c_int32, vp, C.c_size_t, f64p,
                                            i32p, vp]),
            "fq_batch_last_error": (C.c_char_p, [vp]),
            "fq_batch_replica_scratch_size": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
            "fq_batch_run_replicas": (C.c_int, [vp, C.c_int64, vp, vp, vp, C.c_size_t,
                                                C.POINTER(C.c_int32), vp]),
            "fq_batch_run_replicas_static": (C.c_int, [vp, C.c_int64, vp, vp, C.POINTER(C.c_int32), vp]),
            "fq_batch_spectral_scratch_size": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
            "fq_batch_run_spectral": (C.c_int, [vp, C.c_int64, vp, vp, C.c_size_t, C.POINTER(C.c_int32), vp]),
            "fq_batch_destroy": (C.c_int, [vp]),
            "fq_server_create": (C.c_int, [P(ServerConfig), vp, C.c_size_t, P(vp)]),
            "fq_server_submit": (C.c_int, [vp, P(Hamiltonian), P(Params), P(Layout), u64p, C.c_double,
                                           C.c_int64, P(C.c_uint64)]),
            "fq_server_tick": (C.c_int, [vp, vp, i32p, i32p, i32p]),
            "fq_server_poll": (C.c_int, [vp, C.c_uint64, P(RequestInfo)]),
            "fq_server_destroy": (C.c_int, [vp]),
            "fq_server_last_error": (C.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def encode(occ, W=1):
    """Occupation numbers -> W address words (host helper of the library)."""
    o = np.ascontiguousarray(occ, dtype=np.int32)
    out = np.zeros(W, np.uint64)
    rc = lib().fq_encode(_p(o, C.c_int32), len(o), W, _p(out, C.c_uint64))
    if rc:
        raise FqError(rc, "fq_encode")
    return out


def encode_many(occs, W=1):
    occs = np.asarray(occs, dtype=np.int32)
    return np.stack([encode(o, W) for o in occs]) if len(occs) else np.zeros((0, W), np.uint64)


def workspace_size(ham, params, layout):
    nb = C.c_size_t(0)
    lo = Layout()
    rc = lib().fq_workspace_size(C.byref(ham), C.byref(params), C.byref(layout), C.byref(nb),
                                 C.byref(lo))
    if rc:
        msg = lib().fq_last_error(None)
        raise FqError(rc, f"fq_workspace_size: {msg.decode() if msg else ''}")
    return nb.value, lo


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ham_params(model, M, N, t=1.0, u=1.0, dtau=1e-3, target_walkers=1000.0, zeta=0.08, xi=None,
                threshold=1.0, t_rel=1.0, seed=0, addr_words=1, flags=0, lx=0, g=0.0, initiator=None):
    """`initiator`: threshold n_a of the initiator rule (sets FLAG_INITIATOR);
    None leaves the rule off."""
    if xi is None:
        xi = zeta * zeta / 4.0
    if initiator is not None:
        flags |= FLAG_INITIATOR
    return (Hamiltonian(model, M, N, int(lx), float(t), float(u), float(g)),
            Params(dtau, target_walkers, zeta, xi, threshold, t_rel, seed, addr_words, flags,
                   0.0 if initiator is None else float(initiator)))


def _layout(table_capacity=4096, spawn_capacity=16384, buckets=0, lds_slots=0, block=0,
            spawn_block=0):
    return Layout(table_capacity, spawn_capacity, buckets, lds_slots, block, spawn_block)


class Solver:
    """One FCIQMC instance on the current GPU (plain per-step launches)."""

    def __init__(self, model, M, N, t=1.0, u=1.0, dtau=1e-3, target_walkers=1000.0, zeta=0.08,
                 xi=None, threshold=1.0, t_rel=1.0, seed=0, addr_words=1, flags=0,
                 table_capacity=4096, spawn_capacity=16384, buckets=0, lds_slots=0, block=0,
                 spawn_block=0, lx=0, g=0.0, initiator=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the FCIQMC solver needs a GPU")
        self.ham, self.params = _ham_params(model, M, N, t, u, dtau, target_walkers, zeta, xi,
                                            threshold, t_rel, seed, addr_words, flags, lx, g, initiator)
        self.W = addr_words
        nbytes, lay = workspace_size(self.ham, self.params,
                                     _layout(table_capacity, spawn_capacity, buckets, lds_slots,
                                             block, spawn_block))
        self.layout = lay
        self.nbytes = nbytes
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        rc = lib().fq_create(C.byref(self.ham), C.byref(self.params), C.byref(lay),
                             C.c_void_p(self.ws.data_ptr()), nbytes, C.byref(h))
        if rc:
            msg = lib().fq_last_error(None)
            raise FqError(rc, f"fq_create: {msg.decode() if msg else ''}")
        self.h = h
        self.table_capacity = lay.table_capacity
        self.spawn_capacity = lay.spawn_capacity

    def _check(self, rc, what):
        if rc:
            msg = lib().fq_last_error(self.h)
            raise FqError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            lib().fq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _addr(self, addrs):
        a = np.asarray(addrs, dtype=np.uint64)
        if a.ndim == 1:
            a = a[:, None]
        if a.shape[1] < self.W:
            a = np.concatenate([a, np.zeros((len(a), self.W - a.shape[1]), np.uint64)], 1)
        elif a.shape[1] > self.W:
            if np.any(a[:, self.W:]):
                raise ValueError("address does not fit addr_words")
            a = a[:, :self.W]
        return np.ascontiguousarray(a)

    def set_state(self, addrs, vals, shift=0.0, step=0, ref=None, yref=10.0):
        a = self._addr(addrs)
        v = np.ascontiguousarray(vals, dtype=np.float64)
        r = self._addr([a[0] if ref is None else ref])[0].copy()
        self._check(lib().fq_set_state(self.h, _p(a, C.c_uint64), _p(v, C.c_double), len(v),
                                       float(shift), int(step), _p(r, C.c_uint64), float(yref),
                                       _stream()), "fq_set_state")

    def run(self, n_steps):
        out = np.zeros(n_steps, STATS_DTYPE)
        rc = lib().fq_run(self.h, n_steps, C.c_void_p(out.ctypes.data), _stream())
        if rc:
            msg = lib().fq_last_error(self.h)
            err = FqError(rc, f"fq_run: {msg.decode() if msg else ''}")
            err.stats = out
            raise err
        return out

    def last_error(self):
        """fq_last_error() of this handle (also notes inexact sums after a
        successful run)."""
        msg = lib().fq_last_error(self.h)
        return msg.decode() if msg else ""

    def get_state(self, cap=None):
        """Current state (addresses, values, shift, step); order unspecified."""
        if cap is None:
            cap = self.table_capacity + 1024
        for _ in range(2):
            a = np.zeros((cap, self.W), np.uint64)
            v = np.zeros(cap, np.float64)
            n = C.c_int64(0)
            sh = C.c_double(0)
            st = C.c_int64(0)
            rc = lib().fq_get_state(self.h, _p(a, C.c_uint64), _p(v, C.c_double), cap, C.byref(n),
                                    C.byref(sh), C.byref(st), _stream())
            if rc == -2 and n.value > cap:
                cap = n.value
                continue
            self._check(rc, "fq_get_state")
            return a[:n.value].copy(), v[:n.value].copy(), sh.value, st.value
        raise FqError(-2, "fq_get_state: state changed size")

    def spawn_dump(self, cap=None):
        cap = cap or (self.spawn_capacity + self.table_capacity)
        par = np.zeros((cap, self.W), np.uint64)
        att = np.zeros(cap, np.int64)
        dst = np.zeros((cap, self.W), np.uint64)
        val = np.zeros(cap, np.float64)
        n = C.c_int64(0)
        self._check(lib().fq_read_spawn_dump(self.h, _p(par, C.c_uint64), _p(att, C.c_int64),
                                             _p(dst, C.c_uint64), _p(val, C.c_double), cap,
                                             C.byref(n), _stream()), "fq_read_spawn_dump")
        k = n.value
        return par[:k].copy(), att[:k].copy(), dst[:k].copy(), val[:k].copy()

    def merged_dump(self, cap=None):
        cap = cap or (self.spawn_capacity + self.table_capacity)
        a = np.zeros((cap, self.W), np.uint64)
        v = np.zeros(cap, np.float64)
        n = C.c_int64(0)
        self._check(lib().fq_read_merged_dump(self.h, _p(a, C.c_uint64), _p(v, C.c_double), cap,
                                              C.byref(n), _stream()), "fq_read_merged_dump")
        return a[:n.value].copy(), v[:n.value].copy()

    def set_timing(self, on=True):
        self._check(lib().fq_set_timing(self.h, 1 if on else 0), "fq_set_timing")

    def kernel_time(self, reset=False):
        """Summed HIP-event milliseconds of the timed steps as a dict with keys
        merge, spawn, partition (second pass), finalize (reduction and shift
        update), and the number of timed steps."""
        ms = np.zeros(4)
        n = C.c_int64(0)
        self._check(lib().fq_kernel_time(self.h, _p(ms, C.c_double), 4, C.byref(n), 1 if reset else 0),
                    "fq_kernel_time")
        return dict(merge=float(ms[0]), spawn=float(ms[1]), partition=float(ms[2]),
                    finalize=float(ms[3])), n.value

    def debug_counters(self, reset=False):
        out = np.zeros(13)
        self._check(lib().fq_debug_counters(self.h, _p(out, C.c_double), 13, 1 if reset else 0,
                                            _stream()), "fq_debug_counters")
        names = ["init", "merge_table", "merge_slab", "compress", "compact", "spawn_info",
                 "spawn_scan", "spawn_walk", "diag", "ph9"]
        d = {f"ms_{n}": float(out[i]) for i, n in enumerate(names)}
        d.update(probes=float(out[10]), inserts=float(out[11]), max_load=float(out[12]))
        return d

    def get_layout(self):
        lo = Layout()
        self._check(lib().fq_get_layout(self.h, C.byref(lo)), "fq_get_layout")
        return lo

    def copy_state_from(self, other):
        """Copy the state of another solver (same Hamiltonian and parameters,
        any layout) on the device."""
        self._check(lib().fq_copy_state(self.h, other.h, _stream()), "fq_copy_state")

    def autotune(self, candidates, trial_steps=20):
        """Time candidate layouts (dicts of buckets, lds_slots, block,
        spawn_block; capacities default to this solver's) on copies of this
        solver's state.  Returns (ms per step for each candidate, or -1,
        index of the fastest)."""
        lays = (Layout * len(candidates))()
        need = 0
        for i, c in enumerate(candidates):
            lays[i] = _layout(c.get("table_capacity", self.table_capacity),
                              c.get("spawn_capacity", self.spawn_capacity), c.get("buckets", 0),
                              c.get("lds_slots", 0), c.get("block", 0), c.get("spawn_block", 0))
            try:
                need = max(need, workspace_size(self.ham, self.params, lays[i])[0])
            except FqError:
                pass
        import torch
        scratch = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        ms = np.zeros(len(candidates))
        best = C.c_int32(-1)
        self._check(lib().fq_autotune(self.h, lays, len(candidates), int(trial_steps),
                                      C.c_void_p(scratch.data_ptr()), scratch.numel(),
                                      _p(ms, C.c_double), C.byref(best), _stream()), "fq_autotune")
        del scratch
        return ms, best.value


class _Borrowed(Solver):
    """Handle owned by a batch: same calls as a Solver, no ownership."""

    def __init__(self, h, W, ham, params, table_capacity, spawn_capacity):
        self.h = h
        self.W = W
        self.ham = ham
        self.params = params
        self.table_capacity = table_capacity
        self.spawn_capacity = spawn_capacity

    def close(self):
        self.h = None


class Batch:
    """n instances advanced together (one launch per kernel per step).

    `specs` is a list of dicts with the keyword arguments of Solver (model,
    M, N, t, u, dtau, target_walkers, seed, addr_words, threshold, t_rel,
    flags, initiator, table_capacity, spawn_capacity, buckets, lds_slots, block,
    spawn_block).
    """

    def __init__(self, specs):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the FCIQMC batch needs a GPU")
        n = len(specs)
        self.n = n
        self.hams = (Hamiltonian * n)()
        self.params = (Params * n)()
        self.layouts = (Layout * n)()
        lay_keys = ("table_capacity", "spawn_capacity", "buckets", "lds_slots", "block",
                    "spawn_block")
        for i, sp in enumerate(specs):
            hp = {k: v for k, v in sp.items() if k not in lay_keys}
            h, p = _ham_params(**hp)
            self.hams[i], self.params[i] = h, p
            self.layouts[i] = _layout(**{k: v for k, v in sp.items() if k in lay_keys})
        nb = C.c_size_t(0)
        rc = lib().fq_batch_workspace_size(n, self.hams, self.params, self.layouts, C.byref(nb))
        if rc:
            raise FqError(rc, f"fq_batch_workspace_size: {lib().fq_last_error(None).decode()}")
        self.nbytes = nb.value
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        b = C.c_void_p()
        rc = lib().fq_batch_create(n, self.hams, self.params, self.layouts,
                                   C.c_void_p(self.ws.data_ptr()), self.nbytes, C.byref(b))
        if rc:
            raise FqError(rc, f"fq_batch_create: {lib().fq_last_error(None).decode()}")
        self.b = b
        self._ov = None
        self._gs = None
        self._inst = []
        for i in range(n):
            h = C.c_void_p()
            rc = lib().fq_batch_instance(self.b, i, C.byref(h))
            if rc:
                raise FqError(rc, "fq_batch_instance")
            lo = Layout()
            lib().fq_get_layout(h, C.byref(lo))
            self._inst.append(_Borrowed(h, self.params[i].addr_words, self.hams[i], self.params[i],
                                        lo.table_capacity, lo.spawn_capacity))

    def instance(self, i):
        return self._inst[i]

    def run(self, n_steps):
        """Advance every instance; returns statistics of shape (n, n_steps)."""
        out = np.zeros((self.n, n_steps), STATS_DTYPE)
        rc = lib().fq_batch_run(self.b, n_steps, C.c_void_p(out.ctypes.data), _stream())
        if rc:
            i = lib().fq_batch_failed(self.b)
            msg = lib().fq_last_error(self._inst[i].h).decode() if i >= 0 else ""
            err = FqError(rc, f"fq_batch_run: instance {i}: {msg}")
            err.stats = out
            err.instance = i
            raise err
        return out

    def autotune(self, candidates, trial_steps=20):
        """Time candidate shared layouts (dicts of buckets, lds_slots, block,
        spawn_block) for the whole batch on device copies of its states
        (fq_batch_autotune).  Returns (ms per step for each candidate, or -1,
        index of the fastest).  The batch is not changed."""
        import torch
        lays = (Layout * len(candidates))()
        need = 0
        for i, c in enumerate(candidates):
            lays[i] = _layout(0, 0, c.get("buckets", 0), c.get("lds_slots", 0), c.get("block", 0),
                              c.get("spawn_block", 0))
            ls = (Layout * self.n)()
            for j in range(self.n):
                lo = self._inst[j].get_layout()
                ls[j] = _layout(lo.table_capacity, lo.spawn_capacity, c.get("buckets", 0),
                                c.get("lds_slots", 0), c.get("block", 0), c.get("spawn_block", 0))
            nb = C.c_size_t(0)
            if lib().fq_batch_workspace_size(self.n, self.hams, self.params, ls, C.byref(nb)) == 0:
                need = max(need, nb.value)
        scratch = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        ms = np.zeros(len(candidates))
        best = C.c_int32(-1)
        rc = lib().fq_batch_autotune(self.b, lays, len(candidates), int(trial_steps),
                                     C.c_void_p(scratch.data_ptr()), scratch.numel(), _p(ms, C.c_double),
                                     C.byref(best), _stream())
        del scratch
        if rc:
            raise FqError(rc, f"fq_batch_autotune: {lib().fq_batch_last_error(self.b).decode()}")
        return ms, best.value

    def run_replicas(self, n_steps):
        """Advance every instance as replicas of one Hamiltonian (Sec. 4.3)
        and compute the overlap c_A . c_B of every pair A < B after every
        step on the device.  Returns (stats of shape (n, n_steps), overlaps
        of shape (n_steps, P) with pairs (0,1), (0,2), .., (1,2), ..,
        inexact flag)."""
        import torch
        if self._ov is None:
            nb = C.c_size_t(0)
            rc = lib().fq_batch_replica_scratch_size(self.b, C.byref(nb))
            if rc:
                raise FqError(rc, f"fq_batch_replica_scratch_size: {lib().fq_batch_last_error(self.b).decode()}")
            self._ov = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        P = self.n * (self.n - 1) // 2
        out = np.zeros((self.n, n_steps), STATS_DTYPE)
        ovl = np.zeros((n_steps, P), np.float64)
        inexact = C.c_int32(0)
        rc = lib().fq_batch_run_replicas(self.b, n_steps, C.c_void_p(out.ctypes.data),
                                         C.c_void_p(ovl.ctypes.data), C.c_void_p(self._ov.data_ptr()),
                                         self._ov.numel(), C.byref(inexact), _stream())
        if rc:
            i = lib().fq_batch_failed(self.b)
            msg = (lib().fq_last_error(self._inst[i].h).decode() if i >= 0
                   else lib().fq_batch_last_error(self.b).decode())
            err = FqError(rc, f"fq_batch_run_replicas: {msg}")
            err.stats, err.overlaps, err.instance = out, ovl, i
            raise err
        return out, ovl, bool(inexact.value)

    def run_replicas_static(self, n_steps):
        """As run_replicas, with the join's scratch in the library's static
        device array (fq_batch_run_replicas_static: no device allocation;
        calls on one GPU must not overlap)."""
        P = self.n * (self.n - 1) // 2
        out = np.zeros((self.n, n_steps), STATS_DTYPE)
        ovl = np.zeros((n_steps, P), np.float64)
        inexact = C.c_int32(0)
        rc = lib().fq_batch_run_replicas_static(self.b, n_steps, C.c_void_p(out.ctypes.data),
                                                C.c_void_p(ovl.ctypes.data), C.byref(inexact), _stream())
        if rc:
            i = lib().fq_batch_failed(self.b)
            msg = (lib().fq_last_error(self._inst[i].h).decode() if i >= 0
                   else lib().fq_batch_last_error(self.b).decode())
            err = FqError(rc, f"fq_batch_run_replicas_static: {msg}")
            err.stats, err.overlaps, err.instance = out, ovl, i
            raise err
        return out, ovl, bool(inexact.value)

    def run_spectral(self, n_steps):
        """Advance every instance as step-synchronised runs of one
        Hamiltonian with run k orthogonalised against runs 0 .. k-1 after
        every merge (excited states, Sec. 2.2).  Returns (stats of shape
        (n, n_steps), inexact flag)."""
        import torch
        if self._gs is None:
            nb = C.c_size_t(0)
            rc = lib().fq_batch_spectral_scratch_size(self.b, C.byref(nb))
            if rc:
                raise FqError(rc, f"fq_batch_spectral_scratch_size: {lib().fq_batch_last_error(self.b).decode()}")
            self._gs = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        out = np.zeros((self.n, n_steps), STATS_DTYPE)
        inexact = C.c_int32(0)
        rc = lib().fq_batch_run_spectral(self.b, n_steps, C.c_void_p(out.ctypes.data),
                                         C.c_void_p(self._gs.data_ptr()), self._gs.numel(),
                                         C.byref(inexact), _stream())
        if rc:
            i = lib().fq_batch_failed(self.b)
            msg = (lib().fq_last_error(self._inst[i].h).decode() if i >= 0
                   else lib().fq_batch_last_error(self.b).decode())
            err = FqError(rc, f"fq_batch_run_spectral: {msg}")
            err.stats, err.instance = out, i
            raise err
        return out, bool(inexact.value)

    def close(self):
        if getattr(self, "b", None):
            for x in self._inst:
                x.close()
            lib().fq_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous batching of FCIQMC solves (fq_server_* of the C ABI)."""

    def __init__(self, model, pool_bytes, addr_words=1, lds_slots=1024, block=256, spawn_block=256,
                 max_active=64, steps_per_tick=200):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the FCIQMC server needs a GPU")
        self.cfg = ServerConfig(model, addr_words, lds_slots, block, spawn_block, max_active,
                                steps_per_tick)
        self.W = addr_words
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        sv = C.c_void_p()
        rc = lib().fq_server_create(C.byref(self.cfg), C.c_void_p(self.pool.data_ptr()),
                                    self.pool.numel(), C.byref(sv))
        if rc:
            raise FqError(rc, f"fq_server_create: {lib().fq_server_last_error(None).decode()}")
        self.sv = sv

    def _check(self, rc, what):
        if rc:
            raise FqError(rc, f"{what}: {lib().fq_server_last_error(self.sv).decode()}")

    def submit(self, spec, start, start_val=10.0, n_steps=1000):
        lay_keys = ("table_capacity", "spawn_capacity", "buckets", "lds_slots", "block",
                    "spawn_block")
        hp = {k: v for k, v in spec.items() if k not in lay_keys}
        hp.setdefault("addr_words", self.W)
        h, p = _ham_params(**hp)
        lay = _layout(**{k: v for k, v in spec.items() if k in lay_keys})
        a = np.zeros(2, np.uint64)
        st = np.asarray(start, dtype=np.uint64).ravel()
        a[:len(st)] = st
        rid = C.c_uint64(0)
        self._check(lib().fq_server_submit(self.sv, C.byref(h), C.byref(p), C.byref(lay),
                                           _p(a, C.c_uint64), float(start_val), int(n_steps),
                                           C.byref(rid)), "fq_server_submit")
        return rid.value

    def tick(self):
        a, q, f = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        self._check(lib().fq_server_tick(self.sv, _stream(), C.byref(a), C.byref(q), C.byref(f)),
                    "fq_server_tick")
        return a.value, q.value, f.value

    def poll(self, rid):
        info = RequestInfo()
        self._check(lib().fq_server_poll(self.sv, int(rid), C.byref(info)), "fq_server_poll")
        last = {k: getattr(info.last, k) for k, _ in StepStats._fields_}
        return dict(state=info.state, status=info.status, steps_done=info.steps_done, last=last,
                    mean_shift=info.mean_shift, mean_hproj=info.mean_hproj,
                    mean_vproj=info.mean_vproj, n_mean=info.n_mean,
                    workspace_bytes=info.workspace_bytes, walker_steps=info.walker_steps)

    def close(self):
        if getattr(self, "sv", None):
            lib().fq_server_destroy(self.sv)
            self.sv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def source_digest():
    """sha256 of the kernel sources and the C header (identifies the kernels
    a profile was taken with)."""
    import hashlib
    hsh = hashlib.sha256()
    root = os.path.dirname(HERE)
    files = sorted(os.path.join(HERE, "csrc", f) for f in os.listdir(os.path.join(HERE, "csrc"))
                   if f.endswith((".hip", ".hpp")))
    files.append(os.path.join(root, "include", "fciqmc.h"))
    for f in files:
        with open(f, "rb") as fh:
            hsh.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return hsh.hexdigest()


def start_address(model, M, N, W=1):
    """Default starting address: the uniform state in real space (ring or
    lattice, sites in index order), the k = 0 condensate in momentum space."""
    if model == MOM1D:
        occ = [N] + [0] * (M - 1)
    else:
        occ = [N // M + (1 if j < N % M else 0) for j in range(M)]
    return encode(occ, W)
