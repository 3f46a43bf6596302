"""CPU oracle for the FCIQMC hot path of the Rimu.jl paper (arXiv 2601.19505).

TEST INFRASTRUCTURE ONLY: a plain, serial, slow and obviously correct
reference.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the GPU library in ``paper_2601_19505_amd``; the two meet only through the
seeded input generators in ``synthetic``.

Contents (paper sections in brackets):

* Fock addresses, dimension and combinatorial ranking [Sec. 2, Sec. 6.1]
* real- and momentum-space 1D Bose-Hubbard columns [Sec. 2, Sec. 6.2, 6.3],
  the periodic square lattice and Gutzwiller importance sampling [Sec. 3.3,
  Sec. 7.2]
* Philox4x32-10 counter-based draws (published definition, Salmon et al.)
* one serial FCIQMC step and repeated steps [Sec. 3.1, 3.2, 7.1]
* sparse-matrix and matrix-free Lanczos exact diagonalisation [Sec. 5]
* replica overlaps c_A . c_B [Sec. 4.3]; Gram-Schmidt orthogonalisation
  of step-synchronised vectors for excited states [Sec. 2.2]
* blocking analysis, shift estimator, ratio of means, variational energy
  [Sec. 4] (``stats``)

Every function here is pinned by a ``-m "not gpu"`` test against the
paper's printed values, closed forms or independent library routines.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

REAL1D = 0
MOM1D = 1
REAL2D = 2


class Ham(C.Structure):
    _fields_ = [("model", C.c_int32), ("M", C.c_int32), ("N", C.c_int32), ("lx", C.c_int32),
                ("t", C.c_double), ("u", C.c_double), ("g", C.c_double)]


class Params(C.Structure):
    _fields_ = [("h", Ham), ("dtau", C.c_double), ("target", C.c_double), ("zeta", C.c_double),
                ("xi", C.c_double), ("theta", C.c_double), ("t_rel", C.c_double),
                ("seed", C.c_uint64), ("early", C.c_int32), ("initiator", C.c_int32),
                ("n_a", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("len", C.c_int64), ("exact_steps", C.c_int64),
                ("inexact_steps", C.c_int64), ("spawns", C.c_int64), ("shift", C.c_double),
                ("norm", C.c_double), ("hproj", C.c_double), ("vproj", C.c_double)]


EVENT_DTYPE = np.dtype([("parent", np.int64), ("attempt", np.int64), ("dest", np.uint64, (2,)),
                        ("value", np.float64)])
STATS_FIELDS = [f for f, _ in Stats._fields_]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        u64p, f64p, i64p, i32p, u32p = (P(C.c_uint64), P(C.c_double), P(C.c_int64), P(C.c_int32),
                                        P(C.c_uint32))
        L.orc_binom.restype = C.c_uint64
        L.orc_binom.argtypes = [C.c_int, C.c_int]
        L.orc_dimension.restype = C.c_uint64
        L.orc_dimension.argtypes = [C.c_int, C.c_int]
        L.orc_encode.restype = C.c_int
        L.orc_encode.argtypes = [i32p, C.c_int, u64p]
        L.orc_decode.restype = None
        L.orc_decode.argtypes = [u64p, C.c_int, C.c_int, i32p]
        L.orc_rank.restype = C.c_uint64
        L.orc_rank.argtypes = [u64p, C.c_int, C.c_int]
        L.orc_unrank.restype = None
        L.orc_unrank.argtypes = [C.c_uint64, C.c_int, C.c_int, u64p]
        L.orc_philox4x32_10.restype = None
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_draw.restype = None
        L.orc_draw.argtypes = [C.c_uint64, u64p, C.c_uint32, C.c_uint32, C.c_uint32, u32p]
        L.orc_det_log.restype = C.c_double
        L.orc_det_log.argtypes = [C.c_double]
        L.orc_fsum.restype = C.c_double
        L.orc_fsum.argtypes = [f64p, C.c_int64]
        L.orc_column.restype = C.c_int
        L.orc_column.argtypes = [P(Ham), u64p, u64p, f64p, C.c_int, f64p]
        L.orc_row.restype = C.c_int
        L.orc_row.argtypes = [P(Ham), u64p, u64p, f64p, C.c_int]
        L.orc_shift_update.restype = C.c_double
        L.orc_shift_update.argtypes = [C.c_double] * 7
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [P(Params), u64p, f64p, C.c_int64, C.c_double, C.c_int64, u64p,
                               C.c_double, u64p, f64p, C.c_int64, i64p, P(Stats), C.c_void_p,
                               C.c_int64, i64p, u64p, f64p, C.c_int64, i64p]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [P(Params), u64p, f64p, C.c_int64, C.c_double, C.c_int64, C.c_int64,
                              u64p, C.c_double, C.c_int64, u64p, f64p, i64p, P(Stats)]
        L.orc_build_csr.restype = C.c_int
        L.orc_build_csr.argtypes = [P(Ham), i64p, i64p, f64p]
        L.orc_lanczos.restype = C.c_int
        L.orc_lanczos.argtypes = [P(Ham), u64p, C.c_int, f64p, f64p, i32p]
        L.orc_validate.restype = C.c_int
        L.orc_validate.argtypes = [P(Ham)]
        L.orc_sampled_pair.restype = C.c_int
        L.orc_sampled_pair.argtypes = [P(Ham), u64p, C.c_int, i32p, i32p]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")
    return rc


# --------------------------------------------------------------------------
# Fock addresses [Sec. 6.1]
# --------------------------------------------------------------------------

def binom(n, k):
    return int(lib().orc_binom(n, k))


def dimension(M, N):
    """Hilbert dimension C(N+M-1, N) [Sec. 2]."""
    return int(lib().orc_dimension(M, N))


def encode(occ):
    """Occupations -> (word0, word1) of the unary bitstring [Sec. 6.1]."""
    o = np.ascontiguousarray(occ, dtype=np.int32)
    w = np.zeros(2, np.uint64)
    nb = lib().orc_encode(_p(o, C.c_int32), len(o), _p(w, C.c_uint64))
    if nb < 0:
        raise ValueError("address does not fit 128 bits")
    return int(w[0]), int(w[1])


def encode_many(occs):
    occs = np.asarray(occs, dtype=np.int32)
    out = np.zeros((len(occs), 2), np.uint64)
    for i, o in enumerate(occs):
        out[i] = encode(o)
    return out


def decode(words, M, N):
    w = np.asarray([int(words[0]), int(words[1])], np.uint64)
    occ = np.zeros(M, np.int32)
    lib().orc_decode(_p(w, C.c_uint64), M, N, _p(occ, C.c_int32))
    return occ


def bitstring(occ):
    """The paper's printed form: N+M-1 bits, most significant first."""
    occ = list(occ)
    nb = sum(occ) + len(occ) - 1
    w0, w1 = encode(occ)
    v = w0 | (w1 << 64)
    return format(v, "b").zfill(nb)


def rank(words, M, N):
    w = np.asarray([int(words[0]), int(words[1])], np.uint64)
    return int(lib().orc_rank(_p(w, C.c_uint64), M, N))


def unrank(r, M, N):
    w = np.zeros(2, np.uint64)
    lib().orc_unrank(r, M, N, _p(w, C.c_uint64))
    return int(w[0]), int(w[1])


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(o, C.c_uint32))
    return [int(x) for x in o]


def draw(seed, words, step, tag, block):
    a = np.asarray([int(words[0]), int(words[1])], np.uint64)
    o = np.zeros(4, np.uint32)
    lib().orc_draw(seed, _p(a, C.c_uint64), step, tag, block, _p(o, C.c_uint32))
    return [int(x) for x in o]


def det_log(x):
    return float(lib().orc_det_log(x))


def fsum(xs):
    x = np.ascontiguousarray(xs, dtype=np.float64)
    return float(lib().orc_fsum(_p(x, C.c_double), len(x)))


def shift_update(S, N1, N0, Nt, zeta, xi, dtau):
    return float(lib().orc_shift_update(S, N1, N0, Nt, zeta, xi, dtau))


# --------------------------------------------------------------------------
# Hamiltonians [Sec. 6.2]
# --------------------------------------------------------------------------

def ham(model, M, N, t=1.0, u=1.0, lx=0, g=0.0):
    """Hamiltonian: REAL1D ring of M sites, MOM1D with M modes, or REAL2D
    periodic lx x (M / lx) lattice; g is the Gutzwiller importance-sampling
    parameter of the real-space models [Sec. 3.3, Sec. 7.2]."""
    return Ham(model, M, N, int(lx), float(t), float(u), float(g))


def column(h, words, cap=1 << 16):
    """(diagonal, dests[m,2], values[m]) in canonical enumeration order."""
    a = np.asarray([int(words[0]), int(words[1])], np.uint64)
    dest = np.zeros((cap, 2), np.uint64)
    vals = np.zeros(cap, np.float64)
    diag = C.c_double(0.0)
    m = _check(lib().orc_column(C.byref(h), _p(a, C.c_uint64), _p(dest, C.c_uint64),
                                _p(vals, C.c_double), cap, C.byref(diag)), "column")
    return diag.value, dest[:m].copy(), vals[:m].copy()


def row(h, words, cap=1 << 16):
    """(dests[m,2], values[m]): the row of `words` over its column's
    destinations, H_{words,dest} (differs from the column only under
    importance sampling)."""
    a = np.asarray([int(words[0]), int(words[1])], np.uint64)
    dest = np.zeros((cap, 2), np.uint64)
    vals = np.zeros(cap, np.float64)
    m = _check(lib().orc_row(C.byref(h), _p(a, C.c_uint64), _p(dest, C.c_uint64),
                             _p(vals, C.c_double), cap), "row")
    return dest[:m].copy(), vals[:m].copy()


def sampled_pair(h, words, pi):
    """Modes (p, q) of the removal pair with sampling index pi (momentum space)."""
    a = np.asarray([int(words[0]), int(words[1])], np.uint64)
    p, q = C.c_int32(0), C.c_int32(0)
    _check(lib().orc_sampled_pair(C.byref(h), _p(a, C.c_uint64), int(pi), C.byref(p), C.byref(q)),
           "sampled_pair")
    return p.value, q.value


def validate(h):
    return lib().orc_validate(C.byref(h)) == 0


# --------------------------------------------------------------------------
# FCIQMC [Sec. 3]
# --------------------------------------------------------------------------

def params(model, M, N, t=1.0, u=1.0, dtau=1e-3, target=1000.0, zeta=0.08, xi=None,
           theta=1.0, t_rel=1.0, seed=0, early=False, lx=0, g=0.0, initiator=None):
    """FCIQMC parameters; `initiator` is the threshold n_a of the initiator
    rule (None: the rule is off)."""
    if xi is None:
        xi = zeta * zeta / 4.0
    return Params(ham(model, M, N, t, u, lx, g), dtau, target, zeta, xi, theta, t_rel, seed,
                  1 if early else 0, 0 if initiator is None else 1,
                  0.0 if initiator is None else float(initiator))


def _addr2(addrs):
    a = np.zeros((len(addrs), 2), np.uint64)
    if len(addrs):
        arr = np.asarray(addrs, dtype=np.uint64)
        if arr.ndim == 1:
            a[:, 0] = arr
        else:
            a[:, :arr.shape[1]] = arr
    return np.ascontiguousarray(a)


def step(P, addrs, vals, shift, step_index, ref, yref, cap=None, events=False, merged=False):
    """One step c^(n) -> c^(n+1); returns dict with table, stats, dumps."""
    a = _addr2(addrs)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    n = len(v)
    if cap is None:
        cap = max(16, 64 * (n + int(np.abs(v).sum()) + 16))
    oa = np.zeros((cap, 2), np.uint64)
    ov = np.zeros(cap, np.float64)
    on = C.c_int64(0)
    st = Stats()
    r = np.asarray([int(ref[0]), int(ref[1])], np.uint64)
    ev = np.zeros(cap if events else 0, EVENT_DTYPE)
    evn = C.c_int64(0)
    mga = np.zeros((cap if merged else 0, 2), np.uint64)
    mgv = np.zeros(cap if merged else 0, np.float64)
    mgn = C.c_int64(0)
    rc = lib().orc_step(C.byref(P), _p(a, C.c_uint64), _p(v, C.c_double), n, shift, step_index,
                        _p(r, C.c_uint64), yref, _p(oa, C.c_uint64), _p(ov, C.c_double), cap,
                        C.byref(on), C.byref(st),
                        ev.ctypes.data if events else None, len(ev), C.byref(evn),
                        _p(mga, C.c_uint64) if merged else None,
                        _p(mgv, C.c_double) if merged else None, len(mgv), C.byref(mgn))
    _check(rc, "step")
    out = dict(addr=oa[:on.value].copy(), val=ov[:on.value].copy(),
               stats={f: getattr(st, f) for f in STATS_FIELDS})
    if events:
        if evn.value > len(ev):
            raise RuntimeError("event capacity exceeded")
        out["events"] = ev[:evn.value].copy()
    if merged:
        out["merged_addr"] = mga[:mgn.value].copy()
        out["merged_val"] = mgv[:mgn.value].copy()
    return out


def run(P, addrs, vals, shift, first_step, nsteps, ref, yref, cap=None):
    """Repeated steps; returns (stats structured array, final addr, final val)."""
    a = _addr2(addrs)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    if cap is None:
        cap = 1 << 22
    oa = np.zeros((cap, 2), np.uint64)
    ov = np.zeros(cap, np.float64)
    on = C.c_int64(0)
    stats = (Stats * nsteps)()
    r = np.asarray([int(ref[0]), int(ref[1])], np.uint64)
    rc = lib().orc_run(C.byref(P), _p(a, C.c_uint64), _p(v, C.c_double), len(v), shift,
                       first_step, nsteps, _p(r, C.c_uint64), yref, cap, _p(oa, C.c_uint64),
                       _p(ov, C.c_double), C.byref(on), stats)
    _check(rc, "run")
    dt = np.dtype([(f, np.int64 if f in ("step", "len", "exact_steps", "inexact_steps", "spawns")
                    else np.float64) for f in STATS_FIELDS])
    arr = np.zeros(nsteps, dt)
    for k in range(nsteps):
        for f in STATS_FIELDS:
            arr[f][k] = getattr(stats[k], f)
    return arr, oa[:on.value].copy(), ov[:on.value].copy()


# --------------------------------------------------------------------------
# Replica overlaps [Sec. 4.3]
# --------------------------------------------------------------------------

def replica_pairs(R):
    """The pairs (A, B), A < B, of R replicas in the order A = 0.., then B."""
    return [(a, b) for a in range(R) for b in range(a + 1, R)]


def _keys(addrs):
    a = np.ascontiguousarray(np.asarray(addrs, dtype=np.uint64).reshape(len(addrs), -1))
    return a.view(np.dtype((np.void, 8 * a.shape[1]))).ravel()


def overlap(addrs_a, vals_a, addrs_b, vals_b):
    """Dot product c_A . c_B of two sparse vectors [Sec. 4.3, Eq.
    RayleighQuotientReplica, denominator term].

    Addresses present in only one of the vectors contribute nothing.  Each
    product of two amplitudes is rounded to double; the products are summed
    exactly and rounded once (math.fsum).  Address rows must be unique
    within each vector and use the same number of words.
    """
    import math
    ka, kb = _keys(addrs_a), _keys(addrs_b)
    if len(np.unique(ka)) != len(ka) or len(np.unique(kb)) != len(kb):
        raise ValueError("overlap: duplicate address")
    _, ia, ib = np.intersect1d(ka, kb, assume_unique=True, return_indices=True)
    va = np.asarray(vals_a, dtype=np.float64)[ia]
    vb = np.asarray(vals_b, dtype=np.float64)[ib]
    return math.fsum((va * vb).tolist())


def orthogonalise(addrs_k, vals_k, addrs_j, vals_j):
    """Gram-Schmidt projection c_k - (c_j . c_k / c_j . c_j) c_j [Sec. 2.2,
    excited states by orthogonalising step-synchronised vectors].

    c_j . c_k is the exactly rounded overlap and c_j . c_j the exactly
    rounded sum of the rounded squares; their quotient alpha is one IEEE
    division (0 when c_j is empty).  Each entry becomes v_k - (alpha v_j),
    the product rounded first, with v_k = 0 where c_k has no entry; exact
    zeros are dropped.  Returns (addrs, vals, alpha), c_k's entries first in
    their order, then the new addresses in c_j's order.
    """
    import math
    W = max(np.asarray(addrs_k).reshape(len(addrs_k), -1).shape[1] if len(addrs_k) else 1,
            np.asarray(addrs_j).reshape(len(addrs_j), -1).shape[1] if len(addrs_j) else 1)
    A = np.ascontiguousarray(np.asarray(addrs_k, dtype=np.uint64).reshape(len(addrs_k), W))
    Bj = np.ascontiguousarray(np.asarray(addrs_j, dtype=np.uint64).reshape(len(addrs_j), W))
    vk = np.asarray(vals_k, dtype=np.float64)
    vj = np.asarray(vals_j, dtype=np.float64)
    dot = overlap(A, vk, Bj, vj) if len(vk) and len(vj) else 0.0
    nrm2 = math.fsum((vj * vj).tolist())
    alpha = dot / nrm2 if nrm2 > 0.0 else 0.0
    out = {}
    order = []
    for row, v in zip(A, vk):
        key = row.tobytes()
        out[key] = float(v)
        order.append((key, row))
    for row, v in zip(Bj, vj):
        key = row.tobytes()
        if key not in out:
            out[key] = 0.0
            order.append((key, row))
        out[key] = out[key] - alpha * float(v)
    keep = [(row, out[key]) for key, row in order if out[key] != 0.0]
    addrs = np.array([r for r, _ in keep], dtype=np.uint64).reshape(len(keep), W)
    vals = np.array([v for _, v in keep], dtype=np.float64)
    return addrs, vals, alpha


def spectral_run(Ps, starts, ref, nsteps, yref=10.0):
    """R step-synchronised runs of one Hamiltonian (parameters Ps[r], 10
    walkers on starts[r], shift 0, projected energy on ref): after every
    step, vector k is orthogonalised against vectors 0 .. k-1 in turn [Sec.
    2.2].  Returns the statistics rows (R, nsteps) of the steps (describing
    the merged vectors before the orthogonalisation) and the final states."""
    R = len(Ps)
    st = [(_addr2([a]), np.array([10.0]), 0.0) for a in starts]
    rows = [[] for _ in range(R)]
    for n in range(nsteps):
        for r in range(R):
            addrs, vals, S = st[r]
            o = step(Ps[r], addrs, vals, S, n + 1, ref, yref)
            st[r] = (o["addr"], o["val"], o["stats"]["shift"])
            rows[r].append(o["stats"])
        for k in range(1, R):
            for j in range(k):
                a, v, _ = orthogonalise(st[k][0], st[k][1], st[j][0], st[j][1])
                st[k] = (a, v, st[k][2])
    return rows, st


# --------------------------------------------------------------------------
# Exact diagonalisation [Sec. 5]
# --------------------------------------------------------------------------

def csr_matrix(h):
    """H as scipy.sparse CSR over the ranked basis (column j -> rows)."""
    import scipy.sparse as sp
    D = dimension(h.M, h.N)
    indptr = np.zeros(D + 1, np.int64)
    _check(lib().orc_build_csr(C.byref(h), _p(indptr, C.c_int64), None, None), "csr count")
    nnz = int(indptr[-1])
    ind = np.zeros(nnz, np.int64)
    dat = np.zeros(nnz, np.float64)
    _check(lib().orc_build_csr(C.byref(h), _p(indptr, C.c_int64), _p(ind, C.c_int64),
                               _p(dat, C.c_double)), "csr fill")
    # column j stores (row indices, values): this is CSC of H, i.e. CSR of H^T.
    m = sp.csc_matrix((dat, ind, indptr), shape=(D, D))
    return m.tocsr()


def dense_matrix(h):
    return csr_matrix(h).toarray()


def lanczos(h, start, kmax=200):
    """Lowest Ritz value from plain matrix-free Lanczos started at `start`."""
    from scipy.linalg import eigh_tridiagonal
    s = np.asarray([int(start[0]), int(start[1])], np.uint64)
    al = np.zeros(kmax)
    be = np.zeros(kmax)
    k = C.c_int32(0)
    _check(lib().orc_lanczos(C.byref(h), _p(s, C.c_uint64), kmax, _p(al, C.c_double),
                             _p(be, C.c_double), C.byref(k)), "lanczos")
    k = k.value
    w = eigh_tridiagonal(al[:k], be[:k - 1], eigvals_only=True)
    return np.sort(w)


def eigs_sparse(h, k=2):
    from scipy.sparse.linalg import eigsh
    m = csr_matrix(h)
    w = eigsh(m, k=k, which="SA", return_eigenvectors=False, tol=1e-12)
    return np.sort(w)


def start_address(model, M, N):
    """Starting address: the uniform (near_uniform) state in real space (ring
    or lattice, sites in index order); the k = 0 condensate in momentum space
    (reading for the momentum model)."""
    if model == MOM1D:
        occ = [0] * M
        occ[0] = N
    else:
        occ = [N // M + (1 if j < N % M else 0) for j in range(M)]
    return encode(occ)
