"""Pins of the oracle's square-lattice Bose-Hubbard model and of Gutzwiller
importance sampling [Sec. 2, Sec. 3.3, Sec. 7.2].

The lattice Hamiltonian is checked against a first-quantised construction
that shares nothing with the oracle's column code (two bosons: the
symmetric block of T (x) 1 + 1 (x) T + u on the diagonal of the pair space,
with T built from grid coordinates by np.roll), and against the free-boson
closed form.  The importance-sampled Hamiltonian is checked to be a
similarity transform in the stated direction (same spectrum, ground vector
exp(-g H_ii) v0), its rows to be the transpose of its columns, and its
stochastic step to be unbiased.
"""
import numpy as np
import pytest

from test_oracle_step import _dense_T, _to_dense


def _hopping(lx, ly, t):
    """Single-particle hopping matrix of the periodic lx x ly lattice from
    grid shifts; a bond reached in two directions counts twice."""
    M = lx * ly
    idx = np.arange(M).reshape(ly, lx)  # idx[y, x] = x + lx y
    T = np.zeros((M, M))
    for axis in (0, 1):
        for sh in (1, -1):
            nb = np.roll(idx, -sh, axis=axis)
            for s, d in zip(idx.ravel(), nb.ravel()):
                T[d, s] += -t
    return T


def _two_boson_spectrum(lx, ly, t, u):
    T = _hopping(lx, ly, t)
    M = lx * ly
    I = np.eye(M)
    H1 = np.kron(T, I) + np.kron(I, T)
    H1 += u * np.diag([1.0 if i == j else 0.0 for i in range(M) for j in range(M)])
    # symmetric two-boson states |i j> + |j i> (normalised), i <= j
    cols = []
    for i in range(M):
        for j in range(i, M):
            v = np.zeros(M * M)
            v[i * M + j] += 1.0
            v[j * M + i] += 1.0
            cols.append(v / np.linalg.norm(v))
    B = np.array(cols).T
    return np.sort(np.linalg.eigvalsh(B.T @ H1 @ B))


@pytest.mark.parametrize("lx,ly,u", [(3, 3, 2.5), (4, 3, 1.0), (4, 2, 3.0), (2, 2, 0.7)])
def test_two_bosons_match_first_quantised(orc, lx, ly, u):
    h = orc.ham(orc.REAL2D, lx * ly, 2, 1.0, u, lx=lx)
    H = orc.dense_matrix(h)
    assert np.allclose(H, H.T)
    w = np.sort(np.linalg.eigvalsh(H))
    assert np.allclose(w, _two_boson_spectrum(lx, ly, 1.0, u), atol=1e-10)


@pytest.mark.parametrize("lx,ly,N", [(3, 3, 3), (4, 3, 4), (3, 2, 5)])
def test_free_bosons_on_the_torus(orc, lx, ly, N):
    """u = 0: all bosons in the k = 0 orbital, E0 = -4 t N (-2 t per
    direction, a width-2 direction doubling its bond)."""
    t = 0.7
    h = orc.ham(orc.REAL2D, lx * ly, N, t, 0.0, lx=lx)
    E0 = np.sort(np.linalg.eigvalsh(orc.dense_matrix(h)))[0]
    assert abs(E0 - (-4.0 * t * N)) < 1e-10


def test_lattice_rejects_bad_shapes(orc):
    assert not orc.validate(orc.ham(orc.REAL2D, 9, 3, lx=1))
    assert not orc.validate(orc.ham(orc.REAL2D, 10, 3, lx=3))
    assert not orc.validate(orc.ham(orc.REAL2D, 6, 3, lx=6))
    assert not orc.validate(orc.ham(orc.MOM1D, 6, 3, g=0.2))
    assert orc.validate(orc.ham(orc.REAL2D, 6, 3, lx=3, g=0.2))
    assert orc.validate(orc.ham(orc.REAL1D, 6, 3, g=0.2))


@pytest.mark.parametrize("model,M,N,lx,u,g", [(2, 9, 4, 3, 2.0, 0.4), (0, 6, 6, 0, 6.0, 0.25),
                                              (2, 8, 5, 4, 1.0, -0.3)])
def test_gutzwiller_is_the_stated_similarity_transform(orc, model, M, N, lx, u, g):
    h0 = orc.ham(model, M, N, 1.0, u, lx=lx)
    hg = orc.ham(model, M, N, 1.0, u, lx=lx, g=g)
    H = orc.dense_matrix(h0)
    Hg = orc.dense_matrix(hg)
    D = np.diag(H)
    assert np.array_equal(np.diag(Hg), D)
    # same spectrum
    w0 = np.linalg.eigvalsh(H)
    wg = np.sort(np.linalg.eigvals(Hg).real)
    assert np.allclose(w0, wg, atol=1e-9)
    # H~ = G H G^-1 with G = diag(exp(-g H_ii)): ground vector of H~ is G v0
    e, V = np.linalg.eigh(H)
    v0 = V[:, 0]
    f = np.exp(-g * D) * v0
    assert np.allclose(Hg @ f, e[0] * f, atol=1e-9 * np.abs(f).max())


@pytest.mark.parametrize("model,M,N,lx,g", [(2, 9, 4, 3, 0.4), (0, 7, 5, 0, -0.6)])
def test_rows_are_the_transposed_columns(orc, model, M, N, lx, g):
    """Row r's value at destination j equals column j's value at r."""
    h = orc.ham(model, M, N, 1.0, 2.0, lx=lx, g=g)
    rng = np.random.default_rng(5)
    for r in rng.choice(orc.dimension(M, N), 20, replace=False):
        a = orc.unrank(int(r), M, N)
        dests, rv = orc.row(h, a)
        _, cdest, cv = orc.column(h, a)
        assert np.array_equal(dests, cdest)
        for d, x in zip(dests, rv):
            _, back, bv = orc.column(h, d)
            hits = [bv[i] for i in range(len(bv)) if tuple(back[i]) == (a[0], a[1])]
            assert hits and all(y == hits[0] for y in hits)
            assert x == hits[0]


@pytest.mark.parametrize("model,M,N,lx,u,g,early", [(2, 6, 4, 3, 2.0, 0.3, False), (2, 6, 4, 3, 2.0, 0.3, True),
                                                    (0, 5, 5, 0, 6.0, 0.2, False)])
def test_lattice_step_unbiased(orc, model, M, N, lx, u, g, early):
    """E[T~ c] = T c for the lattice and importance-sampled Hamiltonians,
    within 5 standard errors per entry (Sec. 3.2)."""
    rng = np.random.default_rng(23)
    D = orc.dimension(M, N)
    idx = rng.choice(D, size=min(D, 12), replace=False)
    addrs = [orc.unrank(int(i), M, N) for i in idx]
    vals = rng.choice([-1, 1], len(idx)) * rng.uniform(0.2, 40.0, len(idx))
    S, dtau = -1.1, 0.01
    h = orc.ham(model, M, N, 1.0, u, lx=lx, g=g)
    Tc, _ = _dense_T(orc, h, addrs, vals, S, dtau)
    nseed = 2000
    acc = np.zeros(D)
    acc2 = np.zeros(D)
    for s in range(nseed):
        P = orc.params(model, M, N, 1.0, u, dtau=dtau, target=100.0, seed=500 + s, early=early, lx=lx, g=g)
        out = orc.step(P, addrs, vals, S, 3, addrs[0], 1.0)
        x = _to_dense(orc, h, out["addr"], out["val"])
        acc += x
        acc2 += x * x
    mean = acc / nseed
    # an entry reached with probability p ~ |Tc| / theta may never be hit:
    # one hit moves its mean by theta / nseed, the floor of the error
    sd = np.sqrt(np.maximum(acc2 / nseed - mean ** 2, 0.0) / nseed)
    z = np.abs(mean - Tc) / np.maximum(sd, 1.0 / nseed)
    assert np.all(z < 5.0), z.max()


def test_projected_energy_uses_the_row(orc):
    """For the exact importance-sampled ground vector f = G v0 the step's
    y.H~f / y.f (computed on the output state from exact columns, t_rel = 0,
    no compression below theta) equals E0: with the column values instead of
    the row it would not."""
    M, N, lx, u, g = 6, 3, 3, 2.0, 0.5
    h0 = orc.ham(orc.REAL2D, M, N, 1.0, u, lx=lx)
    H = orc.dense_matrix(h0)
    e, V = np.linalg.eigh(H)
    v0 = V[:, 0] * np.sign(V[:, 0].sum())
    f = np.exp(-g * np.diag(H)) * v0
    f = f / np.abs(f).min() * 4.0  # every amplitude >= 4 > theta
    addrs = [orc.unrank(i, M, N) for i in range(len(f))]
    ref = orc.start_address(orc.REAL2D, M, N)
    P = orc.params(orc.REAL2D, M, N, 1.0, u, dtau=1e-3, target=1e9, theta=1e-3, t_rel=0.0, seed=0,
                   lx=lx, g=g)
    out = orc.step(P, addrs, f, e[0], 1, ref, 1.0)
    st = out["stats"]
    # an exact step with S = E0 maps the eigenvector onto itself
    assert abs(st["hproj"] / st["vproj"] - e[0]) < 1e-10
