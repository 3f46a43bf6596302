/*
 * oracle/orc.c -- plain, serial, slow CPU reference for the FCIQMC hot path
 * described in the Rimu.jl paper (arXiv 2601.19505).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library; the product path never does.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Everything is fp64, compiled without floating-point contraction and without
 * fast-math.  Each function cites the passage of the paper it follows.  Where
 * the paper is silent the reading taken is stated in the comment.
 *
 * Address convention (Sec. 6.1, bitstring representation of BoseFS): a Fock
 * state |n_1 ... n_M> is a string of N+M-1 bits; mode 1 occupies the lowest
 * bits as n_1 ones, then one zero separator, then n_2 ones, ...  The string is
 * kept in two 64-bit words (word 0 holds bits 0..63).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXM 128
#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ECAP -2
#define ORC_ENOMEM -4

enum { ORC_REAL1D = 0, ORC_MOM1D = 1, ORC_REAL2D = 2 };

typedef struct {
    int32_t model, M, N;
    int32_t lx;      /* square lattice: sites per row (M = lx * ly); unused in 1D */
    double t, u;
    double g;        /* Gutzwiller importance-sampling parameter (0: none) */
} orc_ham;

typedef struct {
    orc_ham h;
    double dtau, target, zeta, xi, theta, t_rel;
    uint64_t seed;
    int32_t early;   /* 0: late compression (default); 1: early compression (Sec. 7.1) */
    int32_t initiator; /* 1: initiator rule with threshold n_a (Sec. 1, sign-problem paragraph of Sec. 3.2) */
    double n_a;
} orc_params;

typedef struct {
    int64_t step, len, exact_steps, inexact_steps, spawns;
    double shift, norm, hproj, vproj;
} orc_stats;

typedef struct {
    int64_t parent;   /* index of the parent in the input table */
    int64_t attempt;  /* attempt (stochastic) or column entry (exact) */
    uint64_t dest[2];
    double value;
} orc_event;

/* ------------------------------------------------------------------------ */
/* Binomials and the Hilbert dimension, D = C(N+M-1, N)  (Sec. 2)            */
/* ------------------------------------------------------------------------ */

/* C(n, k) from Pascal's triangle C(n,k) = C(n-1,k-1) + C(n-1,k), built once
 * for n < 128 and saturating at UINT64_MAX when a value does not fit. */
static uint64_t pascal[128][128];
static int pascal_ready = 0;

static uint64_t sat_add(uint64_t a, uint64_t b) { return a > UINT64_MAX - b ? UINT64_MAX : a + b; }

uint64_t orc_binom(int n, int k)
{
    if (k < 0 || n < 0 || k > n || n >= 128) return 0;
    if (!pascal_ready) {
        for (int i = 0; i < 128; i++) {
            pascal[i][0] = 1;
            for (int j = 1; j <= i; j++)
                pascal[i][j] = j == i ? 1 : sat_add(pascal[i - 1][j - 1], pascal[i - 1][j]);
        }
        pascal_ready = 1;
    }
    return pascal[n][k];
}

uint64_t orc_dimension(int M, int N) { return orc_binom(N + M - 1, N); }

/* ------------------------------------------------------------------------ */
/* Fock addresses (Sec. 6.1)                                                 */
/* ------------------------------------------------------------------------ */

static inline int getbit(const uint64_t *w, int p) { return (int)((w[p >> 6] >> (p & 63)) & 1u); }
static inline void setbit(uint64_t *w, int p) { w[p >> 6] |= (uint64_t)1 << (p & 63); }

/* Occupation numbers -> unary bitstring.  Returns the number of bits used. */
int orc_encode(const int32_t *occ, int M, uint64_t *w)
{
    w[0] = w[1] = 0;
    int pos = 0;
    for (int j = 0; j < M; j++) {
        for (int r = 0; r < occ[j]; r++) {
            if (pos >= 128) return -1;
            setbit(w, pos++);
        }
        if (j < M - 1) pos++; /* separator zero */
    }
    return pos;
}

void orc_decode(const uint64_t *w, int M, int N, int32_t *occ)
{
    int nb = N + M - 1, pos = 0;
    for (int j = 0; j < M; j++) {
        int n = 0;
        while (pos < nb && getbit(w, pos)) { n++; pos++; }
        occ[j] = n;
        pos++;
    }
}

/* Combinatorial ranking of the bitstring: the positions p_1 < ... < p_N of
 * the ones form an N-subset of {0..N+M-2}; rank = sum_c C(p_c, c).  This is
 * a bijection onto [0, D) and plays the role of the index <-> address
 * translation layer of the matrix-free exact diagonalisation (Sec. 5). */
uint64_t orc_rank(const uint64_t *w, int M, int N)
{
    int nb = N + M - 1, c = 0;
    uint64_t r = 0;
    for (int p = 0; p < nb; p++)
        if (getbit(w, p)) { c++; r += orc_binom(p, c); }
    return r;
}

void orc_unrank(uint64_t r, int M, int N, uint64_t *w)
{
    w[0] = w[1] = 0;
    int p = N + M - 2;
    for (int c = N; c >= 1; c--) {
        while (orc_binom(p, c) > r) p--;
        setbit(w, p);
        r -= orc_binom(p, c);
        p--;
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its       */
/* published definition.  The paper fixes no generator; keying reading:     */
/*   key     = 64-bit seed XOR address word 1                                */
/*   counter = (address word 0 low, high, (tag << 28) | block, step)         */
/* tag 0 draws spawn picks, tag 1 draws the vector-compression uniform.      */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_draw(uint64_t seed, const uint64_t *a, uint32_t step, uint32_t tag, uint32_t block,
              uint32_t *out)
{
    uint64_t k = seed ^ a[1];
    uint32_t key[2] = {(uint32_t)k, (uint32_t)(k >> 32)};
    uint32_t ctr[4] = {(uint32_t)a[0], (uint32_t)(a[0] >> 32), (tag << 28) | block, step};
    orc_philox4x32_10(ctr, key, out);
}

/* Uniform integer in [0, m) from a 32-bit word: floor(r * m / 2^32). */
static inline uint32_t pick(uint32_t r, uint32_t m) { return (uint32_t)(((uint64_t)r * m) >> 32); }

/* ------------------------------------------------------------------------ */
/* Deterministic natural logarithm used by the shift update.  The paper uses */
/* ln (Eq. shift-update, Sec. 3.1); to make the trajectory reproducible      */
/* across machines this oracle and the GPU library each implement the same  */
/* textbook method: x = (1+f) 2^e with 1+f in [sqrt(1/2), sqrt(2)),          */
/* s = f/(2+f), ln(1+f) = 2 atanh(s) = f - (f^2/2 - s (f^2/2 + R)),          */
/* R = sum_{k>=1} 2 s^(2k)/(2k+1), and e ln 2 split into a high part with    */
/* trailing zeros and a low part.                                            */
/* ------------------------------------------------------------------------ */

static double from_bits(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }
static uint64_t to_bits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }

double orc_det_log(double x)
{
    uint64_t b = to_bits(x);
    int e = (int)((b >> 52) & 0x7ff) - 1023;
    double m = from_bits((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > from_bits(0x3FF6A09E667F3BCDull)) { m = m * 0.5; e += 1; }
    double f = m - 1.0;
    double hfsq = (0.5 * f) * f;
    double s = f / (2.0 + f);
    double z = s * s;
    double R = 2.0 / 27.0;
    for (int k = 12; k >= 1; k--) R = R * z + 2.0 / (double)(2 * k + 1);
    R = R * z;
    double lm = f - (hfsq - s * (hfsq + R));
    double de = (double)e;
    return de * from_bits(0x3FE62E42FEE00000ull) + (de * from_bits(0x3DEA39EF35793C76ull) + lm);
}

/* ------------------------------------------------------------------------ */
/* Exact summation: the merge of contributions onto one address (Sec. 3.2,   */
/* "collected and summed together") is defined as the exactly rounded sum.   */
/* Shewchuk's non-overlapping partials with a final half-even correction.    */
/* ------------------------------------------------------------------------ */

double orc_fsum(const double *x, int64_t n)
{
    double part[256];
    int np = 0;
    for (int64_t i = 0; i < n; i++) {
        double v = x[i];
        int k = 0;
        for (int j = 0; j < np; j++) {
            double y = part[j];
            if (fabs(v) < fabs(y)) { double tmp = v; v = y; y = tmp; }
            double hi = v + y;
            double lo = y - (hi - v);
            if (lo != 0.0) part[k++] = lo;
            v = hi;
        }
        part[k] = v;
        np = k + 1;
        if (np >= 255) return NAN; /* cannot happen for finite doubles */
    }
    if (np == 0) return 0.0;
    int j = np - 1;
    double hi = part[j], lo = 0.0;
    while (j > 0) {
        double v = hi;
        double y = part[--j];
        hi = v + y;
        double yr = hi - v;
        lo = y - yr;
        if (lo != 0.0) break;
    }
    if (j > 0 && ((lo < 0.0 && part[j - 1] < 0.0) || (lo > 0.0 && part[j - 1] > 0.0))) {
        double y = lo * 2.0;
        double v = hi + y;
        double yr = v - hi;
        if (y == yr) hi = v;
    }
    return hi;
}

/* ------------------------------------------------------------------------ */
/* Hamiltonians (Sec. 2 Eq. bose-hubbard-hamiltonian; Sec. 6.2)              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;               /* number of off-diagonal entries m_i */
    int cap;
    uint64_t (*dest)[2];
    double *h;
    /* momentum space: pair structure used by the two-stage sampler */
    int npairs;
    int *pair_off;       /* first column entry of each pair, npairs+1 */
    int (*pair_pq)[2];   /* modes (p, q), p <= q, of each pair in column order */
} orc_col;

static void col_free(orc_col *c)
{
    free(c->dest); free(c->h); free(c->pair_off); free(c->pair_pq);
    memset(c, 0, sizeof *c);
}

static int col_push(orc_col *c, const int32_t *occ, int M, double h)
{
    if (c->n == c->cap) {
        int nc = c->cap ? 2 * c->cap : 64;
        void *d = realloc(c->dest, sizeof(uint64_t[2]) * (size_t)nc);
        if (!d) return ORC_ENOMEM;
        c->dest = d;
        void *hh = realloc(c->h, sizeof(double) * (size_t)nc);
        if (!hh) return ORC_ENOMEM;
        c->h = hh;
        c->cap = nc;
    }
    orc_encode(occ, M, c->dest[c->n]);
    c->h[c->n] = h;
    c->n++;
    return ORC_OK;
}

/* Real-space ring (Eq. bose-hubbard-hamiltonian): diagonal (u/2) sum n(n-1). */
static double real_diag(const orc_ham *H, const int32_t *occ)
{
    int64_t s = 0;
    for (int j = 0; j < H->M; j++) s += (int64_t)occ[j] * (occ[j] - 1);
    return (0.5 * H->u) * (double)s;
}

/* Neighbour of site s in direction dir on the periodic lattice.  Sites are
 * numbered s = x + lx y (x fastest).  Directions (reading): 0 = +x, 1 = -x,
 * 2 = +y, 3 = -y; the ring (1D, lx = M) has only the first two. */
static int lattice_neighbour(const orc_ham *H, int s, int dir)
{
    int lx = H->model == ORC_REAL2D ? H->lx : H->M;
    int ly = H->M / lx;
    int x = s % lx, y = s / lx;
    switch (dir) {
    case 0: x = (x + 1) % lx; break;
    case 1: x = (x - 1 + lx) % lx; break;
    case 2: y = (y + 1) % ly; break;
    default: y = (y - 1 + ly) % ly; break;
    }
    return x + lx * y;
}

/* Importance sampling with the Gutzwiller guiding function (Sec. 3.3, a
 * similarity transformation by a diagonal matrix; Sec. 7.2 uses it).
 * Reading: G = diag(exp(-g H_ii)) with H_ii the diagonal element (the
 * interaction energy), H~ = G H G^-1, so H~_ij = H_ij exp(-g (H_ii - H_jj))
 * for destination i and source j.  One boson hopping from a site holding n
 * to one holding nd changes H_ii by u (nd - n + 1); the factor is
 * exp(-(g u) k) with k = nd - n + 1 for the column (source -> destination)
 * and k = -(nd - n + 1) for the row of the source. */
static double gutzwiller_factor(const orc_ham *H, int k)
{
    if (H->g == 0.0) return 1.0;
    return exp(-((H->g * H->u) * (double)k));
}

/* Real-space column on the ring (Eq. bose-hubbard-hamiltonian) or on the
 * periodic square lattice.  Enumeration order (reading; the paper prints it
 * only for the uniform 12/12 ring state in Sec. 6.2): entry k = dir o + i
 * moves one particle from the i-th occupied site (ascending) to its
 * neighbour in direction dir (o = occupied sites; on the ring k < o hops to
 * the next site, k >= o to the previous one).  Value (-t sqrt(n_src (n_dst +
 * 1))) times the Gutzwiller factor, occupations before the hop.  With
 * row != 0 the values are those of the row of the source (the transposed
 * similarity factor), used by the projected energy.  When two directions
 * lead to the same site (a ring of 2 sites, a lattice 2 sites wide) the
 * entry appears twice. */
static int lattice_column(const orc_ham *H, const int32_t *occ, orc_col *c, int row)
{
    int M = H->M;
    int ndir = H->model == ORC_REAL2D ? 4 : 2;
    int list[ORC_MAXM], o = 0;
    for (int j = 0; j < M; j++) if (occ[j] > 0) list[o++] = j;
    int32_t tmp[ORC_MAXM];
    for (int dir = 0; dir < ndir; dir++) {
        for (int k = 0; k < o; k++) {
            int s = list[k];
            int d = lattice_neighbour(H, s, dir);
            int kd = occ[d] - occ[s] + 1;
            double h = ((-H->t) * sqrt((double)(occ[s] * (occ[d] + 1)))) * gutzwiller_factor(H, row ? -kd : kd);
            memcpy(tmp, occ, sizeof(int32_t) * (size_t)M);
            tmp[s] -= 1;
            tmp[d] += 1;
            int rc = col_push(c, tmp, M, h);
            if (rc) return rc;
        }
    }
    return ORC_OK;
}

/* Momentum-space 1D Bose-Hubbard (HubbardMom1D, used in Sec. 6.3).  The
 * paper gives no formula; reading (pinned by the worked example in Sec. 6.3):
 *   H = sum_k eps_k n_k + (u/2M) sum_{p+q = r+s mod M} a+_r a+_s a_q a_p,
 *   eps_k = -2t cos(2 pi k / M). */
static double mom_eps(const orc_ham *H, int j)
{
    return (-2.0 * H->t) * cos((2.0 * 3.14159265358979323846 * (double)j) / (double)H->M);
}

static double mom_diag(const orc_ham *H, const int32_t *occ)
{
    int M = H->M, N = H->N;
    double kin = 0.0;
    int64_t sq = 0;
    for (int j = 0; j < M; j++) {
        if (occ[j] > 0) kin = kin + mom_eps(H, j) * (double)occ[j];
        sq += (int64_t)occ[j] * occ[j];
    }
    double coef = H->u / (2.0 * (double)M);
    double pot = coef * (double)(2 * (int64_t)N * N - N - sq);
    return kin + pot;
}

/* Number of unordered pairs {r <= s} with r + s = K (mod M). */
static int mom_pair_count(int K, int M) { return K / 2 + 1 + (K + M) / 2 - K; }

/* r for the idx-th pair {r, s} of total momentum K: r runs over
 * [0, K/2] and then over [K+1, (K+M)/2]. */
static int mom_r_of(int idx, int K) { return idx <= K / 2 ? idx : K + 1 + (idx - K / 2 - 1); }

/* Momentum-space column: removal pairs {p <= q} over occupied modes in
 * ascending order (p = q only if n_p >= 2); for each, destination pairs
 * {r <= s} with r + s = p + q (mod M) in the order of mom_r_of, skipping the
 * pair itself.  Value (u/2M) c_pq c_rs sqrt(n_p (n_q - d_pq))
 * sqrt((n_r + 1)(n_s + 1 + d_rs)), c = 2 for a pair of distinct modes. */
static int mom_column(const orc_ham *H, const int32_t *occ, orc_col *c)
{
    int M = H->M;
    int list[ORC_MAXM], o = 0;
    for (int j = 0; j < M; j++) if (occ[j] > 0) list[o++] = j;
    double coef = H->u / (2.0 * (double)M);
    int32_t tmp[ORC_MAXM];
    int npairs = 0;
    int *off = malloc(sizeof(int) * (size_t)(o * (o + 1) / 2 + 2));
    int (*pq)[2] = malloc(sizeof(int[2]) * (size_t)(o * (o + 1) / 2 + 2));
    if (!off || !pq) { free(off); free(pq); return ORC_ENOMEM; }
    c->pair_off = off;
    c->pair_pq = pq;
    for (int a = 0; a < o; a++) {
        for (int b = a; b < o; b++) {
            int p = list[a], q = list[b];
            if (p == q && occ[p] < 2) continue;
            pq[npairs][0] = p;
            pq[npairs][1] = q;
            off[npairs++] = c->n;
            int K = (p + q) % M;
            int cnt = mom_pair_count(K, M);
            int cpq = p == q ? 1 : 2;
            int A = occ[p] * (occ[q] - (p == q ? 1 : 0));
            for (int idx = 0; idx < cnt; idx++) {
                int r = mom_r_of(idx, K);
                int s = (K - r + M) % M;
                if (r == p) continue; /* the removal pair itself */
                int crs = r == s ? 1 : 2;
                int B = (occ[r] + 1) * (occ[s] + 1 + (r == s ? 1 : 0));
                double h = (coef * (double)(cpq * crs)) * (sqrt((double)A) * sqrt((double)B));
                memcpy(tmp, occ, sizeof(int32_t) * (size_t)M);
                tmp[p] -= 1; tmp[q] -= 1; tmp[r] += 1; tmp[s] += 1;
                int rc = col_push(c, tmp, M, h);
                if (rc) return rc;
            }
        }
    }
    off[npairs] = c->n;
    c->npairs = npairs;
    return ORC_OK;
}

static double ham_diag(const orc_ham *H, const int32_t *occ)
{
    return H->model == ORC_MOM1D ? mom_diag(H, occ) : real_diag(H, occ);
}

static int ham_column(const orc_ham *H, const int32_t *occ, orc_col *c)
{
    memset(c, 0, sizeof *c);
    return H->model == ORC_MOM1D ? mom_column(H, occ, c) : lattice_column(H, occ, c, 0);
}

/* The off-diagonal entries of row `occ` (same destinations as its column;
 * they differ only under importance sampling). */
static int ham_row(const orc_ham *H, const int32_t *occ, orc_col *c)
{
    memset(c, 0, sizeof *c);
    return H->model == ORC_MOM1D ? mom_column(H, occ, c) : lattice_column(H, occ, c, 1);
}

int orc_validate(const orc_ham *H)
{
    if (H->M < 2 || H->M > ORC_MAXM || H->N < 1 || H->N + H->M - 1 > 127) return ORC_EINVAL;
    if (H->model != ORC_REAL1D && H->model != ORC_MOM1D && H->model != ORC_REAL2D) return ORC_EINVAL;
    if (H->model == ORC_MOM1D && (H->M < 3 || H->g != 0.0)) return ORC_EINVAL;
    if (H->model == ORC_REAL2D && (H->lx < 2 || H->M % H->lx != 0 || H->M / H->lx < 2)) return ORC_EINVAL;
    if (!isfinite(H->g)) return ORC_EINVAL;
    return ORC_OK;
}

/* Exported column: diagonal element plus the off-diagonal entries in the
 * canonical order (Sec. 6.2, operator_column / offdiagonals). */
int orc_column(const orc_ham *H, const uint64_t *a, uint64_t *dest, double *h, int cap,
               double *diag)
{
    if (orc_validate(H)) return ORC_EINVAL;
    int32_t occ[ORC_MAXM];
    orc_decode(a, H->M, H->N, occ);
    *diag = ham_diag(H, occ);
    orc_col c;
    int rc = ham_column(H, occ, &c);
    if (rc) { col_free(&c); return rc; }
    int n = c.n;
    if (n > cap) { col_free(&c); return ORC_ECAP; }
    for (int k = 0; k < n; k++) {
        dest[2 * k] = c.dest[k][0];
        dest[2 * k + 1] = c.dest[k][1];
        h[k] = c.h[k];
    }
    col_free(&c);
    return n;
}

/* Exported row: the off-diagonal entries H_{a,dest} of the row of address a,
 * with the destinations of its column in the same order (they differ from
 * the column's values only under importance sampling). */
int orc_row(const orc_ham *H, const uint64_t *a, uint64_t *dest, double *h, int cap)
{
    if (orc_validate(H)) return ORC_EINVAL;
    int32_t occ[ORC_MAXM];
    orc_decode(a, H->M, H->N, occ);
    orc_col c;
    int rc = ham_row(H, occ, &c);
    if (rc) { col_free(&c); return rc; }
    int n = c.n;
    if (n > cap) { col_free(&c); return ORC_ECAP; }
    for (int k = 0; k < n; k++) {
        dest[2 * k] = c.dest[k][0];
        dest[2 * k + 1] = c.dest[k][1];
        h[k] = c.h[k];
    }
    col_free(&c);
    return n;
}

/* One stochastic pick from a column (Sec. 3.2, matrix compression; Sec. 6.2,
 * random_offdiagonal).  Real space: uniform over the m entries.  Momentum
 * space (reading): a removal pair uniform over the P pairs, then a
 * destination uniform over that pair's R(K) destinations; generation
 * probability 1/(P R).  Returns the column entry and sets *qnum = m or P R,
 * the inverse generation probability. */
/* The uniform pair index of the sampler (Sec. 6.3) names a pair in the
 * sampling order, which need not be the column order: any fixed one-to-one
 * order gives every pair probability 1/P.  Sampling order: first the pairs
 * (p, p) of the modes with n_p >= 2, p ascending; then the pairs of two
 * distinct occupied modes, the i-th and j-th occupied mode (i < j, counted
 * from 0 in ascending mode order) at index j(j-1)/2 + i.  Returns the
 * position of the pair in the column order. */
static int sampled_pair(const orc_col *c, const int32_t *occ, int M, int pi)
{
    int list[ORC_MAXM], o = 0, p = -1, q = -1;
    for (int j = 0; j < M; j++) if (occ[j] > 0) list[o++] = j;
    for (int j = 0; j < M && p < 0; j++) {
        if (occ[j] >= 2) {
            if (pi == 0) p = q = j;
            pi--;
        }
    }
    for (int jj = 1; jj < o && p < 0; jj++) {
        for (int ii = 0; ii < jj && p < 0; ii++) {
            if (pi == 0) { p = list[ii]; q = list[jj]; }
            pi--;
        }
    }
    for (int k = 0; k < c->npairs; k++)
        if (c->pair_pq[k][0] == p && c->pair_pq[k][1] == q) return k;
    return -1; /* not reached for 0 <= pi < P */
}

/* Exported for tests: modes (p, q) of the pair with sampling index pi of the
 * momentum-space parent a. */
int orc_sampled_pair(const orc_ham *H, const uint64_t *a, int pi, int *p, int *q)
{
    if (orc_validate(H) || H->model != ORC_MOM1D) return ORC_EINVAL;
    int32_t occ[ORC_MAXM];
    orc_decode(a, H->M, H->N, occ);
    orc_col c;
    int rc = ham_column(H, occ, &c);
    if (rc) { col_free(&c); return rc; }
    if (pi < 0 || pi >= c.npairs) { col_free(&c); return ORC_EINVAL; }
    int k = sampled_pair(&c, occ, H->M, pi);
    *p = c.pair_pq[k][0];
    *q = c.pair_pq[k][1];
    col_free(&c);
    return ORC_OK;
}

static int column_pick(const orc_ham *H, const orc_col *c, const int32_t *occ, uint32_t r0, uint32_t r1,
                       int64_t *qnum)
{
    if (H->model == ORC_MOM1D) {
        int P = c->npairs;
        int pi = sampled_pair(c, occ, H->M, (int)pick(r0, (uint32_t)P));
        int R = c->pair_off[pi + 1] - c->pair_off[pi];
        int di = (int)pick(r1, (uint32_t)R);
        *qnum = (int64_t)P * R;
        return c->pair_off[pi] + di;
    }
    *qnum = c->n;
    return (int)pick(r0, (uint32_t)c->n);
}

/* ------------------------------------------------------------------------ */
/* One FCIQMC step (Sec. 3.2, Eqs. column-compression, vec-compression and   */
/* the late-compression form of Sec. 7.1; shift update Eq. shift-update;     */
/* projected energy Eq. ProjectedEnergy of Sec. 4.2).                        */
/* ------------------------------------------------------------------------ */

/* kind: 0 diagonal survivor, 1 spawn from an initiator (or any spawn when
 * the initiator rule is off), 2 spawn from a non-initiator */
typedef struct {
    uint64_t a[2];
    double v;
    int32_t kind;
} orc_rec;

static int rec_cmp(const void *x, const void *y)
{
    const orc_rec *p = x, *q = y;
    if (p->a[1] != q->a[1]) return p->a[1] < q->a[1] ? -1 : 1;
    if (p->a[0] != q->a[0]) return p->a[0] < q->a[0] ? -1 : 1;
    return 0;
}

static int addr_cmp(const uint64_t *a, const uint64_t *b)
{
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    return 0;
}

/* Binary search in a table sorted by address; returns the value or 0. */
static double lookup(const uint64_t *addr, const double *val, int64_t n, const uint64_t *key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int c = addr_cmp(addr + 2 * mid, key);
        if (c == 0) return val[mid];
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return 0.0;
}

/* Projected-energy numerator y H c and denominator y c for a reference
 * vector with a single nonzero entry y at address ref (Sec. 4.2).
 * hproj = sum over the row of ref of y (H_rj c_j) plus y (H_rr c_ref),
 * summed exactly.  The row has the destinations of the column of ref; its
 * values equal the column's unless importance sampling makes H~ asymmetric. */
static int proj_energy(const orc_params *P, const uint64_t *addr, const double *val, int64_t n,
                       const uint64_t *ref, double y, double *hproj, double *vproj)
{
    int32_t occ[ORC_MAXM];
    orc_decode(ref, P->h.M, P->h.N, occ);
    orc_col c;
    int rc = ham_row(&P->h, occ, &c);
    if (rc) { col_free(&c); return rc; }
    double *terms = malloc(sizeof(double) * (size_t)(c.n + 1));
    if (!terms) { col_free(&c); return ORC_ENOMEM; }
    double cr = lookup(addr, val, n, ref);
    terms[0] = y * (ham_diag(&P->h, occ) * cr);
    for (int k = 0; k < c.n; k++) terms[k + 1] = y * (c.h[k] * lookup(addr, val, n, c.dest[k]));
    *hproj = orc_fsum(terms, c.n + 1);
    *vproj = y * cr;
    free(terms);
    col_free(&c);
    return ORC_OK;
}

/* Shift update, Eq. shift-update (Sec. 3.1):
 *   S' = S - (zeta/dtau) ln(N1/N0) - (xi/dtau) ln(N1/Nt). */
double orc_shift_update(double S, double N1, double N0, double Nt, double zeta, double xi,
                        double dtau)
{
    double a = zeta / dtau, b = xi / dtau;
    return (S - a * orc_det_log(N1 / N0)) - b * orc_det_log(N1 / Nt);
}

/* Exact-branch criterion (Sec. 7.1, semistochastic threshold; reading):
 * the column is spawned exactly when |c| >= t_rel m, which makes a smaller
 * t_rel give more exact steps and t_rel = infinity none.  A column with no
 * off-diagonal entry is always "exact" (nothing to spawn). */
static int is_exact(double absc, double t_rel, int64_t m) { return m == 0 || absc >= t_rel * (double)m; }

/* The compression rule of Eq. vec-compression for one value w with
 * threshold theta and uniform u in [0, 1): |w| >= theta is kept, otherwise
 * sign(w) theta when u theta < |w|, else 0. */
static double compress1(double w, double theta, double u)
{
    double aw = fabs(w);
    if (aw >= theta) return w;
    if (aw > 0.0 && u * theta < aw) return w < 0.0 ? -theta : theta;
    return 0.0;
}

/* Uniform of the early compression (Sec. 7.1, Eq. early-comp) of one
 * contribution of the parent at address a in step `step`: the diagonal
 * survivor uses tag 2, block 0; spawn attempt k uses tag 4 + (k >> 28),
 * block k mod 2^28. */
static double early_u(uint64_t seed, const uint64_t *a, int64_t step, int diag, int64_t k)
{
    uint32_t r[4];
    if (diag) orc_draw(seed, a, (uint32_t)step, 2, 0, r);
    else orc_draw(seed, a, (uint32_t)step, (uint32_t)(4 + (k >> 28)), (uint32_t)(k & 0x0fffffff), r);
    return (double)r[0] * 0x1p-32;
}

/*
 * orc_step: c^(n) -> c^(n+1) for the step with index `step` (= n+1, the row
 * index of the resulting statistics).  The input table need not be sorted;
 * the output table is sorted by address (word 1, then word 0).
 *
 *  1. every entry i (address a_i, value c_i) contributes its diagonal
 *     survivor c_i (1 + dtau (S - H_ii)) to a_i (Eqs. propagator and
 *     column-compression, j = i);
 *  2. if |c_i| >= t_rel m_i all m_i off-diagonal entries spawn exactly with
 *     value (-(dtau H_ji)) c_i; otherwise n_i = ceil|c_i| picks with
 *     replacement, each ((-(dtau H_ji)) c_i) q with q = qnum / n_i;
 *  3. contributions are summed per address (exactly rounded), exact zeros
 *     dropped (annihilation, Sec. 3.2);
 *  4. vector compression Pi with threshold theta: |w| >= theta kept,
 *     otherwise sign(w) theta if u theta < |w|, else dropped, with
 *     u = r / 2^32 from the tag-1 draw of the address (Eq. vec-compression,
 *     applied after the sum: late compression, Sec. 7.1);
 *  5. statistics and the shift update.
 *
 * With P->early set (early compression, Eq. early-comp of Sec. 7.1, read as
 * compressing each spawn individually), the rule of step 4 is applied
 * instead to every contribution before the sum: to the diagonal survivor
 * with the tag-2 draw of its address and to spawn attempt k with the draw
 * of early_u; contributions compressed to 0 are dropped (they are not
 * spawn events), and the sums are kept as they are.
 *
 * With P->initiator set (the initiator approximation of Cleland, Booth and
 * Alavi, which the paper names in Sec. 1 and in the sign-problem paragraph
 * of Sec. 3.2 without stating it; reading): entry i is an initiator when
 * |c_i| > n_a.  Steps 1 and 2 are unchanged, and every spawn event is still
 * generated, dumped and counted in `spawns`.  In step 3 a spawn of a
 * non-initiator parent counts only when its destination is occupied in
 * c^(n), i.e. is an address of the input table; otherwise it is discarded.
 * Survivors and spawns of initiators always count.  Every input address
 * takes part in the merge (its survivor is recorded even when it is 0), so
 * the merged dump lists the input addresses and the destinations that
 * received a counted spawn.  n_a = 0 makes every nonzero entry an initiator
 * and gives the plain step.
 */
int orc_step(const orc_params *P, const uint64_t *addr, const double *val, int64_t n,
             double shift, int64_t step, const uint64_t *ref, double yref,
             uint64_t *out_addr, double *out_val, int64_t out_cap, int64_t *out_n,
             orc_stats *st, orc_event *ev, int64_t ev_cap, int64_t *ev_n,
             uint64_t *mg_addr, double *mg_val, int64_t mg_cap, int64_t *mg_n)
{
    const orc_ham *H = &P->h;
    if (orc_validate(H)) return ORC_EINVAL;
    if (P->initiator && !(P->n_a >= 0.0)) return ORC_EINVAL;
    int M = H->M, N = H->N;
    int rc = ORC_OK;
    /* pass 1: count records */
    int64_t nrec = n, nexact = 0, ninexact = 0;
    double *absv = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!absv) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++) absv[i] = fabs(val[i]);
    double norm0 = orc_fsum(absv, n);
    free(absv);
    int32_t occ[ORC_MAXM];
    for (int64_t i = 0; i < n; i++) {
        orc_decode(addr + 2 * i, M, N, occ);
        orc_col c;
        rc = ham_column(H, occ, &c);
        if (rc) { col_free(&c); return rc; }
        double ac = fabs(val[i]);
        if (is_exact(ac, P->t_rel, c.n)) nrec += c.n;
        /* the block index of a draw has 28 bits (tag << 28 | block): at most
         * 2^28 blocks of 4 words, i.e. 2^29 momentum-space attempts (two
         * words each) or 2^30 attempts of the other models (one word) */
        else if (ceil(ac) > (H->model == ORC_MOM1D ? 536870912.0 : 1073741824.0)) {
            col_free(&c);
            return ORC_EINVAL;
        }
        else nrec += (int64_t)ceil(ac);
        col_free(&c);
    }
    orc_rec *rec = malloc(sizeof(orc_rec) * (size_t)(nrec > 0 ? nrec : 1));
    if (!rec) return ORC_ENOMEM;
    int64_t nr = 0, nev = 0, nspawn = 0;
    /* pass 2: generate */
    for (int64_t i = 0; i < n; i++) {
        const uint64_t *a = addr + 2 * i;
        double ci = val[i];
        orc_decode(a, M, N, occ);
        double hii = ham_diag(H, occ);
        double g = 1.0 + P->dtau * (shift - hii);
        double sv = ci * g;
        if (P->early) sv = compress1(sv, P->theta, early_u(P->seed, a, step, 1, 0));
        if (sv != 0.0 || P->initiator) {
            rec[nr].a[0] = a[0]; rec[nr].a[1] = a[1]; rec[nr].v = sv; rec[nr].kind = 0; nr++;
        }
        const int32_t skind = (P->initiator && !(fabs(ci) > P->n_a)) ? 2 : 1;
        orc_col c;
        rc = ham_column(H, occ, &c);
        if (rc) { col_free(&c); free(rec); return rc; }
        double ac = fabs(ci);
        if (is_exact(ac, P->t_rel, c.n)) {
            nexact++;
            for (int k = 0; k < c.n; k++) {
                double v = (-(P->dtau * c.h[k])) * ci;
                if (P->early) v = compress1(v, P->theta, early_u(P->seed, a, step, 0, k));
                if (v == 0.0) continue;
                rec[nr].a[0] = c.dest[k][0]; rec[nr].a[1] = c.dest[k][1]; rec[nr].v = v;
                rec[nr].kind = skind; nr++;
                if (ev && nev < ev_cap) {
                    ev[nev].parent = i; ev[nev].attempt = k;
                    ev[nev].dest[0] = c.dest[k][0]; ev[nev].dest[1] = c.dest[k][1];
                    ev[nev].value = v;
                }
                nev++;
                nspawn++;
            }
        } else {
            ninexact++;
            int64_t ni = (int64_t)ceil(ac);
            uint32_t r[4] = {0, 0, 0, 0};
            for (int64_t k = 0; k < ni; k++) {
                uint32_t r0, r1 = 0;
                if (H->model == ORC_MOM1D) {
                    if ((k & 1) == 0) orc_draw(P->seed, a, (uint32_t)step, 0, (uint32_t)(k >> 1), r);
                    r0 = r[2 * (k & 1)];
                    r1 = r[2 * (k & 1) + 1];
                } else {
                    if ((k & 3) == 0) orc_draw(P->seed, a, (uint32_t)step, 0, (uint32_t)(k >> 2), r);
                    r0 = r[k & 3];
                }
                int64_t qnum;
                int e = column_pick(H, &c, occ, r0, r1, &qnum);
                double q = (double)qnum / (double)ni;
                double v = ((-(P->dtau * c.h[e])) * ci) * q;
                if (P->early) v = compress1(v, P->theta, early_u(P->seed, a, step, 0, k));
                if (v == 0.0) continue;
                rec[nr].a[0] = c.dest[e][0]; rec[nr].a[1] = c.dest[e][1]; rec[nr].v = v;
                rec[nr].kind = skind; nr++;
                if (ev && nev < ev_cap) {
                    ev[nev].parent = i; ev[nev].attempt = k;
                    ev[nev].dest[0] = c.dest[e][0]; ev[nev].dest[1] = c.dest[e][1];
                    ev[nev].value = v;
                }
                nev++;
                nspawn++;
            }
        }
        col_free(&c);
    }
    if (ev_n) *ev_n = nev;
    /* annihilation: group by address, exactly rounded sum per group */
    qsort(rec, (size_t)nr, sizeof(orc_rec), rec_cmp);
    double *buf = malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1));
    double *nabs = malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1));
    if (!buf || !nabs) { free(rec); free(buf); free(nabs); return ORC_ENOMEM; }
    int64_t nout = 0, nmg = 0;
    for (int64_t s = 0; s < nr;) {
        int64_t e = s;
        int occupied = 0, counted = 0;
        while (e < nr && rec[e].a[0] == rec[s].a[0] && rec[e].a[1] == rec[s].a[1]) {
            if (rec[e].kind == 0) occupied = 1;
            e++;
        }
        /* the group's counted contributions (all of them without the
         * initiator rule) */
        for (int64_t k = s; k < e; k++)
            if (rec[k].kind != 2 || occupied) buf[counted++] = rec[k].v;
        if (counted == 0) { s = e; continue; }
        double w = orc_fsum(buf, counted);
        if (mg_addr && nmg < mg_cap) {
            mg_addr[2 * nmg] = rec[s].a[0]; mg_addr[2 * nmg + 1] = rec[s].a[1]; mg_val[nmg] = w;
        }
        nmg++;
        double cnew = w;
        if (!P->early && w != 0.0 && fabs(w) < P->theta) {
            uint32_t r[4];
            orc_draw(P->seed, rec[s].a, (uint32_t)step, 1, 0, r);
            cnew = compress1(w, P->theta, (double)r[0] * 0x1p-32);
        }
        if (cnew != 0.0) {
            if (nout >= out_cap) { rc = ORC_ECAP; break; }
            out_addr[2 * nout] = rec[s].a[0]; out_addr[2 * nout + 1] = rec[s].a[1];
            out_val[nout] = cnew;
            nabs[nout] = fabs(cnew);
            nout++;
        }
        s = e;
    }
    if (mg_n) *mg_n = nmg;
    free(rec);
    free(buf);
    if (rc) { free(nabs); return rc; }
    *out_n = nout;
    double norm1 = orc_fsum(nabs, nout);
    free(nabs);
    st->step = step;
    st->len = nout;
    st->exact_steps = nexact;
    st->inexact_steps = ninexact;
    st->spawns = nspawn;
    st->norm = norm1;
    st->shift = norm1 > 0.0 ? orc_shift_update(shift, norm1, norm0, P->target, P->zeta, P->xi, P->dtau)
                            : shift;
    rc = proj_energy(P, out_addr, out_val, nout, ref, yref, &st->hproj, &st->vproj);
    return rc;
}

/* Repeated steps from a given state; stats[k] describes step first_step+k.
 * The final table is returned in out_addr/out_val. */
int orc_run(const orc_params *P, const uint64_t *addr, const double *val, int64_t n, double shift,
            int64_t first_step, int64_t nsteps, const uint64_t *ref, double yref,
            int64_t cap, uint64_t *out_addr, double *out_val, int64_t *out_n, orc_stats *stats)
{
    uint64_t *a0 = malloc(sizeof(uint64_t) * 2 * (size_t)cap);
    double *v0 = malloc(sizeof(double) * (size_t)cap);
    if (!a0 || !v0) { free(a0); free(v0); return ORC_ENOMEM; }
    if (n > cap) { free(a0); free(v0); return ORC_ECAP; }
    memcpy(a0, addr, sizeof(uint64_t) * 2 * (size_t)n);
    memcpy(v0, val, sizeof(double) * (size_t)n);
    int64_t cur = n;
    double S = shift;
    int rc = ORC_OK;
    for (int64_t k = 0; k < nsteps; k++) {
        int64_t nn = 0;
        rc = orc_step(P, a0, v0, cur, S, first_step + k, ref, yref, out_addr, out_val, cap, &nn,
                      &stats[k], NULL, 0, NULL, NULL, NULL, 0, NULL);
        if (rc) break;
        S = stats[k].shift;
        memcpy(a0, out_addr, sizeof(uint64_t) * 2 * (size_t)nn);
        memcpy(v0, out_val, sizeof(double) * (size_t)nn);
        cur = nn;
    }
    if (!rc) {
        memcpy(out_addr, a0, sizeof(uint64_t) * 2 * (size_t)cur);
        memcpy(out_val, v0, sizeof(double) * (size_t)cur);
        *out_n = cur;
    }
    free(a0);
    free(v0);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Exact diagonalisation support (Sec. 5)                                    */
/* ------------------------------------------------------------------------ */

/* Sparse matrix by walking the ranked basis: row i of column j holds H_ij.
 * indptr has D+1 entries; when indices is NULL only the count is returned
 * in indptr[D] (nnz).  Duplicate entries (M = 2 ring) are kept separately. */
int orc_build_csr(const orc_ham *H, int64_t *indptr, int64_t *indices, double *data)
{
    if (orc_validate(H)) return ORC_EINVAL;
    uint64_t D = orc_dimension(H->M, H->N);
    if (D == UINT64_MAX) return ORC_EINVAL;
    int32_t occ[ORC_MAXM];
    uint64_t a[2];
    int64_t nnz = 0;
    for (uint64_t j = 0; j < D; j++) {
        orc_unrank(j, H->M, H->N, a);
        orc_decode(a, H->M, H->N, occ);
        orc_col c;
        int rc = ham_column(H, occ, &c);
        if (rc) { col_free(&c); return rc; }
        indptr[j] = nnz;
        if (indices) {
            indices[nnz] = (int64_t)j;
            data[nnz] = ham_diag(H, occ);
            for (int k = 0; k < c.n; k++) {
                indices[nnz + 1 + k] = (int64_t)orc_rank(c.dest[k], H->M, H->N);
                data[nnz + 1 + k] = c.h[k];
            }
        }
        nnz += 1 + c.n;
        col_free(&c);
    }
    indptr[D] = nnz;
    return ORC_OK;
}

/* Matrix-free H x over the ranked basis (Sec. 5): y = H x, column by column. */
static int matvec(const orc_ham *H, uint64_t D, const double *x, double *y)
{
    int32_t occ[ORC_MAXM];
    uint64_t a[2];
    for (uint64_t i = 0; i < D; i++) y[i] = 0.0;
    for (uint64_t j = 0; j < D; j++) {
        if (x[j] == 0.0) continue;
        orc_unrank(j, H->M, H->N, a);
        orc_decode(a, H->M, H->N, occ);
        y[j] += ham_diag(H, occ) * x[j];
        orc_col c;
        int rc = ham_column(H, occ, &c);
        if (rc) { col_free(&c); return rc; }
        for (int k = 0; k < c.n; k++) y[orc_rank(c.dest[k], H->M, H->N)] += c.h[k] * x[j];
        col_free(&c);
    }
    return ORC_OK;
}

/* Plain Lanczos (three-term recurrence, no re-orthogonalisation) started
 * from the basis vector of `start`; returns alpha[0..k) and beta[0..k-1).
 * The lowest Ritz value converges to the ground-state energy of the
 * symmetry sector of `start`. */
int orc_lanczos(const orc_ham *H, const uint64_t *start, int kmax, double *alpha, double *beta,
                int *kout)
{
    if (orc_validate(H)) return ORC_EINVAL;
    uint64_t D = orc_dimension(H->M, H->N);
    if (D == UINT64_MAX || D > ((uint64_t)1 << 31)) return ORC_EINVAL;
    double *v = calloc(D, sizeof(double)), *vp = calloc(D, sizeof(double)),
           *w = calloc(D, sizeof(double));
    if (!v || !vp || !w) { free(v); free(vp); free(w); return ORC_ENOMEM; }
    v[orc_rank(start, H->M, H->N)] = 1.0;
    double b = 0.0;
    int k = 0;
    for (; k < kmax; k++) {
        int rc = matvec(H, D, v, w);
        if (rc) { free(v); free(vp); free(w); return rc; }
        double a = 0.0;
        for (uint64_t i = 0; i < D; i++) a += w[i] * v[i];
        alpha[k] = a;
        double nn = 0.0;
        for (uint64_t i = 0; i < D; i++) {
            w[i] = w[i] - a * v[i] - b * vp[i];
            nn += w[i] * w[i];
        }
        b = sqrt(nn);
        if (k + 1 < kmax) beta[k] = b;
        if (b < 1e-12) { k++; break; }
        for (uint64_t i = 0; i < D; i++) {
            vp[i] = v[i];
            v[i] = w[i] / b;
        }
    }
    *kout = k;
    free(v); free(vp); free(w);
    return ORC_OK;
}
