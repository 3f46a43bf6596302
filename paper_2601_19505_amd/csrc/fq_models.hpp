// fq_models.hpp -- the two Bose-Hubbard Hamiltonians as device functions.
//
// Column enumeration order, matrix elements and floating-point operation
// order follow the conventions stated for the CPU reference so that spawn
// events agree bit for bit:
//
//  Real space (Sec. 2, Eq. bose-hubbard-hamiltonian; periodic ring of M
//  sites): diagonal (0.5 u) * sum n(n-1); column entry k < o moves one boson
//  from the k-th occupied site to the next site on the ring, entry k >= o
//  from the (k-o)-th occupied site to the previous one; value
//  (-t) * sqrt(n_src (n_dst + 1)).  m = 2 o.
//
//  Momentum space (HubbardMom1D of Sec. 6.3): eps_k = -2t cos(2 pi k / M),
//  V = (u/2M) sum_{p+q = r+s mod M} a+_r a+_s a_q a_p.  Removal pairs
//  {p <= q} over occupied modes in ascending order (p = q when n_p >= 2);
//  destinations {r <= s} with r + s = p + q (mod M), r running over
//  [0, K/2] then [K+1, (K+M)/2], skipping {p, q}; value
//  (coef * c_pq c_rs) * (sqrt(n_p (n_q - d_pq)) * sqrt((n_r + 1)(n_s + 1 + d_rs))).
//  Stochastic picks: a removal pair uniform over the P pairs, then a
//  destination uniform over that pair's R(K); inverse probability P R.
#pragma once
#include "fq_device.hpp"

namespace fq {

constexpr int MOM_MAXM = 32;     // largest M of the momentum model on the device
constexpr int MOM_ROW = 100;     // bytes of per-thread LDS scratch (occ, start, list)

struct ModelConst {
    int M, N, nb;
    double t, u, coef;          // coef = u / (2 M) (momentum)
    const double *sq;           // sq[k] = sqrt(k), correctly rounded, from the host
    const double *eps;          // eps[k] (momentum), from the host
};

// ---------------------------------------------------------------- real space

// number of consecutive ones starting at bit s
template <class T> __device__ __forceinline__ int runlen(T a, int s) { return ctz(~shr(a, s)); }

template <class T> __device__ __forceinline__ T run_starts(T a) { return a & ~shl(a, 1); }

template <class T> __device__ __forceinline__ double real_diag(const ModelConst &C, T a)
{
    T st = run_starts(a);
    i64 s = 0;
    while (!is_zero(st)) {
        int p = ctz(st);
        int n = runlen(a, p);
        s += (i64)n * (n - 1);
        st = st & ~one_at<T>(p);
    }
    return (0.5 * C.u) * (double)s;
}

// column entry k (0 <= k < 2 o) of the real-space ring; o = popc(run_starts)
template <class T>
__device__ __forceinline__ T real_entry(const ModelConst &C, T a, T st, int o, int k, double &h)
{
    const int M = C.M, nb = C.nb;
    bool left = k >= o;
    int s = select(st, left ? k - o : k);
    int n = runlen(a, s);
    int jm = s - popc(a & mask_below<T>(s));
    int nd;
    T d;
    if (!left) {
        if (jm < M - 1) {
            int sep = s + n;
            nd = runlen(a, sep + 1);
            d = a ^ shl(T(one_at<T>(0)) | one_at<T>(1), sep - 1);
        } else {
            nd = runlen(a, 0);
            d = shl(a & ~one_at<T>(nb - 1), 1) | one_at<T>(0);
        }
    } else {
        if (jm > 0) {
            int sep = s - 1;
            T z = ~a & mask_below<T>(sep);
            nd = is_zero(z) ? sep : (sep - 1 - msb(z));
            d = a ^ shl(T(one_at<T>(0)) | one_at<T>(1), sep);
        } else {
            T z = ~a & mask_below<T>(nb);
            nd = (nb - 1) - msb(z);
            d = shr(a, 1) | one_at<T>(nb - 1);
        }
    }
    h = (-C.t) * C.sq[n * (nd + 1)];
    return d;
}

// ---------------------------------------------------------------- momentum

struct MomRow {
    unsigned char *occ, *start, *list;
    int o, o_odd, dbl;
};

__device__ __forceinline__ MomRow mom_row(unsigned char *base)
{
    MomRow r;
    r.occ = base;
    r.start = base + MOM_MAXM;
    r.list = base + 2 * MOM_MAXM;
    r.o = r.o_odd = r.dbl = 0;
    return r;
}

template <class T> __device__ __forceinline__ void mom_decode(const ModelConst &C, T a, MomRow &R)
{
    int pos = 0, o = 0, oo = 0, dbl = 0;
    for (int j = 0; j < C.M; j++) {
        int n = runlen(a, pos);
        R.occ[j] = (unsigned char)n;
        R.start[j] = (unsigned char)pos;
        if (n) {
            R.list[o++] = (unsigned char)j;
            oo += j & 1;
            dbl += n >= 2;
        }
        pos += n + 1;
    }
    R.o = o;
    R.o_odd = oo;
    R.dbl = dbl;
}

__device__ __forceinline__ double mom_diag(const ModelConst &C, const MomRow &R)
{
    double kin = 0.0;
    i64 sq = 0;
    for (int j = 0; j < C.M; j++) {
        int n = R.occ[j];
        if (n > 0) kin = kin + C.eps[j] * (double)n;
        sq += (i64)n * n;
    }
    i64 N = C.N;
    double pot = C.coef * (double)(2 * N * N - N - sq);
    return kin + pot;
}

// destinations per removal pair of total momentum K
__device__ __forceinline__ int mom_R(int K, int M)
{
    return (M & 1) ? (M - 1) / 2 : ((K & 1) ? M / 2 - 1 : M / 2);
}
__device__ __forceinline__ int mom_npairs(const MomRow &R) { return R.o * (R.o - 1) / 2 + R.dbl; }
// column size: sum over pairs of R(K); for even M, pairs of odd K are the
// distinct pairs of one odd and one even mode
__device__ __forceinline__ i64 mom_m(const MomRow &R, int M)
{
    i64 P = mom_npairs(R);
    if (M & 1) return P * ((M - 1) / 2);
    return P * (M / 2) - (i64)R.o_odd * (R.o - R.o_odd);
}

template <class T> __device__ __forceinline__ T del_bit(T a, int x)
{
    return (a & mask_below<T>(x)) | shl(shr(a, x + 1), x);
}
template <class T> __device__ __forceinline__ T ins_one(T a, int x)
{
    return (a & mask_below<T>(x)) | one_at<T>(x) | shl(shr(a, x), x + 1);
}

// move {p,q} -> {r,s} (p <= q, r <= s, disjoint): value and destination
template <class T>
__device__ __forceinline__ T mom_move(const ModelConst &C, T a, const MomRow &R, int p, int q, int di,
                                      double &h)
{
    const int M = C.M;
    int K = (p + q) % M;
    int half = K / 2;
    int idxp = p <= half ? p : half + 1 + (p - K - 1);
    int idx = di < idxp ? di : di + 1;
    int r = idx <= half ? idx : K + 1 + (idx - half - 1);
    int s = (K - r + M) % M;
    int np = R.occ[p], nq = R.occ[q], nr = R.occ[r], ns = R.occ[s];
    int A = np * (nq - (p == q ? 1 : 0));
    int B = (nr + 1) * (ns + 1 + (r == s ? 1 : 0));
    int cc = (p == q ? 1 : 2) * (r == s ? 1 : 2);
    h = (C.coef * (double)cc) * (C.sq[A] * C.sq[B]);
    // four single-bit edits applied from the highest position down, so each
    // edit leaves the positions of the lower ones valid
    int pp = R.start[p], pq = R.start[q], pr = R.start[r], ps = R.start[s];
    // removals at pq >= pp, insertions at ps >= pr; merge descending
    int rem[2] = {pq, pp}, ins[2] = {ps, pr};
    int ir = 0, ii = 0;
    T d = a;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        bool take_ins = ir >= 2 || (ii < 2 && ins[ii] > rem[ir]);
        if (take_ins) { d = ins_one(d, ins[ii]); ii++; }
        else { d = del_bit(d, rem[ir]); ir++; }
    }
    return d;
}

// pair index -> (p, q) in the canonical pair order
__device__ __forceinline__ void mom_pair(const MomRow &R, int pi, int &p, int &q)
{
    const int o = R.o;
    for (int a = 0; a < o; a++) {
        int pa = R.list[a];
        int d = R.occ[pa] >= 2 ? 1 : 0;
        int cnt = o - a - 1 + d;
        if (pi < cnt) {
            p = pa;
            if (d) q = pi == 0 ? pa : R.list[a + pi];
            else q = R.list[a + 1 + pi];
            return;
        }
        pi -= cnt;
    }
    p = q = R.list[0];  // not reached for valid pi
}

// column entry e -> (p, q, di) by walking pairs in canonical order
__device__ __forceinline__ void mom_entry(const MomRow &R, int M, i64 e, int &p, int &q, int &di)
{
    const int o = R.o;
    for (int a = 0; a < o; a++) {
        int pa = R.list[a];
        if (R.occ[pa] >= 2) {
            int Rk = mom_R((2 * pa) % M, M);
            if (e < Rk) { p = q = pa; di = (int)e; return; }
            e -= Rk;
        }
        for (int b = a + 1; b < o; b++) {
            int qb = R.list[b];
            int Rk = mom_R((pa + qb) % M, M);
            if (e < Rk) { p = pa; q = qb; di = (int)e; return; }
            e -= Rk;
        }
    }
    p = q = R.list[0];
    di = 0;
}

}  // namespace fq
