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

// (u/2) sum_j n_j (n_j - 1): a run of n ones holds n - k positions whose k
// higher neighbours are all ones, so sum_j n_j (n_j - 1) / 2 is the sum over
// k >= 1 of popc(a & a>>1 & ... & a>>k); the loop runs as many times as the
// longest run.
template <class T> __device__ __forceinline__ double real_diag_runs(const ModelConst &C, T a)
{
    i64 s = 0;
    T x = a & shr(a, 1);
    while (!is_zero(x)) {
        s += popc(x);
        x = x & shr(x, 1);
    }
    return (0.5 * C.u) * (double)(2 * s);
}

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

// A momentum-space parent decoded into registers.  Occupied modes are the
// runs of ones of the address: `st` marks the first bit of every run, the
// mode of a run starting at bit s is the number of zeros below s, and the
// run of mode j starts after the j-th zero (`z` = zeros inside the N+M-1
// bits).  Everything is bit arithmetic on one or two words.
template <class T> struct MomP {
    T a, st, z;
    int o, o_odd, dbl;
};

template <class T> __device__ __forceinline__ int mom_mode_at(const MomP<T> &P, int s)
{
    return s - popc(P.a & mask_below<T>(s));
}
template <class T> __device__ __forceinline__ int mom_start(const MomP<T> &P, int j)
{
    return j == 0 ? 0 : select(P.z, j - 1) + 1;
}

template <class T> __device__ __forceinline__ MomP<T> mom_parent(const ModelConst &C, T a)
{
    MomP<T> P;
    P.a = a;
    P.st = run_starts(a);
    P.z = ~a & mask_below<T>(C.nb);
    P.o = popc(P.st);
    P.dbl = popc(P.st & shr(a, 1));  // runs of length >= 2
    int oo = 0;
    T x = P.st;
    while (!is_zero(x)) {
        int s = ctz(x);
        x = x & ~one_at<T>(s);
        oo += mom_mode_at(P, s) & 1;
    }
    P.o_odd = oo;
    return P;
}

// Diagonal element in one pass over the M modes in order (a trip count the
// same for every lane; eps[j] is a uniform, scalar load).  Empty modes add
// eps_j * 0 = +-0 to the kinetic sum, which leaves it unchanged (the sum
// starts at +0 and never becomes -0), so the result equals the sum over the
// occupied modes in ascending order bit for bit.
template <class T> __device__ __forceinline__ double mom_diag_modes(const ModelConst &C, T a)
{
    T zz = (~a & mask_below<T>(C.nb)) | one_at<T>(C.nb);  // separators, then the end
    double kin = 0.0;
    int sq = 0, prev = -1;
    for (int j = 0; j < C.M; j++) {
        const int zp = ctz(zz);
        zz = zz & ~one_at<T>(zp);
        const int n = zp - prev - 1;
        prev = zp;
        kin = kin + C.eps[j] * (double)n;
        sq += n * n;
    }
    const i64 N = C.N;
    const double pot = C.coef * (double)(2 * N * N - N - (i64)sq);
    return kin + pot;
}

template <class T> __device__ __forceinline__ double mom_diag(const ModelConst &C, const MomP<T> &P)
{
    double kin = 0.0;
    i64 sq = 0;
    T x = P.st;
    while (!is_zero(x)) {  // occupied modes in ascending order
        int s = ctz(x);
        x = x & ~one_at<T>(s);
        int n = runlen(P.a, s);
        kin = kin + C.eps[mom_mode_at(P, s)] * (double)n;
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
__device__ __forceinline__ int mod_add(int x, int y, int M)
{
    int r = x + y;
    return r >= M ? r - M : r;
}
template <class T> __device__ __forceinline__ int mom_npairs(const MomP<T> &P) { return P.o * (P.o - 1) / 2 + P.dbl; }
// column size: sum over pairs of R(K); for even M, pairs of odd K are the
// distinct pairs of one odd and one even mode
template <class T> __device__ __forceinline__ i64 mom_m(const MomP<T> &P, int M)
{
    i64 np = mom_npairs(P);
    if (M & 1) return np * ((M - 1) / 2);
    return np * (M / 2) - (i64)P.o_odd * (P.o - P.o_odd);
}

// bit i = parity of the set bits of x in [0, i]
__device__ __forceinline__ u32 prefix_xor(u32 x)
{
    x ^= x << 1; x ^= x << 2; x ^= x << 4; x ^= x << 8; x ^= x << 16;
    return x;
}
__device__ __forceinline__ u64 prefix_xor(u64 x)
{
    x ^= x << 1; x ^= x << 2; x ^= x << 4; x ^= x << 8; x ^= x << 16; x ^= x << 32;
    return x;
}
__device__ __forceinline__ U128 prefix_xor(U128 x)
{
    const u64 lo = prefix_xor(x.lo);
    const u64 hi = prefix_xor(x.hi) ^ ((__popcll(x.lo) & 1) ? ~0ull : 0ull);
    return U128{lo, hi};
}

// Column size m of a momentum-space parent without a loop: the parity of
// the mode that starts at bit s is the parity of the separators below s.
template <class T> __device__ __forceinline__ i64 mom_col_size(const ModelConst &C, T a)
{
    const int M = C.M;
    const T st = run_starts(a);
    const int o = popc(st);
    const i64 np = (i64)o * (o - 1) / 2 + popc(st & shr(a, 1));
    if (M & 1) return np * ((M - 1) / 2);
    const T par = shl(prefix_xor(~a & mask_below<T>(C.nb)), 1);  // parity of the mode at each bit
    const int o_odd = popc(st & par);
    return np * (M / 2) - (i64)o_odd * (o - o_odd);
}

template <class T> __device__ __forceinline__ T del_bit(T a, int x)
{
    return (a & mask_below<T>(x)) | shl(shr(a, x + 1), x);
}
template <class T> __device__ __forceinline__ T ins_one(T a, int x)
{
    return (a & mask_below<T>(x)) | one_at<T>(x) | shl(shr(a, x), x + 1);
}

// move {p,q} -> {r,s} (p <= q modes starting at bits sp <= sq; r <= s): value
// and destination
template <class T>
__device__ __forceinline__ T mom_move(const ModelConst &C, const MomP<T> &P, int p, int q, int sp, int sq, int di,
                                      double &h)
{
    const int M = C.M;
    int K = mod_add(p, q, M);
    int half = K / 2;
    int idxp = p <= half ? p : half + 1 + (p - K - 1);
    int idx = di < idxp ? di : di + 1;
    int r = idx <= half ? idx : K + 1 + (idx - half - 1);
    int s = K - r;
    if (s < 0) s += M;
    const int sr = mom_start(P, r), ss = mom_start(P, s);
    int np = runlen(P.a, sp), nq = runlen(P.a, sq), nr = runlen(P.a, sr), ns = runlen(P.a, ss);
    int A = np * (nq - (p == q ? 1 : 0));
    int B = (nr + 1) * (ns + 1 + (r == s ? 1 : 0));
    int cc = (p == q ? 1 : 2) * (r == s ? 1 : 2);
    h = (C.coef * (double)cc) * (C.sq[A] * C.sq[B]);
    // four single-bit edits applied from the highest position down, so each
    // edit leaves the positions of the lower ones valid
    int rem0 = sq, rem1 = sp, ins0 = ss, ins1 = sr;  // each pair descending
    T d = P.a;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        bool take_ins = rem0 < 0 || (ins0 >= 0 && ins0 > rem0);
        if (take_ins) { d = ins_one(d, ins0); ins0 = ins1; ins1 = -1; }
        else { d = del_bit(d, rem0); rem0 = rem1; rem1 = -1; }
    }
    return d;
}

// One stochastic spawn of a momentum-space parent (Sec. 6.3, two-stage
// sampler): w0 picks the removal pair uniformly over the P pairs through the
// sampling order (first the pairs (p, p) of doubly occupied modes, p
// ascending; then the pairs of the i-th and j-th occupied mode, i < j, at
// index j(j-1)/2 + i), w1 picks one of the pair's R(K) destinations in column
// order.  Returns the destination, its matrix element h and qnum = P R, the
// inverse generation probability.  No data-dependent branches, so the lanes
// of a wave stay converged.
template <class T>
__device__ __forceinline__ T mom_stochastic(const ModelConst &C, T a, u32 w0, u32 w1, double &h, i64 &qnum,
                                            const unsigned char *lut)
{
    const int M = C.M;
    const T st = run_starts(a);
    const T z = ~a & mask_below<T>(C.nb);
    const int o = popc(st);
    const T dpos = st & shr(a, 1);  // run starts of modes with n >= 2
    const int D = popc(dpos);
    const int P = o * (o - 1) / 2 + D;
    const int pi = (int)pick(w0, (u32)P);
    const bool diag = pi < D;
    const int t = diag ? 0 : pi - D;
    // j = largest integer with j (j - 1) / 2 <= t; the float root is exact to
    // within one and corrected
    int j = (int)((1.0f + __builtin_amdgcn_sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
    j -= (j * (j - 1) / 2 > t) ? 1 : 0;
    j += ((j + 1) * j / 2 <= t) ? 1 : 0;
    const int i = t - j * (j - 1) / 2;
    const T x = diag ? dpos : st;
    const int sp = select_lut(x, diag ? pi : i, lut);
    const int sq = select_lut(x, diag ? pi : j, lut);
    const int p = sp - popc(a & mask_below<T>(sp));
    const int q = sq - popc(a & mask_below<T>(sq));
    const int K = mod_add(p, q, M);
    const int R = mom_R(K, M);
    const int di = (int)pick(w1, (u32)R);
    const int half = K / 2;
    const int idxp = p <= half ? p : half + 1 + (p - K - 1);
    const int idx = di < idxp ? di : di + 1;
    const int r = idx <= half ? idx : K + 1 + (idx - half - 1);
    int s = K - r;
    if (s < 0) s += M;
    const int sr = r == 0 ? 0 : select_lut(z, r - 1, lut) + 1;
    const int ss = s == 0 ? 0 : select_lut(z, s - 1, lut) + 1;
    const int np = runlen(a, sp), nq = runlen(a, sq), nr = runlen(a, sr), ns = runlen(a, ss);
    const int A = np * (nq - (p == q ? 1 : 0));
    const int B = (nr + 1) * (ns + 1 + (r == s ? 1 : 0));
    const int cc = (p == q ? 1 : 2) * (r == s ? 1 : 2);
    h = (C.coef * (double)cc) * (C.sq[A] * C.sq[B]);
    qnum = (i64)P * R;
    // remove one boson at the start of runs q and p (higher first), then add
    // one at the start of runs r and s, whose starts moved down by one for
    // each removal from a lower mode (higher insertion first)
    T d = del_bit(a, sq);
    d = del_bit(d, sp);
    const int r2 = sr - (p < r ? 1 : 0) - (q < r ? 1 : 0);
    const int s2 = ss - (p < s ? 1 : 0) - (q < s ? 1 : 0);
    d = ins_one(d, max(r2, s2));
    d = ins_one(d, min(r2, s2));
    return d;
}

// pair index -> (p, q) in the canonical pair order: occupied p ascending,
// then (p, p) when n_p >= 2, then (p, q) for occupied q > p
template <class T>
__device__ __forceinline__ void mom_pair(const MomP<T> &P, int pi, int &p, int &q, int &sp, int &sq)
{
    T x = P.st;
    int rank = 0;
    while (!is_zero(x)) {
        const int s = ctz(x);
        x = x & ~one_at<T>(s);
        const int d = is_zero(P.a & one_at<T>(s + 1)) ? 0 : 1;
        const int cnt = P.o - rank - 1 + d;
        if (pi < cnt) {
            sp = s;
            p = mom_mode_at(P, s);
            if (d && pi == 0) { sq = s; q = p; return; }
            sq = select(P.st, rank + 1 + (pi - d));
            q = mom_mode_at(P, sq);
            return;
        }
        pi -= cnt;
        rank++;
    }
    p = q = sp = sq = 0;  // not reached for valid pi
}

// iterator over the column entries of a momentum-space parent in canonical
// order; rows are skipped with closed-form row sizes
template <class T> struct PairIt {
    T xa, xb;               // remaining run starts for the row index / partner
    int sa, pa, sb, pb;     // current pair: bit starts and modes
    int di, Rk;
};

template <class T>
__device__ __forceinline__ bool mom_it_row(const MomP<T> &P, int M, PairIt<T> &it)
{
    // position the iterator on the first pair of row it.sa (already set)
    if (!is_zero(P.a & one_at<T>(it.sa + 1))) {  // (p, p)
        it.sb = it.sa;
        it.pb = it.pa;
        it.Rk = mom_R(mod_add(it.pa, it.pa, M), M);
        it.xb = it.xa;
        return true;
    }
    if (is_zero(it.xa)) return false;
    it.sb = ctz(it.xa);
    it.xb = it.xa & ~one_at<T>(it.sb);
    it.pb = mom_mode_at(P, it.sb);
    it.Rk = mom_R(mod_add(it.pa, it.pb, M), M);
    return true;
}

template <class T>
__device__ __forceinline__ void mom_it_init(const MomP<T> &P, int M, i64 e, PairIt<T> &it)
{
    T x = P.st;
    int rank = 0, odd_seen = 0;
    while (!is_zero(x)) {
        const int s = ctz(x);
        x = x & ~one_at<T>(s);
        const int pm = mom_mode_at(P, s);
        const int d = is_zero(P.a & one_at<T>(s + 1)) ? 0 : 1;
        const i64 pairs = P.o - rank - 1 + d;
        i64 row;
        if (M & 1) {
            row = pairs * ((M - 1) / 2);
        } else {
            const int odd_after = P.o_odd - odd_seen - (pm & 1);
            const int even_after = (P.o - rank - 1) - odd_after;
            row = pairs * (M / 2) - (i64)((pm & 1) ? even_after : odd_after);
        }
        if (e < row) {
            it.sa = s;
            it.pa = pm;
            it.xa = x;
            mom_it_row(P, M, it);
            while (e >= it.Rk) {
                e -= it.Rk;
                it.sb = ctz(it.xb);
                it.xb = it.xb & ~one_at<T>(it.sb);
                it.pb = mom_mode_at(P, it.sb);
                it.Rk = mom_R(mod_add(it.pa, it.pb, M), M);
            }
            it.di = (int)e;
            return;
        }
        e -= row;
        odd_seen += pm & 1;
        rank++;
    }
    it.sa = it.sb = it.pa = it.pb = 0;
    it.di = 0;
    it.Rk = 1;
}

template <class T> __device__ __forceinline__ void mom_it_next(const MomP<T> &P, int M, PairIt<T> &it)
{
    if (++it.di < it.Rk) return;
    it.di = 0;
    if (!is_zero(it.xb)) {
        it.sb = ctz(it.xb);
        it.xb = it.xb & ~one_at<T>(it.sb);
        it.pb = mom_mode_at(P, it.sb);
        it.Rk = mom_R(mod_add(it.pa, it.pb, M), M);
        return;
    }
    while (!is_zero(it.xa)) {  // next row
        it.sa = ctz(it.xa);
        it.xa = it.xa & ~one_at<T>(it.sa);
        it.pa = mom_mode_at(P, it.sa);
        if (mom_it_row(P, M, it)) return;
    }
    it.Rk = 1;  // past the end (not used)
}

// A momentum-space parent with the start bit of every mode packed into
// registers: byte j&3 of word j>>2 is the first bit of the run of mode j, and
// `end` = N+M is where a virtual mode M would start, so a destination's
// occupation and position cost a few instructions.  MAXM (16 or 32) is the
// compile-time bound on M.  The words are separate members, not an array, so
// that no dynamically indexed private memory is created.
template <class T, int MAXM> struct MomD {
    MomP<T> P;
    u32 w0, w1, w2, w3, w4, w5, w6, w7;
    int end;
};

template <class T, int MAXM> __device__ __forceinline__ void mom_set_byte(MomD<T, MAXM> &D, int j, u32 v)
{
    const u32 x = v << ((j & 3) * 8);
    switch (j >> 2) {
    case 0: D.w0 |= x; break;
    case 1: D.w1 |= x; break;
    case 2: D.w2 |= x; break;
    case 3: D.w3 |= x; break;
    case 4: D.w4 |= x; break;
    case 5: D.w5 |= x; break;
    case 6: D.w6 |= x; break;
    default: D.w7 |= x; break;
    }
}

template <class T, int MAXM> __device__ __forceinline__ MomD<T, MAXM> mom_decode_packed(const ModelConst &C, T a)
{
    static_assert(MAXM == 16 || MAXM == 32, "MAXM");
    MomD<T, MAXM> D;
    D.P.a = a;
    D.P.st = run_starts(a);
    D.P.z = ~a & mask_below<T>(C.nb);
    D.P.o = popc(D.P.st);
    D.P.dbl = popc(D.P.st & shr(a, 1));
    D.w0 = D.w1 = D.w2 = D.w3 = D.w4 = D.w5 = D.w6 = D.w7 = 0u;
    D.end = C.nb + 1;
    T zz = D.P.z;  // separators: mode j starts one bit after the j-th zero
    int prev = 0, oo = 0;
#pragma unroll
    for (int j = 1; j < MAXM; j++) {
        if (j < C.M) {
            const int z0 = ctz(zz);
            zz = zz & ~one_at<T>(z0);
            const int sj = z0 + 1;
            oo += ((j - 1) & 1) & (sj - prev - 1 > 0 ? 1 : 0);
            mom_set_byte(D, j, (u32)sj);
            prev = sj;
        }
    }
    // the last mode M-1 ends at the virtual start N+M
    oo += ((C.M - 1) & 1) & (D.end - prev - 1 > 0 ? 1 : 0);
    D.P.o_odd = oo;
    return D;
}

// first bit of mode j (0 <= j <= M; j = M gives N+M)
template <class T, int MAXM> __device__ __forceinline__ int mom_pos(const ModelConst &C, const MomD<T, MAXM> &D, int j)
{
    // the word is picked with masks, not selects between members: a select
    // between two members is turned into one load at a computed address, which
    // sends the whole struct to private memory
    const u32 k = (u32)j >> 2;
    u32 x = (D.w0 & (0u - (u32)(k == 0u))) | (D.w1 & (0u - (u32)(k == 1u))) | (D.w2 & (0u - (u32)(k == 2u))) |
            (D.w3 & (0u - (u32)(k == 3u)));
    if (MAXM > 16)
        x |= (D.w4 & (0u - (u32)(k == 4u))) | (D.w5 & (0u - (u32)(k == 5u))) | (D.w6 & (0u - (u32)(k == 6u))) |
             (D.w7 & (0u - (u32)(k == 7u)));
    const int v = (int)((x >> ((j & 3) * 8)) & 0xffu);
    return j == C.M ? D.end : v;
}

// move {p,q} -> {r,s} using the packed start positions
template <class T, int MAXM>
__device__ __forceinline__ T mom_move_d(const ModelConst &C, const MomD<T, MAXM> &D, int p, int q, int sp, int sq,
                                        int di, double &h)
{
    const int M = C.M;
    int K = mod_add(p, q, M);
    int half = K / 2;
    int idxp = p <= half ? p : half + 1 + (p - K - 1);
    int idx = di < idxp ? di : di + 1;
    int r = idx <= half ? idx : K + 1 + (idx - half - 1);
    int s = K - r;
    if (s < 0) s += M;
    const int sr = mom_pos(C, D, r), ss = mom_pos(C, D, s);
    const int np = mom_pos(C, D, p + 1) - sp - 1, nq = mom_pos(C, D, q + 1) - sq - 1;
    const int nr = mom_pos(C, D, r + 1) - sr - 1, ns = mom_pos(C, D, s + 1) - ss - 1;
    int A = np * (nq - (p == q ? 1 : 0));
    int B = (nr + 1) * (ns + 1 + (r == s ? 1 : 0));
    int cc = (p == q ? 1 : 2) * (r == s ? 1 : 2);
    h = (C.coef * (double)cc) * (C.sq[A] * C.sq[B]);
    int rem0 = sq, rem1 = sp, ins0 = ss, ins1 = sr;
    T d = D.P.a;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        bool take_ins = rem0 < 0 || (ins0 >= 0 && ins0 > rem0);
        if (take_ins) { d = ins_one(d, ins0); ins0 = ins1; ins1 = -1; }
        else { d = del_bit(d, rem0); rem0 = rem1; rem1 = -1; }
    }
    return d;
}

}  // namespace fq
