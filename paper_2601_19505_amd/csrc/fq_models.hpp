// fq_models.hpp -- the Bose-Hubbard Hamiltonians as device functions.
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
//  Stochastic picks: a removal pair uniform over the P pairs (through the
//  sampling order of mom_draw), then a destination uniform over that pair's
//  R(K); inverse probability P R.
//
//  A momentum-space address is handled as bit strings: `st` marks the first
//  bit of every run of ones (an occupied mode), the mode of a run starting at
//  bit s is the number of zeros below s, and mode j starts after the j-th
//  zero of `z` (the zeros inside the N+M-1 bits).
#pragma once
#include "fq_device.hpp"

namespace fq {

constexpr int MOM_MAXM = 32;     // largest M of the momentum model on the device

struct ModelConst {
    int M, N, nb;
    double t, u, coef;          // coef = u / (2 M) (momentum)
    const double *sq;           // sq[k] = sqrt(k), correctly rounded, from the host
    const double *eps;          // eps[k] (momentum), from the host
    int ndir;                   // lattice: hop directions (2 ring, 4 square lattice)
    const unsigned char *nbr;   // lattice: nbr[dir M + site] = neighbouring site
    const double *gz;           // lattice: gz[N + k] = exp(-(g u) k), from the host
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
    h = (-C.t) * gmem(C.sq)[n * (nd + 1)];
    return d;
}

// ---------------------------------------------------------------- lattice

// remove bit x (higher bits move down) / insert a one at bit x (higher bits
// move up)
template <class T> __device__ __forceinline__ T del_bit(T a, int x)
{
    return (a & mask_below<T>(x)) | shl(shr(a, x + 1), x);
}
template <class T> __device__ __forceinline__ T ins_one(T a, int x)
{
    return (a & mask_below<T>(x)) | one_at<T>(x) | shl(shr(a, x), x + 1);
}


// Ring or periodic square lattice, with Gutzwiller importance sampling
// (Sec. 3.3, Sec. 7.2).  Column entry k = dir o + i moves one boson from the
// i-th occupied site to its neighbour in direction dir (+x, -x, +y, -y).
// Returns the destination, h0 = (-t) sqrt(n_src (n_dst + 1)) and kd = n_dst
// - n_src + 1; the matrix element is h0 gz[N + kd] in the column and
// h0 gz[N - kd] in the row of the source.  The destination is the parent
// with the first one of the source run removed and a one inserted at the
// start of the destination run (whose start moves down by one when it lies
// above the removed bit).
template <class T>
__device__ __forceinline__ T lat_entry(const ModelConst &C, T a, T st, int o, int k, double &h0, int &kd,
                                       const unsigned char *lut)
{
    const int dir = (k >= o ? 1 : 0) + (k >= 2 * o ? 1 : 0) + (k >= 3 * o ? 1 : 0);
    const int s = select_lut(st, k - dir * o, lut);
    const int n = runlen(a, s);
    const int j = s - popc(a & mask_below<T>(s));
    const int dj = gmem(C.nbr)[dir * C.M + j];
    const T z = ~a & mask_below<T>(C.nb);
    const int sd = dj == 0 ? 0 : select_lut(z, dj - 1, lut) + 1;
    const int nd = runlen(a, sd);
    kd = nd - n + 1;
    h0 = (-C.t) * gmem(C.sq)[n * (nd + 1)];
    return ins_one(del_bit(a, s), sd > s ? sd - 1 : sd);
}

// ---------------------------------------------------------------- momentum

// Diagonal element in one pass over the M modes in order (a trip count the
// same for every lane; eps[j] is a uniform, scalar load).  Empty modes add
// eps_j * 0 = +-0 to the kinetic sum, which leaves it unchanged (the sum
// starts at +0 and never becomes -0), so the result equals the sum over the
// occupied modes in ascending order bit for bit.
template <class T> __device__ __forceinline__ double mom_diag_modes(const ModelConst &C, T a)
{
    // eps is a host table no kernel writes, and mode j is the same for every
    // lane: read it in the constant address space (scalar loads)
    const __attribute__((address_space(4))) double *eps =
        (const __attribute__((address_space(4))) double *)(uintptr_t)C.eps;
    T zz = (~a & mask_below<T>(C.nb)) | one_at<T>(C.nb);  // separators, then the end
    double kin = 0.0;
    int sq = 0, prev = -1;
    for (int j = 0; j < C.M; j++) {
        const int zp = ctz(zz);
        zz = zz & ~one_at<T>(zp);
        const int n = zp - prev - 1;
        prev = zp;
        kin = kin + eps[j] * (double)n;
        sq += n * n;
    }
    const i64 N = C.N;
    const double pot = C.coef * (double)(2 * N * N - N - (i64)sq);
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


// The move {p,q} -> {r,s} of a momentum-space parent a for the removal pair
// starting at bits sp <= sq (modes p <= q, K = p + q mod M) and its di-th
// destination pair in column order (r runs over [0, K/2], then over
// [K+1, (K+M)/2], skipping r = p).  Returns the destination and the matrix
// element h (Sec. 6.3).
template <class T>
__device__ __forceinline__ T mom_move_to(const ModelConst &C, T a, T z, int sp, int sq, int p, int q, int K, int di,
                                         double &h, const unsigned char *lut)
{
    const int M = C.M;
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
    h = (C.coef * (double)cc) * (gmem(C.sq)[A] * gmem(C.sq)[B]);
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

// What every stochastic draw of one momentum-space parent shares: the run
// starts `st` (occupied modes), the separators `z`, the run starts `dpos`
// of modes with n >= 2, o = occupied modes, D = doubly occupied modes and
// P = C(o, 2) + D removal pairs.
template <class T> struct MomCtx {
    T a, st, z, dpos;
    int o, D, P;
};
template <class T> __device__ __forceinline__ MomCtx<T> mom_ctx(const ModelConst &C, T a)
{
    MomCtx<T> x;
    x.a = a;
    x.st = run_starts(a);
    x.z = ~a & mask_below<T>(C.nb);
    x.o = popc(x.st);
    x.dpos = x.st & shr(a, 1);
    x.D = popc(x.dpos);
    x.P = x.o * (x.o - 1) / 2 + x.D;
    return x;
}

// One stochastic spawn of a momentum-space parent (Sec. 6.3, two-stage
// sampler): w0 picks the removal pair uniformly over the P pairs through the
// sampling order (first the pairs (p, p) of doubly occupied modes, p
// ascending; then the pairs of the i-th and j-th occupied mode, i < j, at
// index j(j-1)/2 + i), w1 picks one of the pair's R(K) destinations in column
// order.  Returns the destination, its matrix element h and R; the inverse
// generation probability is P R.  No data-dependent branches, so the lanes
// of a wave stay converged.
template <class T>
__device__ __forceinline__ T mom_draw(const ModelConst &C, const MomCtx<T> &x, u32 w0, u32 w1, double &h, int &R,
                                      const unsigned char *lut)
{
    const int M = C.M;
    const T a = x.a;
    const int pi = (int)pick(w0, (u32)x.P);
    const bool diag = pi < x.D;
    const int t = diag ? 0 : pi - x.D;
    // j = largest integer with j (j - 1) / 2 <= t; the float root is exact to
    // within one and corrected
    int j = (int)((1.0f + __builtin_amdgcn_sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
    j -= (j * (j - 1) / 2 > t) ? 1 : 0;
    j += ((j + 1) * j / 2 <= t) ? 1 : 0;
    const int i = t - j * (j - 1) / 2;
    const T xs = diag ? x.dpos : x.st;
    const int sp = select_lut(xs, diag ? pi : i, lut);
    const int sq = select_lut(xs, diag ? pi : j, lut);
    const int p = sp - popc(a & mask_below<T>(sp));
    const int q = sq - popc(a & mask_below<T>(sq));
    const int K = mod_add(p, q, M);
    R = mom_R(K, M);
    return mom_move_to(C, a, x.z, sp, sq, p, q, K, (int)pick(w1, (u32)R), h, lut);
}

// ---- momentum space, addresses of at most 31 bits
//
// The same draw as mom_draw for a parent whose address fits 31 bits, with
// what every draw of the parent shares computed once: byte-prefix popcounts
// of the run starts, of the doubly occupied run starts and of the mode
// starts (so each select is a lookup), and a table `tri` of the pair (i, j),
// i < j, at sampling index j (j - 1) / 2 + i.  With 31 bits every shift
// count stays below 32.

// byte k of the result: set bits of w in bytes 0 .. k
__device__ __forceinline__ u32 byte_prefix(u32 w)
{
    u32 c = w - ((w >> 1) & 0x55555555u);
    c = (c & 0x33333333u) + ((c >> 2) & 0x33333333u);
    c = (c + (c >> 4)) & 0x0f0f0f0fu;
    return c * 0x01010101u;
}
// position of the j-th set bit of w (w has more than j), given
// pre = byte_prefix(w)
__device__ __forceinline__ int select_pre(u32 w, u32 pre, int j, const unsigned char *lut)
{
    u32 jj = (u32)(j + 1);
    jj |= jj << 8;
    jj |= jj << 16;
    const u32 ge = ((pre | 0x80808080u) - jj) & 0x80808080u;
    const u32 b8 = 8u * (u32)(4 - __popc(ge));          // 8 x (bytes whose prefix is <= j)
    const u32 before = __builtin_amdgcn_ubfe(pre << 8, b8, 8);  // set bits below that byte
    return (int)b8 + lut[__builtin_amdgcn_ubfe(w, b8, 8) * 8u + ((u32)j - before)];
}
// remove bit x / insert a one at bit x (x <= 31): the bits below x stay,
// the bits above move down / up by one
__device__ __forceinline__ u32 del_bit32(u32 a, int x)
{
    const u32 m = (1u << x) - 1u;
    return (a & m) | ((a >> 1) & ~m);
}
__device__ __forceinline__ u32 ins_one32(u32 a, int x)
{
    const u32 m = (1u << x) - 1u;
    return (a & m) | (((a << 1) | (1u << x)) & ~m);
}
// ones starting at bit s of a 31-bit word (s <= 31)
__device__ __forceinline__ int runlen31(u32 a, int s) { return __builtin_ctz(~(a >> s)); }

struct MomCtx32 {
    u32 a, st, dpos, ms;  // ms: bit j set at the start of mode j, shifted up by one
    u32 pst, pdpos, pms;  // byte_prefix of st, dpos, ms
    int D, P;
};
__device__ __forceinline__ MomCtx32 mom_ctx32(const ModelConst &C, u32 a)
{
    MomCtx32 x;
    x.a = a;
    x.st = a & ~(a << 1);
    x.dpos = x.st & (a >> 1);
    // a separator at bit p starts the next mode at p + 1, and mode 0 starts
    // at bit 0: with ms = (separators << 1) | 1, mode j starts at the j-th
    // set bit of ms
    x.ms = ((~a & ((1u << C.nb) - 1u)) << 1) | 1u;
    x.pst = byte_prefix(x.st);
    x.pdpos = byte_prefix(x.dpos);
    x.pms = byte_prefix(x.ms);
    const int o = (int)(x.pst >> 24);
    x.D = (int)(x.pdpos >> 24);
    x.P = o * (o - 1) / 2 + x.D;
    return x;
}
// tri[t] = i | j << 8 for the pair (i, j), i < j, of sampling index
// t = j (j - 1) / 2 + i; t < nt
constexpr int TRI_N = 512;  // pairs of up to 32 occupied modes
__device__ __forceinline__ void tri_fill(unsigned short *tri, int tid, int nthreads)
{
    for (int t = tid; t < TRI_N; t += nthreads) {
        // j = largest integer with j (j - 1) / 2 <= t: the float root is
        // exact to within one and corrected
        int j = (int)((1.0f + __builtin_amdgcn_sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
        j -= (j * (j - 1) / 2 > t) ? 1 : 0;
        j += ((j + 1) * j / 2 <= t) ? 1 : 0;
        tri[t] = (unsigned short)((t - j * (j - 1) / 2) | (j << 8));
    }
}
__device__ __forceinline__ u32 mom_draw31(const ModelConst &C, const MomCtx32 &x, u32 w0, u32 w1, double &h, int &R,
                                          const unsigned char *lut, const unsigned short *tri)
{
    const int M = C.M;
    const u32 a = x.a;
    const int pi = (int)pick(w0, (u32)x.P);
    const bool diag = pi < x.D;
    const u32 ij = tri[diag ? 0 : pi - x.D];
    const int i = diag ? pi : (int)(ij & 0xffu), j = diag ? pi : (int)(ij >> 8);
    const u32 xs = diag ? x.dpos : x.st, pxs = diag ? x.pdpos : x.pst;
    const int sp = select_pre(xs, pxs, i, lut);
    const int sq = select_pre(xs, pxs, j, lut);
    const int p = sp - __popc(a & ((1u << sp) - 1u));
    const int q = sq - __popc(a & ((1u << sq) - 1u));
    const int K = mod_add(p, q, M);
    R = mom_R(K, M);
    const int di = (int)pick(w1, (u32)R);
    // destination pair (r, s) of index di in column order (r over [0, K/2],
    // then over [K+1, (K+M)/2], skipping r = p)
    const int half = (int)((u32)K >> 1);
    const int idxp = p <= half ? p : half + 1 + (p - K - 1);
    const int idx = di < idxp ? di : di + 1;
    const int r = idx <= half ? idx : K + 1 + (idx - half - 1);
    int s = K - r;
    if (s < 0) s += M;
    const int sr = select_pre(x.ms, x.pms, r, lut);
    const int ss = select_pre(x.ms, x.pms, s, lut);
    const int np = runlen31(a, sp), nq = runlen31(a, sq), nr = runlen31(a, sr), ns = runlen31(a, ss);
    const int A = np * (nq - (p == q ? 1 : 0));
    const int B = (nr + 1) * (ns + 1 + (r == s ? 1 : 0));
    const int cc = (p == q ? 1 : 2) * (r == s ? 1 : 2);
    h = (C.coef * (double)cc) * (gmem(C.sq)[A] * gmem(C.sq)[B]);
    u32 d = del_bit32(a, sq);
    d = del_bit32(d, sp);
    const int r2 = sr - (p < r ? 1 : 0) - (q < r ? 1 : 0);
    const int s2 = ss - (p < s ? 1 : 0) - (q < s ? 1 : 0);
    d = ins_one32(d, max(r2, s2));
    d = ins_one32(d, min(r2, s2));
    return d;
}

// Entry e (0 <= e < m) of the column of a momentum-space parent in column
// order (occupied p ascending; (p, p) first when n_p >= 2, then (p, q) for
// occupied q > p; each pair's R(K) destinations in order), computed without
// walking the column: row sizes follow from popcounts, because R(K) is M/2
// or M/2 - 1 as p + q is even or odd (even M), and (M-1)/2 for odd M.
template <class T>
__device__ __forceinline__ T mom_column_entry(const ModelConst &C, T a, int e, double &h, const unsigned char *lut)
{
    const int M = C.M;
    const bool even = (M & 1) == 0;
    const int hR = even ? M / 2 : (M - 1) / 2;  // R of an even K; every K when M is odd
    const T st = run_starts(a);
    const T z = ~a & mask_below<T>(C.nb);
    const T par = shl(prefix_xor(z), 1);  // parity of the mode at each bit
    // row of the removal mode p: pairs (p, p) if n_p >= 2, then (p, q > p)
    T x = st;
    int sp = ctz(x), dp = 0, pp = 0;
    for (;;) {
        sp = ctz(x);
        x = x & ~one_at<T>(sp);                     // run starts after sp
        dp = is_zero(a & one_at<T>(sp + 1)) ? 0 : 1;  // n_p >= 2
        pp = is_zero(par & one_at<T>(sp)) ? 0 : 1;   // parity of p
        const int later = popc(x);
        const int odd_later = popc(x & par);
        const int mism = even ? (pp ? later - odd_later : odd_later) : 0;
        const int row = (dp + later) * hR - mism;
        if (e < row || is_zero(x)) break;
        e -= row;
    }
    int sq = sp;
    if (!(dp && e < hR)) {
        e -= dp * hR;
        T y = x;
        for (;;) {
            sq = ctz(y);
            y = y & ~one_at<T>(sq);
            const int pq = is_zero(par & one_at<T>(sq)) ? 0 : 1;
            const int R = hR - ((even && pq != pp) ? 1 : 0);
            if (e < R || is_zero(y)) break;
            e -= R;
        }
    }
    const int p = sp - popc(a & mask_below<T>(sp));
    const int q = sq - popc(a & mask_below<T>(sq));
    return mom_move_to(C, a, z, sp, sq, p, q, mod_add(p, q, M), e, h, lut);
}

}  // namespace fq
