// fq_overlap.hpp -- replica overlaps c_A . c_B (Sec. 4.3, Eq.
// RayleighQuotientReplica).
//
// R replicas of one Hamiltonian run in one batch with the same bucket count,
// so an address lies in the same bucket of every replica.  After every step
// one workgroup per (replica A, bucket b), A < R-1, loads bucket b of A's new
// table into an LDS hash (address -> amplitude) and streams bucket b of every
// replica B > A through it; each common address contributes the product of
// its two amplitudes, rounded to double.  The products are summed exactly in
// 192-bit fixed point (96 fractional bits), per bucket, then over buckets by
// one workgroup, and rounded once to the nearest double.  The sums are
// integer additions, so the result does not depend on the bucket count or on
// the order in which threads meet their products.
#pragma once
#include "fq_step.hpp"

namespace fq {

// ------------------------------------------------ 192-bit fixed point

constexpr int OV_FRAC = 96;

struct Fx3 {
    u64 w0, w1, w2;  // two's complement, w2 most significant
};

__device__ __forceinline__ Fx3 fx3_zero() { return Fx3{0, 0, 0}; }

__device__ __forceinline__ void fx3_add(Fx3 &a, const Fx3 &b)
{
    const u64 s0 = a.w0 + b.w0;
    const u64 c0 = s0 < a.w0 ? 1ull : 0ull;
    const u64 s1 = a.w1 + b.w1;
    u64 c1 = s1 < a.w1 ? 1ull : 0ull;
    const u64 s1c = s1 + c0;
    c1 += s1c < s1 ? 1ull : 0ull;
    a.w2 = a.w2 + b.w2 + c1;
    a.w1 = s1c;
    a.w0 = s0;
}

__device__ __forceinline__ void fx3_neg(Fx3 &a)
{
    a.w0 = ~a.w0;
    a.w1 = ~a.w1;
    a.w2 = ~a.w2;
    const Fx3 one{1, 0, 0};
    fx3_add(a, one);
}

// v * 2^96 as a 192-bit integer.  Exact when v is a multiple of 2^-96 (every
// double with |v| >= 2^-43 is); otherwise rounded half-even and *inexact set.
// |v| >= 2^95 or a non-finite v sets *ovf.
__device__ __forceinline__ Fx3 to_fx3(double v, int &inexact, int &ovf)
{
    const u64 b = dbits(v);
    int e = (int)((b >> 52) & 0x7ff);
    u64 m = b & 0x000FFFFFFFFFFFFFull;
    if (e == 0x7ff) { ovf = 1; return fx3_zero(); }
    if (e == 0) { e = 1; } else { m |= 1ull << 52; }
    const int sh = e - 1075 + OV_FRAC;  // v = m 2^(e - 1075)
    Fx3 x = fx3_zero();
    if (sh > 138) { ovf = 1; return x; }
    if (sh >= 128) {
        x.w2 = m << (sh - 128);
    } else if (sh >= 64) {
        const int s = sh - 64;
        x.w1 = m << s;
        x.w2 = s ? m >> (64 - s) : 0ull;
    } else if (sh >= 0) {
        x.w0 = m << sh;
        x.w1 = sh ? m >> (64 - sh) : 0ull;
    } else {
        const int s = -sh;
        u64 q = 0;
        if (s <= 53) {
            q = m >> s;
            const u64 rem = m & ((1ull << s) - 1), half = 1ull << (s - 1);
            if (rem) inexact = 1;
            if (rem > half || (rem == half && (q & 1ull))) q++;
        } else if (m) {
            inexact = 1;
        }
        x.w0 = q;
    }
    if (b >> 63) fx3_neg(x);
    return x;
}

__device__ __forceinline__ u64 fx3_word(const Fx3 &x, int i)
{
    return i == 0 ? x.w0 : i == 1 ? x.w1 : i == 2 ? x.w2 : 0ull;
}
__device__ __forceinline__ int fx3_bit(const Fx3 &x, int i) { return (int)((fx3_word(x, i >> 6) >> (i & 63)) & 1ull); }
// any bit below position i (i >= 0)
__device__ __forceinline__ bool fx3_any_below(const Fx3 &x, int i)
{
    const int w = i >> 6, r = i & 63;
    bool any = r ? (fx3_word(x, w) & ((1ull << r) - 1)) != 0 : false;
    if (w > 0) any = any || x.w0 != 0;
    if (w > 1) any = any || x.w1 != 0;
    return any;
}
// bits [s, s + 53) of x (0 < s < 192)
__device__ __forceinline__ u64 fx3_bits53(const Fx3 &x, int s)
{
    const int w = s >> 6, r = s & 63;
    const u64 lo = fx3_word(x, w), hi = fx3_word(x, w + 1);
    const u64 v = r ? (lo >> r) | (hi << (64 - r)) : lo;
    return v & ((1ull << 53) - 1);
}

// nearest double (half-even) of x 2^-96
__device__ __forceinline__ double from_fx3(Fx3 x)
{
    const bool neg = (i64)x.w2 < 0;
    if (neg) fx3_neg(x);
    if ((x.w0 | x.w1 | x.w2) == 0) return 0.0;
    const int p = x.w2 ? 128 + msb(x.w2) : x.w1 ? 64 + msb(x.w1) : msb(x.w0);
    double r;
    if (p <= 52) {
        r = (double)x.w0 * bitsd((u64)(1023 - OV_FRAC) << 52);
    } else {
        int s = p - 52;
        u64 mant = fx3_bits53(x, s);
        const int rb = fx3_bit(x, s - 1);
        const bool sticky = s >= 2 ? fx3_any_below(x, s - 1) : false;
        if (rb && (sticky || (mant & 1ull))) mant++;
        if (mant == (1ull << 53)) { mant >>= 1; s++; }
        const u64 ex = (u64)(s - OV_FRAC + 52 + 1023);
        r = bitsd((ex << 52) | (mant & 0x000FFFFFFFFFFFFFull));
    }
    return neg ? -r : r;
}

__device__ __forceinline__ Fx3 fx3_shfl_down(const Fx3 &x, int o)
{
    return Fx3{(u64)__shfl_down((unsigned long long)x.w0, o, 64), (u64)__shfl_down((unsigned long long)x.w1, o, 64),
               (u64)__shfl_down((unsigned long long)x.w2, o, 64)};
}

// ------------------------------------------------ replica join

struct Overlap {
    const Inst *const *rep;  // replicas in caller order
    int R, P, B;
    Fx3 *part;               // [B][P] per-bucket partial sums
    double *ring;            // [ring_cap][P] rows of the current chunk
    i64 ring_cap;
    int *flags;              // [0] LDS hash full, [1] inexact product, [2] out of range
};

// index of pair (A, B), A < B, in the order A = 0.., then B
__device__ __host__ __forceinline__ int pair_index(int A, int B, int R) { return A * (2 * R - A - 1) / 2 + (B - A - 1); }

template <int W> __device__ __forceinline__ void tab_entry(const Inst &I, int par, i64 e, u64 &a0, u64 &a1, double &v)
{
    a0 = I.tab_a[par][0][e];
    a1 = W == 2 ? I.tab_a[par][1][e] : 0ull;
    v = I.tab_v[par][e];
}

template <int BS> __device__ __forceinline__ Fx3 block_sum_fx3(Fx3 x, Fx3 *tmp)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        const Fx3 y = fx3_shfl_down(x, o);
        fx3_add(x, y);
    }
    if (lane == 0) tmp[wid] = x;
    __syncthreads();
    Fx3 s = fx3_zero();
    if (tid == 0)
        for (int w = 0; w < BS / 64; w++) fx3_add(s, tmp[w]);
    __syncthreads();
    return s;  // valid in thread 0
}

// workgroup (A, b): partial sums of bucket b for the pairs (A, B), B > A
template <int W, int BS> __device__ void overlap_bucket(const Overlap &O, const int A, const int b, char *smem)
{
    const Inst &IA = const_inst(O.rep[A]);
    const int slots = IA.slots;
    Lds L;
    L.k0 = (u64 *)smem;
    double *val = (double *)(smem + sizeof(u64) * slots);
    L.k1 = W == 2 ? (u64 *)(smem + 2 * sizeof(u64) * slots) : nullptr;
    L.state = W == 2 ? (u32 *)(smem + 3 * sizeof(u64) * slots) : nullptr;
    L.lo = L.hi = nullptr;
    L.misc = nullptr;
    L.mask = slots - 1;
    Fx3 *tmp = (Fx3 *)(smem + (W == 2 ? 3 * sizeof(u64) + sizeof(u32) : 2 * sizeof(u64)) * slots);
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    for (int s = tid; s < slots; s += BS) {
        L.k0[s] = EMPTY;
        if (W == 2) { L.k1[s] = EMPTY; L.state[s] = 0u; }
    }
    if (tid == 0) s_flag = 0;
    __syncthreads();
    const int pA = IA.ctrl->parity;
    const i64 nA = min((i64)IA.tab_n[pA][b], IA.cap_t);
    const i64 ba = (i64)b * IA.cap_t;
    int np = 0;
    for (i64 i = tid; i < nA; i += BS) {
        u64 a0, a1;
        double v;
        tab_entry<W>(IA, pA, ba + i, a0, a1, v);
        const int s = lds_slot<W>(L, a0, a1, addr_hash(AddrOf<W>::make(a0, a1)), np);
        if (s < 0) s_flag = 1;
        else val[s] = v;
    }
    __syncthreads();
    if (s_flag && tid == 0) atomicOr(&O.flags[0], 1);
    int inexact = 0, ovf = 0;
    for (int Bi = A + 1; Bi < O.R; Bi++) {
        const Inst &IB = const_inst(O.rep[Bi]);
        const int pB = IB.ctrl->parity;
        const i64 nB = min((i64)IB.tab_n[pB][b], IB.cap_t);
        const i64 bb = (i64)b * IB.cap_t;
        Fx3 acc = fx3_zero();
        for (i64 j = tid; j < nB; j += BS) {
            u64 a0, a1;
            double v;
            tab_entry<W>(IB, pB, bb + j, a0, a1, v);
            const int s = lds_find<W>(L, a0, a1, addr_hash(AddrOf<W>::make(a0, a1)));
            if (s >= 0) {
                const Fx3 t = to_fx3(val[s] * v, inexact, ovf);
                fx3_add(acc, t);
            }
        }
        const Fx3 sum = block_sum_fx3<BS>(acc, tmp);
        if (tid == 0) O.part[(i64)b * O.P + pair_index(A, Bi, O.R)] = sum;
    }
    if (inexact) atomicOr(&O.flags[1], 1);
    if (ovf) atomicOr(&O.flags[2], 1);
}

// one workgroup: the overlaps of all pairs for the step just completed.
// A pair whose replicas are not both error-free at the same step gets NaN.
template <int BS> __device__ void overlap_finalize(const Overlap &O)
{
    __shared__ Fx3 tmp[BS / 64];
    const int tid = threadIdx.x;
    const Ctrl *c0 = O.rep[0]->ctrl;
    const i64 row = c0->step - c0->ring_base;
    for (int k = 0; k < O.P; k++) {
        Fx3 acc = fx3_zero();
        for (int b = tid; b < O.B; b += BS) fx3_add(acc, O.part[(i64)b * O.P + k]);
        const Fx3 sum = block_sum_fx3<BS>(acc, tmp);
        if (tid == 0 && row >= 0 && row < O.ring_cap) {
            int A = 0, rem = k;
            while (rem >= O.R - 1 - A) { rem -= O.R - 1 - A; A++; }
            const int Bi = A + 1 + rem;
            const Ctrl *ca = O.rep[A]->ctrl, *cb = O.rep[Bi]->ctrl;
            const bool ok = ca->error == 0 && cb->error == 0 && ca->step == c0->step && cb->step == c0->step;
            O.ring[row * O.P + k] = ok ? from_fx3(sum) : __longlong_as_double(0x7ff8000000000000ll);
        }
    }
}

// ------------------------------------------------ excited states
//
// Step-synchronised runs of one Hamiltonian, run k orthogonalised against
// runs 0 .. k-1 in turn after every merge (Sec. 2.2, Gram-Schmidt): c_k <-
// c_k - alpha c_j with alpha = (c_j . c_k) / (c_j . c_j).  The merged tables
// (parity 1 - ctrl.parity while the step runs) are updated before the spawn
// kernel reads them, so the next step starts from the orthogonal vector.
// gs_dot: per bucket, c_j . c_k and c_j . c_j (products rounded, summed in
// 192-bit fixed point); gs_alpha: one workgroup, the exactly rounded sums and
// one division; gs_update: per bucket, the union of the two buckets in an
// LDS hash of twice the merge's size, v_k - (alpha v_j) per address of c_j,
// compaction of the non-zero values in slot order back into c_k's table and
// the bucket's exact 1-norm; gs_norm (after the finalize kernel): that norm
// becomes the norm the next shift update starts from.

struct Spectral {
    const Inst *const *rep;  // runs in caller order
    int R, B;
    Fx3 *dots;               // [B][2]: c_j . c_k, c_j . c_j of the pair being projected
    Fx3 *norms;              // [R][B]: per-bucket 1-norm of c_k after its last projection
    double *alpha;           // [1]
    int *updated;            // [R]: run k was projected in the current step
    int *flags;              // [0] inexact product or norm term
};

__device__ __forceinline__ bool gs_idle(const Spectral &S, int j, int k)
{
    return halted(S.rep[j]->ctrl) != 0 || halted(S.rep[k]->ctrl) != 0;
}

template <int W> __device__ __forceinline__ Lds gs_lds(char *smem, int slots)
{
    Lds L;
    L.k0 = (u64 *)smem;
    L.k1 = W == 2 ? (u64 *)(smem + 2 * sizeof(u64) * slots) : nullptr;
    L.state = W == 2 ? (u32 *)(smem + 3 * sizeof(u64) * slots) : nullptr;
    L.lo = L.hi = nullptr;
    L.misc = nullptr;
    L.mask = slots - 1;
    return L;
}
// bytes of the hash in gs_lds layout: keys, values (after the keys), W = 2
// second words and slot states
template <int W> __device__ __forceinline__ size_t gs_lds_bytes(int slots)
{
    return (size_t)slots * (W == 2 ? 3 * sizeof(u64) + sizeof(u32) : 2 * sizeof(u64));
}

template <int W, int BS> __device__ void gs_dot(const Spectral &S, const int j, const int k, const int b, char *smem)
{
    if (gs_idle(S, j, k)) return;
    const Inst &IJ = const_inst(S.rep[j]), &IK = const_inst(S.rep[k]);
    const int slots = 2 * IJ.slots;  // a projected run may hold the union of two buckets
    Lds L = gs_lds<W>(smem, slots);
    double *val = (double *)(smem + sizeof(u64) * slots);
    Fx3 *tmp = (Fx3 *)(smem + gs_lds_bytes<W>(slots));
    __shared__ int s_full;
    const int tid = threadIdx.x;
    for (int s = tid; s < slots; s += BS) {
        L.k0[s] = EMPTY;
        if (W == 2) { L.k1[s] = EMPTY; L.state[s] = 0u; }
    }
    if (tid == 0) s_full = 0;
    __syncthreads();
    const int pj = 1 - IJ.ctrl->parity, pk = 1 - IK.ctrl->parity;
    const i64 nJ = min((i64)IJ.tab_n[pj][b], IJ.cap_t), nK = min((i64)IK.tab_n[pk][b], IK.cap_t);
    const i64 bj = (i64)b * IJ.cap_t, bk = (i64)b * IK.cap_t;
    int inexact = 0, ovf = 0, np = 0;
    Fx3 sq = fx3_zero();
    for (i64 i = tid; i < nJ; i += BS) {
        u64 a0, a1;
        double v;
        tab_entry<W>(IJ, pj, bj + i, a0, a1, v);
        const int s = lds_slot<W>(L, a0, a1, addr_hash(AddrOf<W>::make(a0, a1)), np);
        if (s < 0) s_full = 1;
        else val[s] = v;
        fx3_add(sq, to_fx3(v * v, inexact, ovf));
    }
    __syncthreads();
    if (s_full && tid == 0) set_error(IK.ctrl, FQE_CAP_LDS, b);
    Fx3 dot = fx3_zero();
    for (i64 i = tid; i < nK; i += BS) {
        u64 a0, a1;
        double v;
        tab_entry<W>(IK, pk, bk + i, a0, a1, v);
        const int s = lds_find<W>(L, a0, a1, addr_hash(AddrOf<W>::make(a0, a1)));
        if (s >= 0) fx3_add(dot, to_fx3(val[s] * v, inexact, ovf));
    }
    const Fx3 d = block_sum_fx3<BS>(dot, tmp);
    const Fx3 q = block_sum_fx3<BS>(sq, tmp);
    if (tid == 0) {
        S.dots[2 * (i64)b] = d;
        S.dots[2 * (i64)b + 1] = q;
    }
    if (inexact) atomicOr(&S.flags[0], 1);
    if (ovf) set_error(IK.ctrl, FQE_DIVERGED, b);
}

template <int BS> __device__ void gs_alpha(const Spectral &S, const int j, const int k)
{
    __shared__ Fx3 tmp[BS / 64];
    if (gs_idle(S, j, k)) return;
    const int tid = threadIdx.x;
    Fx3 d = fx3_zero(), q = fx3_zero();
    for (int b = tid; b < S.B; b += BS) {
        fx3_add(d, S.dots[2 * (i64)b]);
        fx3_add(q, S.dots[2 * (i64)b + 1]);
    }
    const Fx3 ds = block_sum_fx3<BS>(d, tmp);
    const Fx3 qs = block_sum_fx3<BS>(q, tmp);
    if (tid == 0) {
        const double nq = from_fx3(qs);
        *S.alpha = nq > 0.0 ? from_fx3(ds) / nq : 0.0;
    }
}

template <int W, int BS> __device__ void gs_update(const Spectral &S, const int j, const int k, const int b, char *smem)
{
    if (gs_idle(S, j, k)) return;
    const Inst &IJ = const_inst(S.rep[j]), &IK = const_inst(S.rep[k]);
    const int slots = 2 * IK.slots;  // the union of two buckets
    Lds L = gs_lds<W>(smem, slots);
    double *val = (double *)(smem + sizeof(u64) * slots);
    char *rest = smem + gs_lds_bytes<W>(slots);
    Fx3 *tmp = (Fx3 *)rest;
    i64 *scan = (i64 *)(rest + sizeof(Fx3) * (BS / 64));
    __shared__ int s_full;
    const int tid = threadIdx.x;
    for (int s = tid; s < slots; s += BS) {
        L.k0[s] = EMPTY;
        if (W == 2) { L.k1[s] = EMPTY; L.state[s] = 0u; }
        val[s] = 0.0;
    }
    if (tid == 0) s_full = 0;
    __syncthreads();
    const int pj = 1 - IJ.ctrl->parity, pk = 1 - IK.ctrl->parity;
    const i64 nJ = min((i64)IJ.tab_n[pj][b], IJ.cap_t), nK = min((i64)IK.tab_n[pk][b], IK.cap_t);
    const i64 bj = (i64)b * IJ.cap_t, bk = (i64)b * IK.cap_t;
    int np = 0;
    for (i64 i = tid; i < nK; i += BS) {
        u64 a0, a1;
        double v;
        tab_entry<W>(IK, pk, bk + i, a0, a1, v);
        const int s = lds_slot<W>(L, a0, a1, addr_hash(AddrOf<W>::make(a0, a1)), np);
        if (s < 0) s_full = 1;
        else val[s] = v;
    }
    __syncthreads();
    const double alpha = *S.alpha;
    for (i64 i = tid; i < nJ; i += BS) {
        u64 a0, a1;
        double v;
        tab_entry<W>(IJ, pj, bj + i, a0, a1, v);
        const int s = lds_slot<W>(L, a0, a1, addr_hash(AddrOf<W>::make(a0, a1)), np);
        if (s < 0) {
            s_full = 1;
        } else {
            const double p = alpha * v;
            val[s] = val[s] - p;
        }
    }
    __syncthreads();
    if (s_full) {
        if (tid == 0) set_error(IK.ctrl, FQE_CAP_LDS, b);
        return;
    }
    // compaction in slot order: thread t owns slots [t c, (t + 1) c)
    const int per = slots / BS;
    const int s0 = tid * per;
    i64 mine = 0;
    for (int s = s0; s < s0 + per; s++) {
        const bool occ = W == 1 ? L.k0[s] != EMPTY : L.state[s] == 2u;
        mine += (occ && val[s] != 0.0) ? 1 : 0;
    }
    i64 total;
    i64 o = block_excl_scan<BS>(mine, scan, total);
    int inexact = 0, ovf = 0;
    Fx3 nrm = fx3_zero();
    if (total > IK.cap_t) {
        if (tid == 0) set_error(IK.ctrl, FQE_CAP_TABLE, b);
        return;
    }
    for (int s = s0; s < s0 + per; s++) {
        const bool occ = W == 1 ? L.k0[s] != EMPTY : L.state[s] == 2u;
        if (occ && val[s] != 0.0) {
            IK.tab_a[pk][0][bk + o] = L.k0[s];
            if (W == 2) IK.tab_a[pk][1][bk + o] = L.k1[s];
            IK.tab_v[pk][bk + o] = val[s];
            fx3_add(nrm, to_fx3(fabs(val[s]), inexact, ovf));
            o++;
        }
    }
    const Fx3 ns = block_sum_fx3<BS>(nrm, tmp);
    if (tid == 0) {
        IK.tab_n[pk][b] = (int)total;
        S.norms[(i64)k * S.B + b] = ns;
        if (b == 0) S.updated[k] = 1;
    }
    if (inexact) atomicOr(&S.flags[0], 1);
    if (ovf) set_error(IK.ctrl, FQE_DIVERGED, b);
}

// after the finalize kernel: the orthogonalised norm of every projected run
template <int BS> __device__ void gs_norm(const Spectral &S, const int k)
{
    __shared__ Fx3 tmp[BS / 64];
    __shared__ int s_go;
    const int tid = threadIdx.x;
    Ctrl *c = S.rep[k]->ctrl;
    if (tid == 0) s_go = S.updated[k] && __hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    __syncthreads();
    if (!s_go) return;
    Fx3 a = fx3_zero();
    for (int b = tid; b < S.B; b += BS) fx3_add(a, S.norms[(i64)k * S.B + b]);
    const Fx3 t = block_sum_fx3<BS>(a, tmp);
    if (tid == 0) {
        c->norm = from_fx3(t);
        S.updated[k] = 0;
    }
}

}  // namespace fq
