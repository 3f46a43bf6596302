// fq_step.hpp -- one FCIQMC step for one hash bucket, run by one workgroup.
//
// Data layout in HBM (per instance, two parities p = 0, 1):
//   table[p]: B buckets x cap_t entries, struct of arrays: address word 0,
//             address word 1 (W = 2), value (f64); count per bucket.
//   slab[p]:  B buckets x cap_s spawn records (array of structs: address
//             words + value; 12 B when the address fits 32 bits, else 16 B
//             for W = 1, 24 B for W = 2; with the initiator rule a record of
//             a non-initiator parent carries a flag bit above the address
//             bits); count per bucket.
// An address lives in bucket bucket_index(address): the top log2 B bits of
// a hash of the address.
//
// Step n -> n+1 for bucket b (Sec. 3.2; the two phases of the paper's
// segmented product in Sec. 6.4 become one pass per bucket):
//   1. merge: the diagonal survivors c (1 + dtau (S^(n) - H_aa)) of table[p]
//      and every spawn record of slab[p] are summed per address in an LDS
//      open-addressing hash with exact 128-bit fixed-point accumulators;
//   2. compress: |w| >= theta kept, else sign(w) theta with probability
//      |w|/theta using the address-keyed tag-1 draw of step n+1;
//   3. projected energy: the entries of the reference column that live in
//      this bucket are looked up in the LDS hash;
//   4. compact survivors into table[1-p] and into LDS;
//   5. spawn for step n+2 from every survivor (a separate kernel): exact
//      columns when |c| >= t_rel m, attempt by attempt over the workgroup;
//      else ceil|c| Philox picks, in units of four consecutive attempts of
//      one parent per thread.  Records are partitioned in rounds: every thread holds
//      its round's records in registers, takes a rank inside each record's
//      destination group with an LDS atomic, one global atomic per group
//      reserves a contiguous run, and the records are stored into the runs.
//      With B <= 64 the groups are the buckets of slab[1-p]; otherwise they
//      are G coarse groups and the partition kernel splits every group into
//      its B/G buckets.
// A separate one-workgroup kernel reduces the per-bucket partial statistics,
// performs the shift update (Eq. shift-update) and writes the statistics row.
#pragma once
#include <type_traits>

#include "fq_models.hpp"

namespace fq {

constexpr u64 EMPTY = ~0ull;
enum { FQE_CAP_TABLE = 1, FQE_CAP_SLAB = 2, FQE_CAP_LDS = 3, FQE_DIVERGED = 4, FQE_ATTEMPTS = 5,
       FQE_BARRIER = 6 };

struct StepStats {  // mirrors fq_step_stats
    i64 step, len, exact_steps, inexact_steps, spawns;
    double shift, norm, hproj, vproj;
    i64 flags;
};
constexpr i64 ROW_INEXACT = 1;  // FQ_ROW_INEXACT

struct Ctrl {
    i64 step;          // index n of the current state c^(n)
    int parity;        // parity holding c^(n) and its spawns
    int error;         // 0 or an FQE_* code
    double shift;      // S^(n)
    double norm;       // ||c^(n)||_1
    u32 inexact_in;    // the norm of a state being set was rounded (reported in the next row)
    u32 max_load;      // largest LDS hash occupancy seen
    i64 ring_base;     // step number stored in ring row 0
    u64 acc_norm[2];   // norm of a state being set (set_state only)
    i64 dump_spawn_n, dump_merged_n;
    i64 stop_step;     // batch: do not advance past this step
    int err_bucket, spawn_par;  // spawn_par: parity of the slab being produced
    u64 phase[10];     // summed wall-clock ticks per phase (opt-in diagnostics)
    u64 probes;        // LDS hash probes summed over all inserts (diagnostics)
    u64 inserts;
    i64 first_inexact; // first step whose row has ROW_INEXACT since the state was set, 0 if none
};

// per-bucket partial statistics, written with plain stores by the workgroup
// that merges the bucket and reduced by the finalize kernel (no same-address
// atomics on the step's critical path)
struct Part {
    u64 norm[2], hproj[2], vproj[2];
    i64 len, load, inexact;
};
struct SpawnPart {
    i64 exact, inexact, spawns, pad;
};

struct Inst {
    ModelConst mc;
    int model, W;
    double dtau, target, zeta, xi, theta, t_rel;
    u64 seed;
    int log2B, B, slots, flags;
    i64 cap_t, cap_s;
    u64 *tab_a[2][2];
    double *tab_v[2];
    int *tab_n[2];
    char *slab[2];
    int *slab_n[2];
    int ref_n, ref_self;
    u64 *ref_a[2];
    double *ref_h;
    int *ref_off;
    double yref;
    Ctrl *ctrl;
    StepStats *ring;
    i64 ring_cap;
    u64 *dsp_parent, *dsp_dest;
    i64 *dsp_attempt;
    double *dsp_val;
    u64 *dmg_addr;
    double *dmg_val;
    i64 dump_cap;
    Part *part;          // [B]
    SpawnPart *spart[2]; // [row parity][B]
    // two-pass spawn partition (B > 64): G = 2^log2G groups of B/G buckets,
    // each with SUB = 2^log2SUB coarse sub-slabs of cap_c records
    int two_pass, log2G, log2SUB;
    int rec;  // bytes per spawn record: 12 (one address word that fits 32 bits), 16 or 24
    i64 cap_c;
    // initiator rule: parents with |c| > n_a are initiators; a record of a
    // non-initiator carries iflag (a bit above every address bit of the
    // last address word); iflag = 0 without the rule
    u64 iflag;
    double n_a;
    char *coarse;
    int *coarse_n;
};

// Kernels never write a descriptor, so a workgroup reads its descriptor in
// the constant address space: scalar loads, loaded once rather than again
// after every store the kernel makes, and the pointers it holds are known to
// address device memory (global, not flat, loads and stores).  The integer
// round trip keeps the compiler from folding the cast away.
typedef const __attribute__((address_space(4))) Inst ConstInst;
__device__ __forceinline__ const Inst &const_inst(const Inst *p)
{
    return *(const Inst *)(ConstInst *)(uintptr_t)p;
}

__device__ __forceinline__ void set_error(Ctrl *c, int code, int bucket)
{
    if (atomicCAS(&c->error, 0, code) == 0) c->err_bucket = bucket;
}

// an instance does no work once it has failed or has reached its stop step
// (instances of a batch stop independently; all kernels of one step see the
// same step number, which only the finalize kernel advances)
// Parity dumps may keep a sample of the addresses: with k = flags bits 8..12
// (0 = keep all), an address is kept when bits 24 .. 24+k-1 of its hash are
// zero, a fixed 2^-k fraction independent of the bucket and LDS slot bits.
__device__ __forceinline__ bool dump_keeps(int flags, u64 h)
{
    const int k = (flags >> 8) & 31;
    return k == 0 || ((h >> 24) & ((1ull << k) - 1)) == 0;
}

// the compression rule of Eq. vec-compression for one value: |w| >= theta
// kept, otherwise sign(w) theta when u theta < |w| (u = r 2^-32), else 0
__device__ __forceinline__ double compress1(double w, double theta, u32 r)
{
    const double aw = fabs(w);
    if (aw >= theta) return w;
    const double u = (double)r * 0x1p-32;
    return (aw > 0.0 && u * theta < aw) ? (w < 0.0 ? -theta : theta) : 0.0;
}

constexpr int FLAG_EARLY = 32;  // early compression (FQ_FLAG_EARLY_COMPRESSION)

__device__ __forceinline__ int halted(Ctrl *c)
{
    const int e = __hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return e != 0 || c->step >= c->stop_step;
}

template <int W> struct Rec;
template <> struct Rec<1> {
    u64 a;
    double v;
};
template <> struct Rec<2> {
    u64 a0, a1;
    double v;
};

// Spawn records in the slabs: address words then the value.  When the
// address fits 32 bits (one word, N+M-1 <= 32) a record is three 32-bit words
// (12 bytes, rec = 12); otherwise 16 or 24 bytes.  `base` is the start of a
// slab or sub-slab, i the record index.
template <int W> __device__ __forceinline__ void store_rec(int rec, char *base, i64 i, typename AddrOf<W>::T d, double v);
template <> __device__ __forceinline__ void store_rec<1>(int rec, char *base, i64 i, u64 d, double v)
{
    const u64 vb = dbits(v);
    if (rec == 12) {
        uint3 x;
        x.x = (u32)d;
        x.y = (u32)vb;
        x.z = (u32)(vb >> 32);
        *gmem((uint3 *)(base + 12 * i)) = x;
    } else {
        ulonglong2 x;
        x.x = d;
        x.y = vb;
        *gmem((ulonglong2 *)base + i) = x;
    }
}
template <> __device__ __forceinline__ void store_rec<2>(int, char *base, i64 i, U128 d, double v)
{
    FQ_GAS Rec<2> *r = gmem((Rec<2> *)base + i);
    r->a0 = d.lo;
    r->a1 = d.hi;
    r->v = v;
}
template <int W> __device__ __forceinline__ void load_rec(int rec, const char *base, i64 i, u64 &a0, u64 &a1, double &v);
template <> __device__ __forceinline__ void load_rec<1>(int rec, const char *base, i64 i, u64 &a0, u64 &a1, double &v)
{
    a1 = 0;
    if (rec == 12) {
        const uint3 x = *gmem((const uint3 *)(base + 12 * i));
        a0 = x.x;
        v = bitsd(((u64)x.z << 32) | x.y);
    } else {
        const ulonglong2 x = *gmem((const ulonglong2 *)base + i);
        a0 = x.x;
        v = bitsd(x.y);
    }
}
template <> __device__ __forceinline__ void load_rec<2>(int, const char *base, i64 i, u64 &a0, u64 &a1, double &v)
{
    const FQ_GAS Rec<2> *r = gmem((const Rec<2> *)base + i);
    a0 = r->a0;
    a1 = r->a1;
    v = r->v;
}

// ---------------------------------------------------------------- block scan

template <int BS> __device__ __forceinline__ i64 block_excl_scan(i64 v, i64 *tmp, i64 &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    i64 x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        i64 y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) tmp[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        i64 s = 0;
        for (int w = 0; w < BS / 64; w++) {
            i64 t = tmp[w];
            tmp[w] = s;
            s += t;
        }
        tmp[BS / 64] = s;
    }
    __syncthreads();
    i64 r = tmp[wid] + x - v;
    total = tmp[BS / 64];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- LDS hash

struct Lds {
    u64 *k0, *k1;   // keys (word 0, word 1)
    u32 *state;     // W = 2 slot state: 0 empty, 1 busy, 2 full
    u64 *lo, *hi;   // fixed-point accumulators; later reused for survivors
    i64 *misc;      // scan scratch and block accumulators
    unsigned char *occ;  // initiator rule: 1 where the slot holds an address of c^(n)
    int mask;
};

// find or insert the slot of address (a0, a1); returns -1 when full
template <int W> __device__ __forceinline__ int lds_slot(const Lds &L, u64 a0, u64 a1, u64 h, int &np)
{
    int s = (int)(h & (u64)L.mask);
    for (int probe = 0; probe <= L.mask; probe++) {
        np++;
        if (W == 1) {
            // one compare-and-swap per probe: it claims an empty slot, and
            // returns the key already there otherwise
            const u64 old = atomicCAS((unsigned long long *)&L.k0[s], EMPTY, a0);
            if (old == EMPTY || old == a0) return s;
        } else {
            for (;;) {
                // claim an empty slot (0 -> 1), or learn its state: 2 full,
                // 1 busy while another lane writes the key
                u32 st = 0u;
                if (__hip_atomic_compare_exchange_strong(&L.state[s], &st, 1u, __ATOMIC_ACQUIRE, __ATOMIC_ACQUIRE,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP)) {
                    L.k0[s] = a0;
                    L.k1[s] = a1;
                    __hip_atomic_store(&L.state[s], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                    return s;
                }
                if (st == 2u) {
                    if (L.k0[s] == a0 && L.k1[s] == a1) return s;
                    break;
                }
                // busy: another lane is writing the key; look again
            }
        }
        s = (s + 1) & L.mask;
    }
    return -1;
}

// read-only lookup; -1 if absent
template <int W> __device__ __forceinline__ int lds_find(const Lds &L, u64 a0, u64 a1, u64 h)
{
    int s = (int)(h & (u64)L.mask);
    for (int probe = 0; probe <= L.mask; probe++) {
        bool occ = W == 1 ? L.k0[s] != EMPTY : L.state[s] == 2u;
        if (!occ) return -1;
        if (L.k0[s] == a0 && (W == 1 || L.k1[s] == a1)) return s;
        s = (s + 1) & L.mask;
    }
    return -1;
}

// Slot of an address in the merge's LDS hash: a 32-bit finalizer (two
// multiplies) of the address words folded to 32 bits.  The bucket is chosen
// by the top bits of the 64-bit address hash; inside a bucket any well-mixed
// function serves, and this one costs a third of the instructions.
__device__ __forceinline__ u64 slot_hash(u64 a0, u64 a1)
{
    u32 x = (u32)a0 ^ ((u32)(a0 >> 32) * 0x85EBCA6Bu) ^ ((u32)a1 * 0xC2B2AE35u) ^ ((u32)(a1 >> 32) * 0x27D4EB2Fu);
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return (u64)x;
}

// Insert NB values of this thread at once: the fixed-point conversions
// first, then every first-probe compare-and-swap, then every accumulator
// add, so the LDS round trips of the NB inserts overlap instead of running
// one after another.  ok[e] selects the values to insert.  Sums are exact,
// so the order of the adds does not matter.  One-word keys: the CAS is on
// the key itself.  Two-word keys: the CAS claims the slot's state word
// (0 -> 1); the claiming lane then writes the key and publishes the slot
// (state 2) before any lane continues a probe, so a lane that found the
// slot busy finds it full when it looks again.
template <int W, int NB>
__device__ __forceinline__ void lds_add_n(const Lds &L, const Inst &I, const u64 *a0, const u64 *a1,
                                          const double *v, const bool *ok, int b, int &np, int &inx)
{
    u64 lo[NB], hi[NB], old[NB];
    int s[NB];
    bool go[NB];
#pragma unroll
    for (int e = 0; e < NB; e++) {
        go[e] = ok[e];
        lo[e] = hi[e] = 0;
        if (go[e]) {
            int ovf = 0;
            to_fixed(v[e], lo[e], hi[e], ovf, inx);
            if (ovf) { set_error(I.ctrl, FQE_DIVERGED, b); go[e] = false; }
        }
    }
    if (W == 1) {
#pragma unroll
        for (int e = 0; e < NB; e++) {
            s[e] = 0;
            old[e] = EMPTY;
            if (go[e]) {
                s[e] = (int)(slot_hash(a0[e], 0ull) & (u64)L.mask);
                np++;
                old[e] = atomicCAS((unsigned long long *)&L.k0[s[e]], EMPTY, a0[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < NB; e++) {
            if (go[e] && old[e] != EMPTY && old[e] != a0[e]) {
                // collision: continue the linear probe from the next slot
                s[e] = lds_slot<W>(L, a0[e], 0ull, (u64)(s[e] + 1), np);
                if (s[e] < 0) { set_error(I.ctrl, FQE_CAP_LDS, b); go[e] = false; }
            }
        }
    } else {
        u32 st[NB];
        bool claimed[NB];
#pragma unroll
        for (int e = 0; e < NB; e++) {
            s[e] = 0;
            st[e] = 0u;
            claimed[e] = false;
            if (go[e]) {
                s[e] = (int)(slot_hash(a0[e], a1[e]) & (u64)L.mask);
                np++;
                claimed[e] = __hip_atomic_compare_exchange_strong(&L.state[s[e]], &st[e], 1u, __ATOMIC_ACQUIRE,
                                                                  __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
#pragma unroll
        for (int e = 0; e < NB; e++) {
            if (go[e] && claimed[e]) {
                L.k0[s[e]] = a0[e];
                L.k1[s[e]] = a1[e];
                __hip_atomic_store(&L.state[s[e]], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
#pragma unroll
        for (int e = 0; e < NB; e++) {
            if (go[e] && !claimed[e]) {
                // full with another key: probe on from the next slot; busy:
                // look at this slot again (its key is being written)
                const bool hit = st[e] == 2u && L.k0[s[e]] == a0[e] && L.k1[s[e]] == a1[e];
                if (!hit) {
                    s[e] = lds_slot<W>(L, a0[e], a1[e], (u64)(s[e] + (st[e] == 2u ? 1 : 0)), np);
                    if (s[e] < 0) { set_error(I.ctrl, FQE_CAP_LDS, b); go[e] = false; }
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < NB; e++)
        if (go[e]) old[e] = atomicAdd((unsigned long long *)&L.lo[s[e]], (unsigned long long)lo[e]);
#pragma unroll
    for (int e = 0; e < NB; e++) {
        if (go[e]) {
            const u64 h = hi[e] + ((old[e] + lo[e]) < old[e] ? 1ull : 0ull);
            if (h) atomicAdd((unsigned long long *)&L.hi[s[e]], (unsigned long long)h);
        }
    }
}

// Initiator rule: add NB contributions of non-initiator parents (ok[e])
// only onto addresses of c^(n).  Called after the table entries are in the
// hash and L.occ marks them; every slot on the probe path of such an address
// was full before any spawn record was inserted, so the lookup finds it
// while other lanes insert concurrently, and a miss or an unmarked slot
// means the destination is not occupied: the contribution is discarded.
template <int W, int NB>
__device__ __forceinline__ void lds_add_occupied(const Lds &L, const Inst &I, const u64 *a0, const u64 *a1,
                                                 const double *v, const bool *ok, int b, int &inx)
{
#pragma unroll
    for (int e = 0; e < NB; e++) {
        if (!ok[e]) continue;
        const int s = lds_find<W>(L, a0[e], a1[e], slot_hash(a0[e], W == 2 ? a1[e] : 0ull));
        if (s < 0 || !L.occ[s]) continue;
        u64 lo = 0, hi = 0;
        int ovf = 0;
        to_fixed(v[e], lo, hi, ovf, inx);
        if (ovf) { set_error(I.ctrl, FQE_DIVERGED, b); continue; }
        const u64 old = atomicAdd((unsigned long long *)&L.lo[s], (unsigned long long)lo);
        const u64 h = hi + ((old + lo) < old ? 1ull : 0ull);
        if (h) atomicAdd((unsigned long long *)&L.hi[s], (unsigned long long)h);
    }
}

// ---------------------------------------------------------------- spawn info

template <int W, int MODEL>
__device__ __forceinline__ void spawn_info(const Inst &I, typename AddrOf<W>::T a, double c, u32 &cnt, bool &exact,
                                           int &bad)
{
    i64 m;
    if (MODEL == 0) m = 2 * popc(run_starts(a));
    else if (MODEL == 3) m = I.mc.ndir * popc(run_starts(a));
    else if (MODEL == 1 || (W == 1 && I.mc.nb <= 32)) m = mom_col_size<u32>(I.mc, (u32)word0(a));
    else m = mom_col_size(I.mc, a);
    double ac = fabs(c);
    exact = (m == 0) || ac >= I.t_rel * (double)m;
    if (exact) {
        cnt = (u32)m;
    } else {
        // the 28-bit block index of the draw counter allows 2^28 blocks: two
        // momentum-space attempts per block, four of the other models
        double n = ceil(ac);
        if (!(n <= (MODEL == 1 || MODEL == 2 ? 536870912.0 : 1073741824.0))) { bad = 1; n = 0.0; }
        cnt = (u32)n;
    }
}

// ---------------------------------------------------------------- spawn records

// Partition of spawn records into destination groups, one round at a time:
// every thread holds up to NR records, takes a rank inside the record's group
// from an LDS counter, one thread per group reserves a contiguous run with
// one global atomic, then the records are stored into the runs.  With the
// two-pass partition a group is a coarse group of buckets and the run lies in
// the coarse sub-slab of the producing bucket (bucket mod 64); otherwise a group
// is a bucket and the run lies in its slab.
// COUNT: also count the records emitted (early compression drops records, so
// the spawn count is not the attempt count)
template <int W, bool COUNT> struct SpawnOut {
    typedef typename AddrOf<W>::T T;
    const Inst &I;
    const Lds &L;
    int out_par, G, gshift, sub;
    __device__ SpawnOut(const Inst &I_, const Lds &L_, int out_par_, int b) : I(I_), L(L_), out_par(out_par_)
    {
        const int log2G = I.two_pass ? I.log2G : I.log2B;
        G = 1 << log2G;
        gshift = I.log2B - log2G;
        sub = b & ((1 << I.log2SUB) - 1);
    }
    __device__ int *gcnt() const { return (int *)(L.misc + 64); }  // G <= 64 counters
    __device__ i64 *gbase() const { return L.misc + 96; }          // G <= 64 run bases
    __device__ void begin() const
    {
        if ((int)threadIdx.x < G) gcnt()[threadIdx.x] = 0;
        __syncthreads();
    }
    __device__ int group(const T &d) const { return (int)(bucket_index(d, I.log2B, I.mc.nb <= 32) >> gshift); }
    __device__ int rank(int g) const { return atomicAdd(&gcnt()[g], 1); }
    __device__ void reserve() const
    {
        __syncthreads();
        const int tid = threadIdx.x;
        if (tid < G) {
            const int cg = gcnt()[tid];
            int *cn = I.two_pass ? &I.coarse_n[(tid << I.log2SUB) + sub] : &I.slab_n[out_par][tid];
            gbase()[tid] = cg ? (i64)gatomic_add(cn, cg) : 0;
            if (COUNT && cg) atomicAdd((unsigned long long *)&L.misc[60], (unsigned long long)cg);
        }
        __syncthreads();
    }
    // ni: the parent is not an initiator; its flag I.iflag (0 without the
    // initiator rule) goes into the record's address, not into the dump
    __device__ void put(int g, int rk, const T &d, double v, u64 pa0, u64 pa1, u32 k, bool ni) const
    {
        const i64 pos = gbase()[g] + rk;
        const u64 fl = ni ? I.iflag : 0ull;
        const T df = AddrOf<W>::make(W == 1 ? word0(d) | fl : word0(d), W == 2 ? word1(d) | fl : 0ull);
        if (I.two_pass) {
            const i64 cs = ((i64)g << I.log2SUB) + sub;
            if (pos < I.cap_c) store_rec<W>(I.rec, I.coarse, cs * I.cap_c + pos, df, v);
            else set_error(I.ctrl, FQE_CAP_SLAB, g);
        } else {
            if (pos < I.cap_s) store_rec<W>(I.rec, I.slab[out_par], (i64)g * I.cap_s + pos, df, v);
            else set_error(I.ctrl, FQE_CAP_SLAB, g);
        }
        if ((I.flags & 1) && dump_keeps(I.flags, addr_hash(d))) {
            i64 di = atomicAdd((unsigned long long *)&I.ctrl->dump_spawn_n, 1ull);
            if (di < I.dump_cap) {
                I.dsp_parent[di * W] = pa0;
                if (W == 2) I.dsp_parent[di * W + 1] = pa1;
                I.dsp_attempt[di] = (i64)k;
                I.dsp_dest[di * W] = word0(d);
                if (W == 2) I.dsp_dest[di * W + 1] = word1(d);
                I.dsp_val[di] = v;
            }
        }
    }
};

// Spawns of the exact parents (Sec. 7.1, exact columns): an exact parent
// with column size m has m attempts, attempt k being column entry k with
// weight 1.  The A attempts of the nX exact parents (permuted indices
// 0 .. nX-1, attempt offsets in info[2 w], count word in info[2 w + 1]) are
// enumerated flat: in each round thread t takes attempts base + r BS + t
// (r < NR), finds each attempt's parent by a binary search over the short
// range a coarse index of the bucket leaves, and computes the column entry
// directly (no walk of the column).  NR records per thread and round make
// the runs appended to each destination group longer.
#ifndef FQ_SPAWN_NR
#define FQ_SPAWN_NR 4
#endif
constexpr int SPAWN_COARSE = 512;  // entries of the coarse parent index of a bucket

template <int W, int MODEL, int BS, bool EARLY>
__device__ __forceinline__ void spawn_exact(const Inst &I, const Lds &L, const int b, const int par,
                                            const u32 spawn_step, const int nX, const u32 *info, const u32 *perm,
                                            const i64 A, const unsigned char *lut, int *coarse)
{
    typedef typename AddrOf<W>::T T;
    constexpr int NR = FQ_SPAWN_NR;
    const int tid = threadIdx.x;
    const SpawnOut<W, EARLY> out(I, L, par, b);
    // the address fits 32 bits (same for every lane; always for model variant 1)
    const bool narrow = MODEL == 1 || (W == 1 && I.mc.nb <= 32);
    // Coarse index: coarse[j] is the parent of attempt j 2^cs (the last entry
    // whose first attempt is at or before it), for j < nc.  The parent of
    // attempt k then lies between coarse[k >> cs] and the next coarse entry,
    // a short range searched per attempt.
    int top = 1;
    while (2 * top <= nX) top *= 2;
    int cs = 5;
    while ((A >> cs) >= SPAWN_COARSE) cs++;
    const int nc = (int)(A >> cs) + 1;
    for (int j = tid; j < nc; j += BS) {
        const u32 kj = (u32)((i64)j << cs);  // A < 2^32 (checked by the caller)
        int lo = 0;
        for (int stp = top; stp > 0; stp >>= 1) {
            const int nx = lo + stp;
            if (nx < nX && info[2 * nx] <= kj) lo = nx;
        }
        coarse[j] = lo;
    }
    __syncthreads();
    for (i64 base = 0; base < A; base += (i64)NR * BS) {
        out.begin();
        T d[NR];
        double v[NR];
        int g[NR], rk[NR];
        u64 pa0[NR], pa1[NR];
        bool ni[NR];
        u32 kk[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const i64 kf = base + (i64)r * BS + tid;
            d[r] = AddrOf<W>::make(0, 0);
            v[r] = 0.0;
            g[r] = -1;
            rk[r] = 0;
            pa0[r] = pa1[r] = 0;
            ni[r] = false;
            kk[r] = 0;
            if (kf < A) {
                // A < 2^32 (checked by the caller): 32-bit offsets suffice
                const u32 k32 = (u32)kf;
                const int j = (int)(kf >> cs);
                int lo = coarse[j], hi = j + 1 < nc ? coarse[j + 1] : nX - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (info[2 * mid] <= k32) lo = mid;
                    else hi = mid - 1;
                }
                const int w = lo;
                const u32 k = k32 - info[2 * w];
                const i64 e = (i64)b * I.cap_t + perm[w];
                const u64 a0 = gmem(I.tab_a[par][0])[e];
                const u64 a1 = W == 2 ? gmem(I.tab_a[par][1])[e] : 0;
                const double c = gmem(I.tab_v[par])[e];
                const T a = AddrOf<W>::make(a0, a1);
                double h;
                T dd;
                if (MODEL == 0) {
                    const T st = run_starts(a);
                    dd = real_entry(I.mc, a, st, popc(st), (int)k, h);
                } else if (MODEL == 3) {
                    const T st = run_starts(a);
                    int kd;
                    dd = lat_entry(I.mc, a, st, popc(st), (int)k, h, kd, lut);
                    h = h * gmem(I.mc.gz)[I.mc.N + kd];
                } else if (narrow) {
                    dd = AddrOf<W>::make((u64)mom_column_entry<u32>(I.mc, (u32)a0, (int)k, h, lut), 0);
                } else {
                    dd = mom_column_entry(I.mc, a, (int)k, h, lut);
                }
                d[r] = dd;
                v[r] = (-(I.dtau * h)) * c;
                pa0[r] = a0;
                pa1[r] = a1;
                ni[r] = !(fabs(c) > I.n_a);
                kk[r] = k;
                if (EARLY && fabs(v[r]) < I.theta) {
                    const R4 rc = draw(I.seed, a0, a1, spawn_step, 4u + (k >> 28), k & 0x0fffffffu);
                    v[r] = compress1(v[r], I.theta, rc.x);
                }
                if (!EARLY || v[r] != 0.0) {
                    g[r] = out.group(dd);
                    rk[r] = out.rank(g[r]);
                }
            }
        }
        out.reserve();
#pragma unroll
        for (int r = 0; r < NR; r++)
            if (g[r] >= 0) out.put(g[r], rk[r], d[r], v[r], pa0[r], pa1[r], kk[r], ni[r]);
    }
}

// Spawns of the stochastic parents (Sec. 3.2, Eqs. spawning and
// column-compression): a parent with ceil|c| = n attempts draws n column
// entries independently, attempt k from its Philox block (k >> 1 in
// momentum space, two words per attempt; k >> 2 otherwise, one word).  The
// attempts are cut into units of U = SPAWN_UNIT consecutive attempts:
// parent w has floor(n / U) full units (attempts U j .. U j + U - 1) and,
// when U does not divide n, one partial unit with the last n mod U
// attempts.  Units are
// enumerated full units first (flat over the parents, unit offsets in
// info[2 w]), then the partial units in the order of the parents
// w = w0 .. w0 + nP - 1, which the caller sorted by n mod U descending, so
// that the lanes of a wave run loops of equal length.  Each thread takes
// one unit per round: it finds and loads the parent once, prepares what
// every draw of that parent shares (run starts, pair counts, the weight
// m / n or the two values of P R / n), computes each Philox block once for
// the attempts that share it, and generates the unit's records.
#ifndef FQ_SPAWN_UNIT
#define FQ_SPAWN_UNIT 4
#endif
constexpr int SPAWN_UNIT = FQ_SPAWN_UNIT;
// a unit starts at an attempt that is a multiple of SPAWN_UNIT, and the
// draws of a unit assume that its Philox blocks start with it: four
// attempts per block in real space, two in momentum space
static_assert(SPAWN_UNIT % 4 == 0, "units must align with the Philox blocks");

template <int W, int MODEL, int BS, bool EARLY>
__device__ __forceinline__ void spawn_units(const Inst &I, const Lds &L, const int b, const int par,
                                            const u32 spawn_step, const int w0, const int nS, const int nP,
                                            const u32 *info, const u32 *perm, const i64 FU,
                                            const unsigned char *lut, const unsigned short *tri)
{
    typedef typename AddrOf<W>::T T;
    // records of model variant 1 (addresses of at most 31 bits) are held as
    // 32-bit words until they are stored
    constexpr bool R32 = MODEL == 1 && W == 1;
    typedef typename std::conditional<R32, u32, T>::type RA;
    auto wide = [](RA x) -> T {
        if constexpr (R32) return AddrOf<W>::make((u64)x, 0ull);
        else return x;
    };
    constexpr int U = SPAWN_UNIT;
    const int tid = threadIdx.x;
    const SpawnOut<W, EARLY> out(I, L, par, b);
    const int ns = nS - w0;  // stochastic parents
    int top = 1;
    while (2 * top <= ns) top *= 2;
    const i64 NU = FU + nP;
    for (i64 ubase = 0; ubase < NU; ubase += BS) {
        out.begin();
        RA d[U];
        double v[U];
        int gr[U];  // destination group << 16 | rank inside the round (ranks < BS U <= 8192), -1 if none
        u64 pa0 = 0, pa1 = 0;
        bool ni = false;
        u32 k0 = 0;
        int size = 0;
#pragma unroll
        for (int i = 0; i < U; i++) {
            d[i] = RA{};
            v[i] = 0.0;
            gr[i] = -1;
        }
        const i64 u = ubase + tid;
        int w = -1;
        if (u < FU) {
            // the last stochastic parent whose first full unit is at or before u
            // (FU < 2^29: 32-bit offsets suffice)
            const u32 u32_ = (u32)u;
            int lo = w0;
            for (int stp = top; stp > 0; stp >>= 1) {
                const int nx = lo + stp;
                if (nx < nS && info[2 * nx] <= u32_) lo = nx;
            }
            w = lo;
            k0 = (u32)U * (u32_ - info[2 * w]);
            size = U;
        } else if (u < NU) {
            w = w0 + (int)(u - FU);
            const u32 cnt = info[2 * w + 1] & 0x7fffffffu;
            k0 = cnt & ~(u32)(U - 1);
            size = (int)(cnt & (u32)(U - 1));
        }
        if (w >= 0) {
            const u32 cnt = info[2 * w + 1] & 0x7fffffffu;
            const i64 e = (i64)b * I.cap_t + perm[w];
            pa0 = gmem(I.tab_a[par][0])[e];
            pa1 = W == 2 ? gmem(I.tab_a[par][1])[e] : 0;
            const double c = gmem(I.tab_v[par])[e];
            const T a = AddrOf<W>::make(pa0, pa1);
            const double cn = (double)cnt;
            ni = !(fabs(c) > I.n_a);
            if constexpr (MODEL == 0 || MODEL == 3) {
                const T st = run_starts(a);
                const int o = popc(st);
                const int m = (MODEL == 0 ? 2 : I.mc.ndir) * o;
                const double q = (double)m / cn;
                R4 rr;
#pragma unroll
                for (int i = 0; i < U; i++) {
                    if (i < size) {
                        if ((i & 3) == 0) rr = draw(I.seed, pa0, pa1, spawn_step, 0u, (k0 + (u32)i) >> 2);
                        const u32 rw = (i & 3) == 0 ? rr.x : (i & 3) == 1 ? rr.y : (i & 3) == 2 ? rr.z : rr.w;
                        double h;
                        if constexpr (MODEL == 0) {
                            d[i] = real_entry(I.mc, a, st, o, (int)pick(rw, (u32)m), h);
                        } else {
                            int kd;
                            d[i] = lat_entry(I.mc, a, st, o, (int)pick(rw, (u32)m), h, kd, lut);
                            h = h * gmem(I.mc.gz)[I.mc.N + kd];
                        }
                        v[i] = ((-(I.dtau * h)) * c) * q;
                    }
                }
            } else if constexpr (R32) {
                // momentum space, one-word addresses of at most 31 bits
                const MomCtx32 x = mom_ctx32(I.mc, (u32)pa0);
                const int hR = mom_R(0, I.mc.M);
                const double qa = (double)((i64)x.P * hR) / cn, qb = (double)((i64)x.P * (hR - 1)) / cn;
                R4 rr;
#pragma unroll
                for (int i = 0; i < U; i++) {
                    if (i < size) {
                        if ((i & 1) == 0) rr = draw(I.seed, pa0, 0ull, spawn_step, 0u, (k0 + (u32)i) >> 1);
                        const u32 x0 = (i & 1) ? rr.z : rr.x, x1 = (i & 1) ? rr.w : rr.y;
                        double h;
                        int R;
                        d[i] = mom_draw31(I.mc, x, x0, x1, h, R, lut, tri);
                        v[i] = ((-(I.dtau * h)) * c) * (R == hR ? qa : qb);
                    }
                }
            } else {
                const MomCtx<T> x = mom_ctx<T>(I.mc, a);
                const int hR = mom_R(0, I.mc.M);
                const double qa = (double)((i64)x.P * hR) / cn, qb = (double)((i64)x.P * (hR - 1)) / cn;
                R4 rr;
#pragma unroll
                for (int i = 0; i < U; i++) {
                    if (i < size) {
                        if ((i & 1) == 0) rr = draw(I.seed, pa0, pa1, spawn_step, 0u, (k0 + (u32)i) >> 1);
                        const u32 x0 = (i & 1) ? rr.z : rr.x, x1 = (i & 1) ? rr.w : rr.y;
                        double h;
                        int R;
                        d[i] = mom_draw<T>(I.mc, x, x0, x1, h, R, lut);
                        v[i] = ((-(I.dtau * h)) * c) * (R == hR ? qa : qb);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < U; i++) {
                if (i < size) {
                    if (EARLY && fabs(v[i]) < I.theta) {
                        const u32 k = k0 + (u32)i;
                        const R4 rc = draw(I.seed, pa0, pa1, spawn_step, 4u + (k >> 28), k & 0x0fffffffu);
                        v[i] = compress1(v[i], I.theta, rc.x);
                    }
                    if (!EARLY || v[i] != 0.0) {
                        const int g = out.group(wide(d[i]));
                        gr[i] = (g << 16) | out.rank(g);
                    }
                }
            }
        }
        out.reserve();
#pragma unroll
        for (int i = 0; i < U; i++)
            if (gr[i] >= 0) out.put(gr[i] >> 16, gr[i] & 0xffff, wide(d[i]), v[i], pa0, pa1, k0 + (u32)i, ni);
    }
}

// ---------------------------------------------------------------- the step

#ifndef FQ_MERGE_MT
#define FQ_MERGE_MT 2  // table entries in flight per merge thread
#endif
#ifndef FQ_MERGE_MS
#define FQ_MERGE_MS 2  // spawn records in flight per merge thread (and per batch of LDS inserts)
#endif
#ifndef FQ_MERGE_PREFETCH
#define FQ_MERGE_PREFETCH 1  // load the next batch before inserting the current one
#endif

// Merge of bucket b for step n+1: the diagonal survivors of table[p] and the
// spawn records of slab[p] are summed per address in an LDS hash table, the
// sums are compressed, the projected-energy terms of the bucket's reference
// entries are accumulated, and the survivors are written to table[1-p]
// together with the bucket's partial statistics.
template <int W, int MODEL, int BS, bool EARLY>
__device__ void merge_bucket(const Inst &I, const int b, char *smem)
{
    typedef typename AddrOf<W>::T T;
    const int tid = threadIdx.x;
    Ctrl *ctrl = I.ctrl;
    const int slots = I.slots;
    __shared__ int s_err;

    // one memory round trip before the barrier: the halt state (thread 0),
    // the step parameters and the counts of both parities (the kernel that
    // ran before wrote them; nothing in this launch does)
    if (tid == 0) s_err = halted(ctrl);
    const i64 n = ctrl->step;
    const int p = ctrl->parity;
    const double S = ctrl->shift;
    const int tn0 = I.tab_n[0][b], tn1 = I.tab_n[1][b];
    const int sn0 = I.slab_n[0][b], sn1 = I.slab_n[1][b];
    const int r_beg = I.ref_off[b], r_end = I.ref_off[b + 1];  // this bucket's reference entries
    __syncthreads();
    if (s_err) return;

    // LDS carve-up
    Lds L;
    char *q = smem;
    L.k0 = (u64 *)q; q += (size_t)slots * 8;
    L.k1 = (u64 *)q; if (W == 2) q += (size_t)slots * 8;
    L.lo = (u64 *)q; q += (size_t)slots * 8;
    L.hi = (u64 *)q; q += (size_t)slots * 8;
    L.state = (u32 *)q; if (W == 2) q += (size_t)slots * 4;
    L.misc = (i64 *)q; q += 160 * 8;
    L.occ = (unsigned char *)q;  // slots bytes, present with the initiator rule only
    L.mask = slots - 1;
    const bool init = I.iflag != 0;

    const bool timing = (I.flags & 4) != 0;
    u64 tprev = timing ? wall_clock64() : 0;
    auto mark = [&](int ph) {
        if (timing && tid == 0) {
            u64 t = wall_clock64();
            atomicAdd((unsigned long long *)&ctrl->phase[ph], (unsigned long long)(t - tprev));
            tprev = t;
        }
    };
    const int out_par = 1 - p;
    // the address fits 32 bits (same for every lane; always for model variant 1)
    const bool narrow = MODEL == 1 || (W == 1 && I.mc.nb <= 32);
    const int spt = slots / BS;  // candidate slots per thread (contiguous), <= 8

    // candidate survivors of this thread: address words and value (0 = none)
    u64 r0[8], r1[8];
    double rc[8];
#pragma unroll
    for (int k = 0; k < 8; k++) { r0[k] = 0; r1[k] = 0; rc[k] = 0.0; }

    int used = 0;  // occupied LDS slots of this thread
    int inx = 0;   // some contribution of this thread was rounded to the fixed-point grid
    {
        // ------------------------------------------------ 1. merge
        int nprobe = 0;
        const int nt = p ? tn1 : tn0;
        const i64 tb = (i64)b * I.cap_t;
        const int ns = min(p ? sn1 : sn0, (int)I.cap_s);
        const char *sb = I.slab[p] + (i64)b * I.cap_s * (i64)I.rec;
        // Loads in flight per thread: the first MT table entries and the
        // first MS spawn records are requested before the LDS hash is
        // cleared, so their latency overlaps the clearing, and each later
        // batch is requested while the current one is inserted.
        constexpr int MT = FQ_MERGE_MT, MS = FQ_MERGE_MS;
        u64 x0[MS], x1[MS];
        double xv[MS];
#pragma unroll
        for (int e = 0; e < MS; e++) {
            const int i = e * BS + tid;
            if (i < ns) load_rec<W>(I.rec, sb, i, x0[e], x1[e], xv[e]);
        }
        u64 t0[MT], t1[MT];
        double tc[MT];
#pragma unroll
        for (int e = 0; e < MT; e++) {
            const int i = e * BS + tid;
            t0[e] = t1[e] = 0;
            tc[e] = 0.0;
            if (i < nt) {
                t0[e] = gmem(I.tab_a[p][0])[tb + i];
                t1[e] = W == 2 ? gmem(I.tab_a[p][1])[tb + i] : 0;
                tc[e] = gmem(I.tab_v[p])[tb + i];
            }
        }
        for (int s = tid; s < slots; s += BS) {
            L.k0[s] = EMPTY;
            if (W == 2) { L.k1[s] = EMPTY; L.state[s] = 0u; }
            L.lo[s] = 0;
            L.hi[s] = 0;
        }
        if (tid < 64) L.misc[tid] = 0;
        __syncthreads();
        mark(0);
        for (int i0 = 0; i0 < nt; i0 += MT * BS) {
            double tw[MT];
            bool tok[MT];
#pragma unroll
            for (int e = 0; e < MT; e++) {
                const int i = i0 + e * BS + tid;
                tw[e] = 0.0;
                tok[e] = false;
                if (i < nt) {
                    const T a = AddrOf<W>::make(t0[e], t1[e]);
                    double hii;
                    if (MODEL == 0 || MODEL == 3)
                        hii = narrow ? real_diag_runs<u32>(I.mc, (u32)t0[e]) : real_diag_runs(I.mc, a);
                    else hii = narrow ? mom_diag_modes<u32>(I.mc, (u32)t0[e]) : mom_diag_modes(I.mc, a);
                    const double g = 1.0 + I.dtau * (S - hii);
                    double w = tc[e] * g;
                    if (EARLY && fabs(w) < I.theta)
                        w = compress1(w, I.theta, draw(I.seed, t0[e], t1[e], (u32)(n + 1), 2u, 0u).x);
                    tw[e] = w;
                    // with the initiator rule every address of c^(n) enters
                    // the hash, even with a zero survivor: it is occupied
                    tok[e] = w != 0.0 || init;
                }
            }
            if (FQ_MERGE_PREFETCH) {
                // the next batch is in flight while this one is inserted
                u64 n0[MT], n1[MT];
#pragma unroll
                for (int e = 0; e < MT; e++) {
                    const int i = i0 + (MT + e) * BS + tid;
                    n0[e] = n1[e] = 0;
                    if (i < nt) {
                        n0[e] = gmem(I.tab_a[p][0])[tb + i];
                        n1[e] = W == 2 ? gmem(I.tab_a[p][1])[tb + i] : 0;
                        tc[e] = gmem(I.tab_v[p])[tb + i];
                    }
                }
                lds_add_n<W, MT>(L, I, t0, t1, tw, tok, b, nprobe, inx);
#pragma unroll
                for (int e = 0; e < MT; e++) {
                    t0[e] = n0[e];
                    t1[e] = n1[e];
                }
            } else {
                lds_add_n<W, MT>(L, I, t0, t1, tw, tok, b, nprobe, inx);
                // next batch
#pragma unroll
                for (int e = 0; e < MT; e++) {
                    const int i = i0 + (MT + e) * BS + tid;
                    if (i < nt) {
                        t0[e] = gmem(I.tab_a[p][0])[tb + i];
                        t1[e] = W == 2 ? gmem(I.tab_a[p][1])[tb + i] : 0;
                        tc[e] = gmem(I.tab_v[p])[tb + i];
                    }
                }
            }
        }
        if (timing) { __syncthreads(); mark(1); }
        if (init) {
            // the hash now holds exactly the addresses of c^(n)
            __syncthreads();
            for (int s = tid; s < slots; s += BS) L.occ[s] = (W == 1 ? L.k0[s] != EMPTY : L.state[s] == 2u) ? 1 : 0;
            __syncthreads();
        }
        for (int i0 = 0; i0 < ns; i0 += MS * BS) {
            bool xok[MS], xni[MS];
#pragma unroll
            for (int e = 0; e < MS; e++) {
                const bool in = i0 + e * BS + tid < ns;
                // records of non-initiator parents carry I.iflag (0 without the rule)
                const bool ni = in && ((W == 1 ? x0[e] : x1[e]) & I.iflag) != 0;
                if (W == 1) x0[e] &= ~I.iflag;
                else x1[e] &= ~I.iflag;
                xok[e] = in && !ni;
                xni[e] = ni;
            }
            if (FQ_MERGE_PREFETCH) {
                // the next batch is in flight while this one is inserted
                u64 y0[MS], y1[MS];
                double yv[MS];
#pragma unroll
                for (int e = 0; e < MS; e++) {
                    const int i = i0 + (MS + e) * BS + tid;
                    y0[e] = y1[e] = 0;
                    yv[e] = 0.0;
                    if (i < ns) load_rec<W>(I.rec, sb, i, y0[e], y1[e], yv[e]);
                }
                lds_add_n<W, MS>(L, I, x0, x1, xv, xok, b, nprobe, inx);
                if (init) lds_add_occupied<W, MS>(L, I, x0, x1, xv, xni, b, inx);
#pragma unroll
                for (int e = 0; e < MS; e++) {
                    x0[e] = y0[e];
                    x1[e] = y1[e];
                    xv[e] = yv[e];
                }
            } else {
                lds_add_n<W, MS>(L, I, x0, x1, xv, xok, b, nprobe, inx);
                if (init) lds_add_occupied<W, MS>(L, I, x0, x1, xv, xni, b, inx);
                // next batch
#pragma unroll
                for (int e = 0; e < MS; e++) {
                    const int i = i0 + (MS + e) * BS + tid;
                    if (i < ns) load_rec<W>(I.rec, sb, i, x0[e], x1[e], xv[e]);
                }
            }
        }
        __syncthreads();
        mark(2);
        if (timing) {
            i64 tp, ti;
            block_excl_scan<BS>((i64)nprobe, L.misc, tp);
            i64 mine_ins = (nt > tid ? (nt - tid + BS - 1) / BS : 0) + (ns > tid ? (ns - tid + BS - 1) / BS : 0);
            block_excl_scan<BS>(mine_ins, L.misc, ti);
            if (tid == 0) {
                atomicAdd((unsigned long long *)&ctrl->probes, (unsigned long long)tp);
                atomicAdd((unsigned long long *)&ctrl->inserts, (unsigned long long)ti);
            }
            mark(8);
        }

        // ------------------------------------------------ 2. compress (per slot, owner thread)
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (k >= spt) break;
            int s = tid * spt + k;
            u64 a0 = L.k0[s];
            u64 a1 = W == 2 ? L.k1[s] : 0;
            bool occ = W == 1 ? a0 != EMPTY : L.state[s] == 2u;
            double cn = 0.0;
            if (occ) {
                used++;
                double w = from_fixed(L.lo[s], L.hi[s]);
                if ((I.flags & 2) && dump_keeps(I.flags, addr_hash(AddrOf<W>::make(a0, a1)))) {
                    i64 di = atomicAdd((unsigned long long *)&ctrl->dump_merged_n, 1ull);
                    if (di < I.dump_cap) {
                        I.dmg_addr[di * W] = a0;
                        if (W == 2) I.dmg_addr[di * W + 1] = a1;
                        I.dmg_val[di] = w;
                    }
                }
                cn = w;
                if (!EARLY && w != 0.0 && fabs(w) < I.theta)
                    cn = compress1(w, I.theta, draw(I.seed, a0, a1, (u32)(n + 1), 1u, 0u).x);
            }
            r0[k] = a0;
            r1[k] = a1;
            rc[k] = cn;
        }
        // expose compressed values for the projected-energy lookups
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < spt) L.lo[tid * spt + k] = dbits(rc[k]);
        if (timing) __syncthreads();
        mark(3);
        // 128-bit accumulators: [40,41] norm, [42,43] y.Hc, [44,45] y.c;
        // [46] inexact flag of the bucket
        if (tid < 7) L.misc[40 + tid] = 0;
        __syncthreads();

        // ------------------------------------------------ 3. projected energy
        {
            for (int e = r_beg + tid; e < r_end; e += BS) {
                u64 a0 = gmem(I.ref_a[0])[e];
                u64 a1 = W == 2 ? gmem(I.ref_a[1])[e] : 0;
                int s = lds_find<W>(L, a0, a1, slot_hash(a0, W == 2 ? a1 : 0ull));
                double cv = s >= 0 ? bitsd(L.lo[s]) : 0.0;
                double term = I.yref * (gmem(I.ref_h)[e] * cv);
                u64 lo, hi;
                int ovf = 0;
                to_fixed(term, lo, hi, ovf, inx);
                lds_acc128((u64 *)&L.misc[42], (u64 *)&L.misc[43], lo, hi);
                if (e == I.ref_self) {
                    to_fixed(I.yref * cv, lo, hi, ovf, inx);
                    lds_acc128((u64 *)&L.misc[44], (u64 *)&L.misc[45], lo, hi);
                }
            }
        }
    }

    // ---------------------------------------------------- 4. compaction and partial statistics
    int mine = 0;
    u64 nlo = 0, nhi = 0;  // fixed-point partial norm
#pragma unroll
    for (int k = 0; k < 8; k++) {
        if (k < spt && rc[k] != 0.0) {
            mine++;
            u64 lo, hi;
            int ovf = 0;
            to_fixed(fabs(rc[k]), lo, hi, ovf, inx);
            add128(nlo, nhi, lo, hi);
        }
    }
    // one scan gives the compaction offsets (low half) and the number of
    // occupied slots (high half; the largest per bucket is reported)
    i64 packed;
    const i64 base = block_excl_scan<BS>((i64)mine | ((i64)used << 32), L.misc, packed) & 0xffffffffll;
    const i64 total = packed & 0xffffffffll, occupied = packed >> 32;
    if (total > I.cap_t) {
        if (tid == 0) set_error(ctrl, FQE_CAP_TABLE, b);
        return;
    }
    {
        const i64 ob = (i64)b * I.cap_t;
        int w = (int)base;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (k < spt && rc[k] != 0.0) {
                gmem(I.tab_a[out_par][0])[ob + w] = r0[k];
                if (W == 2) gmem(I.tab_a[out_par][1])[ob + w] = r1[k];
                gmem(I.tab_v[out_par])[ob + w] = rc[k];
                w++;
            }
        }
    }
    // exact wave reduction first: one LDS accumulation per wave instead of
    // one per thread on the same address
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const u64 x = __shfl_down(nlo, o, 64), y = __shfl_down(nhi, o, 64);
        add128(nlo, nhi, x, y);
    }
    if ((tid & 63) == 0 && (nlo | nhi)) lds_acc128((u64 *)&L.misc[40], (u64 *)&L.misc[41], nlo, nhi);
    if (__any(inx) && (tid & 63) == 0) atomicOr((unsigned long long *)&L.misc[46], 1ull);
    __syncthreads();
    if (tid == 0) {
        I.tab_n[out_par][b] = (int)total;
        Part pt;
        pt.norm[0] = (u64)L.misc[40];
        pt.norm[1] = (u64)L.misc[41];
        pt.hproj[0] = (u64)L.misc[42];
        pt.hproj[1] = (u64)L.misc[43];
        pt.vproj[0] = (u64)L.misc[44];
        pt.vproj[1] = (u64)L.misc[45];
        pt.len = total;
        pt.load = occupied;
        pt.inexact = L.misc[46];
        I.part[b] = pt;
    }
    mark(4);
}

// ---------------------------------------------------------------- spawn kernel

// Spawns of the entries of table[par] in bucket b for step spawn_step
// (mode 0: the table just produced by the merge; mode 1: a state that was
// set).  Per entry the attempt count is computed (m exact entries when
// |c| >= t_rel m, else ceil|c| picks); entries are ordered exact first by an
// index permutation so that waves run one kind of unit; units of 4 attempts
// are scanned and walked by spawn_units.
template <int W, int MODEL, int BS, bool EARLY>
__device__ void spawn_bucket(const Inst &I, const int b, const int mode, char *smem)
{
    typedef typename AddrOf<W>::T T;
    const int tid = threadIdx.x;
    Ctrl *ctrl = I.ctrl;
    __shared__ int s_err;
    // the halt state, the step parameters and both parities' table counts
    // in one memory round trip before the barrier
    if (tid == 0) s_err = halted(ctrl);
    const i64 n = ctrl->step;
    const int p = ctrl->parity;
    const int tn0 = I.tab_n[0][b], tn1 = I.tab_n[1][b];
    __syncthreads();
    if (s_err) return;
    // mode 0 runs after the merge of step n+1 (state in table[1-p]), mode 1 on c^(n)
    const int par = mode == 0 ? 1 - p : p;
    const u32 spawn_step = (u32)(mode == 0 ? n + 2 : n + 1);
    Lds L;
    L.misc = (i64 *)smem;
    const bool timing = (I.flags & 4) != 0;
    u64 tprev = timing ? wall_clock64() : 0;
    auto mark = [&](int ph) {
        if (timing && tid == 0) {
            u64 t = wall_clock64();
            atomicAdd((unsigned long long *)&ctrl->phase[ph], (unsigned long long)(t - tprev));
            tprev = t;
        }
    };
    // info[2 i] holds entry i's count word until the units are scanned, then
    // unit offsets in exact-first order; info[2 w + 1] the count word of the
    // w-th entry in that order and perm[w] its table index
    u32 *info = (u32 *)(smem + 160 * 8);
    u32 *perm = info + 2 * I.cap_t;
    unsigned char *lut = (unsigned char *)(perm + I.cap_t);  // select table, 2048 bytes
    for (int i = tid; i < 2048; i += BS) lut[i] = select_lut_entry(i);
    // then the coarse parent index of the exact parents and the pair table
    if (MODEL == 1 || MODEL == 2)
        tri_fill((unsigned short *)(lut + 2048 + sizeof(int) * SPAWN_COARSE), tid, BS);
    const int nS = par ? tn1 : tn0;
    const i64 tb = (i64)b * I.cap_t;
    const int chunk = (nS + BS - 1) / BS;
    const int i0 = min(nS, tid * chunk), i1 = min(nS, i0 + chunk);
    // order classes: 0 exact parents, then the stochastic parents by n mod U
    // descending (U = SPAWN_UNIT; class U - (n mod U) for n mod U > 0, class
    // U for n mod U = 0); ranks inside a class come from LDS counters (the
    // order inside a class does not matter)
    int *cls = (int *)(L.misc + 20);  // [0..8] counts, [9..18] offsets, [19..27] fill
    if (tid < 28) cls[tid] = 0;
    int bad = 0;
    // four entries at a time: their loads are in flight together
    for (int i = i0; i < i1; i += 4) {
        u64 e0[4], e1[4];
        double ec[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            e0[k] = e1[k] = 0;
            ec[k] = 0.0;
            if (i + k < i1) {
                e0[k] = gmem(I.tab_a[par][0])[tb + i + k];
                e1[k] = W == 2 ? gmem(I.tab_a[par][1])[tb + i + k] : 0;
                ec[k] = gmem(I.tab_v[par])[tb + i + k];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (i + k < i1) {
                u32 cnt;
                bool ex;
                spawn_info<W, MODEL>(I, AddrOf<W>::make(e0[k], e1[k]), ec[k], cnt, ex, bad);
                info[2 * (i + k)] = cnt | (ex ? 0x80000000u : 0u);
            }
        }
    }
    if (bad) set_error(ctrl, FQE_ATTEMPTS, b);
    __syncthreads();
    mark(5);
    auto cls_of = [](u32 cw) -> int {
        const u32 r = cw & (u32)(SPAWN_UNIT - 1);
        return (cw >> 31) ? 0 : (r ? 1 + (SPAWN_UNIT - 1) - (int)r : SPAWN_UNIT);
    };
    for (int i = i0; i < i1; i++) atomicAdd(&cls[cls_of(info[2 * i])], 1);
    __syncthreads();
    if (tid == 0) {
        int o = 0;
        for (int k = 0; k <= SPAWN_UNIT; k++) {
            cls[9 + k] = o;
            o += cls[k];
        }
        cls[9 + SPAWN_UNIT + 1] = o;
        L.misc[60] = 0;  // spawn records emitted by this bucket
        if (b == 0) ctrl->spawn_par = par;
    }
    __syncthreads();
    for (int i = i0; i < i1; i++) {
        const u32 ce = info[2 * i];
        const int k = cls_of(ce);
        const int w = cls[9 + k] + atomicAdd(&cls[19 + k], 1);
        perm[w] = (u32)i;
        info[2 * w + 1] = ce;
    }
    const int tot_e = cls[9 + 1];                  // exact parents: w < tot_e
    const int nP = cls[9 + SPAWN_UNIT] - tot_e;   // stochastic parents with a partial unit
    i64 sum_r = 0;
    for (int k = 1; k < SPAWN_UNIT; k++) sum_r += (i64)cls[k] * (SPAWN_UNIT - k);
    __syncthreads();
    // offsets in the new order: attempt offsets of the exact parents (low 32
    // bits) and full-unit offsets of the stochastic parents (high 32 bits)
    i64 packed;
    {
        i64 x = 0;
        for (int i = i0; i < i1; i++) {
            const u32 cw = info[2 * i + 1], cnt = cw & 0x7fffffffu;
            x += (cw >> 31) ? (i64)cnt : ((i64)(cnt / SPAWN_UNIT) << 32);
        }
        const i64 ab = block_excl_scan<BS>(x, L.misc, packed);
        u32 ae = (u32)ab, fu = (u32)(ab >> 32);
        for (int i = i0; i < i1; i++) {
            const u32 cw = info[2 * i + 1], cnt = cw & 0x7fffffffu;
            if (cw >> 31) { info[2 * i] = ae; ae += cnt; }
            else { info[2 * i] = fu; fu += cnt / SPAWN_UNIT; }
        }
    }
    const i64 A_ex = packed & 0xffffffffll, FU = packed >> 32;
    const i64 atot = A_ex + (i64)SPAWN_UNIT * FU + sum_r;
    if (atot >= ((i64)1 << 32) || A_ex >= ((i64)1 << 31)) {
        if (tid == 0) set_error(ctrl, FQE_CAP_SLAB, b);
        return;
    }
    // partial statistics: with late compression every attempt is a record;
    // early compression counts the records that survive it
    SpawnPart sp;
    sp.exact = tot_e;
    sp.inexact = nS - tot_e;
    sp.spawns = atot;
    sp.pad = 0;
    if (!EARLY && tid == 0) I.spart[spawn_step & 1][b] = sp;
    __syncthreads();
    mark(6);
    spawn_exact<W, MODEL, BS, EARLY>(I, L, b, par, spawn_step, tot_e, info, perm, A_ex, lut, (int *)(lut + 2048));
    spawn_units<W, MODEL, BS, EARLY>(I, L, b, par, spawn_step, tot_e, nS, nP, info, perm, FU, lut,
                                     (const unsigned short *)(lut + 2048 + sizeof(int) * SPAWN_COARSE));
    if (EARLY) {
        __syncthreads();
        if (tid == 0) {
            sp.spawns = L.misc[60];
            I.spart[spawn_step & 1][b] = sp;
        }
    }
    mark(7);
}

// ---------------------------------------------------------------- partition

// Second pass of the spawn partition: workgroup cs reads coarse sub-slab cs
// (group g = cs >> log2SUB) and splits it into the F = B/G <= 256 buckets of
// the group in rounds of RPT records per thread.  Each round takes ranks
// inside the destination buckets from LDS counters, reserves one run per
// bucket with one global atomic, and sorts the round's records by bucket in
// LDS, so that consecutive lanes store consecutive records of one run (whole
// cache lines instead of one scattered record per lane).  Releases the
// coarse sub-slab.
template <int W, int BS, int RPT, int FMAX> __device__ void partition_coarse(const Inst &I, const int cs)
{
    static_assert(BS >= FMAX && BS % 64 == 0, "the scan of the F <= FMAX counts needs FMAX threads");
    static_assert(FMAX == 256 || FMAX == 512, "groups of at most 256 or 512 buckets");
    typedef typename std::conditional<FMAX <= 256, unsigned char, unsigned short>::type Dst;
    constexpr int NRND = BS * RPT;  // records per round
    __shared__ int s_err;
    __shared__ int cnt[FMAX];       // per bucket of the group: count, then run start in the sorted round
    __shared__ int wsum[FMAX / 64];
    __shared__ i64 off[FMAX];       // reserved run start minus the run start in the sorted round
    __shared__ u64 st_a0[NRND];
    __shared__ u64 st_a1[W == 2 ? NRND : 1];
    __shared__ double st_v[NRND];
    __shared__ Dst st_d[NRND];
    Ctrl *ctrl = I.ctrl;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) s_err = halted(ctrl);
    __syncthreads();
    if (s_err) return;
    const int q = ctrl->spawn_par;
    const int g = cs >> I.log2SUB;
    const int log2F = I.log2B - I.log2G;
    const int F = 1 << log2F;  // <= FMAX (the host picks FMAX from B / G)
    const int n = min(I.coarse_n[cs], (int)I.cap_c);
    const char *src = I.coarse + (i64)cs * I.cap_c * (i64)I.rec;
    for (int r0 = 0; r0 < n; r0 += NRND) {
        if (tid < F) cnt[tid] = 0;
        __syncthreads();
        u64 a0[RPT], a1[RPT];
        double v[RPT];
        int lb[RPT], rk[RPT];
#pragma unroll
        for (int e = 0; e < RPT; e++) {
            const int i = r0 + e * BS + tid;
            lb[e] = -1;
            if (i < n) {
                load_rec<W>(I.rec, src, i, a0[e], a1[e], v[e]);
                // the bucket of the address without the non-initiator flag
                const typename AddrOf<W>::T a =
                    AddrOf<W>::make(W == 1 ? a0[e] & ~I.iflag : a0[e], W == 2 ? a1[e] & ~I.iflag : 0ull);
                lb[e] = (int)(bucket_index(a, I.log2B, I.mc.nb <= 32) & (u32)(F - 1));
            }
        }
#pragma unroll
        for (int e = 0; e < RPT; e++)
            if (lb[e] >= 0) rk[e] = atomicAdd(&cnt[lb[e]], 1);
        __syncthreads();
        // exclusive scan of the F counts (threads 0 .. F-1, at most FMAX / 64 waves)
        const int c = tid < F ? cnt[tid] : 0;
        int x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63 && wid < FMAX / 64) wsum[wid] = x;
        __syncthreads();
        if (tid < F) {
            int st = x - c;
            for (int w = 0; w < wid; w++) st += wsum[w];
            const i64 b0 = c ? (i64)gatomic_add(&I.slab_n[q][(g << log2F) + tid], c) : 0;
            off[tid] = b0 - st;
            cnt[tid] = st;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < RPT; e++) {
            if (lb[e] < 0) continue;
            const int j = cnt[lb[e]] + rk[e];
            st_a0[j] = a0[e];
            if (W == 2) st_a1[W == 2 ? j : 0] = a1[e];
            st_v[j] = v[e];
            st_d[j] = (Dst)lb[e];
        }
        __syncthreads();
        const int nr = min(NRND, n - r0);
        for (int j = tid; j < nr; j += BS) {
            const int d = st_d[j];
            const i64 pos = off[d] + j;
            const i64 dg = ((i64)g << log2F) + d;
            if (pos < I.cap_s)
                store_rec<W>(I.rec, I.slab[q], dg * I.cap_s + pos,
                             AddrOf<W>::make(st_a0[j], W == 2 ? st_a1[W == 2 ? j : 0] : 0ull), st_v[j]);
            else set_error(ctrl, FQE_CAP_SLAB, (int)dg);
        }
        __syncthreads();
    }
    if (tid == 0) I.coarse_n[cs] = 0;
}

// ---------------------------------------------------------------- finalize

// One workgroup: reduce the per-bucket partials of the step that just ran,
// update the shift (Eq. shift-update), write the statistics row, release the
// consumed spawn slab.  Exact integer reductions, so the result does not
// depend on the number of buckets.
template <int BS> __device__ void finalize_instance(const Inst &I)
{
    __shared__ u64 red[BS / 64][12];  // the 12th word: inexact flags
    __shared__ int s_err;
    Ctrl *ctrl = I.ctrl;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) s_err = halted(ctrl);
    __syncthreads();
    if (s_err) return;
    const i64 n = ctrl->step;
    const int p = ctrl->parity;
    const double S = ctrl->shift;
    u64 nl = 0, nh = 0, hl = 0, hh = 0, vl = 0, vh = 0;
    i64 len = 0, load = 0, ex = 0, in = 0, sp = 0, inx = 0;
    const SpawnPart *spp = I.spart[(n + 1) & 1];
    for (int b = tid; b < I.B; b += BS) {
        const Part pt = I.part[b];
        add128(nl, nh, pt.norm[0], pt.norm[1]);
        add128(hl, hh, pt.hproj[0], pt.hproj[1]);
        add128(vl, vh, pt.vproj[0], pt.vproj[1]);
        len += pt.len;
        load = max(load, pt.load);
        inx |= pt.inexact;
        const SpawnPart q = spp[b];
        ex += q.exact;
        in += q.inexact;
        sp += q.spawns;
    }
    // wave reduction (integer adds are exact and associative)
    for (int o = 32; o > 0; o >>= 1) {
        u64 x = __shfl_down(nl, o, 64), y = __shfl_down(nh, o, 64);
        add128(nl, nh, x, y);
        x = __shfl_down(hl, o, 64); y = __shfl_down(hh, o, 64);
        add128(hl, hh, x, y);
        x = __shfl_down(vl, o, 64); y = __shfl_down(vh, o, 64);
        add128(vl, vh, x, y);
        len += __shfl_down(len, o, 64);
        load = max(load, (i64)__shfl_down(load, o, 64));
        inx |= __shfl_down(inx, o, 64);
        ex += __shfl_down(ex, o, 64);
        in += __shfl_down(in, o, 64);
        sp += __shfl_down(sp, o, 64);
    }
    if (lane == 0) {
        red[wid][0] = nl; red[wid][1] = nh; red[wid][2] = hl; red[wid][3] = hh;
        red[wid][4] = vl; red[wid][5] = vh; red[wid][6] = (u64)len; red[wid][7] = (u64)load;
        red[wid][8] = (u64)ex; red[wid][9] = (u64)in; red[wid][10] = (u64)sp; red[wid][11] = (u64)inx;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < BS / 64; w++) {
            add128(nl, nh, red[w][0], red[w][1]);
            add128(hl, hh, red[w][2], red[w][3]);
            add128(vl, vh, red[w][4], red[w][5]);
            len += (i64)red[w][6];
            load = max(load, (i64)red[w][7]);
            ex += (i64)red[w][8];
            in += (i64)red[w][9];
            sp += (i64)red[w][10];
            inx |= (i64)red[w][11];
        }
        const double N1 = from_fixed(nl, nh);
        const double hp = from_fixed(hl, hh);
        const double vp = from_fixed(vl, vh);
        const double N0 = ctrl->norm;
        double S1 = S;
        if (N1 > 0.0) {
            const double za = I.zeta / I.dtau, xb = I.xi / I.dtau;
            S1 = (S - za * det_log(N1 / N0)) - xb * det_log(N1 / I.target);
        }
        if ((u32)load > ctrl->max_load) ctrl->max_load = (u32)load;
        inx |= ctrl->inexact_in ? 1 : 0;
        if (!(N1 < 17592186044416.0) || !(S1 == S1)) {
            set_error(ctrl, FQE_DIVERGED, -1);
            s_err = 1;
        } else {
            const i64 row = n + 1 - ctrl->ring_base;
            if (row >= 0 && row < I.ring_cap) {
                StepStats &R = I.ring[row];
                R.step = n + 1;
                R.len = len;
                R.exact_steps = ex;
                R.inexact_steps = in;
                R.spawns = sp;
                R.shift = S1;
                R.norm = N1;
                R.hproj = hp;
                R.vproj = vp;
                R.flags = inx ? ROW_INEXACT : 0;
            }
            ctrl->shift = S1;
            ctrl->norm = N1;
            ctrl->inexact_in = 0;
            if (inx && ctrl->first_inexact == 0) ctrl->first_inexact = n + 1;
            ctrl->step = n + 1;
            ctrl->parity = 1 - p;
        }
    }
    __syncthreads();
    if (s_err) return;
    for (int i = tid; i < I.B; i += BS) I.slab_n[p][i] = 0;  // consumed spawns
}

}  // namespace fq
