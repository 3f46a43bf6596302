// fq_step.hpp -- one FCIQMC step for one hash bucket, run by one workgroup.
//
// Data layout in HBM (per instance, two parities p = 0, 1):
//   table[p]: B buckets x cap_t entries, struct of arrays: address word 0,
//             address word 1 (W = 2), value (f64); count per bucket.
//   slab[p]:  B buckets x cap_s spawn records (array of structs: address
//             words + value, 16 B for W = 1, 24 B for W = 2); count per bucket.
// An address lives in bucket hash(address) >> (64 - log2 B).
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
//   5. spawn for step n+2 from every survivor: exact columns when
//      |c| >= t_rel m, else ceil|c| Philox picks; attempts are expanded over
//      the workgroup by a prefix sum over 4-attempt units and scattered to
//      the destination buckets of slab[1-p] (atomic slot allocation).
// The last workgroup to finish (completion counter) performs the shift
// update (Eq. shift-update), writes the statistics row and resets counters.
#pragma once
#include "fq_models.hpp"

namespace fq {

constexpr u64 EMPTY = ~0ull;
enum { FQE_CAP_TABLE = 1, FQE_CAP_SLAB = 2, FQE_CAP_LDS = 3, FQE_DIVERGED = 4, FQE_ATTEMPTS = 5,
       FQE_BARRIER = 6 };

struct StepStats {  // mirrors fq_step_stats
    i64 step, len, exact_steps, inexact_steps, spawns;
    double shift, norm, hproj, vproj;
};

struct Ctrl {
    i64 step;          // index n of the current state c^(n)
    int parity;        // parity holding c^(n) and its spawns
    int error;         // 0 or an FQE_* code
    double shift;      // S^(n)
    double norm;       // ||c^(n)||_1
    u32 pad1;
    u32 max_load;      // largest LDS hash occupancy seen
    i64 ring_base;     // step number stored in ring row 0
    u64 acc_norm[2];   // norm of a state being set (set_state only)
    i64 dump_spawn_n, dump_merged_n;
    i64 stop_step;     // batch: do not advance past this step
    int err_bucket, pad0;
    u64 phase[10];     // summed wall-clock ticks per phase (opt-in diagnostics)
    u64 probes;        // LDS hash probes summed over all inserts (diagnostics)
    u64 inserts;
};

// per-bucket partial statistics, written with plain stores by the workgroup
// that merges the bucket and reduced by the finalize kernel (no same-address
// atomics on the step's critical path)
struct Part {
    u64 norm[2], hproj[2], vproj[2];
    i64 len, load;
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
};

__device__ __forceinline__ void set_error(Ctrl *c, int code, int bucket)
{
    if (atomicCAS(&c->error, 0, code) == 0) c->err_bucket = bucket;
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

template <int W> __device__ __forceinline__ void store_rec(char *base, i64 i, typename AddrOf<W>::T d, double v);
template <> __device__ __forceinline__ void store_rec<1>(char *base, i64 i, u64 d, double v)
{
    Rec<1> *r = (Rec<1> *)base + i;
    ulonglong2 x;
    x.x = d;
    x.y = dbits(v);
    *(ulonglong2 *)r = x;
}
template <> __device__ __forceinline__ void store_rec<2>(char *base, i64 i, U128 d, double v)
{
    Rec<2> *r = (Rec<2> *)base + i;
    r->a0 = d.lo;
    r->a1 = d.hi;
    r->v = v;
}
template <int W> __device__ __forceinline__ void load_rec(const char *base, i64 i, u64 &a0, u64 &a1, double &v);
template <> __device__ __forceinline__ void load_rec<1>(const char *base, i64 i, u64 &a0, u64 &a1, double &v)
{
    ulonglong2 x = *((const ulonglong2 *)base + i);
    a0 = x.x;
    a1 = 0;
    v = bitsd(x.y);
}
template <> __device__ __forceinline__ void load_rec<2>(const char *base, i64 i, u64 &a0, u64 &a1, double &v)
{
    const Rec<2> *r = (const Rec<2> *)base + i;
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
    unsigned char *rows;
    int mask;
};

// find or insert the slot of address (a0, a1); returns -1 when full
template <int W> __device__ __forceinline__ int lds_slot(const Lds &L, u64 a0, u64 a1, u64 h, int &np)
{
    int s = (int)(h & (u64)L.mask);
    for (int probe = 0; probe <= L.mask; probe++) {
        np++;
        if (W == 1) {
            u64 k = __hip_atomic_load(&L.k0[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k == a0) return s;
            if (k == EMPTY) {
                u64 old = atomicCAS((unsigned long long *)&L.k0[s], EMPTY, a0);
                if (old == EMPTY || old == a0) return s;
            }
        } else {
            for (;;) {
                u32 st = __hip_atomic_load(&L.state[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (st == 2u) {
                    if (L.k0[s] == a0 && L.k1[s] == a1) return s;
                    break;
                }
                if (st == 0u) {
                    u32 old = atomicCAS(&L.state[s], 0u, 1u);
                    if (old == 0u) {
                        L.k0[s] = a0;
                        L.k1[s] = a1;
                        __hip_atomic_store(&L.state[s], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                        return s;
                    }
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

template <int W> __device__ __forceinline__ void lds_add(const Lds &L, const Inst &I, u64 a0, u64 a1,
                                                        double v, int b, int &np)
{
    typedef typename AddrOf<W>::T T;
    u64 h = addr_hash(AddrOf<W>::make(a0, a1));
    int s = lds_slot<W>(L, a0, a1, h, np);
    if (s < 0) { set_error(I.ctrl, FQE_CAP_LDS, b); return; }
    u64 lo, hi;
    int ovf = 0;
    to_fixed(v, lo, hi, ovf);
    if (ovf) { set_error(I.ctrl, FQE_DIVERGED, b); return; }
    lds_acc128(&L.lo[s], &L.hi[s], lo, hi);
    (void)sizeof(T);
}

// ---------------------------------------------------------------- spawn info

template <int W, int MODEL>
__device__ __forceinline__ void spawn_info(const Inst &I, typename AddrOf<W>::T a, double c,
                                           unsigned char *row, u32 &cnt, bool &exact, int &bad)
{
    i64 m;
    if (MODEL == 0) {
        m = 2 * popc(run_starts(a));
    } else {
        MomRow R = mom_row(row);
        mom_decode(I.mc, a, R);
        m = mom_m(R, I.mc.M);
    }
    double ac = fabs(c);
    exact = (m == 0) || ac >= I.t_rel * (double)m;
    if (exact) {
        cnt = (u32)m;
    } else {
        double n = ceil(ac);
        if (!(n <= 1073741824.0)) { bad = 1; n = 0.0; }
        cnt = (u32)n;
    }
}

// ---------------------------------------------------------------- the step

template <int W, int MODEL, int BS>
__device__ void process_bucket(const Inst &I, const int b, const int mode, char *smem)
{
    typedef typename AddrOf<W>::T T;
    const int tid = threadIdx.x;
    Ctrl *ctrl = I.ctrl;
    const int slots = I.slots;
    __shared__ int s_err;

    if (tid == 0) s_err = __hip_atomic_load(&ctrl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (s_err) return;

    const i64 n = ctrl->step;
    const int p = ctrl->parity;
    const double S = ctrl->shift;

    // LDS carve-up
    Lds L;
    char *q = smem;
    L.k0 = (u64 *)q; q += (size_t)slots * 8;
    L.k1 = (u64 *)q; if (W == 2) q += (size_t)slots * 8;
    L.lo = (u64 *)q; q += (size_t)slots * 8;
    L.hi = (u64 *)q; q += (size_t)slots * 8;
    L.state = (u32 *)q; if (W == 2) q += (size_t)slots * 4;
    L.misc = (i64 *)q; q += 64 * 8;
    L.rows = (unsigned char *)q;
    L.mask = slots - 1;
    unsigned char *myrow = L.rows + (size_t)tid * MOM_ROW;

    const bool timing = (I.flags & 4) != 0;
    u64 tprev = timing ? wall_clock64() : 0;
    auto mark = [&](int ph) {
        if (timing && tid == 0) {
            u64 t = wall_clock64();
            atomicAdd((unsigned long long *)&ctrl->phase[ph], (unsigned long long)(t - tprev));
            tprev = t;
        }
    };
    int nprobe = 0;
    const int out_par = mode == 0 ? 1 - p : p;
    const u32 spawn_step = (u32)(mode == 0 ? n + 2 : n + 1);
    int nS = 0;  // survivors held in LDS for the spawn phase

    if (mode == 0) {
        // ------------------------------------------------ 1. merge
        for (int s = tid; s < slots; s += BS) {
            L.k0[s] = EMPTY;
            if (W == 2) { L.k1[s] = EMPTY; L.state[s] = 0u; }
            L.lo[s] = 0;
            L.hi[s] = 0;
        }
        if (tid < 64) L.misc[tid] = 0;
        __syncthreads();
        mark(0);
        const int nt = I.tab_n[p][b];
        const i64 tb = (i64)b * I.cap_t;
        for (int i = tid; i < nt; i += BS) {
            u64 a0 = I.tab_a[p][0][tb + i];
            u64 a1 = W == 2 ? I.tab_a[p][1][tb + i] : 0;
            double c = I.tab_v[p][tb + i];
            T a = AddrOf<W>::make(a0, a1);
            double hii;
            if (MODEL == 0) hii = real_diag(I.mc, a);
            else { MomRow R = mom_row(myrow); mom_decode(I.mc, a, R); hii = mom_diag(I.mc, R); }
            double g = 1.0 + I.dtau * (S - hii);
            lds_add<W>(L, I, a0, a1, c * g, b, nprobe);
        }
        if (timing) { __syncthreads(); mark(1); }
        const int ns = min(I.slab_n[p][b], (int)I.cap_s);
        const char *sb = I.slab[p] + (i64)b * I.cap_s * (i64)sizeof(Rec<W>);
        for (int i = tid; i < ns; i += BS) {
            u64 a0, a1;
            double v;
            load_rec<W>(sb, i, a0, a1, v);
            lds_add<W>(L, I, a0, a1, v, b, nprobe);
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
        const int spt = slots / BS;  // slots per thread (contiguous), <= 8
        u64 r0[8], r1[8];
        double rc[8];
        int mine = 0, used = 0;
        u64 nlo = 0, nhi = 0;  // fixed-point partial norm
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
                if (I.flags & 2) {
                    i64 di = atomicAdd((unsigned long long *)&ctrl->dump_merged_n, 1ull);
                    if (di < I.dump_cap) {
                        I.dmg_addr[di * W] = a0;
                        if (W == 2) I.dmg_addr[di * W + 1] = a1;
                        I.dmg_val[di] = w;
                    }
                }
                double aw = fabs(w);
                if (aw >= I.theta) {
                    cn = w;
                } else if (aw > 0.0) {
                    R4 r = draw(I.seed, a0, a1, (u32)(n + 1), 1u, 0u);
                    double u = (double)r.x * 0x1p-32;
                    if (u * I.theta < aw) cn = w < 0.0 ? -I.theta : I.theta;
                }
            }
            r0[k] = a0;
            r1[k] = a1;
            rc[k] = cn;
            if (cn != 0.0) {
                mine++;
                u64 lo, hi;
                int ovf = 0;
                to_fixed(fabs(cn), lo, hi, ovf);
                add128(nlo, nhi, lo, hi);
            }
        }
        mark(3);
        // expose compressed values for the projected-energy lookups
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < spt) L.lo[tid * spt + k] = dbits(rc[k]);
        __syncthreads();

        // ------------------------------------------------ 3. projected energy
        if (tid == 0) { L.misc[42] = 0; L.misc[43] = 0; L.misc[44] = 0; L.misc[45] = 0; }
        __syncthreads();
        {
            const int r_beg = I.ref_off[b], r_end = I.ref_off[b + 1];
            for (int e = r_beg + tid; e < r_end; e += BS) {
                u64 a0 = I.ref_a[0][e];
                u64 a1 = W == 2 ? I.ref_a[1][e] : 0;
                u64 h = addr_hash(AddrOf<W>::make(a0, a1));
                int s = lds_find<W>(L, a0, a1, h);
                double cv = s >= 0 ? bitsd(L.lo[s]) : 0.0;
                double term = I.yref * (I.ref_h[e] * cv);
                u64 lo, hi;
                int ovf = 0;
                to_fixed(term, lo, hi, ovf);
                lds_acc128((u64 *)&L.misc[42], (u64 *)&L.misc[43], lo, hi);
                if (e == I.ref_self) {
                    to_fixed(I.yref * cv, lo, hi, ovf);
                    lds_acc128((u64 *)&L.misc[44], (u64 *)&L.misc[45], lo, hi);
                }
            }
        }
        // occupancy statistic (largest number of distinct addresses in a bucket)
        {
            i64 tot;
            i64 u = block_excl_scan<BS>(used, L.misc, tot);
            (void)u;
            if (tid == 0) L.misc[46] = tot;
        }
        // ------------------------------------------------ 4. compact
        i64 total;
        i64 base = block_excl_scan<BS>(mine, L.misc, total);
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
                    L.k0[w] = r0[k];
                    if (W == 2) L.k1[w] = r1[k];
                    L.lo[w] = dbits(rc[k]);
                    I.tab_a[out_par][0][ob + w] = r0[k];
                    if (W == 2) I.tab_a[out_par][1][ob + w] = r1[k];
                    I.tab_v[out_par][ob + w] = rc[k];
                    w++;
                }
            }
        }
        // block totals of len and norm
        if (tid == 0) { L.misc[40] = 0; L.misc[41] = 0; }
        __syncthreads();
        if (nlo | nhi) lds_acc128((u64 *)&L.misc[40], (u64 *)&L.misc[41], nlo, nhi);
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
            pt.load = L.misc[46];
            I.part[b] = pt;
        }
        nS = (int)total;
        mark(4);
    } else {
        // spawn-only pass: survivors are the stored entries of table[p]
        nS = I.tab_n[p][b];
        const i64 tb = (i64)b * I.cap_t;
        for (int i = tid; i < nS; i += BS) {
            L.k0[i] = I.tab_a[p][0][tb + i];
            if (W == 2) L.k1[i] = I.tab_a[p][1][tb + i];
            L.lo[i] = dbits(I.tab_v[p][tb + i]);
        }
        if (tid < 64) L.misc[tid] = 0;
    }
    __syncthreads();

    // ---------------------------------------------------- 5. spawn
    {
        // per-survivor attempt counts -> 4-attempt units, scanned
        const int chunk = (nS + BS - 1) / BS;
        const int i0 = min(nS, tid * chunk), i1 = min(nS, i0 + chunk);
        i64 units = 0, nex = 0, nin = 0, nsp = 0;
        int bad = 0;
        u32 *info = (u32 *)L.hi;  // [2 i] = unit offset, [2 i + 1] = count | exact << 31
        for (int i = i0; i < i1; i++) {
            T a = AddrOf<W>::make(L.k0[i], W == 2 ? L.k1[i] : 0);
            double c = bitsd(L.lo[i]);
            u32 cnt;
            bool ex;
            spawn_info<W, MODEL>(I, a, c, myrow, cnt, ex, bad);
            info[2 * i + 1] = cnt | (ex ? 0x80000000u : 0u);
            units += (cnt + 3) / 4;
            nsp += cnt;
            if (ex) nex++; else nin++;
        }
        if (bad) set_error(ctrl, FQE_ATTEMPTS, b);
        mark(5);
        i64 utot;
        i64 ubase = block_excl_scan<BS>(units, L.misc, utot);
        for (int i = i0; i < i1; i++) {
            info[2 * i] = (u32)ubase;
            ubase += ((info[2 * i + 1] & 0x7fffffffu) + 3) / 4;
        }
        // spawn statistics belong to row spawn_step (parents of c^(spawn_step - 1))
        {
            i64 t_ex, t_in, t_sp;
            block_excl_scan<BS>(nex, L.misc, t_ex);
            block_excl_scan<BS>(nin, L.misc, t_in);
            block_excl_scan<BS>(nsp, L.misc, t_sp);
            if (tid == 0) {
                SpawnPart sp;
                sp.exact = t_ex;
                sp.inexact = t_in;
                sp.spawns = t_sp;
                sp.pad = 0;
                I.spart[spawn_step & 1][b] = sp;
            }
        }

        mark(6);
        char *ob = I.slab[out_par];
        int *on = I.slab_n[out_par];
        const double dtau = I.dtau;
        for (i64 j = tid; j < utot; j += BS) {
            // parent: largest i with offset[i] <= j
            int lo_i = 0, hi_i = nS - 1;
            while (lo_i < hi_i) {
                int mid = (lo_i + hi_i + 1) >> 1;
                if ((i64)info[2 * mid] <= j) lo_i = mid; else hi_i = mid - 1;
            }
            const int i = lo_i;
            const u32 inf = info[2 * i + 1];
            const u32 cnt = inf & 0x7fffffffu;
            const bool ex = inf >> 31;
            const u32 qu = (u32)(j - (i64)info[2 * i]);
            const u64 a0 = L.k0[i], a1 = W == 2 ? L.k1[i] : 0;
            const T a = AddrOf<W>::make(a0, a1);
            const double c = bitsd(L.lo[i]);
            const u32 k0 = 4 * qu, k1 = min(cnt, k0 + 4);
            // scatter one spawn record to its destination bucket
            auto emit = [&](const T &dd, double vv, u32 k) {
                const u64 hh = addr_hash(dd);
                const u32 db = bucket_of(hh, I.log2B);
                const int pos = atomicAdd(&on[db], 1);
                if (pos < I.cap_s) store_rec<W>(ob, (i64)db * I.cap_s + pos, dd, vv);
                else set_error(ctrl, FQE_CAP_SLAB, (int)db);
                if (I.flags & 1) {
                    i64 di = atomicAdd((unsigned long long *)&ctrl->dump_spawn_n, 1ull);
                    if (di < I.dump_cap) {
                        I.dsp_parent[di * W] = a0;
                        if (W == 2) I.dsp_parent[di * W + 1] = a1;
                        I.dsp_attempt[di] = (i64)k;
                        I.dsp_dest[di * W] = word0(dd);
                        if (W == 2) I.dsp_dest[di * W + 1] = word1(dd);
                        I.dsp_val[di] = vv;
                    }
                }
            };
            if (MODEL == 0) {
                const T st = run_starts(a);
                const int o = popc(st);
                const u32 m = 2 * o;
                R4 r = {0, 0, 0, 0};
                double qd = 0.0;
                if (!ex) {
                    r = draw(I.seed, a0, a1, spawn_step, 0u, qu);
                    qd = (double)m / (double)cnt;
                }
                for (u32 k = k0; k < k1; k++) {
                    int idx = ex ? (int)k : (int)pick(rword(r, (int)(k - k0)), m);
                    double h;
                    T dd = real_entry(I.mc, a, st, o, idx, h);
                    double vv = (-(dtau * h)) * c;
                    if (!ex) vv = vv * qd;
                    emit(dd, vv, k);
                }
            } else {
                MomRow R = mom_row(myrow);
                mom_decode(I.mc, a, R);
                const int P = mom_npairs(R);
                R4 r = {0, 0, 0, 0};
                for (u32 k = k0; k < k1; k++) {
                    int pp, qq, di;
                    double h;
                    if (ex) {
                        mom_entry(R, I.mc.M, (i64)k, pp, qq, di);
                        T dd = mom_move(I.mc, a, R, pp, qq, di, h);
                        emit(dd, (-(dtau * h)) * c, k);
                    } else {
                        if ((k & 1u) == 0u || k == k0) r = draw(I.seed, a0, a1, spawn_step, 0u, k >> 1);
                        u32 w0 = rword(r, 2 * (int)(k & 1u)), w1 = rword(r, 2 * (int)(k & 1u) + 1);
                        mom_pair(R, (int)pick(w0, (u32)P), pp, qq);
                        const int Rk = mom_R((pp + qq) % I.mc.M, I.mc.M);
                        di = (int)pick(w1, (u32)Rk);
                        T dd = mom_move(I.mc, a, R, pp, qq, di, h);
                        const double qn = (double)((i64)P * Rk) / (double)cnt;
                        emit(dd, ((-(dtau * h)) * c) * qn, k);
                    }
                }
            }
        }
    }
    if (timing) { __syncthreads(); mark(7); }
}

// ---------------------------------------------------------------- finalize

// One workgroup: reduce the per-bucket partials of the step that just ran,
// update the shift (Eq. shift-update), write the statistics row, release the
// consumed spawn slab.  Exact integer reductions, so the result does not
// depend on the number of buckets.
template <int BS> __device__ void finalize_instance(const Inst &I)
{
    __shared__ u64 red[BS / 64][12];
    __shared__ int s_err;
    Ctrl *ctrl = I.ctrl;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) s_err = __hip_atomic_load(&ctrl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (s_err) return;
    const i64 n = ctrl->step;
    const int p = ctrl->parity;
    const double S = ctrl->shift;
    u64 nl = 0, nh = 0, hl = 0, hh = 0, vl = 0, vh = 0;
    i64 len = 0, load = 0, ex = 0, in = 0, sp = 0;
    const SpawnPart *spp = I.spart[(n + 1) & 1];
    for (int b = tid; b < I.B; b += BS) {
        const Part pt = I.part[b];
        add128(nl, nh, pt.norm[0], pt.norm[1]);
        add128(hl, hh, pt.hproj[0], pt.hproj[1]);
        add128(vl, vh, pt.vproj[0], pt.vproj[1]);
        len += pt.len;
        load = max(load, pt.load);
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
        ex += __shfl_down(ex, o, 64);
        in += __shfl_down(in, o, 64);
        sp += __shfl_down(sp, o, 64);
    }
    if (lane == 0) {
        red[wid][0] = nl; red[wid][1] = nh; red[wid][2] = hl; red[wid][3] = hh;
        red[wid][4] = vl; red[wid][5] = vh; red[wid][6] = (u64)len; red[wid][7] = (u64)load;
        red[wid][8] = (u64)ex; red[wid][9] = (u64)in; red[wid][10] = (u64)sp;
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
            }
            ctrl->shift = S1;
            ctrl->norm = N1;
            ctrl->step = n + 1;
            ctrl->parity = 1 - p;
        }
    }
    __syncthreads();
    if (s_err) return;
    for (int i = tid; i < I.B; i += BS) I.slab_n[p][i] = 0;  // consumed spawns
}

}  // namespace fq
