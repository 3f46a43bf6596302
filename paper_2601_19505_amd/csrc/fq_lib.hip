// fq_lib.hip -- kernels and host runtime behind the C ABI of include/fciqmc.h.
//
// One step is four launches on the caller's stream with no host
// synchronisation between them: k_merge (one workgroup per bucket:
// annihilation, compression, projected energy, compaction into the other
// table), k_spawn (one workgroup per bucket: spawn records of the new table
// for the next step), k_part (second pass of the spawn partition, only when
// there are more than 64 buckets) and k_finalize (one workgroup: exact
// reduction of the per-bucket partial sums and the shift update).  The host
// synchronises only at the end of a chunk of steps, to copy the statistics
// rows and check the error word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>

#include "fciqmc.h"
#include "fq_kernels.hpp"
#include "fq_overlap.hpp"
#include "fq_step.hpp"

using namespace fq;

// ------------------------------------------------------------------ kernels
//
// The merge and spawn kernels (fq_kernels.hpp) are instantiated in
// fq_inst.hip, one translation unit per (W, model variant).

FQ_EXTERN_STEP_KERNELS

// one workgroup per instance
#ifndef FQ_FIN_BS
#define FQ_FIN_BS 256
#endif
constexpr int FIN_BS = FQ_FIN_BS;  // threads of the finalize workgroup
__global__ __launch_bounds__(FIN_BS) void k_finalize(const Inst *const *insts)
{
    finalize_instance<FIN_BS>(const_inst(insts[blockIdx.x]));
}

// Second partition pass; map entry = instance << 14 | coarse sub-slab.  The
// host orders the entries so that all sub-slabs of one coarse group run on
// the same XCD (workgroups are dispatched round-robin over the 8 XCDs): the
// runs that different workgroups append to one bucket's slab then meet in
// that XCD's L2, which merges partial cache lines before they are written
// back.
// Threads per workgroup and records per thread and round, by address words
// (measured at both benchmark sizes: 1024 x 3 records per round is faster
// than 2048 or 4096 per round, and than other shapes of 3072).
#ifndef FQ_PART1_BS
#define FQ_PART1_BS 1024
#endif
#ifndef FQ_PART1_RPT
#define FQ_PART1_RPT 3
#endif
#ifndef FQ_PART2_BS
#define FQ_PART2_BS 1024
#endif
#ifndef FQ_PART2_RPT
#define FQ_PART2_RPT 3
#endif
template <int W> struct PartShape;
template <> struct PartShape<1> { static constexpr int BS = FQ_PART1_BS, RPT = FQ_PART1_RPT; };
template <> struct PartShape<2> { static constexpr int BS = FQ_PART2_BS, RPT = FQ_PART2_RPT; };

// FMAX: the most buckets per coarse group the workgroup splits into (256, or
// 512 with more than 16384 buckets)
template <int W, int FMAX>
__global__ __launch_bounds__(PartShape<W>::BS) void k_part(const Inst *const *insts, const u32 *map)
{
    const u32 m = map[blockIdx.x];
    partition_coarse<W, PartShape<W>::BS, PartShape<W>::RPT, FMAX>(const_inst(insts[m >> 14]),
                                                                   (int)(m & 0x3fffu));
}

// start of a chunk of steps: statistics rows are stored from row 0
__global__ void k_begin_chunk(const Inst *const *insts, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        Ctrl *c = insts[i]->ctrl;
        c->ring_base = c->step + 1;
    }
}

// every instance stops after `steps` more steps
__global__ void k_set_stop(const Inst *const *insts, int n, i64 steps)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        Ctrl *c = insts[i]->ctrl;
        c->stop_step = c->step + steps;
    }
}

// copy the control blocks of n instances into one array
__global__ void k_gather_ctrl(const Inst *const *insts, int n, Ctrl *out)
{
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const u32 *src = (const u32 *)insts[i]->ctrl;
        u32 *dst = (u32 *)(out + i);
        for (int k = threadIdx.x; k < (int)(sizeof(Ctrl) / 4); k += blockDim.x) dst[k] = src[k];
    }
}

// replica overlaps: workgroup A * B + b joins bucket b of replica A with the
// same bucket of every replica after A; then one workgroup sums the buckets
constexpr int OV_BS = 256;
template <int W> __global__ __launch_bounds__(OV_BS) void k_overlap(Overlap O)
{
    extern __shared__ __align__(16) char smem[];
    overlap_bucket<W, OV_BS>(O, (int)blockIdx.x / O.B, (int)blockIdx.x % O.B, smem);
}
__global__ __launch_bounds__(1024) void k_overlap_fin(Overlap O) { overlap_finalize<1024>(O); }
// excited states: Gram-Schmidt projection of run k against run j, per bucket
template <int W> __global__ __launch_bounds__(OV_BS) void k_gs_dot(Spectral S, int j, int k)
{
    extern __shared__ __align__(16) char smem[];
    gs_dot<W, OV_BS>(S, j, k, (int)blockIdx.x, smem);
}
__global__ __launch_bounds__(1024) void k_gs_alpha(Spectral S, int j, int k) { gs_alpha<1024>(S, j, k); }
template <int W> __global__ __launch_bounds__(OV_BS) void k_gs_update(Spectral S, int j, int k)
{
    extern __shared__ __align__(16) char smem[];
    gs_update<W, OV_BS>(S, j, k, (int)blockIdx.x, smem);
}
// one workgroup per projected run k = 1 .. R-1
__global__ __launch_bounds__(1024) void k_gs_norm(Spectral S) { gs_norm<1024>(S, (int)blockIdx.x + 1); }
__global__ void k_fill_i32(int *p, int n, int v)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// insert host-staged entries into table[parity] and accumulate the norm
template <int W>
__global__ __launch_bounds__(256) void k_insert(const Inst *Ip, const u64 *sa, const double *sv, i64 n)
{
    const Inst &I = *Ip;
    Ctrl *ctrl = I.ctrl;
    const int p = ctrl->parity;
    __shared__ u64 acc[2];
    if (threadIdx.x == 0) acc[0] = acc[1] = 0;
    __syncthreads();
    u64 nlo = 0, nhi = 0;
    int inx = 0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        u64 a0 = sa[i * W], a1 = W == 2 ? sa[i * W + 1] : 0;
        double v = sv[i];
        u32 b = bucket_index(AddrOf<W>::make(a0, a1), I.log2B, I.mc.nb <= 32);
        int pos = atomicAdd(&I.tab_n[p][b], 1);
        if (pos >= I.cap_t) { set_error(ctrl, FQE_CAP_TABLE, (int)b); continue; }
        i64 o = (i64)b * I.cap_t + pos;
        I.tab_a[p][0][o] = a0;
        if (W == 2) I.tab_a[p][1][o] = a1;
        I.tab_v[p][o] = v;
        u64 lo, hi;
        int ovf = 0;
        to_fixed(fabs(v), lo, hi, ovf, inx);
        if (ovf) set_error(ctrl, FQE_DIVERGED, (int)b);
        add128(nlo, nhi, lo, hi);
    }
    if (inx) atomicOr(&ctrl->inexact_in, 1u);
    if (nlo | nhi) lds_acc128(&acc[0], &acc[1], nlo, nhi);
    __syncthreads();
    if (threadIdx.x == 0 && (acc[0] | acc[1])) glb_acc128(ctrl->acc_norm, acc[0], acc[1]);
}

// finish set_state: norm of the inserted vector -> ctrl->norm
__global__ void k_take_norm(const Inst *Ip)
{
    Ctrl *c = Ip->ctrl;
    c->norm = from_fixed(c->acc_norm[0], c->acc_norm[1]);
    c->acc_norm[0] = c->acc_norm[1] = 0;
}

// row of the reference address over its column's destinations: entry 0 is
// the diagonal, then the off-diagonal entries in column order (equal to the
// column's values unless importance sampling makes H asymmetric); bucket of
// every destination
template <int W, int MODEL>
__global__ void k_ref(const Inst *Ip, u64 r0, u64 r1, u64 *oa, double *oh, int *ob, int *on, int cap)
{
    const Inst &I = *Ip;
    typedef typename AddrOf<W>::T T;
    __shared__ unsigned char lut[2048];
    for (int i = threadIdx.x; i < 2048; i += blockDim.x) lut[i] = select_lut_entry(i);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const T a = AddrOf<W>::make(r0, r1);
    const T st = run_starts(a);
    const int o = popc(st);
    double hd;
    i64 m;
    if (MODEL == 0 || MODEL == 3) {
        hd = real_diag_runs(I.mc, a);
        m = (MODEL == 0 ? 2 : I.mc.ndir) * o;
    } else {
        hd = mom_diag_modes(I.mc, a);
        m = mom_col_size(I.mc, a);
    }
    if (m + 1 > cap) { *on = -1; return; }
    oa[0] = r0;
    oa[1] = r1;
    oh[0] = hd;
    ob[0] = (int)bucket_index(a, I.log2B, I.mc.nb <= 32);
    for (i64 e = 0; e < m; e++) {
        double h;
        T d;
        if (MODEL == 0) {
            d = real_entry(I.mc, a, st, o, (int)e, h);
        } else if (MODEL == 3) {
            // the row of the reference: the inverse importance-sampling factor
            int kd;
            d = lat_entry(I.mc, a, st, o, (int)e, h, kd, lut);
            h = h * I.mc.gz[I.mc.N - kd];
        } else {
            d = mom_column_entry(I.mc, a, (int)e, h, lut);
        }
        oa[2 * (e + 1)] = word0(d);
        oa[2 * (e + 1) + 1] = word1(d);
        oh[e + 1] = h;
        ob[e + 1] = (int)bucket_index(d, I.log2B, I.mc.nb <= 32);
    }
    *on = (int)m + 1;
}

// copy table[parity] into contiguous arrays
template <int W>
__global__ __launch_bounds__(256) void k_pack(const Inst *Ip, u64 *oa, double *ov, unsigned long long *cnt)
{
    const Inst &I = *Ip;
    const int p = I.ctrl->parity;
    for (int b = blockIdx.x; b < I.B; b += gridDim.x) {
        const int nb = I.tab_n[p][b];
        __shared__ unsigned long long base;
        if (threadIdx.x == 0) base = nb ? atomicAdd(cnt, (unsigned long long)nb) : 0ull;
        __syncthreads();
        for (int i = threadIdx.x; i < nb; i += blockDim.x) {
            i64 s = (i64)b * I.cap_t + i, d = (i64)base + i;
            oa[d * W] = I.tab_a[p][0][s];
            if (W == 2) oa[d * W + 1] = I.tab_a[p][1][s];
            ov[d] = I.tab_v[p][s];
        }
        __syncthreads();
    }
}

__global__ void k_set_i64(i64 *p, i64 v) { *p = v; }

// ------------------------------------------------------------------ host side

namespace {

constexpr i64 RING = 4096;
constexpr int MAX_BUCKETS = 32768;  // 15 bits of a workgroup map entry
constexpr int NEV = 5;  // timing events per step: merge | spawn | partition | finalize
constexpr int REFCAP = 1 << 15;

template <int W, int MODEL, bool E>
const void *pick_bs(int bs, bool spawn)
{
    switch (bs) {
    case 256: return spawn ? (const void *)k_spawn<W, MODEL, 256, E> : (const void *)k_merge<W, MODEL, 256, E>;
    case 512: return spawn ? (const void *)k_spawn<W, MODEL, 512, E> : (const void *)k_merge<W, MODEL, 512, E>;
    default: return spawn ? (const void *)k_spawn<W, MODEL, 1024, E> : (const void *)k_merge<W, MODEL, 1024, E>;
    }
}
template <int W, int MODEL>
const void *pick_kernel(int bs, bool spawn, bool early)
{
    return early ? pick_bs<W, MODEL, true>(bs, spawn) : pick_bs<W, MODEL, false>(bs, spawn);
}

// kernel variant: 0 real-space ring, 1 momentum space with addresses of one
// word and at most 31 bits (N + M - 1 <= 31), 2 other momentum space, 3
// lattice (the square lattice, or the ring with importance sampling); plus 4
// with early compression
int variant(int model, int M, int N, int W, double g, int flags)
{
    const int base = model == FQ_MOM1D ? ((W == 1 && N + M - 1 <= 31) ? 1 : 2)
                                       : (model == FQ_REAL2D || g != 0.0) ? 3 : 0;
    return base + ((flags & FQ_FLAG_EARLY_COMPRESSION) ? 4 : 0);
}

template <int W> const void *step_kernel_w(int m, int bs, bool spawn, bool e)
{
    switch (m) {
    case 0: return pick_kernel<W, 0>(bs, spawn, e);
    case 1: return pick_kernel<W, 1>(bs, spawn, e);
    case 2: return pick_kernel<W, 2>(bs, spawn, e);
    default: return pick_kernel<W, 3>(bs, spawn, e);
    }
}

const void *step_kernel(int W, int var, int bs, bool spawn)
{
    const bool e = var >= 4;
    const int m = var % 4;
    return W == 1 ? step_kernel_w<1>(m, bs, spawn, e) : step_kernel_w<2>(m, bs, spawn, e);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int ilog2(i64 x)
{
    int r = 0;
    while (((i64)1 << r) < x) r++;
    return r;
}

// bytes per spawn record (see store_rec)
// nb address bits, plus the non-initiator flag bit with the initiator rule
size_t rec_bytes(int W, int nb, bool init) { return W == 2 ? 24 : (nb + (init ? 1 : 0) <= 32 ? 12 : 16); }

// The non-initiator flag of a spawn record: the top bit of the last address
// word as stored (bit 31 of a 12-byte record, bit 63 otherwise), above every
// address bit; 0 without the initiator rule.
u64 initiator_flag_bit(bool init, int rec) { return !init ? 0ull : rec == 12 ? (1ull << 31) : (1ull << 63); }

// merge kernel: the LDS hash table (keys, 128-bit accumulators, W = 2 slot
// states), the scratch words and, with the initiator rule, one occupancy
// byte per slot
size_t lds_bytes(int W, int slots, bool init)
{
    size_t per = 8 + (W == 2 ? 8 : 0) + 8 + 8 + (W == 2 ? 4 : 0) + (init ? 1 : 0);
    return (size_t)slots * per + 160 * 8;
}

// spawn kernel: three 32-bit words per table entry (unit offset, count word,
// permutation), the scratch words, the 2048-byte select table, the coarse
// parent index of the exact parents and the pair table of the momentum draw
size_t lds_spawn_bytes(i64 cap_t) { return (size_t)cap_t * 12 + 160 * 8 + 2048 + sizeof(int) * SPAWN_COARSE + 2 * TRI_N; }

constexpr size_t LDS_MAX = 160 * 1024;
static_assert(sizeof(Ctrl) % 4 == 0, "Ctrl is copied in 32-bit words");
static_assert(sizeof(StepStats) == sizeof(fq_step_stats), "StepStats mirrors fq_step_stats");

// A set of instances stepped together: one launch per kernel per step.
struct Exec {
    int W = 1, var = 0, block = 512, spawn_block = 256;
    size_t lds_m = 0, lds_s = 0;  // dynamic LDS of the merge and spawn kernels
    int n = 0;                    // instances
    const Inst *const *insts = nullptr;
    const u32 *map = nullptr;     // merge / spawn workgroup map (nullptr: one instance)
    int grid = 0;
    const u32 *pmap = nullptr;    // second-pass partition map
    int pgrid = 0;
    bool wide_groups = false;     // coarse groups of more than 256 buckets
};

struct Resolved {
    int W, nb, B, log2B, slots, block, spawn_block, two_pass, log2G, log2SUB;
    bool init;  // the initiator rule
    i64 cap_t, cap_s, cap_c, dump_cap;
    size_t rec, slab_bytes;  // bytes per spawn record; bytes of one slab
    size_t off_ctrl, off_inst, off_iptr, off_pmap, off_sq, off_eps, off_nbr, off_gz, off_ref_a, off_ref_h, off_ref_b, off_ref_off, off_ref_tmp, off_ring,
        off_tab_a[2][2], off_tab_v[2], off_tab_n[2], off_slab[2], off_slab_n[2], off_dsp_parent,
        off_dsp_attempt, off_dsp_dest, off_dsp_val, off_dmg_addr, off_dmg_val, off_part, off_spart[2], off_coarse,
        off_coarse_n, total;
    int nsq;
};

// Upper bound on the spectral width E_max - E_0 of the Hamiltonian, from
// Weyl's inequality applied to H = T + V: the hopping term T of N bosons has
// its spectrum in [-z t N, z t N] (the one-boson hopping matrix has z
// entries of size t per row, z = 2 on the ring, 4 on the square lattice;
// momentum space is the ring in another basis), and V = (u/2) sum n(n-1) has
// its spectrum between 0 and (u/2) N (N - 1).  Importance sampling is a
// similarity transformation and keeps the spectrum.
double spectral_width_bound(const fq_hamiltonian *h)
{
    const double z = h->model == FQ_REAL2D ? 4.0 : 2.0;
    const double N = h->N;
    return std::fabs(h->u) * 0.5 * N * (N - 1.0) + 2.0 * z * std::fabs(h->t) * N;
}

int validate(const fq_hamiltonian *h, const fq_params *p, std::string &err)
{
    if (!h || !p) { err = "null argument"; return FQ_EINVAL; }
    if (h->model != FQ_REAL1D && h->model != FQ_MOM1D && h->model != FQ_REAL2D) { err = "unknown model"; return FQ_EINVAL; }
    if (h->M < 2 || h->N < 1) { err = "need M >= 2 and N >= 1"; return FQ_EINVAL; }
    if (h->model == FQ_MOM1D && (h->M < 3 || h->M > MOM_MAXM)) { err = "momentum model needs 3 <= M <= 32"; return FQ_EINVAL; }
    if (h->model == FQ_REAL2D && (h->lx < 2 || h->M % h->lx != 0 || h->M / h->lx < 2)) {
        err = "square lattice needs lx >= 2 and M / lx >= 2 rows of lx sites";
        return FQ_EINVAL;
    }
    if (!std::isfinite(h->g) || (h->model == FQ_MOM1D && h->g != 0.0)) {
        err = "g must be finite, and 0 for the momentum model";
        return FQ_EINVAL;
    }
    if (p->addr_words != 1 && p->addr_words != 2) { err = "addr_words must be 1 or 2"; return FQ_EINVAL; }
    int nb = h->N + h->M - 1;
    if (nb > (p->addr_words == 1 ? 62 : 126)) { err = "N+M-1 too large for addr_words"; return FQ_EINVAL; }
    if (!(p->dtau > 0) || !(p->target_walkers > 0) || !(p->threshold > 0) || !(p->t_rel >= 0) ||
        !(p->zeta >= 0) || !(p->xi >= 0) || !std::isfinite(p->dtau) || !std::isfinite(p->target_walkers) ||
        !std::isfinite(p->threshold) || !std::isfinite(p->zeta) || !std::isfinite(p->xi)) {
        err = "dtau, target_walkers, threshold must be finite and > 0; t_rel >= 0; zeta, xi finite and >= 0";
        return FQ_EINVAL;
    }
    if (!std::isfinite(h->t) || !std::isfinite(h->u)) { err = "t and u must be finite"; return FQ_EINVAL; }
    if ((p->flags & FQ_FLAG_INITIATOR) && !(p->initiator_threshold >= 0.0)) {
        err = "initiator_threshold must be >= 0 (not NaN) with FQ_FLAG_INITIATOR";
        return FQ_EINVAL;
    }
    // Stability of the projector (Sec. 3.1): dtau < 2 / (E_max - E_0).
    const double width = spectral_width_bound(h);
    if (!(p->flags & FQ_FLAG_UNCHECKED_DTAU) && !(p->dtau * width < 2.0)) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "dtau = %.6g violates the stability bound dtau < 2 / (E_max - E_0) = %.6g (spectral width "
                 "at most %.6g); FQ_FLAG_UNCHECKED_DTAU skips this check",
                 p->dtau, 2.0 / width, width);
        err = msg;
        return FQ_EINVAL;
    }
    return FQ_OK;
}

int resolve(const fq_hamiltonian *h, const fq_params *p, const fq_layout *lin, Resolved &R, fq_layout &lout,
            std::string &err)
{
    int rc = validate(h, p, err);
    if (rc) return rc;
    if (!lin || lin->table_capacity < 1 || lin->spawn_capacity < 1) {
        err = "layout capacities must be >= 1";
        return FQ_EINVAL;
    }
    fq_layout L = *lin;
    L.spawn_capacity = std::max(L.spawn_capacity, L.table_capacity);
    R.W = p->addr_words;
    R.nb = h->N + h->M - 1;
    R.init = (p->flags & FQ_FLAG_INITIATOR) != 0;
    if (L.lds_slots == 0) L.lds_slots = 4096;
    if (L.lds_slots < 1024 || L.lds_slots > 8192 || (L.lds_slots & (L.lds_slots - 1))) {
        err = "lds_slots must be a power of two in [1024, 8192]";
        return FQ_EINVAL;
    }
    if (L.block == 0) L.block = h->model == FQ_MOM1D ? 512 : 1024;
    if (L.block != 256 && L.block != 512 && L.block != 1024) { err = "block must be 256, 512 or 1024"; return FQ_EINVAL; }
    if (L.lds_slots > 8 * L.block) { err = "lds_slots must be <= 8 * block"; return FQ_EINVAL; }
    if (L.spawn_block == 0) L.spawn_block = 256;
    if (L.spawn_block != 256 && L.spawn_block != 512 && L.spawn_block != 1024) {
        err = "spawn_block must be 256, 512 or 1024";
        return FQ_EINVAL;
    }
    if (lds_bytes(R.W, L.lds_slots, R.init) > LDS_MAX) { err = "LDS budget exceeded: lower lds_slots or block"; return FQ_EINVAL; }
    if (L.buckets == 0) {
        double uniq = (double)L.table_capacity + 0.25 * (double)L.spawn_capacity;
        i64 b = (i64)std::ceil(uniq / (0.55 * L.lds_slots));
        L.buckets = (int)((i64)1 << ilog2(std::min<i64>(std::max<i64>(b, 1), MAX_BUCKETS)));
    }
    if (L.buckets < 1 || (L.buckets & (L.buckets - 1)) || L.buckets > MAX_BUCKETS) {
        err = "buckets must be a power of two <= 32768";
        return FQ_EINVAL;
    }
    R.B = L.buckets;
    R.log2B = ilog2(R.B);
    R.slots = L.lds_slots;
    R.block = L.block;
    R.spawn_block = L.spawn_block;
    auto cap = [](double mean) {
        double c = mean + 8.0 * std::sqrt(mean) + 64.0;
        return (i64)std::ceil(c);
    };
    R.cap_t = std::min<i64>(cap((double)L.table_capacity / R.B), R.slots);
    R.cap_s = cap((double)L.spawn_capacity / R.B);
    // spawn partition: one pass into the buckets for B <= 64, otherwise G
    // coarse groups (B/G <= 256 buckets each) with 64 sub-slabs per group
    R.two_pass = R.B > 64;
    R.log2G = R.two_pass ? std::min(6, std::max(4, R.log2B - 8)) : R.log2B;
    R.log2SUB = 6;
    R.cap_c = R.two_pass ? cap((double)L.spawn_capacity / (double)((i64)1 << (R.log2G + R.log2SUB))) + 256 : 1;
    {
        // sampled dumps keep about 2^-k of the events; twice that plus slack
        const int k = (p->flags >> 8) & 31;
        const i64 all = L.spawn_capacity + L.table_capacity;
        R.dump_cap = (p->flags & (FQ_FLAG_DUMP_SPAWNS | FQ_FLAG_DUMP_MERGED)) ? (k ? 2 * (all >> k) + 65536 : all) : 0;
    }
    R.nsq = (h->N + 2) * (h->N + 2) + 8;
    // a slab also stages a whole table (8W + 8 bytes per entry) for
    // set_state, get_state and copy_state
    R.rec = rec_bytes(R.W, R.nb, R.init);
    R.slab_bytes = std::max(R.rec * (size_t)R.B * R.cap_s, (size_t)(8 * R.W + 8) * (size_t)R.B * R.cap_t + 256);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    R.off_ctrl = take(sizeof(Ctrl));
    R.off_inst = take(sizeof(Inst));
    R.off_iptr = take(sizeof(Inst *));
    R.off_pmap = take(sizeof(u32) << (R.log2G + R.log2SUB));
    R.off_sq = take(sizeof(double) * R.nsq);
    R.off_eps = take(sizeof(double) * MOM_MAXM);
    R.off_nbr = take(4 * (size_t)h->M);
    R.off_gz = take(sizeof(double) * (2 * (size_t)h->N + 1));
    R.off_ref_a = take(sizeof(u64) * 2 * REFCAP);
    R.off_ref_h = take(sizeof(double) * REFCAP);
    R.off_ref_b = take(sizeof(int) * REFCAP);
    R.off_ref_off = take(sizeof(int) * (R.B + 1));
    R.off_ref_tmp = take((sizeof(u64) * 2 + sizeof(double) + sizeof(int)) * REFCAP + 64);
    R.off_ring = take(sizeof(StepStats) * RING);
    R.off_part = take(sizeof(Part) * R.B);
    R.off_spart[0] = take(sizeof(SpawnPart) * R.B);
    R.off_spart[1] = take(sizeof(SpawnPart) * R.B);
    const i64 tn = (i64)R.B * R.cap_t;
    for (int q = 0; q < 2; q++) {
        R.off_tab_a[q][0] = take(sizeof(u64) * tn);
        R.off_tab_a[q][1] = R.W == 2 ? take(sizeof(u64) * tn) : 0;
        R.off_tab_v[q] = take(sizeof(double) * tn);
        R.off_tab_n[q] = take(sizeof(int) * R.B);
        R.off_slab[q] = take(R.slab_bytes);
        R.off_slab_n[q] = take(sizeof(int) * R.B);
    }
    R.off_coarse = take(R.rec * (size_t)R.cap_c << (R.log2G + R.log2SUB));
    R.off_coarse_n = take(sizeof(int) << (R.log2G + R.log2SUB));
    const i64 dc = std::max<i64>(R.dump_cap, 1);
    R.off_dsp_parent = take(sizeof(u64) * R.W * dc);
    R.off_dsp_attempt = take(sizeof(i64) * dc);
    R.off_dsp_dest = take(sizeof(u64) * R.W * dc);
    R.off_dsp_val = take(sizeof(double) * dc);
    R.off_dmg_addr = take(sizeof(u64) * R.W * dc);
    R.off_dmg_val = take(sizeof(double) * dc);
    R.total = o;
    lout = L;
    return FQ_OK;
}

// The dynamic-LDS limit is a property of the kernel, shared by every handle
// in the process: only ever raise it, to the largest size any handle needs.
hipError_t ensure_lds(const void *kf, size_t bytes)
{
    static std::mutex mu;
    static std::map<const void *, size_t> limit;
    std::lock_guard<std::mutex> lock(mu);
    size_t &cur = limit[kf];
    if (bytes <= cur) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) cur = bytes;
    return e;
}

// Entries of the second-pass map for instance `inst` whose first workgroup
// is a multiple of 8: local workgroup x runs on XCD x mod 8 and takes coarse
// group ((x / 8) / 64) * 8 + x mod 8, sub-slab (x / 8) mod 64, so the 64
// sub-slabs of a group share one XCD.  Needs at least 8 groups.
void append_pmap(const Resolved &R, u32 inst, std::vector<u32> &out)
{
    if (!R.two_pass) return;
    const int nblk = 1 << (R.log2G + R.log2SUB);
    for (int x = 0; x < nblk; x++) {
        const int xcd = x & 7, j = x >> 3;
        const int g = ((j >> R.log2SUB) << 3) | xcd;
        const int sub = j & ((1 << R.log2SUB) - 1);
        out.push_back((inst << 14) | (u32)((g << R.log2SUB) | sub));
    }
}

hipError_t launch_spawn(const Exec &X, int mode, hipStream_t s, hipEvent_t mid = nullptr)
{
    const void *kf = step_kernel(X.W, X.var, X.spawn_block, true);
    void *args[] = {(void *)&X.insts, (void *)&X.map, (void *)&mode};
    hipError_t e = hipLaunchKernel(kf, dim3(X.grid), dim3(X.spawn_block), args, X.lds_s, s);
    if (e == hipSuccess && mid) e = hipEventRecord(mid, s);
    if (e == hipSuccess && X.pgrid > 0) {
        // groups of more than 256 buckets (more than 16384 buckets in all)
        // take the kernel with the larger count arrays
        if (X.W == 1) {
            if (X.wide_groups) hipLaunchKernelGGL((k_part<1, 512>), dim3(X.pgrid), dim3(PartShape<1>::BS), 0, s, X.insts, X.pmap);
            else hipLaunchKernelGGL((k_part<1, 256>), dim3(X.pgrid), dim3(PartShape<1>::BS), 0, s, X.insts, X.pmap);
        } else {
            if (X.wide_groups) hipLaunchKernelGGL((k_part<2, 512>), dim3(X.pgrid), dim3(PartShape<2>::BS), 0, s, X.insts, X.pmap);
            else hipLaunchKernelGGL((k_part<2, 256>), dim3(X.pgrid), dim3(PartShape<2>::BS), 0, s, X.insts, X.pmap);
        }
        e = hipGetLastError();
    }
    return e;
}

// Excited-state runs: the Gram-Schmidt launches inside every step (all
// instances of the group are the runs).
struct GsRun {
    Spectral S;
    int W = 1;
    size_t lds_dot = 0, lds_upd = 0;
};

size_t gs_dot_lds(int W, int slots) { return (size_t)(2 * slots) * (W == 2 ? 28 : 16) + sizeof(Fx3) * (OV_BS / 64); }
size_t gs_upd_lds(int W, int slots)
{
    return (size_t)(2 * slots) * (W == 2 ? 28 : 16) + sizeof(Fx3) * (OV_BS / 64) + sizeof(i64) * (OV_BS / 64 + 1);
}

hipError_t launch_gs_projections(const GsRun &g, hipStream_t s)
{
    Spectral S = g.S;
    const void *kd = g.W == 1 ? (const void *)k_gs_dot<1> : (const void *)k_gs_dot<2>;
    const void *ku = g.W == 1 ? (const void *)k_gs_update<1> : (const void *)k_gs_update<2>;
    hipError_t e = hipSuccess;
    for (int k = 1; k < S.R && e == hipSuccess; k++) {
        for (int j = 0; j < k && e == hipSuccess; j++) {
            void *args[] = {(void *)&S, (void *)&j, (void *)&k};
            e = hipLaunchKernel(kd, dim3(S.B), dim3(OV_BS), args, g.lds_dot, s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_gs_alpha, dim3(1), dim3(1024), 0, s, S, j, k);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipLaunchKernel(ku, dim3(S.B), dim3(OV_BS), args, g.lds_upd, s);
        }
    }
    return e;
}

// one step of every instance of X: merge, spawn, second partition pass,
// finalize; with `ev`, NEV events: before the merge and after each of the
// four kernels.  With gs, the Gram-Schmidt projections run between the merge
// and the spawn kernel, and the orthogonalised norms are set after the
// finalize kernel.
hipError_t exec_step(const Exec &X, hipStream_t s, hipEvent_t *ev, const GsRun *gs = nullptr)
{
    hipError_t e = hipSuccess;
    if (ev) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) {
        const void *kf = step_kernel(X.W, X.var, X.block, false);
        void *args[] = {(void *)&X.insts, (void *)&X.map};
        e = hipLaunchKernel(kf, dim3(X.grid), dim3(X.block), args, X.lds_m, s);
    }
    if (ev && e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess && gs) e = launch_gs_projections(*gs, s);
    if (e == hipSuccess) e = launch_spawn(X, 0, s, ev ? ev[2] : nullptr);
    if (ev && e == hipSuccess) e = hipEventRecord(ev[3], s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_finalize, dim3(X.n), dim3(FIN_BS), 0, s, X.insts);
        e = hipGetLastError();
    }
    if (e == hipSuccess && gs) {
        hipLaunchKernelGGL(k_gs_norm, dim3(gs->S.R - 1), dim3(1024), 0, s, gs->S);
        e = hipGetLastError();
    }
    if (ev && e == hipSuccess) e = hipEventRecord(ev[4], s);
    return e;
}

}  // namespace

struct fq_handle {
    fq_hamiltonian h;
    fq_params p;
    fq_layout L;
    Resolved R;
    char *ws;
    Inst inst;      // host copy
    Inst *d_inst;
    Ctrl *d_ctrl;
    Exec X;         // this instance alone
    uint64_t ref[2];
    double yref;
    int have_state;
    i64 step;
    int parity;
    std::string err;
    int timing;
    double time_ms[NEV - 1];
    i64 launches;
    std::vector<hipEvent_t> ev;
    std::vector<StepStats> ring_host;
    std::vector<int> ref_bucket_host;
};

static thread_local std::string g_err;  // errors of calls that have no handle yet

static int hip_fail(fq_handle *q, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (q) q->err = m;
    g_err = m;
    return FQ_EHIP;
}

#define HIPCHK(q, call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(q, e_, #call); \
    } while (0)

static int read_ctrl(fq_handle *q, Ctrl &c, hipStream_t s);
static int load_state(fq_handle *q, const u64 *sa, const double *sv, i64 n, double shift, i64 step,
                      const uint64_t *ref_addr, double ref_val, hipStream_t s);

// text of fq_last_error after a successful run in which some sum was not
// exactly rounded (its rows carry FQ_ROW_INEXACT)
static std::string inexact_note(i64 step)
{
    return "note: from step " + std::to_string(step) +
           " on, some sums were not exactly rounded: a contribution below 2^-27 was rounded to a "
           "multiple of 2^-80 (rows flagged FQ_ROW_INEXACT)";
}

static const char *fqe_name(int e)
{
    switch (e) {
    case FQE_CAP_TABLE: return "table bucket capacity exceeded";
    case FQE_CAP_SLAB: return "spawn slab capacity exceeded";
    case FQE_CAP_LDS: return "LDS hash of a bucket is full (use more buckets or lds_slots)";
    case FQE_DIVERGED: return "walker number diverged or became non-finite";
    case FQE_ATTEMPTS: return "too many spawn attempts from one address (more than 2^29 in momentum space, 2^30 otherwise)";
    case FQE_BARRIER: return "grid barrier timed out";
    default: return "unknown device error";
    }
}

static int fqe_status(int e)
{
    switch (e) {
    case FQE_DIVERGED: return FQ_EDIVERGED;
    case FQE_ATTEMPTS: return FQ_EINVAL;
    case FQE_BARRIER: return FQ_EHIP;
    default: return FQ_ECAPACITY;
    }
}

extern "C" {

const char *fq_version(void) { return "fciqmc-mi355x 0.1 (gfx950)"; }

int fq_encode(const int32_t *occ, int32_t M, int32_t W, uint64_t *out)
{
    if (!occ || !out || M < 1 || (W != 1 && W != 2)) return FQ_EINVAL;
    uint64_t w[2] = {0, 0};
    int pos = 0;
    for (int j = 0; j < M; j++) {
        if (occ[j] < 0) return FQ_EINVAL;
        for (int r = 0; r < occ[j]; r++) {
            if (pos >= 64 * W) return FQ_EINVAL;
            w[pos >> 6] |= 1ull << (pos & 63);
            pos++;
        }
        if (j < M - 1) pos++;
    }
    if (pos > 64 * W) return FQ_EINVAL;
    for (int i = 0; i < W; i++) out[i] = w[i];
    return FQ_OK;
}

int fq_workspace_size(const fq_hamiltonian *h, const fq_params *p, const fq_layout *layout, size_t *bytes,
                      fq_layout *layout_out)
{
    Resolved R;
    fq_layout L;
    std::string err;
    int rc = resolve(h, p, layout, R, L, err);
    if (rc) { g_err = err; return rc; }
    if (bytes) *bytes = R.total;
    if (layout_out) *layout_out = L;
    return FQ_OK;
}

int fq_create(const fq_hamiltonian *h, const fq_params *p, const fq_layout *layout, void *workspace, size_t bytes,
              fq_handle **out)
{
    if (!out) return FQ_EINVAL;
    *out = nullptr;
    fq_handle *q = new (std::nothrow) fq_handle();
    if (!q) return FQ_ENOMEM;
    int rc = resolve(h, p, layout, q->R, q->L, q->err);
    if (rc) { g_err = q->err; delete q; return rc; }
    if (!workspace || bytes < q->R.total || ((uintptr_t)workspace & 255)) {
        delete q;
        return workspace ? FQ_ENOMEM : FQ_EINVAL;
    }
    q->h = *h;
    q->p = *p;
    q->ws = (char *)workspace;
    const Resolved &R = q->R;
    Inst &I = q->inst;
    memset(&I, 0, sizeof I);
    I.mc.M = h->M;
    I.mc.N = h->N;
    I.mc.nb = R.nb;
    I.mc.t = h->t;
    I.mc.u = h->u;
    I.mc.coef = h->u / (2.0 * (double)h->M);
    I.mc.sq = (const double *)(q->ws + R.off_sq);
    I.mc.eps = (const double *)(q->ws + R.off_eps);
    I.mc.ndir = h->model == FQ_REAL2D ? 4 : 2;
    I.mc.nbr = (const unsigned char *)(q->ws + R.off_nbr);
    I.mc.gz = (const double *)(q->ws + R.off_gz);
    I.model = h->model;
    I.W = R.W;
    I.dtau = p->dtau;
    I.target = p->target_walkers;
    I.zeta = p->zeta;
    I.xi = p->xi;
    I.theta = p->threshold;
    I.t_rel = p->t_rel;
    I.seed = p->seed;
    I.log2B = R.log2B;
    I.B = R.B;
    I.slots = R.slots;
    I.flags = p->flags;
    I.cap_t = R.cap_t;
    I.cap_s = R.cap_s;
    for (int k = 0; k < 2; k++) {
        I.tab_a[k][0] = (u64 *)(q->ws + R.off_tab_a[k][0]);
        I.tab_a[k][1] = R.W == 2 ? (u64 *)(q->ws + R.off_tab_a[k][1]) : nullptr;
        I.tab_v[k] = (double *)(q->ws + R.off_tab_v[k]);
        I.tab_n[k] = (int *)(q->ws + R.off_tab_n[k]);
        I.slab[k] = q->ws + R.off_slab[k];
        I.slab_n[k] = (int *)(q->ws + R.off_slab_n[k]);
    }
    I.ref_a[0] = (u64 *)(q->ws + R.off_ref_a);
    I.ref_a[1] = I.ref_a[0] + REFCAP;
    I.ref_h = (double *)(q->ws + R.off_ref_h);
    I.ref_off = (int *)(q->ws + R.off_ref_off);
    I.ctrl = (Ctrl *)(q->ws + R.off_ctrl);
    I.ring = (StepStats *)(q->ws + R.off_ring);
    I.ring_cap = RING;
    I.dsp_parent = (u64 *)(q->ws + R.off_dsp_parent);
    I.dsp_attempt = (i64 *)(q->ws + R.off_dsp_attempt);
    I.dsp_dest = (u64 *)(q->ws + R.off_dsp_dest);
    I.dsp_val = (double *)(q->ws + R.off_dsp_val);
    I.dmg_addr = (u64 *)(q->ws + R.off_dmg_addr);
    I.dmg_val = (double *)(q->ws + R.off_dmg_val);
    I.dump_cap = R.dump_cap;
    I.part = (Part *)(q->ws + R.off_part);
    I.two_pass = R.two_pass;
    I.log2G = R.log2G;
    I.log2SUB = R.log2SUB;
    I.cap_c = R.cap_c;
    I.rec = (int)R.rec;
    I.iflag = initiator_flag_bit(R.init, I.rec);
    I.n_a = R.init ? p->initiator_threshold : 0.0;
    I.coarse = q->ws + R.off_coarse;
    I.coarse_n = (int *)(q->ws + R.off_coarse_n);
    I.spart[0] = (SpawnPart *)(q->ws + R.off_spart[0]);
    I.spart[1] = (SpawnPart *)(q->ws + R.off_spart[1]);
    q->d_inst = (Inst *)(q->ws + R.off_inst);
    q->d_ctrl = I.ctrl;
    // host tables: correctly rounded square roots and the momentum dispersion
    std::vector<double> sq(R.nsq), eps(MOM_MAXM, 0.0);
    for (int k = 0; k < R.nsq; k++) sq[k] = std::sqrt((double)k);
    for (int j = 0; j < h->M && j < MOM_MAXM; j++)
        eps[j] = (-2.0 * h->t) * std::cos((2.0 * 3.14159265358979323846 * (double)j) / (double)h->M);
    const void *km = step_kernel(R.W, variant(h->model, h->M, h->N, R.W, h->g, p->flags), R.block, false);
    const void *ks = step_kernel(R.W, variant(h->model, h->M, h->N, R.W, h->g, p->flags), R.spawn_block, true);
    // lattice neighbours (sites x + lx y; +x, -x, +y, -y) and the
    // importance-sampling factors gz[N + k] = exp(-(g u) k), k = -N .. N
    const int lx = h->model == FQ_REAL2D ? h->lx : h->M, ly = h->M / lx;
    std::vector<unsigned char> nbr(4 * (size_t)h->M, 0);
    for (int site = 0; site < h->M; site++) {
        const int x = site % lx, y = site / lx;
        nbr[0 * h->M + site] = (unsigned char)((x + 1) % lx + lx * y);
        nbr[1 * h->M + site] = (unsigned char)((x + lx - 1) % lx + lx * y);
        nbr[2 * h->M + site] = (unsigned char)(x + lx * ((y + 1) % ly));
        nbr[3 * h->M + site] = (unsigned char)(x + lx * ((y + ly - 1) % ly));
    }
    std::vector<double> gz(2 * (size_t)h->N + 1, 1.0);
    if (h->g != 0.0)
        for (int k = -h->N; k <= h->N; k++) gz[h->N + k] = std::exp(-((h->g * h->u) * (double)k));
    hipError_t e = hipMemcpy(q->ws + R.off_sq, sq.data(), sizeof(double) * R.nsq, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(q->ws + R.off_eps, eps.data(), sizeof(double) * MOM_MAXM, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(q->ws + R.off_nbr, nbr.data(), nbr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(q->ws + R.off_gz, gz.data(), sizeof(double) * gz.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(q->d_inst, &I, sizeof(Inst), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(q->ws + R.off_ctrl, 0, sizeof(Ctrl));
    const Inst *iptr = q->d_inst;
    if (e == hipSuccess) e = hipMemcpy(q->ws + R.off_iptr, &iptr, sizeof iptr, hipMemcpyHostToDevice);
    std::vector<u32> pm;
    append_pmap(R, 0, pm);
    if (e == hipSuccess && !pm.empty())
        e = hipMemcpy(q->ws + R.off_pmap, pm.data(), sizeof(u32) * pm.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) { hip_fail(q, e, "fq_create: workspace initialisation"); delete q; return FQ_EHIP; }
    e = ensure_lds(km, lds_bytes(R.W, R.slots, R.init));
    if (e == hipSuccess) e = ensure_lds(ks, lds_spawn_bytes(R.cap_t));
    if (e != hipSuccess) { hip_fail(q, e, "fq_create: hipFuncSetAttribute(step kernels)"); delete q; return FQ_EHIP; }
    Exec &X = q->X;
    X.W = R.W;
    X.var = variant(h->model, h->M, h->N, R.W, h->g, p->flags);
    X.block = R.block;
    X.spawn_block = R.spawn_block;
    X.lds_m = lds_bytes(R.W, R.slots, R.init);
    X.lds_s = lds_spawn_bytes(R.cap_t);
    X.n = 1;
    X.insts = (const Inst *const *)(q->ws + R.off_iptr);
    X.map = nullptr;
    X.grid = R.B;
    X.pmap = (const u32 *)(q->ws + R.off_pmap);
    X.pgrid = (int)pm.size();
    X.wide_groups = R.two_pass && R.log2B - R.log2G > 8;
    q->ring_host.resize(RING);
    *out = q;
    return FQ_OK;
}

int fq_destroy(fq_handle *q)
{
    if (!q) return FQ_EINVAL;
    for (auto e : q->ev) (void)hipEventDestroy(e);
    delete q;
    return FQ_OK;
}

const char *fq_last_error(const fq_handle *q) { return q ? q->err.c_str() : g_err.c_str(); }

int fq_debug_counters(fq_handle *q, double *out, int32_t n, int32_t reset, void *stream)
{
    if (!q || !out || n < 13) return FQ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Ctrl c;
    int rc = read_ctrl(q, c, s);
    if (rc) return rc;
    int rate = 0;
    HIPCHK(q, hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, 0));
    for (int k = 0; k < 10; k++) out[k] = rate > 0 ? (double)c.phase[k] / ((double)rate * 1e3) * 1e3 : 0.0;  // ms
    out[10] = (double)c.probes;
    out[11] = (double)c.inserts;
    out[12] = (double)c.max_load;
    if (reset) {
        Ctrl z = c;
        memset(z.phase, 0, sizeof z.phase);
        z.probes = z.inserts = 0;
        z.max_load = 0;
        HIPCHK(q, hipMemcpyAsync(&q->d_ctrl->phase, &z.phase, sizeof z.phase, hipMemcpyHostToDevice, s));
        HIPCHK(q, hipMemcpyAsync(&q->d_ctrl->probes, &z.probes, 16, hipMemcpyHostToDevice, s));
        HIPCHK(q, hipMemcpyAsync(&q->d_ctrl->max_load, &z.max_load, 4, hipMemcpyHostToDevice, s));
        HIPCHK(q, hipStreamSynchronize(s));
    }
    return FQ_OK;
}

int fq_get_layout(const fq_handle *q, fq_layout *layout)
{
    if (!q || !layout) return FQ_EINVAL;
    *layout = q->L;
    return FQ_OK;
}

static int read_ctrl(fq_handle *q, Ctrl &c, hipStream_t s)
{
    HIPCHK(q, hipMemcpyAsync(&c, q->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIPCHK(q, hipStreamSynchronize(s));
    return FQ_OK;
}

static bool valid_address(const uint64_t *a, int W, int M, int N)
{
    int nb = N + M - 1, ones = 0;
    for (int w = 0; w < W; w++) {
        uint64_t x = a[w];
        int lo = 64 * w, hi = 64 * (w + 1);
        if (nb < hi) {
            int keep = std::max(0, nb - lo);
            uint64_t mask = keep >= 64 ? ~0ull : ((1ull << keep) - 1);
            if (x & ~mask) return false;
        }
        ones += __builtin_popcountll(x);
    }
    return ones == N;
}

int fq_set_state(fq_handle *q, const uint64_t *addrs, const double *vals, int64_t n, double shift, int64_t step,
                 const uint64_t *ref_addr, double ref_val, void *stream)
{
    if (!q || (n > 0 && (!addrs || !vals)) || n < 1 || !ref_addr || step < 0) {
        if (q) q->err = "set_state needs n >= 1 entries, a reference address and step >= 0";
        return FQ_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const Resolved &R = q->R;
    const int W = R.W;
    // host-side validation: addresses well formed and distinct, values finite
    std::vector<std::pair<uint64_t, uint64_t>> keys((size_t)n);
    for (i64 i = 0; i < n; i++) {
        if (!valid_address(addrs + i * W, W, q->h.M, q->h.N) || !std::isfinite(vals[i]) || vals[i] == 0.0) {
            q->err = "invalid address or value at entry " + std::to_string(i);
            return FQ_EINVAL;
        }
        keys[i] = {W == 2 ? addrs[i * W + 1] : 0, addrs[i * W]};
    }
    std::sort(keys.begin(), keys.end());
    for (size_t i = 1; i < keys.size(); i++)
        if (keys[i] == keys[i - 1]) { q->err = "duplicate address in state"; return FQ_EINVAL; }
    if (!valid_address(ref_addr, W, q->h.M, q->h.N)) { q->err = "invalid reference address"; return FQ_EINVAL; }
    if ((size_t)n * (8 * W + 8) > R.slab_bytes || n > (i64)R.B * R.cap_t) {
        q->err = "state larger than the workspace capacity";
        return FQ_ECAPACITY;
    }
    // stage entries in the parity-1 slab, then build the instance from them
    u64 *sa = (u64 *)q->inst.slab[1];
    double *sv = (double *)(q->inst.slab[1] + sizeof(u64) * W * n);
    HIPCHK(q, hipMemcpyAsync(sa, addrs, sizeof(u64) * W * n, hipMemcpyHostToDevice, s));
    HIPCHK(q, hipMemcpyAsync(sv, vals, sizeof(double) * n, hipMemcpyHostToDevice, s));
    return load_state(q, sa, sv, n, shift, step, ref_addr, ref_val, s);
}

// State c^(step) from device arrays (n entries staged in the parity-1 slab
// region or elsewhere outside the tables), shift, reference vector: insert
// into table[0], reference column, spawns of c^(step) for step+1.
static int load_state(fq_handle *q, const u64 *sa, const double *sv, i64 n, double shift, i64 step,
                      const uint64_t *ref_addr, double ref_val, hipStream_t s)
{
    const Resolved &R = q->R;
    const int W = R.W;
    // fresh control block
    Ctrl c;
    memset(&c, 0, sizeof c);
    c.step = step;
    c.parity = 0;
    c.shift = shift;
    c.ring_base = step + 1;
    c.stop_step = INT64_MAX;
    HIPCHK(q, hipMemcpyAsync(q->d_ctrl, &c, sizeof c, hipMemcpyHostToDevice, s));
    for (int k = 0; k < 2; k++) {
        HIPCHK(q, hipMemsetAsync(q->inst.tab_n[k], 0, sizeof(int) * R.B, s));
        HIPCHK(q, hipMemsetAsync(q->inst.slab_n[k], 0, sizeof(int) * R.B, s));
    }
    HIPCHK(q, hipMemsetAsync(q->inst.coarse_n, 0, sizeof(int) << (R.log2G + R.log2SUB), s));
    int grid = (int)std::min<i64>((n + 255) / 256, 4096);
    if (W == 1) hipLaunchKernelGGL(k_insert<1>, dim3(grid), dim3(256), 0, s, (const Inst *)q->d_inst, (const u64 *)sa, (const double *)sv, (i64)n);
    else hipLaunchKernelGGL(k_insert<2>, dim3(grid), dim3(256), 0, s, (const Inst *)q->d_inst, (const u64 *)sa, (const double *)sv, (i64)n);
    HIPCHK(q, hipGetLastError());
    hipLaunchKernelGGL(k_take_norm, dim3(1), dim3(1), 0, s, (const Inst *)q->d_inst);
    // reference column (on the device), sorted by bucket on the host
    u64 *ra = (u64 *)(q->ws + R.off_ref_tmp);
    double *rh = (double *)(ra + 2 * REFCAP);
    int *rb = (int *)(rh + REFCAP);
    int *rn = rb + REFCAP;
    u64 r0 = ref_addr[0], r1 = W == 2 ? ref_addr[1] : 0;
#define REFK(W_, M_) hipLaunchKernelGGL((k_ref<W_, M_>), dim3(1), dim3(64), 0, s, (const Inst *)q->d_inst, r0, r1, ra, rh, rb, rn, REFCAP)
    const int vm = variant(q->h.model, q->h.M, q->h.N, W, q->h.g, 0);
    if (W == 1) { if (vm == 0) REFK(1, 0); else if (vm == 3) REFK(1, 3); else REFK(1, 1); }
    else { if (vm == 0) REFK(2, 0); else if (vm == 3) REFK(2, 3); else REFK(2, 1); }
#undef REFK
    HIPCHK(q, hipGetLastError());
    int m = 0;
    HIPCHK(q, hipMemcpyAsync(&m, rn, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(q, hipStreamSynchronize(s));
    if (m < 1) { q->err = "reference column too long"; return FQ_ECAPACITY; }
    std::vector<u64> ha(2 * (size_t)m);
    std::vector<double> hh(m);
    std::vector<int> hb(m);
    HIPCHK(q, hipMemcpy(ha.data(), ra, sizeof(u64) * 2 * m, hipMemcpyDeviceToHost));
    HIPCHK(q, hipMemcpy(hh.data(), rh, sizeof(double) * m, hipMemcpyDeviceToHost));
    HIPCHK(q, hipMemcpy(hb.data(), rb, sizeof(int) * m, hipMemcpyDeviceToHost));
    std::vector<int> order(m);
    for (int i = 0; i < m; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return hb[x] < hb[y]; });
    std::vector<u64> sa0(m), sa1(m);
    std::vector<double> sh(m);
    std::vector<int> off(R.B + 1, 0);
    int self = -1;
    for (int k = 0; k < m; k++) {
        int i = order[k];
        sa0[k] = ha[2 * i];
        sa1[k] = ha[2 * i + 1];
        sh[k] = hh[i];
        off[hb[i] + 1]++;
        if (i == 0) self = k;
    }
    for (int b = 0; b < R.B; b++) off[b + 1] += off[b];
    q->inst.ref_n = m;
    q->inst.ref_self = self;
    q->inst.yref = ref_val;
    HIPCHK(q, hipMemcpy(q->inst.ref_a[0], sa0.data(), sizeof(u64) * m, hipMemcpyHostToDevice));
    HIPCHK(q, hipMemcpy(q->inst.ref_a[1], sa1.data(), sizeof(u64) * m, hipMemcpyHostToDevice));
    HIPCHK(q, hipMemcpy(q->inst.ref_h, sh.data(), sizeof(double) * m, hipMemcpyHostToDevice));
    HIPCHK(q, hipMemcpy(q->inst.ref_off, off.data(), sizeof(int) * (R.B + 1), hipMemcpyHostToDevice));
    HIPCHK(q, hipMemcpy(q->d_inst, &q->inst, sizeof(Inst), hipMemcpyHostToDevice));
    // spawns of c^(step) for step+1
    HIPCHK(q, launch_spawn(q->X, 1, s));
    Ctrl cc;
    int rc;
    rc = read_ctrl(q, cc, s);
    if (rc) return rc;
    if (cc.error) {
        q->err = std::string("set_state: ") + fqe_name(cc.error);
        return fqe_status(cc.error);
    }
    q->have_state = 1;
    q->step = step;
    q->parity = 0;
    q->ref[0] = ref_addr[0];
    q->ref[1] = W == 2 ? ref_addr[1] : 0;
    q->yref = ref_val;
    return FQ_OK;
}

int fq_set_timing(fq_handle *q, int32_t enable)
{
    if (!q) return FQ_EINVAL;
    q->timing = enable;
    return FQ_OK;
}

int fq_kernel_time(fq_handle *q, double *ms, int32_t n, int64_t *steps, int32_t reset)
{
    if (!q || (ms && n < 1)) return FQ_EINVAL;
    for (int j = 0; ms && j < n && j < NEV - 1; j++) ms[j] = q->time_ms[j];
    for (int j = NEV - 1; ms && j < n; j++) ms[j] = 0.0;
    if (steps) *steps = q->launches;
    if (reset) {
        for (double &t : q->time_ms) t = 0;
        q->launches = 0;
    }
    return FQ_OK;
}

int fq_run(fq_handle *q, int64_t n_steps, fq_step_stats *stats_out, void *stream)
{
    if (!q || n_steps < 0) return FQ_EINVAL;
    if (!q->have_state) { q->err = "run before set_state"; return FQ_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (q->p.flags & (FQ_FLAG_DUMP_SPAWNS | FQ_FLAG_DUMP_MERGED)) {
        hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, &q->d_ctrl->dump_spawn_n, (i64)0);
        hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, &q->d_ctrl->dump_merged_n, (i64)0);
    }
    hipLaunchKernelGGL(k_set_stop, dim3(1), dim3(64), 0, s, q->X.insts, 1, (i64)n_steps);
    i64 done = 0;
    while (done < n_steps) {
        const i64 chunk = std::min<i64>(RING, n_steps - done);
        hipLaunchKernelGGL(k_begin_chunk, dim3(1), dim3(64), 0, s, q->X.insts, 1);
        if (q->timing && (i64)q->ev.size() < NEV * chunk) {
            size_t old = q->ev.size();
            q->ev.resize(NEV * chunk);
            for (size_t k = old; k < q->ev.size(); k++) HIPCHK(q, hipEventCreate(&q->ev[k]));
        }
        for (i64 k = 0; k < chunk; k++) HIPCHK(q, exec_step(q->X, s, q->timing ? &q->ev[NEV * k] : nullptr));
        Ctrl c;
        int rc = read_ctrl(q, c, s);
        if (rc) return rc;
        if (q->timing) {
            for (i64 k = 0; k < chunk; k++)
                for (int j = 0; j < NEV - 1; j++) {
                    float ms = 0;
                    HIPCHK(q, hipEventElapsedTime(&ms, q->ev[NEV * k + j], q->ev[NEV * k + j + 1]));
                    q->time_ms[j] += ms;
                }
            q->launches += chunk;
        }
        const i64 completed = c.step - q->step;
        if (completed > 0 && stats_out) {
            HIPCHK(q, hipMemcpy(stats_out + done, q->inst.ring, sizeof(StepStats) * completed, hipMemcpyDeviceToHost));
        }
        done += std::max<i64>(completed, 0);
        q->step = c.step;
        q->parity = c.parity;
        if (c.error) {
            q->err = std::string(fqe_name(c.error)) + " at step " + std::to_string(c.step + 1) +
                     (c.err_bucket >= 0 ? " (bucket " + std::to_string(c.err_bucket) + ")" : "");
            return fqe_status(c.error);
        }
        if (completed != chunk) { q->err = "step count mismatch"; return FQ_EHIP; }
        if (c.first_inexact) q->err = inexact_note(c.first_inexact);
    }
    return FQ_OK;
}

int fq_get_state(fq_handle *q, uint64_t *addrs, double *vals, int64_t cap, int64_t *n, double *shift, int64_t *step,
                 void *stream)
{
    if (!q || !n) return FQ_EINVAL;
    if (!q->have_state) { q->err = "no state"; return FQ_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    const Resolved &R = q->R;
    const int W = R.W;
    Ctrl c;
    int rc = read_ctrl(q, c, s);
    if (rc) return rc;
    // pack into the free slab (parity 1 - p)
    char *buf = q->inst.slab[1 - c.parity];
    unsigned long long *cnt = (unsigned long long *)buf;
    u64 *oa = (u64 *)(buf + 256);
    const i64 total_cap = (i64)R.B * R.cap_t;
    double *ov = (double *)(oa + (size_t)W * total_cap);
    if (256 + (8 * W + 8) * (size_t)total_cap > R.slab_bytes) {
        q->err = "slab too small to stage the table";
        return FQ_ECAPACITY;
    }
    HIPCHK(q, hipMemsetAsync(cnt, 0, 8, s));
    int grid = std::min(R.B, 4096);
    if (W == 1) hipLaunchKernelGGL(k_pack<1>, dim3(grid), dim3(256), 0, s, (const Inst *)q->d_inst, oa, ov, cnt);
    else hipLaunchKernelGGL(k_pack<2>, dim3(grid), dim3(256), 0, s, (const Inst *)q->d_inst, oa, ov, cnt);
    HIPCHK(q, hipGetLastError());
    unsigned long long tot = 0;
    HIPCHK(q, hipMemcpyAsync(&tot, cnt, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(q, hipStreamSynchronize(s));
    *n = (int64_t)tot;
    if (shift) *shift = c.shift;
    if (step) *step = c.step;
    if ((i64)tot > cap) { q->err = "get_state: capacity too small"; return FQ_ECAPACITY; }
    if (tot) {
        if (addrs) HIPCHK(q, hipMemcpy(addrs, oa, sizeof(u64) * W * tot, hipMemcpyDeviceToHost));
        if (vals) HIPCHK(q, hipMemcpy(vals, ov, sizeof(double) * tot, hipMemcpyDeviceToHost));
    }
    return FQ_OK;
}

int fq_read_spawn_dump(fq_handle *q, uint64_t *parent, int64_t *attempt, uint64_t *dest, double *value, int64_t cap,
                       int64_t *n, void *stream)
{
    if (!q || !n) return FQ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Ctrl c;
    int rc = read_ctrl(q, c, s);
    if (rc) return rc;
    *n = c.dump_spawn_n;
    if (c.dump_spawn_n > q->R.dump_cap || c.dump_spawn_n > cap) { q->err = "dump capacity exceeded"; return FQ_ECAPACITY; }
    i64 k = c.dump_spawn_n;
    const int W = q->R.W;
    if (k) {
        HIPCHK(q, hipMemcpy(parent, q->inst.dsp_parent, sizeof(u64) * W * k, hipMemcpyDeviceToHost));
        HIPCHK(q, hipMemcpy(attempt, q->inst.dsp_attempt, sizeof(i64) * k, hipMemcpyDeviceToHost));
        HIPCHK(q, hipMemcpy(dest, q->inst.dsp_dest, sizeof(u64) * W * k, hipMemcpyDeviceToHost));
        HIPCHK(q, hipMemcpy(value, q->inst.dsp_val, sizeof(double) * k, hipMemcpyDeviceToHost));
    }
    return FQ_OK;
}

int fq_read_merged_dump(fq_handle *q, uint64_t *addr, double *value, int64_t cap, int64_t *n, void *stream)
{
    if (!q || !n) return FQ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Ctrl c;
    int rc = read_ctrl(q, c, s);
    if (rc) return rc;
    *n = c.dump_merged_n;
    if (c.dump_merged_n > q->R.dump_cap || c.dump_merged_n > cap) { q->err = "dump capacity exceeded"; return FQ_ECAPACITY; }
    i64 k = c.dump_merged_n;
    const int W = q->R.W;
    if (k) {
        HIPCHK(q, hipMemcpy(addr, q->inst.dmg_addr, sizeof(u64) * W * k, hipMemcpyDeviceToHost));
        HIPCHK(q, hipMemcpy(value, q->inst.dmg_val, sizeof(double) * k, hipMemcpyDeviceToHost));
    }
    return FQ_OK;
}

// ------------------------------------------------------------------ copy and autotuning

int fq_copy_state(fq_handle *dst, fq_handle *src, void *stream)
{
    if (!dst || !src || dst == src) return FQ_EINVAL;
    if (!src->have_state) { dst->err = "copy_state: source has no state"; return FQ_EINVAL; }
    const fq_hamiltonian &a = dst->h, &b = src->h;
    const fq_params &x = dst->p, &y = src->p;
    if (a.model != b.model || a.M != b.M || a.N != b.N || a.t != b.t || a.u != b.u || x.dtau != y.dtau ||
        x.target_walkers != y.target_walkers || x.zeta != y.zeta || x.xi != y.xi || x.threshold != y.threshold ||
        x.t_rel != y.t_rel || x.seed != y.seed || x.addr_words != y.addr_words) {
        dst->err = "copy_state: different Hamiltonian or parameters";
        return FQ_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int W = dst->R.W;
    Ctrl c;
    int rc = read_ctrl(src, c, s);
    if (rc) return rc;
    if (c.error) { dst->err = "copy_state: source is in an error state"; return FQ_EINVAL; }
    const i64 nmax = (i64)src->R.B * src->R.cap_t;
    if (256 + (8 * W + 8) * (size_t)nmax > dst->R.slab_bytes) {
        dst->err = "copy_state: destination slab too small to stage the source table";
        return FQ_ECAPACITY;
    }
    char *buf = dst->inst.slab[1];
    unsigned long long *cnt = (unsigned long long *)buf;
    u64 *oa = (u64 *)(buf + 256);
    double *ov = (double *)(oa + (size_t)W * nmax);
    HIPCHK(dst, hipMemsetAsync(cnt, 0, 8, s));
    const int grid = std::min(src->R.B, 4096);
    if (W == 1) hipLaunchKernelGGL(k_pack<1>, dim3(grid), dim3(256), 0, s, (const Inst *)src->d_inst, oa, ov, cnt);
    else hipLaunchKernelGGL(k_pack<2>, dim3(grid), dim3(256), 0, s, (const Inst *)src->d_inst, oa, ov, cnt);
    HIPCHK(dst, hipGetLastError());
    unsigned long long tot = 0;
    HIPCHK(dst, hipMemcpyAsync(&tot, cnt, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(dst, hipStreamSynchronize(s));
    if ((i64)tot > (i64)dst->R.B * dst->R.cap_t || tot == 0) {
        dst->err = "copy_state: state does not fit the destination";
        return FQ_ECAPACITY;
    }
    return load_state(dst, oa, ov, (i64)tot, c.shift, c.step, src->ref, src->yref, s);
}

int fq_autotune(fq_handle *src, const fq_layout *cand, int32_t n, int32_t trial_steps, void *scratch,
                size_t scratch_bytes, double *ms, int32_t *best, void *stream)
{
    if (!src || !cand || n < 1 || trial_steps < 1 || !scratch || !ms || !best) return FQ_EINVAL;
    *best = -1;
    double tbest = 0.0;
    for (int i = 0; i < n; i++) {
        ms[i] = -1.0;
        size_t need = 0;
        fq_layout lo;
        if (fq_workspace_size(&src->h, &src->p, &cand[i], &need, &lo) != FQ_OK || need > scratch_bytes) continue;
        fq_handle *t = nullptr;
        if (fq_create(&src->h, &src->p, &cand[i], scratch, scratch_bytes, &t) != FQ_OK) continue;
        bool ok = fq_copy_state(t, src, stream) == FQ_OK && fq_run(t, 1, nullptr, stream) == FQ_OK;
        if (ok) {
            fq_set_timing(t, 1);
            ok = fq_run(t, trial_steps, nullptr, stream) == FQ_OK;
        }
        if (ok) {
            ms[i] = (t->time_ms[0] + t->time_ms[1] + t->time_ms[2] + t->time_ms[3]) / (double)t->launches;
            if (*best < 0 || ms[i] < tbest) { *best = i; tbest = ms[i]; }
        }
        fq_destroy(t);
    }
    if (*best < 0) { src->err = "autotune: no candidate ran"; return FQ_EINVAL; }
    return FQ_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ groups of instances

namespace {

// Host side of instances stepped together in one set of launches.
struct Group {
    std::vector<fq_handle *> h;  // in grid order
    Exec X;
    Ctrl *d_ctrl_out = nullptr;
    std::vector<Ctrl> ctrl;
};

size_t group_header_bytes(i64 n, i64 buckets, i64 pblocks)
{
    return align256(sizeof(Inst *) * n) + align256(sizeof(u32) * buckets) + align256(sizeof(u32) * pblocks) +
           align256(sizeof(Ctrl) * n);
}

i64 pmap_blocks(const Resolved &R) { return R.two_pass ? ((i64)1 << (R.log2G + R.log2SUB)) : 0; }

// Builds the launch maps of `hs` in the device header `hdr`.  Instances are
// placed in decreasing bucket count, so the first workgroup of every
// instance with more than 64 buckets is a multiple of 64: the spawn
// workgroups that append to one coarse sub-slab (bucket mod 64) then share
// an XCD, and the second-pass map of every instance starts on XCD 0.
int group_build(Group &G, std::vector<fq_handle *> hs, char *hdr, std::string &err)
{
    std::stable_sort(hs.begin(), hs.end(), [](const fq_handle *a, const fq_handle *b) { return a->R.B > b->R.B; });
    const int n = (int)hs.size();
    std::vector<const Inst *> ip(n);
    std::vector<u32> map, pmap;
    size_t lds_s = 0, lds_m = 0;
    for (int i = 0; i < n; i++) {
        ip[i] = hs[i]->d_inst;
        for (int b = 0; b < hs[i]->R.B; b++) map.push_back(((u32)i << 15) | (u32)b);
        append_pmap(hs[i]->R, (u32)i, pmap);
        lds_s = std::max(lds_s, hs[i]->X.lds_s);
        lds_m = std::max(lds_m, hs[i]->X.lds_m);
    }
    char *o = hdr;
    const Inst **d_ip = (const Inst **)o;
    o += align256(sizeof(Inst *) * n);
    u32 *d_map = (u32 *)o;
    o += align256(sizeof(u32) * map.size());
    u32 *d_pmap = (u32 *)o;
    o += align256(sizeof(u32) * pmap.size());
    G.d_ctrl_out = (Ctrl *)o;
    hipError_t e = hipMemcpy(d_ip, ip.data(), sizeof(Inst *) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_map, map.data(), sizeof(u32) * map.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !pmap.empty())
        e = hipMemcpy(d_pmap, pmap.data(), sizeof(u32) * pmap.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) { err = std::string("group maps: ") + hipGetErrorString(e); return FQ_EHIP; }
    G.h = hs;
    G.X = hs[0]->X;
    G.X.n = n;
    G.X.insts = d_ip;
    G.X.map = d_map;
    G.X.grid = (int)map.size();
    G.X.pmap = d_pmap;
    G.X.pgrid = (int)pmap.size();
    // instances are sorted by bucket count: the first has the widest groups
    G.X.wide_groups = hs[0]->X.wide_groups;
    G.X.lds_s = lds_s;
    G.X.lds_m = lds_m;
    G.ctrl.resize(n);
    return FQ_OK;
}

// Replica overlaps computed after every step of a group (all instances of
// the group are the replicas).  `out` receives rows of P doubles (advanced).
struct OvRun {
    Overlap O;
    int W = 1;
    size_t lds = 0;
    double *out = nullptr;
};

size_t overlap_lds_bytes(int W, int slots)
{
    return (size_t)slots * (W == 2 ? 28 : 16) + sizeof(Fx3) * (OV_BS / 64);
}

hipError_t launch_overlap(const OvRun &ov, hipStream_t s)
{
    const void *kf = ov.W == 1 ? (const void *)k_overlap<1> : (const void *)k_overlap<2>;
    Overlap O = ov.O;
    void *args[] = {(void *)&O};
    hipError_t e = hipLaunchKernel(kf, dim3((O.R - 1) * O.B), dim3(OV_BS), args, ov.lds, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_overlap_fin, dim3(1), dim3(1024), 0, s, O);
        e = hipGetLastError();
    }
    return e;
}

// Runs `steps` steps of every instance of G (an instance that has failed or
// reached its stop step does no work).  When rows is given, the statistics
// rows of grid position j are appended at (*rows)[j] (advanced), if not
// null.  With ov, the replica overlaps of every step are computed and their
// rows appended at ov->out.  Returns the status of the first failing
// instance (grid position in *failed) after the chunk in which it failed.
int group_steps(Group &G, i64 steps, fq_step_stats **rows, hipStream_t s, int *failed, std::string &err,
                OvRun *ov = nullptr, const GsRun *gs = nullptr)
{
    const Exec &X = G.X;
    i64 launched = 0;
    int rc = FQ_OK;
    while (launched < steps && rc == FQ_OK) {
        const i64 chunk = std::min<i64>(RING, steps - launched);
        hipLaunchKernelGGL(k_begin_chunk, dim3(1), dim3(256), 0, s, X.insts, X.n);
        hipError_t e = hipGetLastError();
        for (i64 k = 0; k < chunk && e == hipSuccess; k++) {
            e = exec_step(X, s, nullptr, gs);
            if (e == hipSuccess && ov) e = launch_overlap(*ov, s);
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_gather_ctrl, dim3(std::min(X.n, 1024)), dim3(64), 0, s, X.insts, X.n, G.d_ctrl_out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(G.ctrl.data(), G.d_ctrl_out, sizeof(Ctrl) * X.n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { err = std::string("group step: ") + hipGetErrorString(e); return FQ_EHIP; }
        if (ov) {
            i64 done = chunk;
            for (int j = 0; j < X.n; j++) done = std::min<i64>(done, G.ctrl[j].step - G.h[j]->step);
            if (done > 0) {
                e = hipMemcpy(ov->out, ov->O.ring, sizeof(double) * ov->O.P * done, hipMemcpyDeviceToHost);
                if (e != hipSuccess) { err = std::string("overlap rows: ") + hipGetErrorString(e); return FQ_EHIP; }
                ov->out += ov->O.P * done;
            }
        }
        for (int j = 0; j < X.n; j++) {
            fq_handle *q = G.h[j];
            const Ctrl &c = G.ctrl[j];
            const i64 completed = c.step - q->step;
            if (completed > 0 && rows && rows[j]) {
                e = hipMemcpy(rows[j], q->inst.ring, sizeof(StepStats) * completed, hipMemcpyDeviceToHost);
                if (e != hipSuccess) { err = std::string("group rows: ") + hipGetErrorString(e); return FQ_EHIP; }
                rows[j] += completed;
            }
            q->step = c.step;
            q->parity = c.parity;
            if (c.error && rc == FQ_OK) {
                q->err = std::string(fqe_name(c.error)) + " at step " + std::to_string(c.step + 1) +
                         (c.err_bucket >= 0 ? " (bucket " + std::to_string(c.err_bucket) + ")" : "");
                err = q->err;
                rc = fqe_status(c.error);
                if (failed) *failed = j;
            }
        }
        launched += chunk;
    }
    return rc;
}

}  // namespace

// ------------------------------------------------------------------ batch

struct fq_batch {
    std::vector<fq_handle *> inst;  // caller order
    std::vector<int> pos;           // caller index -> grid position
    Group G;
    int failed = -1;
    int device = -1;                // current device at creation (owns the workspace)
    std::string err;
};

namespace {

int batch_plan(int n, const fq_hamiltonian *h, const fq_params *p, const fq_layout *lay, std::vector<size_t> &off,
               size_t &total, std::string &err)
{
    if (n < 1 || n > (1 << 17) || !h || !p || !lay) { err = "batch: need 1 <= n <= 131072 and arrays"; return FQ_EINVAL; }
    i64 nb = 0, np = 0;
    std::vector<size_t> sz(n);
    Resolved R0;
    for (int i = 0; i < n; i++) {
        Resolved R;
        fq_layout L;
        int rc = resolve(&h[i], &p[i], &lay[i], R, L, err);
        if (rc) { err = "batch instance " + std::to_string(i) + ": " + err; return rc; }
        if (i == 0) R0 = R;
        if (R.W != R0.W || variant(h[i].model, h[i].M, h[i].N, p[i].addr_words, h[i].g, p[i].flags) !=
                                   variant(h[0].model, h[0].M, h[0].N, p[0].addr_words, h[0].g, p[0].flags) ||
            R.block != R0.block ||
            R.spawn_block != R0.spawn_block || R.slots != R0.slots) {
            err = "batch instance " + std::to_string(i) +
                  ": instances must share the model kind, the compression style (early or late), addr_words, "
                  "lds_slots, block and spawn_block";
            return FQ_EINVAL;
        }
        sz[i] = align256(R.total);
        nb += R.B;
        np += pmap_blocks(R);
    }
    size_t o = group_header_bytes(n, nb, np);
    off.resize(n);
    for (int i = 0; i < n; i++) { off[i] = o; o += sz[i]; }
    total = o;
    return FQ_OK;
}

}  // namespace

extern "C" {

int fq_batch_workspace_size(int32_t n, const fq_hamiltonian *h, const fq_params *p, const fq_layout *lay,
                            size_t *bytes)
{
    std::vector<size_t> off;
    size_t total = 0;
    int rc = batch_plan(n, h, p, lay, off, total, g_err);
    if (rc) return rc;
    if (bytes) *bytes = total;
    return FQ_OK;
}

int fq_batch_create(int32_t n, const fq_hamiltonian *h, const fq_params *p, const fq_layout *lay, void *workspace,
                    size_t bytes, fq_batch **out)
{
    if (!out) return FQ_EINVAL;
    *out = nullptr;
    std::vector<size_t> off;
    size_t total = 0;
    int rc = batch_plan(n, h, p, lay, off, total, g_err);
    if (rc) return rc;
    if (!workspace || ((uintptr_t)workspace & 255)) { g_err = "batch: workspace must be 256-byte aligned"; return FQ_EINVAL; }
    if (bytes < total) { g_err = "batch: workspace too small"; return FQ_ENOMEM; }
    fq_batch *b = new (std::nothrow) fq_batch();
    if (!b) return FQ_ENOMEM;
    if (hipGetDevice(&b->device) != hipSuccess) b->device = -1;
    char *ws = (char *)workspace;
    for (int i = 0; i < n; i++) {
        fq_handle *q = nullptr;
        size_t sz = (i + 1 < n ? off[i + 1] : total) - off[i];
        rc = fq_create(&h[i], &p[i], &lay[i], ws + off[i], sz, &q);
        if (rc) {
            g_err = "batch instance " + std::to_string(i) + ": " + g_err;
            for (auto x : b->inst) fq_destroy(x);
            delete b;
            return rc;
        }
        b->inst.push_back(q);
    }
    rc = group_build(b->G, b->inst, ws, g_err);
    if (rc) {
        for (auto x : b->inst) fq_destroy(x);
        delete b;
        return rc;
    }
    b->pos.resize(n);
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++)
            if (b->G.h[j] == b->inst[i]) b->pos[i] = j;
    *out = b;
    return FQ_OK;
}

int fq_batch_instance(fq_batch *b, int32_t i, fq_handle **out)
{
    if (!b || !out || i < 0 || i >= (int)b->inst.size()) return FQ_EINVAL;
    *out = b->inst[i];
    return FQ_OK;
}

int fq_batch_run(fq_batch *b, int64_t n_steps, fq_step_stats *stats, void *stream)
{
    if (!b || n_steps < 0) return FQ_EINVAL;
    const int n = (int)b->inst.size();
    for (int i = 0; i < n; i++)
        if (!b->inst[i]->have_state) { b->err = "batch: instance " + std::to_string(i) + " has no state"; return FQ_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_set_stop, dim3(1), dim3(256), 0, s, b->G.X.insts, n, (i64)n_steps);
    std::vector<fq_step_stats *> rows(n, nullptr);
    if (stats)
        for (int i = 0; i < n; i++) rows[b->pos[i]] = stats + (size_t)i * n_steps;
    int failed = -1;
    b->failed = -1;
    int rc = group_steps(b->G, n_steps, rows.data(), s, &failed, b->err);
    if (failed >= 0)
        for (int i = 0; i < n; i++)
            if (b->pos[i] == failed) b->failed = i;
    return rc;
}

// The batch as a set of replicas: at least 2 and at most FQ_MAX_REPLICAS
// instances of one Hamiltonian with one bucket count.
static int replica_check(fq_batch *b, std::string &err)
{
    const int n = (int)b->inst.size();
    if (n < 2 || n > FQ_MAX_REPLICAS) {
        err = "replicas: need 2 to " + std::to_string(FQ_MAX_REPLICAS) + " instances";
        return FQ_EINVAL;
    }
    const fq_handle *q0 = b->inst[0];
    for (int i = 1; i < n; i++) {
        const fq_handle *q = b->inst[i];
        if (q->h.model != q0->h.model || q->h.M != q0->h.M || q->h.N != q0->h.N ||
            (q->h.model == FQ_REAL2D && q->h.lx != q0->h.lx) ||
            memcmp(&q->h.t, &q0->h.t, sizeof(double)) || memcmp(&q->h.u, &q0->h.u, sizeof(double)) ||
            memcmp(&q->h.g, &q0->h.g, sizeof(double)) ||
            q->R.B != q0->R.B || q->R.W != q0->R.W || q->R.slots != q0->R.slots) {
            err = "replicas: instance " + std::to_string(i) +
                  " differs from instance 0 in its Hamiltonian, addr_words, buckets or lds_slots";
            return FQ_EINVAL;
        }
    }
    return FQ_OK;
}

struct OvScratch {
    size_t rep, part, ring, flags, total;
};

static OvScratch ov_scratch(int R, int B)
{
    const int P = R * (R - 1) / 2;
    OvScratch o;
    o.rep = 0;
    o.part = align256(sizeof(Inst *) * R);
    o.ring = o.part + align256(sizeof(Fx3) * (size_t)B * P);
    o.flags = o.ring + align256(sizeof(double) * (size_t)RING * P);
    o.total = o.flags + 256;
    return o;
}

int fq_batch_replica_scratch_size(fq_batch *b, size_t *bytes)
{
    if (!b || !bytes) return FQ_EINVAL;
    int rc = replica_check(b, b->err);
    if (rc) return rc;
    *bytes = ov_scratch((int)b->inst.size(), b->inst[0]->R.B).total;
    return FQ_OK;
}

}  // extern "C"

// Replica steps with overlaps (shared by fq_batch_run_replicas and the
// allocation-free fq_batch_run_replicas_static): `sc` is device scratch of
// at least ov_scratch(R, B).total bytes, 256-byte aligned.  Makes no device
// allocation and no host container: R <= FQ_MAX_REPLICAS fits fixed arrays.
static int run_replicas(fq_batch *b, int64_t n_steps, fq_step_stats *stats, double *overlaps, char *sc,
                        int32_t *inexact, hipStream_t s)
{
    const int R = (int)b->inst.size(), P = R * (R - 1) / 2;
    const fq_handle *q0 = b->inst[0];
    const OvScratch lay = ov_scratch(R, q0->R.B);
    for (int i = 0; i < R; i++) {
        if (!b->inst[i]->have_state) { b->err = "replicas: instance " + std::to_string(i) + " has no state"; return FQ_EINVAL; }
        if (b->inst[i]->step != q0->step) { b->err = "replicas: instances are at different steps"; return FQ_EINVAL; }
    }
    const Inst *rep[FQ_MAX_REPLICAS];
    for (int i = 0; i < R; i++) rep[i] = b->inst[i]->d_inst;
    OvRun ov;
    ov.W = q0->R.W;
    ov.lds = overlap_lds_bytes(ov.W, q0->R.slots);
    ov.out = overlaps;
    ov.O.rep = (const Inst *const *)(sc + lay.rep);
    ov.O.R = R;
    ov.O.P = P;
    ov.O.B = q0->R.B;
    ov.O.part = (Fx3 *)(sc + lay.part);
    ov.O.ring = (double *)(sc + lay.ring);
    ov.O.ring_cap = RING;
    ov.O.flags = (int *)(sc + lay.flags);
    hipError_t e = ensure_lds(ov.W == 1 ? (const void *)k_overlap<1> : (const void *)k_overlap<2>, ov.lds);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)ov.O.rep, rep, sizeof(Inst *) * R, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        // the flags start at zero (a fill kernel: the scratch may hold the
        // flags of an earlier call)
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, ov.O.flags, 4, 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { b->err = std::string("replicas: ") + hipGetErrorString(e); return FQ_EHIP; }
    hipLaunchKernelGGL(k_set_stop, dim3(1), dim3(256), 0, s, b->G.X.insts, R, (i64)n_steps);
    fq_step_stats *rows[FQ_MAX_REPLICAS] = {};
    if (stats)
        for (int i = 0; i < R; i++) rows[b->pos[i]] = stats + (size_t)i * n_steps;
    int failed = -1;
    b->failed = -1;
    int rc = group_steps(b->G, n_steps, rows, s, &failed, b->err, &ov);
    if (failed >= 0)
        for (int i = 0; i < R; i++)
            if (b->pos[i] == failed) b->failed = i;
    int fl[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(fl, ov.O.flags, sizeof(fl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { b->err = std::string("replicas: ") + hipGetErrorString(e); return FQ_EHIP; }
    if (inexact) *inexact = fl[1];
    if (rc) return rc;
    if (fl[0]) { b->err = "replicas: a table bucket does not fit the overlap hash (lds_slots)"; return FQ_ECAPACITY; }
    if (fl[2]) { b->err = "replicas: an amplitude product is out of the overlap range"; return FQ_EDIVERGED; }
    return FQ_OK;
}

// Device scratch of fq_batch_run_replicas_static: a file-scope array, one
// copy per GPU the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address): it uses the address hipGetSymbolAddress returns,
// taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[FQ_STATIC_SCRATCH_BYTES];
constexpr int STATIC_MAX_DEVICES = 64;
static char *g_scratch_ptr[STATIC_MAX_DEVICES];
static std::mutex g_scratch_mu;

static int static_scratch(int dev, char **out, std::string &err)
{
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) { err = "static scratch: device index out of range"; return FQ_EINVAL; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("static scratch: hipGetSymbolAddress: ") + hipGetErrorString(e);
            return FQ_EHIP;
        }
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return FQ_OK;
}

extern "C" {

int fq_batch_run_replicas(fq_batch *b, int64_t n_steps, fq_step_stats *stats, double *overlaps, void *scratch_,
                          size_t scratch_bytes, int32_t *inexact, void *stream)
{
    if (!b || n_steps < 0 || !overlaps) return FQ_EINVAL;
    int rc = replica_check(b, b->err);
    if (rc) return rc;
    const OvScratch lay = ov_scratch((int)b->inst.size(), b->inst[0]->R.B);
    if (!scratch_ || ((uintptr_t)scratch_ & 255) || scratch_bytes < lay.total) {
        b->err = "replicas: scratch must be 256-byte aligned and at least fq_batch_replica_scratch_size bytes";
        return FQ_EINVAL;
    }
    return run_replicas(b, n_steps, stats, overlaps, (char *)scratch_, inexact, (hipStream_t)stream);
}

int fq_batch_run_replicas_static(fq_batch *b, int64_t n_steps, fq_step_stats *stats, double *overlaps,
                                 int32_t *inexact, void *stream)
{
    if (!b || n_steps < 0 || !overlaps) return FQ_EINVAL;
    int rc = replica_check(b, b->err);
    if (rc) return rc;
    const OvScratch lay = ov_scratch((int)b->inst.size(), b->inst[0]->R.B);
    if (lay.total > FQ_STATIC_SCRATCH_BYTES) {
        b->err = "replicas (static scratch): " + std::to_string(lay.total) + " bytes of scratch needed, the static "
                 "scratch holds " + std::to_string((size_t)FQ_STATIC_SCRATCH_BYTES) +
                 " (fewer replicas or buckets, or fq_batch_run_replicas with a caller buffer)";
        return FQ_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device) {
        b->err = "replicas (static scratch): the current device is not the batch's device";
        return FQ_EINVAL;
    }
    char *sc = nullptr;
    rc = static_scratch(dev, &sc, b->err);
    if (rc) return rc;
    return run_replicas(b, n_steps, stats, overlaps, sc, inexact, (hipStream_t)stream);
}

struct GsScratch {
    size_t rep, dots, norms, alpha, updated, flags, total;
};

static GsScratch gs_scratch(int R, int B)
{
    GsScratch o;
    o.rep = 0;
    o.dots = align256(sizeof(Inst *) * R);
    o.norms = o.dots + align256(sizeof(Fx3) * 2 * (size_t)B);
    o.alpha = o.norms + align256(sizeof(Fx3) * (size_t)R * B);
    o.updated = o.alpha + 256;
    o.flags = o.updated + align256(sizeof(int) * R);
    o.total = o.flags + 256;
    return o;
}

static int spectral_check(fq_batch *b, std::string &err)
{
    int rc = replica_check(b, err);
    if (rc) return rc;
    const fq_handle *q0 = b->inst[0];
    if (gs_upd_lds(q0->R.W, q0->R.slots) > LDS_MAX) {
        err = "excited states: lds_slots too large for the orthogonalisation hash (twice lds_slots)";
        return FQ_EINVAL;
    }
    return FQ_OK;
}

int fq_batch_spectral_scratch_size(fq_batch *b, size_t *bytes)
{
    if (!b || !bytes) return FQ_EINVAL;
    int rc = spectral_check(b, b->err);
    if (rc) return rc;
    *bytes = gs_scratch((int)b->inst.size(), b->inst[0]->R.B).total;
    return FQ_OK;
}

int fq_batch_run_spectral(fq_batch *b, int64_t n_steps, fq_step_stats *stats, void *scratch, size_t scratch_bytes,
                          int32_t *inexact, void *stream)
{
    if (!b || n_steps < 0) return FQ_EINVAL;
    int rc = spectral_check(b, b->err);
    if (rc) return rc;
    const int R = (int)b->inst.size();
    const fq_handle *q0 = b->inst[0];
    const GsScratch lay = gs_scratch(R, q0->R.B);
    if (!scratch || ((uintptr_t)scratch & 255) || scratch_bytes < lay.total) {
        b->err = "excited states: scratch must be 256-byte aligned and at least fq_batch_spectral_scratch_size bytes";
        return FQ_EINVAL;
    }
    for (int i = 0; i < R; i++) {
        if (!b->inst[i]->have_state) { b->err = "excited states: run " + std::to_string(i) + " has no state"; return FQ_EINVAL; }
        if (b->inst[i]->step != q0->step) { b->err = "excited states: runs are at different steps"; return FQ_EINVAL; }
    }
    hipStream_t s = (hipStream_t)stream;
    char *sc = (char *)scratch;
    std::vector<const Inst *> rep(R);
    for (int i = 0; i < R; i++) rep[i] = b->inst[i]->d_inst;
    GsRun g;
    g.W = q0->R.W;
    g.lds_dot = gs_dot_lds(g.W, q0->R.slots);
    g.lds_upd = gs_upd_lds(g.W, q0->R.slots);
    g.S.rep = (const Inst *const *)(sc + lay.rep);
    g.S.R = R;
    g.S.B = q0->R.B;
    g.S.dots = (Fx3 *)(sc + lay.dots);
    g.S.norms = (Fx3 *)(sc + lay.norms);
    g.S.alpha = (double *)(sc + lay.alpha);
    g.S.updated = (int *)(sc + lay.updated);
    g.S.flags = (int *)(sc + lay.flags);
    hipError_t e = ensure_lds(g.W == 1 ? (const void *)k_gs_dot<1> : (const void *)k_gs_dot<2>, g.lds_dot);
    if (e == hipSuccess)
        e = ensure_lds(g.W == 1 ? (const void *)k_gs_update<1> : (const void *)k_gs_update<2>, g.lds_upd);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)g.S.rep, rep.data(), sizeof(Inst *) * R, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, g.S.updated, R, 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, g.S.flags, 4, 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { b->err = std::string("excited states: ") + hipGetErrorString(e); return FQ_EHIP; }
    hipLaunchKernelGGL(k_set_stop, dim3(1), dim3(256), 0, s, b->G.X.insts, R, (i64)n_steps);
    std::vector<fq_step_stats *> rows(R, nullptr);
    if (stats)
        for (int i = 0; i < R; i++) rows[b->pos[i]] = stats + (size_t)i * n_steps;
    int failed = -1;
    b->failed = -1;
    rc = group_steps(b->G, n_steps, rows.data(), s, &failed, b->err, nullptr, &g);
    if (failed >= 0)
        for (int i = 0; i < R; i++)
            if (b->pos[i] == failed) b->failed = i;
    int fl[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(fl, g.S.flags, sizeof(fl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { b->err = std::string("excited states: ") + hipGetErrorString(e); return FQ_EHIP; }
    if (inexact) *inexact = fl[0];
    return rc;
}

int fq_batch_autotune(fq_batch *b, const fq_layout *cand, int32_t n, int32_t trial_steps, void *scratch,
                      size_t scratch_bytes, double *ms, int32_t *best, void *stream)
{
    if (!b || !cand || n < 1 || trial_steps < 1 || !scratch || !ms || !best) return FQ_EINVAL;
    const int ni = (int)b->inst.size();
    for (int j = 0; j < ni; j++)
        if (!b->inst[j]->have_state) { b->err = "batch autotune: instance " + std::to_string(j) + " has no state"; return FQ_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    std::vector<fq_hamiltonian> h(ni);
    std::vector<fq_params> p(ni);
    std::vector<fq_layout> lay(ni);
    for (int j = 0; j < ni; j++) {
        h[j] = b->inst[j]->h;
        p[j] = b->inst[j]->p;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        b->err = "batch autotune: hipEventCreate failed";
        if (e0) hipEventDestroy(e0);
        return FQ_EHIP;
    }
    *best = -1;
    double tbest = 0.0;
    for (int i = 0; i < n; i++) {
        ms[i] = -1.0;
        // each instance keeps its capacities and takes the candidate's shared
        // shape; the bucket count follows from the capacities when 0
        for (int j = 0; j < ni; j++) {
            lay[j] = b->inst[j]->L;
            lay[j].buckets = cand[i].buckets;
            lay[j].lds_slots = cand[i].lds_slots;
            lay[j].block = cand[i].block;
            lay[j].spawn_block = cand[i].spawn_block;
        }
        size_t need = 0;
        if (fq_batch_workspace_size(ni, h.data(), p.data(), lay.data(), &need) != FQ_OK || need > scratch_bytes) continue;
        fq_batch *t = nullptr;
        if (fq_batch_create(ni, h.data(), p.data(), lay.data(), scratch, scratch_bytes, &t) != FQ_OK) continue;
        bool ok = true;
        for (int j = 0; j < ni && ok; j++) ok = fq_copy_state(t->inst[j], b->inst[j], stream) == FQ_OK;
        ok = ok && fq_batch_run(t, 1, nullptr, stream) == FQ_OK;
        float el = 0.0f;
        ok = ok && hipEventRecord(e0, s) == hipSuccess;
        ok = ok && fq_batch_run(t, trial_steps, nullptr, stream) == FQ_OK;
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&el, e0, e1) == hipSuccess;
        if (ok) {
            ms[i] = (double)el / (double)trial_steps;
            if (*best < 0 || ms[i] < tbest) { *best = i; tbest = ms[i]; }
        }
        fq_batch_destroy(t);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (*best < 0) { b->err = "batch autotune: no candidate ran"; return FQ_EINVAL; }
    return FQ_OK;
}

const char *fq_batch_last_error(const fq_batch *b) { return b ? b->err.c_str() : g_err.c_str(); }

int32_t fq_batch_failed(const fq_batch *b) { return b ? b->failed : -1; }

int fq_batch_destroy(fq_batch *b)
{
    if (!b) return FQ_EINVAL;
    for (auto q : b->inst) fq_destroy(q);
    delete b;
    return FQ_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ server

namespace {

struct Req {
    fq_hamiltonian h;
    fq_params p;
    fq_layout L;
    uint64_t start[2];
    double start_val;
    i64 n_steps;
    size_t bytes = 0, off = 0;
    fq_handle *q = nullptr;
    fq_request_info info;
    double sum_s = 0, sum_h = 0, sum_v = 0;
};

}  // namespace

struct fq_server {
    fq_server_config cfg;
    char *hdr = nullptr, *arena = nullptr;
    size_t arena_bytes = 0;
    std::map<size_t, size_t> free_;  // arena offset -> bytes, coalesced
    std::deque<uint64_t> queue;
    std::vector<uint64_t> active;
    std::unordered_map<uint64_t, Req> reqs;
    uint64_t next_id = 1;
    Group G;
    bool dirty = true;
    std::vector<fq_step_stats> rowbuf;
    std::string err;

    bool alloc(size_t bytes, size_t &off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

namespace {

constexpr int SERVER_MAX_ACTIVE = 1024;

size_t server_header_bytes(int max_active)
{
    return group_header_bytes(max_active, (i64)max_active * MAX_BUCKETS, (i64)max_active * 4096);
}

void retire(fq_server *sv, Req &r)
{
    if (r.q) fq_destroy(r.q);
    r.q = nullptr;
    sv->release(r.off, r.bytes);
}

}  // namespace

extern "C" {

int fq_server_create(const fq_server_config *cfg, void *pool, size_t pool_bytes, fq_server **out)
{
    if (!out || !cfg) return FQ_EINVAL;
    *out = nullptr;
    if ((cfg->model != FQ_REAL1D && cfg->model != FQ_MOM1D) || (cfg->addr_words != 1 && cfg->addr_words != 2) ||
        cfg->max_active < 1 || cfg->max_active > SERVER_MAX_ACTIVE || cfg->steps_per_tick < 1 ||
        cfg->steps_per_tick > RING) {
        g_err = "server: invalid configuration";
        return FQ_EINVAL;
    }
    if (!pool || ((uintptr_t)pool & 255)) { g_err = "server: pool must be 256-byte aligned"; return FQ_EINVAL; }
    const size_t hb = server_header_bytes(cfg->max_active);
    if (pool_bytes < hb + 256) { g_err = "server: pool too small"; return FQ_ENOMEM; }
    fq_server *sv = new (std::nothrow) fq_server();
    if (!sv) return FQ_ENOMEM;
    sv->cfg = *cfg;
    sv->hdr = (char *)pool;
    sv->arena = (char *)pool + hb;
    sv->arena_bytes = (pool_bytes - hb) & ~(size_t)255;
    sv->free_[0] = sv->arena_bytes;
    *out = sv;
    return FQ_OK;
}

const char *fq_server_last_error(const fq_server *sv) { return sv ? sv->err.c_str() : g_err.c_str(); }

int fq_server_submit(fq_server *sv, const fq_hamiltonian *h, const fq_params *p, const fq_layout *layout,
                     const uint64_t *start, double start_val, int64_t n_steps, uint64_t *id)
{
    if (!sv || !h || !p || !layout || !start || !id || n_steps < 1 || !std::isfinite(start_val) || start_val == 0.0)
        return FQ_EINVAL;
    if (h->model != sv->cfg.model || p->addr_words != sv->cfg.addr_words) {
        sv->err = "submit: model or addr_words differ from the server's";
        return FQ_EINVAL;
    }
    if (p->flags & FQ_FLAG_EARLY_COMPRESSION) {
        sv->err = "submit: the server runs late compression only";
        return FQ_EINVAL;
    }
    if (h->model == FQ_REAL1D && h->g != 0.0) {
        sv->err = "submit: a ring server runs without importance sampling (g = 0)";
        return FQ_EINVAL;
    }
    Req r;
    r.h = *h;
    r.p = *p;
    r.L = *layout;
    r.L.lds_slots = sv->cfg.lds_slots;
    r.L.block = sv->cfg.block;
    r.L.spawn_block = sv->cfg.spawn_block;
    size_t bytes = 0;
    fq_layout lo;
    int rc = fq_workspace_size(&r.h, &r.p, &r.L, &bytes, &lo);
    if (rc) { sv->err = "submit: " + g_err; return rc; }
    if (h->model == FQ_MOM1D && (p->addr_words != 1 || h->N + h->M - 1 > 31)) {
        sv->err = "submit: a momentum-space server takes one-word addresses of at most 31 bits (N + M - 1 <= 31)";
        return FQ_EINVAL;
    }
    r.bytes = align256(bytes);
    if (r.bytes > sv->arena_bytes) { sv->err = "submit: the request can never fit the pool"; return FQ_EINVAL; }
    r.start[0] = start[0];
    r.start[1] = p->addr_words == 2 ? start[1] : 0;
    r.start_val = start_val;
    r.n_steps = n_steps;
    memset(&r.info, 0, sizeof r.info);
    r.info.state = FQ_REQ_QUEUED;
    r.info.workspace_bytes = (int64_t)r.bytes;
    const uint64_t rid = sv->next_id++;
    sv->reqs.emplace(rid, r);
    sv->queue.push_back(rid);
    *id = rid;
    return FQ_OK;
}

int fq_server_tick(fq_server *sv, void *stream, int32_t *n_active, int32_t *n_queued, int32_t *n_finished)
{
    if (!sv) return FQ_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int finished = 0;
    // admission in arrival order while memory and slots allow
    while (!sv->queue.empty() && (int)sv->active.size() < sv->cfg.max_active) {
        const uint64_t rid = sv->queue.front();
        Req &r = sv->reqs[rid];
        if (!sv->alloc(r.bytes, r.off)) break;
        sv->queue.pop_front();
        int rc = fq_create(&r.h, &r.p, &r.L, sv->arena + r.off, r.bytes, &r.q);
        if (rc == FQ_OK) rc = fq_set_state(r.q, r.start, &r.start_val, 1, 0.0, 0, r.start, r.start_val, stream);
        if (rc == FQ_OK) {
            hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, &r.q->d_ctrl->stop_step, (i64)r.n_steps);
            if (hipGetLastError() != hipSuccess) rc = FQ_EHIP;
        }
        if (rc != FQ_OK) {
            r.info.state = FQ_REQ_FAILED;
            r.info.status = rc;
            retire(sv, r);
            finished++;
            continue;
        }
        r.info.state = FQ_REQ_RUNNING;
        sv->active.push_back(rid);
        sv->dirty = true;
    }
    if (!sv->active.empty()) {
        if (sv->dirty) {
            std::vector<fq_handle *> hs;
            for (auto rid : sv->active) hs.push_back(sv->reqs[rid].q);
            int rc = group_build(sv->G, hs, sv->hdr, sv->err);
            if (rc) return rc;
            sv->dirty = false;
        }
        const int n = (int)sv->G.h.size();
        const i64 T = sv->cfg.steps_per_tick;
        sv->rowbuf.resize((size_t)n * T);
        std::vector<fq_step_stats *> rows(n);
        for (int j = 0; j < n; j++) rows[j] = sv->rowbuf.data() + (size_t)j * T;
        int failed = -1;
        std::string err;
        int rc = group_steps(sv->G, T, rows.data(), s, &failed, err);
        if (rc == FQ_EHIP) { sv->err = err; return rc; }
        // account the rows and retire finished or failed solves
        std::unordered_map<const fq_handle *, int> posof;
        for (int j = 0; j < n; j++) posof[sv->G.h[j]] = j;
        std::vector<uint64_t> keep;
        for (auto rid : sv->active) {
            Req &r = sv->reqs[rid];
            const int j = posof[r.q];
            const fq_step_stats *b0 = sv->rowbuf.data() + (size_t)j * T;
            for (const fq_step_stats *x = b0; x < rows[j]; x++) {
                r.info.last = *x;
                r.info.walker_steps += x->norm;
                if (2 * x->step > r.n_steps) {
                    r.sum_s += x->shift;
                    r.sum_h += x->hproj;
                    r.sum_v += x->vproj;
                    r.info.n_mean++;
                }
            }
            r.info.steps_done = r.q->step;
            const Ctrl &c = sv->G.ctrl[j];
            if (c.error) {
                r.info.state = FQ_REQ_FAILED;
                r.info.status = fqe_status(c.error);
            } else if (r.q->step >= r.n_steps) {
                r.info.state = FQ_REQ_DONE;
            }
            if (r.info.n_mean > 0) {
                r.info.mean_shift = r.sum_s / (double)r.info.n_mean;
                r.info.mean_hproj = r.sum_h / (double)r.info.n_mean;
                r.info.mean_vproj = r.sum_v / (double)r.info.n_mean;
            }
            if (r.info.state == FQ_REQ_RUNNING) {
                keep.push_back(rid);
            } else {
                retire(sv, r);
                finished++;
                sv->dirty = true;
            }
        }
        sv->active.swap(keep);
    }
    if (n_active) *n_active = (int32_t)sv->active.size();
    if (n_queued) *n_queued = (int32_t)sv->queue.size();
    if (n_finished) *n_finished = finished;
    return FQ_OK;
}

int fq_server_poll(fq_server *sv, uint64_t id, fq_request_info *info)
{
    if (!sv || !info) return FQ_EINVAL;
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return FQ_ENOTFOUND;
    *info = it->second.info;
    return FQ_OK;
}

int fq_server_destroy(fq_server *sv)
{
    if (!sv) return FQ_EINVAL;
    for (auto &kv : sv->reqs)
        if (kv.second.q) fq_destroy(kv.second.q);
    delete sv;
    return FQ_OK;
}

}  // extern "C"
