// fq_kernels.hpp -- the merge and spawn kernel templates of the FCIQMC step.
//
// Their instantiations (address words W, model variant, workgroup size,
// compression style) are compiled in separate translation units, one per
// (W, model variant) pair (fq_inst.hip built with FQ_INST_W and
// FQ_INST_MODEL), so that they build in parallel; the host runtime declares
// them with FQ_EXTERN_STEP_KERNELS and launches them through their handles.
#pragma once
#include "fq_step.hpp"

// The step kernels run over a set of instances: one, or a batch.  `insts` is
// a device array of instance descriptors.  A merge or spawn workgroup finds
// its instance and bucket through `map` (entry = instance << 15 | bucket);
// without a map there is one instance and workgroup b takes bucket b.

__device__ __forceinline__ const fq::Inst &locate(const fq::Inst *const *insts, const fq::u32 *map, int &b)
{
    if (map) {
        const fq::u32 m = map[blockIdx.x];
        b = (int)(m & 0x7fffu);
        return fq::const_inst(insts[m >> 15]);
    }
    b = (int)blockIdx.x;
    return fq::const_inst(insts[0]);
}

// EARLY: early compression (separate kernels, so the late-compression
// kernels carry none of its code and registers)
template <int W, int MODEL, int BS, bool EARLY>
__global__ __launch_bounds__(BS) void k_merge(const fq::Inst *const *insts, const fq::u32 *map)
{
    extern __shared__ __align__(16) char smem[];
    int b;
    const fq::Inst &I = locate(insts, map, b);
    fq::merge_bucket<W, MODEL, BS, EARLY>(I, b, smem);
}

// waves per SIMD the spawn kernel's register budget must allow (1: no
// constraint beyond the workgroup size)
#ifndef FQ_SPAWN_WAVES
#define FQ_SPAWN_WAVES 1
#endif
template <int W, int MODEL, int BS, bool EARLY>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(FQ_SPAWN_WAVES))) void k_spawn(const fq::Inst *const *insts, const fq::u32 *map, int mode)
{
    extern __shared__ __align__(16) char smem[];
    int b;
    const fq::Inst &I = locate(insts, map, b);
    fq::spawn_bucket<W, MODEL, BS, EARLY>(I, b, mode, smem);
}

// explicit instantiations (EXT = extern: declaration only) of the merge and
// spawn kernels of one (W, model variant) pair, all workgroup sizes and both
// compression styles
#define FQ_STEP_KERNEL_SET(EXT, W_, M_)                                                       \
    EXT template __global__ void k_merge<W_, M_, 256, false>(const fq::Inst *const *, const fq::u32 *); \
    EXT template __global__ void k_merge<W_, M_, 512, false>(const fq::Inst *const *, const fq::u32 *); \
    EXT template __global__ void k_merge<W_, M_, 1024, false>(const fq::Inst *const *, const fq::u32 *); \
    EXT template __global__ void k_merge<W_, M_, 256, true>(const fq::Inst *const *, const fq::u32 *); \
    EXT template __global__ void k_merge<W_, M_, 512, true>(const fq::Inst *const *, const fq::u32 *); \
    EXT template __global__ void k_merge<W_, M_, 1024, true>(const fq::Inst *const *, const fq::u32 *); \
    EXT template __global__ void k_spawn<W_, M_, 256, false>(const fq::Inst *const *, const fq::u32 *, int); \
    EXT template __global__ void k_spawn<W_, M_, 512, false>(const fq::Inst *const *, const fq::u32 *, int); \
    EXT template __global__ void k_spawn<W_, M_, 1024, false>(const fq::Inst *const *, const fq::u32 *, int); \
    EXT template __global__ void k_spawn<W_, M_, 256, true>(const fq::Inst *const *, const fq::u32 *, int); \
    EXT template __global__ void k_spawn<W_, M_, 512, true>(const fq::Inst *const *, const fq::u32 *, int); \
    EXT template __global__ void k_spawn<W_, M_, 1024, true>(const fq::Inst *const *, const fq::u32 *, int);

#define FQ_EXTERN_STEP_KERNELS                                                                \
    FQ_STEP_KERNEL_SET(extern, 1, 0) FQ_STEP_KERNEL_SET(extern, 1, 1) FQ_STEP_KERNEL_SET(extern, 1, 2)        \
    FQ_STEP_KERNEL_SET(extern, 1, 3) FQ_STEP_KERNEL_SET(extern, 2, 0) FQ_STEP_KERNEL_SET(extern, 2, 1)        \
    FQ_STEP_KERNEL_SET(extern, 2, 2) FQ_STEP_KERNEL_SET(extern, 2, 3)
