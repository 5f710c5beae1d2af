// at_kernels.hpp -- gfx950 tile kernels: one workgroup of 256 threads runs the
// tile step of at_tile.hpp for one work item (non-persistent) or strides over
// the work list (persistent).  Own-point state and the S stage right-hand sides
// live in registers, tile data in dynamic LDS.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "at_plan.hpp"
#include "at_variants.hpp"

namespace atk {

template <class C>
struct GpuRT {
    TS<C> ts;
    __device__ int nthreads() const { return (int)blockDim.x; }
    template <class Fn>
    __device__ void each(Fn&& f) {
        // the thread index is opaque to the optimiser in each phase, so that values
        // derived from it are computed where they are used instead of being hoisted
        // out of the tile loop and held in registers across every phase
        int tid = (int)threadIdx.x;
        __asm__ volatile("" : "+v"(tid));
        f(tid, ts);
    }
    // Workgroup barrier for LDS traffic only: the wave's own LDS operations are complete
    // (lgkmcnt(0)) before the barrier, and the compiler moves no memory operation across
    // it.  Unlike __syncthreads() it does not wait for the wave's global loads and stores
    // (vmcnt): no phase reads global memory that another wave of the workgroup wrote in
    // the same launch.
    __device__ void sync() {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0xC07F);   // gfx9 encoding: lgkmcnt(0), vmcnt/expcnt unconstrained
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    // Barrier that also drains the wave's vector-memory operations (vmcnt(0)): after
    // direct global-to-LDS copies, which complete on that counter.
    __device__ void sync_mem() { __syncthreads(); }
};

// Work item order with consecutive items on one XCD: workgroup i runs on XCD
// i mod 8, so item = (first item of that XCD's share) + i / 8.
__device__ __forceinline__ int xcd_item(int it, int n) {
    const int q = n >> 3, r = n & 7, x = it & 7, j = it >> 3;
    return x * q + (x < r ? x : r) + j;
}

// The tile list, the problem descriptors and the step counter are not written while a
// tile kernel runs: they are read through the constant address space, so that their
// uniform reads are scalar loads (one request per cache line, no per-lane loads and
// register moves) also inside the tile loop, where the compiler could not otherwise
// rule out an aliasing store.
template <class T>
__device__ __forceinline__ const AT_CONST T& const_ref(const T* p) {
    return *(const AT_CONST T*)p;
}

template <class C, bool STEP, bool STAGED = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(STEP ? C::WAVES_STEP : C::WAVES_PER_EU)))
void at_tile_kernel(KArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    GpuRT<C> rt;
    const int64_t n = (a.step_ptr ? const_ref(a.step_ptr) : 0) + a.step_off;
    const bool remap = (a.flags & KF_XCD) && (int)gridDim.x == a.ntiles;
    for (int it = blockIdx.x; it < a.ntiles; it += gridDim.x) {
        const int ti = remap ? xcd_item(it, a.ntiles) : it;
        const Tile t = const_ref(a.tiles + ti);
        tile_step<C, STEP, STAGED>(rt, a, t, const_ref(a.tprobs + ti), n, lds);
        if (it + (int)gridDim.x < a.ntiles) rt.sync();   // LDS reused by the next tile
    }
}

template <class C, bool STEP, bool STAGED>
hipError_t launch_form(const KArgs& a, int grid, hipStream_t s) {
    // the dynamic-LDS limit is a property of the kernel on each device: raised once per
    // device (the current one, which the stream belongs to); safe under concurrent launches
    static std::atomic<uint64_t> attr_done{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev < 64 ? uint64_t(1) << dev : 0;
    if (!(attr_done.load(std::memory_order_acquire) & bit)) {
        e = hipFuncSetAttribute((const void*)at_tile_kernel<C, STEP, STAGED>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_done.fetch_or(bit, std::memory_order_acq_rel);
    }
    hipLaunchKernelGGL((at_tile_kernel<C, STEP, STAGED>), dim3(grid), dim3(BLOCK), (size_t)a.lds_bytes, s, a);
    return hipGetLastError();
}

// whole steps take the kernel whose stage range is fixed at compile time; the scalar FD
// kind with its strips staged in LDS (run option halo_lds) takes kernels of their own
template <class C>
hipError_t launch_variant(const KArgs& a, int grid, hipStream_t s) {
    const bool whole = a.s_begin == 0 && a.s_end == C::S - 1 && !(a.flags & KF_STAGE_IO);
    if constexpr (C::KIND == K_ADR) {
        if (a.flags & KF_HALO_LDS)
            return whole ? launch_form<C, true, true>(a, grid, s) : launch_form<C, false, true>(a, grid, s);
    }
    return whole ? launch_form<C, true, false>(a, grid, s) : launch_form<C, false, false>(a, grid, s);
}

// per-kind dispatchers (one translation unit each); return false if the key is not theirs
bool launch_adr(const VariantKey& k, const KArgs& a, int grid, hipStream_t s, hipError_t* e);
bool launch_adr32(const VariantKey& k, const KArgs& a, int grid, hipStream_t s, hipError_t* e);
bool launch_rns(const VariantKey& k, const KArgs& a, int grid, hipStream_t s, hipError_t* e);
bool launch_rns32(const VariantKey& k, const KArgs& a, int grid, hipStream_t s, hipError_t* e);
bool launch_wscal(const VariantKey& k, const KArgs& a, int grid, hipStream_t s, hipError_t* e);
bool launch_eul(const VariantKey& k, const KArgs& a, int grid, hipStream_t s, hipError_t* e);
bool launch_reul(const VariantKey& k, const KArgs& a, int grid, hipStream_t s, hipError_t* e);

}  // namespace atk

#define AT_LAUNCH_CASE(K, H_, S_, F32_, PPT_)                                         \
    if (k.kind == (K) && k.H == (H_) && k.S == (S_) && k.f32 == ((F32_) != 0) &&      \
        k.ppt == (PPT_)) {                                                            \
        *e = launch_variant<AT_CFG(K, H_, S_, F32_, PPT_)>(a, grid, s);               \
        return true;                                                                  \
    }

#define AT_DEFINE_LAUNCHER(NAME, LIST)                                                           \
    namespace atk {                                                                              \
    bool NAME(const VariantKey& k, const KArgs& a, int grid, hipStream_t s, hipError_t* e) {     \
        LIST(AT_LAUNCH_CASE)                                                                     \
        return false;                                                                            \
    }                                                                                            \
    }
