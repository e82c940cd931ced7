// tfft_ragged_kernel.hpp -- the persistent kernel for ragged batches.
//
// Workgroups pull work items from an atomic queue until it is empty and run
// the item's plan through a switch over the ragged plan list, every case
// inlined.  Descriptors are read through wave-uniform constant-space
// pointers, so the per-class arguments sit in scalar registers as kernel
// arguments do in a plain launch.  All plans share one dynamic LDS buffer,
// preceded by a slot for the item index.  Included once per ABFT mode
// (inst_ragged_ft*.hip) so the three kernels compile in parallel.
#pragma once

#include "tfft_ragged.hpp"
#include "tfft_ragged_plans.hpp"

namespace tfft {

extern __shared__ __align__(16) char tfft_ragged_smem[];

template <int FT> constexpr int ragged_plan_smem() {
    int m = 0;
#define TFFT_SMEM_MAX(id, kind, Ns, E, WC, B, ...)                                                   \
    {                                                                                                \
        constexpr int b = Smem<float2, TFFT_PLAN_T(id, kind, Ns, E, WC, B, __VA_ARGS__), FT, true>::BYTES; \
        m = m > b ? m : b;                                                                           \
    }
    TFFT_RAGGED_PLANS(TFFT_SMEM_MAX)
#undef TFFT_SMEM_MAX
    return m;
}
template <int FT> constexpr int ragged_smem() { return kRaggedSlotBytes + ragged_plan_smem<FT>(); }
static_assert(ragged_smem<2>() <= 65536, "ragged plans must fit 64 KiB of LDS");

#define TFFT_CHECK_WIDTH(id, kind, Ns, E, WC, B, ...)                                              \
    static_assert(TFFT_PLAN_T(id, kind, Ns, E, WC, B, __VA_ARGS__)::THREADS == kRaggedThreads, \
                  "every ragged plan runs 256-lane workgroups");
TFFT_RAGGED_PLANS(TFFT_CHECK_WIDTH)
#undef TFFT_CHECK_WIDTH

// ---- wave-uniform values and constant-space views ----
template <class T> using cptr = const __attribute__((address_space(4))) T*;

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni(long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}
template <class T> __device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)(unsigned long long)uni(reinterpret_cast<long long>(p));
}
// copy of a descriptor from constant space (scalar loads)
template <class T> __device__ __forceinline__ T cload(cptr<T> p) {
    static_assert(sizeof(T) % 4 == 0, "descriptors are whole dwords");
    T v;
    unsigned* dv = reinterpret_cast<unsigned*>(&v);
    const cptr<unsigned> s = (cptr<unsigned>)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dv[i] = s[i];
    return v;
}

// Publish thread 0's item index to the whole workgroup.  The leading
// barrier also ends the previous item's use of the LDS buffer.
__device__ __forceinline__ long long share_item(long long mine) {
    volatile long long* slot = reinterpret_cast<volatile long long*>(tfft_ragged_smem);
    __syncthreads();
    if (threadIdx.x == 0) *slot = mine;
    __syncthreads();
    return uni(*slot);
}


// One work item.  Column passes write the workspace with coherent stores and
// row passes read it with coherent loads, so handing results from one pass
// to the other needs no cache-wide write-back or invalidation: the column
// pass waits for its stores to complete before it counts itself done, and a
// row pass starts loading only after every count of its group is in.
// Thread 0 waits until *ctr reaches need (bounded; see kMaxPolls).
__device__ __forceinline__ void wait_count(const RaggedCall& c, const RaggedDesc& d, unsigned* ctr,
                                           unsigned need) {
    unsigned polls = 0;
    need += c.wait_extra;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (++polls > c.max_polls ||
            __hip_atomic_load(&d.q->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull) {
            atomicOr(&d.q->err, 1ull);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

template <class PL, int FT, int... Rs>
__device__ __forceinline__ void ragged_step(const RaggedCall& c, const RaggedDesc& d,
                                            cptr<RClass> cl, const RItem& it) {
    constexpr int COH = PL::KIND == kColPass ? 1 : PL::KIND == kRowPass ? 2 : 0;
    const int blk = it.blk, nblk = it.nblk;
    const int tiles = cl->tiles;
    const int need = cl->need;
    const int grp = tiles > 0 ? blk / tiles : 0;
    const int cnt = cl->cnt_base + grp;
    if constexpr (PL::KIND == kColPass) {
        // windowed workspace: the half this batch writes has been read out
        if (it.wait_batch >= 0) {
            if (threadIdx.x == 0) wait_count(c, d, &d.cnt_r[it.wait_batch], (unsigned)it.wait_need);
            __syncthreads();
        }
    }
    if constexpr (PL::KIND == kRowPass) {
        // every column-pass item of this group has finished
        if (threadIdx.x == 0) {
            wait_count(c, d, &d.cnt_a[cnt], (unsigned)need);
            // the last row-pass item of the group resets both counters for
            // the next launch; the others have all passed their wait
            if (atomicAdd(&d.cnt_b[cnt], 1u) == (unsigned)(cl->items_per_group - 1)) {
                atomicExch(&d.cnt_a[cnt], 0u);
                atomicExch(&d.cnt_b[cnt], 0u);
            }
        }
        __syncthreads();
    }
    // the class's arguments are read in place from constant memory (scalar
    // loads the compiler may repeat instead of holding them in registers, as
    // it does for kernel arguments); only the per-call part is built here
    const KArgs<float2>& ka = *(const KArgs<float2>*)&cl->args;
    const int final_pass = PL::KIND != kColPass;
    KCall<float> kc{};
    kc.conj_in = PL::KIND == kRowPass ? 0 : c.conj;
    kc.conj_out = final_pass ? c.conj : 0;
    kc.scale = (final_pass && c.conj && !c.unit_scale) ? 1.0f / (float)ka.N : 1.0f;
    kc.counts = c.counts;
    kc.stats = c.stats;
    {
        // pass 0: the single pass or the column pass; pass 1: the row pass
        constexpr int kPass = PL::KIND == kRowPass ? 1 : 0;
        constexpr int kPasses = PL::KIND == kSingle ? 1 : 2;
        const int want = c.inj_pass < 0 ? kPasses - 1 : c.inj_pass;
        kc.inj_signal = want == kPass ? c.inj_signal : -1;
        kc.inj_signal2 = want == kPass ? c.inj_signal2 : -1;
        kc.inj_stage = c.inj_stage < 0 ? (int)sizeof...(Rs) - 1 : c.inj_stage;
    }
    kc.inj_elem = c.inj_elem;
    kc.inj_part = c.inj_part;
    kc.inj_bit = c.inj_bit;
    const float2* src = PL::KIND == kRowPass ? d.ws : c.x;
    float2* dst = PL::KIND == kColPass ? d.ws : c.y;
    const int nblocks = cl->nblocks;
    for (int b = blk; b < blk + nblk; ++b) {
        if (b != blk) __syncthreads();   // the previous block is done with the LDS buffer
        fft_body<float2, PL, FT, true, COH, false, Rs...>(src, dst, ka, kc, b, nblocks,
                                                   tfft_ragged_smem + kRaggedSlotBytes);
    }
    if constexpr (PL::KIND == kColPass) {
        __builtin_amdgcn_s_waitcnt(0);   // this lane's workspace stores are complete
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&d.cnt_a[cnt], 1u);
    }
    if constexpr (PL::KIND == kRowPass) {
        if (it.batch >= 0) {   // this item's workspace reads are complete
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (threadIdx.x == 0) atomicAdd(&d.cnt_r[it.batch], 1u);
        }
    }
}

template <int FT>
__device__ __forceinline__ void ragged_loop(const RaggedCall& c, const RaggedDesc* dp) {
    const long long n_items = cload(as_const(dp)).n_items;
    long long item = share_item(threadIdx.x == 0 ? (long long)atomicAdd(&cload(as_const(dp)).q->next, 1ull) : 0);
    while (item < n_items) {
        // the descriptor is read again each item (an opaque pointer keeps the
        // compiler from holding all of it in registers across the item)
        const RaggedDesc* dpi = dp;
        asm volatile("" : "+s"(dpi));
        const RaggedDesc d = cload(as_const(dpi));
        // take the next item now; its index is waited for only after this one.
        // Every item waits only on items queued before it, so an item taken
        // while this one waits is never one it waits for.
        unsigned long long pre = 0;
        if (threadIdx.x == 0) pre = atomicAdd(&d.q->next, 1ull);
        const RItem it = cload(as_const(d.items) + item);
        cptr<RClass> cl = as_const(d.classes) + it.cls;
        switch (cl->plan) {
#define TFFT_CASE(id, kind, Ns, E, WC, B, ...)                                                 \
    case id:                                                                                    \
        ragged_step<TFFT_PLAN_T(id, kind, Ns, E, WC, B, __VA_ARGS__), FT, __VA_ARGS__>(c, d, cl, \
                                                                                      it);       \
        break;
            TFFT_RAGGED_PLANS(TFFT_CASE)
#undef TFFT_CASE
            default:   // not a plan of this list: the host never queues one
                break;
        }
        item = share_item((long long)pre);
    }
    // the last workgroup out resets the queue and the batch counters for the
    // next launch
    const RaggedDesc d = cload(as_const(dp));
    const long long last =
        share_item(threadIdx.x == 0 && atomicAdd(&d.q->done, 1ull) == (unsigned long long)gridDim.x - 1ull
                       ? 1
                       : 0);
    if (last) {
        // every other workgroup has left the loop, so every item has finished
        // and no counter changes any more
        const unsigned long long err =
            uni((long long)__hip_atomic_load(&d.q->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        for (long long i = threadIdx.x; i < d.n_batches; i += kRaggedThreads) atomicExch(&d.cnt_r[i], 0u);
        if (err != 0ull) {
            // a wait gave up: the per-group counters may be out of step
            for (long long i = threadIdx.x; i < d.n_groups; i += kRaggedThreads) {
                atomicExch(&d.cnt_a[i], 0u);
                atomicExch(&d.cnt_b[i], 0u);
            }
        }
        if (threadIdx.x == 0) {
            if (err != 0ull) {
                atomicAdd(&d.q->err_launches, 1ull);
                if (c.counts) atomicAdd(&c.counts->sched_errors, 1ull);
                atomicExch(&d.q->err, 0ull);
            }
            atomicExch(&d.q->next, 0ull);
            atomicExch(&d.q->done, 0ull);
        }
    }
}

// The register budget is the compiler's choice (two workgroups per CU for
// the ABFT modes) or held to three workgroups per CU, at the price of a few
// spilled values; which is faster is a measured, per-plan choice.
template <int FT>
__global__ __launch_bounds__(kRaggedThreads) void k_ragged(RaggedCall c, const RaggedDesc* dp) {
    ragged_loop<FT>(c, dp);
}
template <int FT>
__global__ __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void
k_ragged_w3(RaggedCall c, const RaggedDesc* dp) {
    ragged_loop<FT>(c, dp);
}

template <int FT, bool W3>
hipError_t launch_ragged(const RaggedCall& c, const RaggedDesc* d, int grid, hipStream_t s) {
    if constexpr (W3)
        hipLaunchKernelGGL((k_ragged_w3<FT>), dim3(grid), dim3(kRaggedThreads), ragged_smem<FT>(), s, c, d);
    else
        hipLaunchKernelGGL((k_ragged<FT>), dim3(grid), dim3(kRaggedThreads), ragged_smem<FT>(), s, c, d);
    return hipGetLastError();
}

template <int FT, bool W3> RaggedKernel make_ragged_kernel() {
    RaggedKernel k{};
    k.launch = &launch_ragged<FT, W3>;
    k.lds_bytes = ragged_smem<FT>();
    int n = 0;
    hipError_t e;
    if constexpr (W3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ragged_w3<FT>, kRaggedThreads, ragged_smem<FT>());
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ragged<FT>, kRaggedThreads, ragged_smem<FT>());
    k.blocks_per_cu = e == hipSuccess ? n : 0;
    return k;
}

}  // namespace tfft
