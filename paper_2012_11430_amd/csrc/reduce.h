// Deterministic multi-workgroup reduction used by the fused kernels: every
// workgroup of a launch stores one row of `tot` pairs; the last workgroup to
// finish in each group of kFanIn rows sums them (FP64, row order) into a row of
// the next level, until one workgroup holds the total and hands each entry to
// `emit(o, re, im)`. Loads of a group are issued together.
//
// Cross-XCD visibility without cache-wide fences: the rows are written and read
// with agent-scope relaxed atomic stores/loads (global_store/load ... sc1 on
// gfx950, coherent across the XCDs' L2s), every thread waits for its stores to
// complete (s_waitcnt vmcnt(0)) before the workgroup barrier and the counter
// atomic, so a workgroup that sees the group count complete reads complete rows.
// An agent-scope __threadfence would write back and invalidate the whole L2 of
// the XCD for every workgroup. Every counter is back at zero before the launch
// ends.
#pragma once

#include <cstdint>

#include "common.h"

namespace prony {

constexpr int kFanIn = 16;

// Tree nodes above the leaves for `count` rows (rows of `upper` and counters used).
__host__ __device__ inline int tree_nodes(int count) {
    int nodes = 0;
    for (int c = count; c > 1; c = (c + kFanIn - 1) / kFanIn) nodes += (c + kFanIn - 1) / kFanIn;
    return nodes;
}

// Agent-coherent (cross-XCD) store and load of one pair.
__device__ __forceinline__ void store_coherent(float2* p, float2 v) {
    uint64_t bits;
    __builtin_memcpy(&bits, &v, sizeof(bits));
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent(double2* p, double2 v) {
    __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float2 load_coherent(const float2* p) {
    const uint64_t bits = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    float2 v;
    __builtin_memcpy(&v, &bits, sizeof(v));
    return v;
}
__device__ __forceinline__ double2 load_coherent(const double2* p) {
    return make_double2(__hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Wait until this thread's earlier stores have completed (vmcnt = 0).
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0); }

// Sum of rows [beg, end) (at most kFanIn) of a row-major array of `tot` pairs,
// column o, in FP64 and row order; all loads are issued before the additions.
template <typename P2>
__device__ __forceinline__ void sum_rows(const P2* __restrict__ src, int tot, int beg, int end, int o, double& re,
                                         double& im) {
    P2 v[kFanIn];
#pragma unroll
    for (int u = 0; u < kFanIn; ++u)
        if (beg + u < end) v[u] = load_coherent(&src[(size_t)(beg + u) * tot + o]);
    re = 0.0;
    im = 0.0;
#pragma unroll
    for (int u = 0; u < kFanIn; ++u)
        if (beg + u < end) {
            re += (double)v[u].x;
            im += (double)v[u].y;
        }
}

// Called by every thread of every workgroup after the workgroup's leaf row
// (`leaves` + slot * tot) has been stored with store_coherent; count > 1 rows.
template <int THREADS, typename P2, typename Emit>
__device__ __forceinline__ void tree_reduce(const P2* __restrict__ leaves, double2* __restrict__ upper,
                                            unsigned* __restrict__ counters, int count, int slot, int tot,
                                            int* s_last, Emit emit) {
    const int tid = threadIdx.x;
    int cbase = 0, rbase = 0;
    bool first_level = true;
    for (;;) {
        wait_stores();
        __syncthreads();
        const int grp = slot / kFanIn;
        const int beg = grp * kFanIn;
        const int end = min(beg + kFanIn, count);
        if (tid == 0)
            *s_last = __hip_atomic_fetch_add(&counters[cbase + grp], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                      (unsigned)(end - beg - 1);
        __syncthreads();
        if (!*s_last) return;
        const int groups = (count + kFanIn - 1) / kFanIn;
        double2* dst = upper + (size_t)(rbase + grp) * tot;
        for (int o = tid; o < tot; o += THREADS) {
            double re, im;
            if (first_level)
                sum_rows(leaves, tot, beg, end, o, re, im);
            else
                sum_rows(upper + (size_t)(rbase - count) * tot, tot, beg, end, o, re, im);
            if (groups == 1)
                emit(o, re, im);
            else
                store_coherent(&dst[o], make_double2(re, im));
        }
        if (tid == 0) __hip_atomic_store(&counters[cbase + grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (groups == 1) return;
        cbase += groups;
        rbase += groups;
        count = groups;
        slot = grp;
        first_level = false;
    }
}

}  // namespace prony
