// Deterministic multi-workgroup reduction used by the fused kernels: every
// workgroup of a launch stores one row of `tot` pairs; the last workgroup to
// finish in each group of kFanIn rows sums them (FP64, row order) into a row of
// the next level, until one workgroup holds the total and hands each entry to
// `emit(o, re, im)`. Loads of a group are issued together. Release/acquire
// fences (__threadfence) order rows written on other XCDs before the counter
// atomics and the reads; every counter is back at zero before the launch ends.
#pragma once

#include "common.h"

namespace prony {

constexpr int kFanIn = 16;

// Tree nodes above the leaves for `count` rows (rows of `upper` and counters used).
__host__ __device__ inline int tree_nodes(int count) {
    int nodes = 0;
    for (int c = count; c > 1; c = (c + kFanIn - 1) / kFanIn) nodes += (c + kFanIn - 1) / kFanIn;
    return nodes;
}

// Sum of rows [beg, end) (at most kFanIn) of a row-major array of `tot` pairs,
// column o, in FP64 and row order; all loads are issued before the additions.
template <typename P2>
__device__ __forceinline__ void sum_rows(const P2* __restrict__ src, int tot, int beg, int end, int o, double& re,
                                         double& im) {
    P2 v[kFanIn];
#pragma unroll
    for (int u = 0; u < kFanIn; ++u)
        if (beg + u < end) v[u] = src[(size_t)(beg + u) * tot + o];
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
// (`leaves` + slot * tot) has been stored; count > 1 rows in the launch.
template <int THREADS, typename P2, typename Emit>
__device__ __forceinline__ void tree_reduce(const P2* __restrict__ leaves, double2* __restrict__ upper,
                                            unsigned* __restrict__ counters, int count, int slot, int tot,
                                            int* s_last, Emit emit) {
    const int tid = threadIdx.x;
    int cbase = 0, rbase = 0;
    bool first_level = true;
    for (;;) {
        __threadfence();
        __syncthreads();
        const int grp = slot / kFanIn;
        const int beg = grp * kFanIn;
        const int end = min(beg + kFanIn, count);
        if (tid == 0) *s_last = atomicAdd(&counters[cbase + grp], 1u) == (unsigned)(end - beg - 1);
        __syncthreads();
        if (!*s_last) return;
        __threadfence();
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
                dst[o] = make_double2(re, im);
        }
        if (tid == 0) counters[cbase + grp] = 0u;
        if (groups == 1) return;
        cbase += groups;
        rbase += groups;
        count = groups;
        slot = grp;
        first_level = false;
    }
}

}  // namespace prony
