// Deterministic reduction of per-workgroup partial rows in a separate launch.
//
// The fused kernels store one row of `tot` pairs per workgroup. A finishing
// launch (visibility of the rows is given by the kernel boundary) sums them:
// a workgroup of 256 threads owns 16 consecutive outputs; thread (row lane rl,
// output o) sums rows rl, rl+16, ... in order, with up to 16 loads in flight,
// then the 16 row lanes of each output are added in lane order (FP64). The
// result does not depend on scheduling.
#pragma once

#include "common.h"

namespace prony {

constexpr int kFinishThreads = 256;
constexpr int kFinishOuts = 16;                         // outputs per workgroup
constexpr int kFinishLanes = kFinishThreads / kFinishOuts;

// Sum over `nrows` rows of column o0 + (tid % 16) of the row-major array `rows`
// (row length tot). Calls emit(o, re, im) once per owned output (o < tot).
template <typename P2, typename Emit>
__device__ __forceinline__ void finish_rows(const P2* __restrict__ rows, int nrows, int tot, int o0, Emit emit) {
    __shared__ double2 red[kFinishLanes][kFinishOuts];
    const int tid = threadIdx.x;
    const int oi = tid % kFinishOuts, rl = tid / kFinishOuts;
    const int o = o0 + oi;
    double re = 0.0, im = 0.0;
    if (o < tot) {
        constexpr int kBatch = 16;
        for (int r0 = rl; r0 < nrows; r0 += kBatch * kFinishLanes) {
            P2 v[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int r = r0 + u * kFinishLanes;
                if (r < nrows) v[u] = rows[(size_t)r * tot + o];
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (r0 + u * kFinishLanes < nrows) {
                    re += (double)v[u].x;
                    im += (double)v[u].y;
                }
            }
        }
    }
    red[rl][oi] = make_double2(re, im);
    __syncthreads();
    if (rl == 0 && o < tot) {
        re = 0.0;
        im = 0.0;
        for (int k = 0; k < kFinishLanes; ++k) {
            re += red[k][oi].x;
            im += red[k][oi].y;
        }
        emit(o, re, im);
    }
}

}  // namespace prony
