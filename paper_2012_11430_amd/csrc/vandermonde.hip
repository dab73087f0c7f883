// Vandermonde products of the coefficient least-squares step (Sec. 1, eq. ls_probl;
// Algorithm 1, last line): A^T[k,j] = prod_l z_j(l)^{k_l}, gram = (A^T)^* A^T and
// rhs = (A^T)^* f_I, reduced over k in I_n. FP64 throughout.
//
// coeffs_tiles: a workgroup evaluates rows of A^T into LDS 16 at a time
//               (integer powers by binary exponentiation), optionally writes
//               them out, and accumulates its part of the Gram matrix and
//               right-hand side.
// coeffs_finish: sums the parts in a fixed order (reduce.h).
#include <algorithm>

#include "common.h"
#include "reduce.h"

namespace prony {
namespace {

constexpr int kRows = 16;        // rows of A^T per chunk
constexpr int kThreads = 256;
constexpr int kMaxM = 64;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ double2 cpow_int(double2 z, int e) {
    double2 r = make_double2(1.0, 0.0);
    double2 b = z;
    while (e) {
        if (e & 1) r = cmul(r, b);
        e >>= 1;
        if (e) b = cmul(b, b);
    }
    return r;
}

constexpr int kEntries = (kMaxM * kMaxM + kMaxM + kThreads - 1) / kThreads;

// Entry e of (A^T)^* [A^T | f_I]: the first m*m are the Gram matrix, the last m the rhs.
__device__ __forceinline__ void emit_gram(int m, double2* __restrict__ gram, double2* __restrict__ rhs, int e,
                                          double re, double im) {
    if (e < m * m)
        gram[e] = make_double2(re, im);
    else
        rhs[e - m * m] = make_double2(re, im);
}

// One workgroup takes `chunks` consecutive 16-row chunks of I_n. Per chunk the
// rows of A^T are evaluated into LDS, then every thread accumulates its fixed
// entries of (A^T)^* [A^T | f_I] over the chunk in FP64 registers. The
// workgroup's sums are stored as one row of partials; coeffs_finish adds the
// rows in workgroup order (bitwise reproducible) and writes gram and rhs.
__global__ __launch_bounds__(kThreads) void coeffs_tiles(int d, int n, int N, int m, int chunks,
                                                         const double2* __restrict__ z,
                                                         const double2* __restrict__ f, double2* __restrict__ at_out,
                                                         double2* __restrict__ part) {
    __shared__ double2 sz[kMaxM * 3];
    __shared__ double2 sa[kRows * kMaxM];
    __shared__ double2 sf[kRows];
    const int tid = threadIdx.x;
    const int tot = m * m + m;
    for (int i = tid; i < m * d; i += kThreads) sz[i] = z[i];
    const int c0 = grid_center(d, n);
    const int P = n + 1;
    double re[kEntries], im[kEntries];
#pragma unroll
    for (int u = 0; u < kEntries; ++u) re[u] = im[u] = 0.0;

    const int nchunks = (N + kRows - 1) / kRows;
    const int c_end = min((blockIdx.x + 1) * chunks, nchunks);
    for (int ch = blockIdx.x * chunks; ch < c_end; ++ch) {
        const int k0 = ch * kRows;
        __syncthreads();
        for (int r = tid; r < kRows; r += kThreads) {
            const int k = k0 + r;
            sf[r] = k < N ? f[grid_offset_of_index(k, d, n) + c0] : make_double2(0.0, 0.0);
        }
        for (int e = tid; e < kRows * m; e += kThreads) {
            const int r = e / m, j = e - (e / m) * m;
            const int k = k0 + r;
            double2 a = make_double2(0.0, 0.0);
            if (k < N) {
                a = make_double2(1.0, 0.0);
                int rem = k;
                for (int l = d - 1; l >= 0; --l) {
                    const int q = rem / P;
                    a = cmul(a, cpow_int(sz[j * d + l], rem - q * P));
                    rem = q;
                }
                if (at_out) at_out[(size_t)k * m + j] = a;
            }
            sa[r * kMaxM + j] = a;
        }
        __syncthreads();
        const int rows = min(kRows, N - k0);
#pragma unroll
        for (int u = 0; u < kEntries; ++u) {
            const int e = tid + u * kThreads;
            if (e < tot) {
                const int i = e < m * m ? e / m : e - m * m;
                const int j = e < m * m ? e - (e / m) * m : -1;
                for (int r = 0; r < rows; ++r) {
                    const double2 ai = sa[r * kMaxM + i];
                    const double2 b = j >= 0 ? sa[r * kMaxM + j] : sf[r];
                    // conj(ai) * b
                    re[u] = fma(ai.x, b.x, fma(ai.y, b.y, re[u]));
                    im[u] = fma(ai.x, b.y, fma(-ai.y, b.x, im[u]));
                }
            }
        }
    }
    double2* out = part + (size_t)blockIdx.x * tot;
#pragma unroll
    for (int u = 0; u < kEntries; ++u) {
        const int e = tid + u * kThreads;
        if (e < tot) out[e] = make_double2(re[u], im[u]);
    }
}

// Sum of the workgroup parts (reduce.h) into gram and rhs.
__global__ __launch_bounds__(kFinishThreads) void coeffs_finish(int m, int rows, const double2* __restrict__ part,
                                                                double2* __restrict__ gram,
                                                                double2* __restrict__ rhs) {
    finish_rows(part, rows, m * m + m, blockIdx.x * kFinishOuts,
                [&](int e, double re, double im) { emit_gram(m, gram, rhs, e, re, im); });
}

constexpr int kMaxWorkgroups = 256;   // one 16-row chunk each for N <= 4096

}  // namespace

size_t coeffs_workspace_bytes(int d, int n, int m) {
    (void)d;
    (void)n;
    return align_up((size_t)kMaxWorkgroups * (m * m + m) * sizeof(double2), 256);
}

}  // namespace prony

using namespace prony;

extern "C" prony_status_t prony_coeffs(prony_handle_t h, int d, int n, int m, const double* z, const double* f,
                                       double* gram, double* rhs, double* AT_out) {
    if (!h) return PRONY_EINVAL;
    prony_status_t st = check_dn(h, d, n);
    if (st != PRONY_OK) return st;
    const int64_t N = ipow(n + 1, d);
    if (m < 1 || m > N) return fail(h, PRONY_EINVAL, "prony_coeffs: m must be in 1..N");
    if (m > kMaxM) return fail(h, PRONY_ENOTSUP, "prony_coeffs: m > 64 is not supported");
    if (!z || !f || !gram || !rhs) return fail(h, PRONY_EINVAL, "prony_coeffs: null pointer");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    if ((st = ensure_workspace(h, coeffs_workspace_bytes(d, n, m))) != PRONY_OK) return st;
    const int nchunks = (int)((N + kRows - 1) / kRows);
    const int chunks = (nchunks + kMaxWorkgroups - 1) / kMaxWorkgroups;
    const int wgs = (nchunks + chunks - 1) / chunks;
    double2* part = static_cast<double2*>(h->ws);
    {
        ProfileScope prof(h, "coeffs_tiles");
        coeffs_tiles<<<wgs, kThreads, 0, h->stream>>>(d, n, (int)N, m, chunks, reinterpret_cast<const double2*>(z),
                                                      reinterpret_cast<const double2*>(f),
                                                      reinterpret_cast<double2*>(AT_out), part);
    }
    if ((st = check_launch(h, "coeffs_tiles")) != PRONY_OK) return st;
    {
        ProfileScope prof(h, "coeffs_finish");
        const int tot = m * m + m;
        coeffs_finish<<<(tot + kFinishOuts - 1) / kFinishOuts, kFinishThreads, 0, h->stream>>>(
            m, wgs, part, reinterpret_cast<double2*>(gram), reinterpret_cast<double2*>(rhs));
    }
    return check_launch(h, "coeffs_finish");
}
