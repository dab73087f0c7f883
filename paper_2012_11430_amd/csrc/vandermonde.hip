// Vandermonde products of the coefficient least-squares step (Sec. 1, eq. ls_probl;
// Algorithm 1, last line): A^T[k,j] = prod_l z_j(l)^{k_l}, gram = (A^T)^* A^T and
// rhs = (A^T)^* f_I, reduced over k in I_n. FP64 throughout.
//
// coeffs_tiles: one workgroup per 64 rows k. The rows of A^T are evaluated into
//               LDS (integer powers by binary exponentiation), optionally
//               written out, then the 64-row partial Gram matrix and right-hand
//               side are formed from LDS and stored.
// coeffs_reduce: sums the per-tile partials in a fixed order.
#include <algorithm>

#include "common.h"

namespace prony {
namespace {

constexpr int kRows = 64;
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

__global__ __launch_bounds__(kThreads) void coeffs_tiles(int d, int n, int N, int m, const double2* __restrict__ z,
                                                         const double2* __restrict__ f, double2* __restrict__ at_out,
                                                         double2* __restrict__ part) {
    __shared__ double2 sz[kMaxM * 3];
    __shared__ double2 sa[kRows * kMaxM];
    __shared__ double2 sf[kRows];
    const int tid = threadIdx.x;
    const int k0 = blockIdx.x * kRows;
    for (int i = tid; i < m * d; i += kThreads) sz[i] = z[i];
    const int c0 = grid_center(d, n);
    for (int r = tid; r < kRows; r += kThreads) {
        const int k = k0 + r;
        sf[r] = k < N ? f[grid_offset_of_index(k, d, n) + c0] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int P = n + 1;
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
    double2* out = part + (size_t)blockIdx.x * (m * m + m);
    const int rows = min(kRows, N - k0);
    for (int e = tid; e < m * m + m; e += kThreads) {
        const int i = e < m * m ? e / m : e - m * m;
        const int j = e < m * m ? e - (e / m) * m : -1;
        double re = 0.0, im = 0.0;
        for (int r = 0; r < rows; ++r) {
            const double2 ai = sa[r * kMaxM + i];
            const double2 b = j >= 0 ? sa[r * kMaxM + j] : sf[r];
            // conj(ai) * b
            re = fma(ai.x, b.x, fma(ai.y, b.y, re));
            im = fma(ai.x, b.y, fma(-ai.y, b.x, im));
        }
        out[e] = make_double2(re, im);
    }
}

__global__ __launch_bounds__(kThreads) void coeffs_reduce(int m, int tiles, const double2* __restrict__ part,
                                                          double2* __restrict__ gram, double2* __restrict__ rhs) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    const int tot = m * m + m;
    if (e >= tot) return;
    double re = 0.0, im = 0.0;
    for (int t = 0; t < tiles; ++t) {
        const double2 v = part[(size_t)t * tot + e];
        re += v.x;
        im += v.y;
    }
    if (e < m * m)
        gram[e] = make_double2(re, im);
    else
        rhs[e - m * m] = make_double2(re, im);
}

}  // namespace

size_t coeffs_workspace_bytes(int d, int n, int m) {
    const int64_t N = ipow(n + 1, d);
    const int64_t tiles = (N + kRows - 1) / kRows;
    return align_up((size_t)tiles * (m * m + m) * sizeof(double2), 256);
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
    const int tiles = (int)((N + kRows - 1) / kRows);
    double2* part = static_cast<double2*>(h->ws);
    {
        ProfileScope prof(h, "coeffs_tiles");
        coeffs_tiles<<<tiles, kThreads, 0, h->stream>>>(d, n, (int)N, m, reinterpret_cast<const double2*>(z),
                                                        reinterpret_cast<const double2*>(f),
                                                        reinterpret_cast<double2*>(AT_out), part);
    }
    if ((st = check_launch(h, "coeffs_tiles")) != PRONY_OK) return st;
    const int tot = m * m + m;
    {
        ProfileScope prof(h, "coeffs_reduce");
        coeffs_reduce<<<(tot + kThreads - 1) / kThreads, kThreads, 0, h->stream>>>(
            m, tiles, part, reinterpret_cast<double2*>(gram), reinterpret_cast<double2*>(rhs));
    }
    return check_launch(h, "coeffs_reduce");
}
