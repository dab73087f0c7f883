// Materialised multilevel Toeplitz matrices T = [f(k-h)] and T_l = [f(k-h+e_l)]
// (Sec. 1). The write of N*N complex128 values is the whole cost, so the kernel
// streams rows with coalesced 16-byte stores: each block writes kRows rows of
// kCols columns and strides over the rows when N/kRows exceeds the grid.
// Ordinary stores measured faster than non-temporal ones here (6.9 against
// 5.2 TB/s for N = 4096), and few rows per block keep every CU busy.
#include "common.h"

namespace prony {
namespace {

constexpr int kCols = 256;     // threads per block = columns per block
constexpr int kRows = 4;       // rows per block and row stride step
constexpr int kMaxRowBlocks = 65535;
typedef double vdouble2 __attribute__((ext_vector_type(2)));   // one 16-byte access

__global__ __launch_bounds__(kCols) void toeplitz_kernel(int d, int n, int N, int base,
                                                         const vdouble2* __restrict__ f,
                                                         vdouble2* __restrict__ out, int64_t ld) {
    const int h = blockIdx.x * kCols + threadIdx.x;
    if (h >= N) return;
    const int gh = grid_offset_of_index(h, d, n);
    for (int k0 = blockIdx.y * kRows; k0 < N; k0 += gridDim.y * kRows) {
        const int kend = min(k0 + kRows, N);
        for (int k = k0; k < kend; ++k) {
            const int gk = grid_offset_of_index(k, d, n);   // uniform across the block
            out[(int64_t)k * ld + h] = f[gk - gh + base];
        }
    }
}

}  // namespace
}  // namespace prony

using namespace prony;

extern "C" prony_status_t prony_build_T(prony_handle_t h, int d, int n, int which, const double* f,
                                        double* out, int64_t ld) {
    if (!h) return PRONY_EINVAL;
    prony_status_t st = check_dn(h, d, n);
    if (st != PRONY_OK) return st;
    if (which < 0 || which > d) return fail(h, PRONY_EINVAL, "prony_build_T: which must be in 0..d");
    if (!f || !out) return fail(h, PRONY_EINVAL, "prony_build_T: null pointer");
    const int64_t N = ipow(n + 1, d);
    if (ld < N) return fail(h, PRONY_EINVAL, "prony_build_T: ld < N");
    if ((double)N * (double)ld >= 4.0e18) return fail(h, PRONY_ENOTSUP, "prony_build_T: matrix too large");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    const int base = grid_center(d, n) + grid_shift(d, n, which);
    dim3 grid((unsigned)((N + kCols - 1) / kCols), (unsigned)std::min<int64_t>((N + kRows - 1) / kRows, kMaxRowBlocks));
    {
        ProfileScope prof(h, "toeplitz");
        toeplitz_kernel<<<grid, kCols, 0, h->stream>>>(d, n, (int)N, base, reinterpret_cast<const vdouble2*>(f),
                                                       reinterpret_cast<vdouble2*>(out), ld);
    }
    return check_launch(h, "toeplitz_kernel");
}
