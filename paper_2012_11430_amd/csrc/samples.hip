// Samples of the exponential sum on the grid {-n..n+1}^d (Sec. 1, eq. exp_sum),
// with the additive noise model of Sec. 4.
#include "common.h"

namespace prony {
namespace {

constexpr int kThreads = 64;    // small blocks: grids of 1e4 points still spread over all CUs
constexpr int kTermsPerStage = 256;   // nodes/coefficients staged in LDS per pass

// One thread per grid point p; the m terms are staged through LDS in groups.
__global__ __launch_bounds__(kThreads) void samples_kernel(int d, int n, int m, int gsize,
                                                           const double* __restrict__ t,
                                                           const double2* __restrict__ c,
                                                           const double2* __restrict__ noise,
                                                           double2* __restrict__ f) {
    __shared__ double st[kTermsPerStage * 3];
    __shared__ double2 sc[kTermsPerStage];
    const int gidx = blockIdx.x * kThreads + threadIdx.x;
    const int Q = 2 * n + 2;
    double p[3] = {0.0, 0.0, 0.0};
    {
        int r = gidx < gsize ? gidx : 0;
        for (int l = d - 1; l >= 0; --l) {
            const int q = r / Q;
            p[l] = double(r - q * Q - n);
            r = q;
        }
    }
    double re = 0.0, im = 0.0;
    for (int base = 0; base < m; base += kTermsPerStage) {
        const int cnt = min(kTermsPerStage, m - base);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * d; i += kThreads) st[i] = t[base * d + i];
        for (int i = threadIdx.x; i < cnt; i += kThreads) sc[i] = c[base + i];
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            double theta = 0.0;
            for (int l = 0; l < d; ++l) theta = fma(st[j * d + l], p[l], theta);
            theta -= rint(theta);   // exp(-2 pi i x) has period 1 in x
            double s, co;
            sincospi(2.0 * theta, &s, &co);
            // c_j * (cos - i sin)
            const double2 cj = sc[j];
            re = fma(cj.x, co, fma(cj.y, s, re));
            im = fma(cj.y, co, fma(-cj.x, s, im));
        }
    }
    if (gidx < gsize) {
        if (noise) {
            const double2 nz = noise[gidx];
            re += nz.x;
            im += nz.y;
        }
        f[gidx] = make_double2(re, im);
    }
}

}  // namespace
}  // namespace prony

using namespace prony;

extern "C" prony_status_t prony_samples(prony_handle_t h, int d, int n, int m, const double* t,
                                        const double* c, const double* noise, double* f) {
    if (!h) return PRONY_EINVAL;
    prony_status_t st = check_dn(h, d, n);
    if (st != PRONY_OK) return st;
    if (m < 1 || m > 4096) return fail(h, PRONY_EINVAL, "prony_samples: m must be in 1..4096");
    if (!t || !c || !f) return fail(h, PRONY_EINVAL, "prony_samples: null pointer");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    const int gsize = (int)ipow(2 * n + 2, d);
    const int blocks = (gsize + kThreads - 1) / kThreads;
    {
        ProfileScope prof(h, "samples");
        samples_kernel<<<blocks, kThreads, 0, h->stream>>>(d, n, m, gsize, t, reinterpret_cast<const double2*>(c),
                                                           reinterpret_cast<const double2*>(noise),
                                                           reinterpret_cast<double2*>(f));
    }
    return check_launch(h, "samples_kernel");
}
