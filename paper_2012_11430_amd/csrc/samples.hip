// Samples of the exponential sum on the grid {-n..n+1}^d (Sec. 1, eq. exp_sum),
// with the additive noise model of Sec. 4.
#include "common.h"

namespace prony {
namespace {

constexpr int kThreads = 256;
constexpr int kLanesPerPoint = 4;     // the terms of one grid point are split over a lane quad
constexpr int kPointsPerBlock = kThreads / kLanesPerPoint;
constexpr int kTermsPerStage = 256;   // nodes/coefficients staged in LDS per pass

// Lane quad q of a block evaluates grid point p; lane s of the quad sums the
// terms j = s, s+4, ... . The quad adds its four sums in lane order (DPP
// quad permutations, fixed order), and lane 0 adds the noise and stores.
template <int S>
__device__ __forceinline__ double quad_lane(double x) {
    constexpr int sel = S * 0x55;   // quad_perm [S, S, S, S]
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(v & 0xffffffffll), sel, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), sel, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ __launch_bounds__(kThreads) void samples_kernel(int d, int n, int m, int gsize,
                                                           const double* __restrict__ t,
                                                           const double2* __restrict__ c,
                                                           const double2* __restrict__ noise,
                                                           double2* __restrict__ f) {
    __shared__ double st[kTermsPerStage * 3];
    __shared__ double2 sc[kTermsPerStage];
    const int sub = threadIdx.x & (kLanesPerPoint - 1);
    const int gidx = blockIdx.x * kPointsPerBlock + threadIdx.x / kLanesPerPoint;
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
        for (int j = sub; j < cnt; j += kLanesPerPoint) {
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
    // every lane of the block is active here (no early exit above)
    const double re_sum = ((quad_lane<0>(re) + quad_lane<1>(re)) + quad_lane<2>(re)) + quad_lane<3>(re);
    const double im_sum = ((quad_lane<0>(im) + quad_lane<1>(im)) + quad_lane<2>(im)) + quad_lane<3>(im);
    if (sub == 0 && gidx < gsize) {
        double2 v = make_double2(re_sum, im_sum);
        if (noise) {
            const double2 nz = noise[gidx];
            v.x += nz.x;
            v.y += nz.y;
        }
        f[gidx] = v;
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
    const int blocks = (gsize + kPointsPerBlock - 1) / kPointsPerBlock;
    {
        ProfileScope prof(h, "samples");
        samples_kernel<<<blocks, kThreads, 0, h->stream>>>(d, n, m, gsize, t, reinterpret_cast<const double2*>(c),
                                                           reinterpret_cast<const double2*>(noise),
                                                           reinterpret_cast<double2*>(f));
    }
    return check_launch(h, "samples_kernel");
}
