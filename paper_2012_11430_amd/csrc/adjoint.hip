// Adjoint of the pencil map f -> S_l = U^* T_l(f) V Sigma^{-1} (Sec. 1, eq.
// generateSl), with U, Sigma, V held fixed: given gS_l = dL/dS_l (PyTorch's
// convention, grad = dL/dRe + i dL/dIm), the gradient on the sample grid is
//     grad(p) = sum_l sum_{k - h + e_l = p} X_l[k, h],   X_l = U gS_l Sigma^{-1} V^*.
// With k' = k + e_l as in the forward kernel (row-extended form), all d terms are
// one product of the row-extended matrix
//     Z[k', q] = sum_l (U gS_l Sigma^{-1})[k' - e_l, q]   (k' in {0..n+1}^d; a term
//                 is zero where k' - e_l leaves I_n)          ((n+2)^d x m)
// with the conjugated factor W[h, q] = conj(V[h, q]), h in I_n:
//     grad(p) = sum_{k' - h = p} (Z W^T)[k', h],
// i.e. the (n+2)^d x N product (inner dimension m) is summed along its Toeplitz
// diagonals.
//
// adjoint_pack   forms Z (FP64, stored in T), packs W as (Re, Im) pairs,
//                writes the G(h) table and zeroes the gradient;
// adjoint_tiles  one workgroup = 64 rows k' x one chunk of h: for every block of
//                16 h the tile of Z W^T is formed on MFMA (K = m; three real
//                products per complex one: Re z Re w, Im z Im w and
//                (Re z + Im z)(Re w + Im w)), and each
//                entry is added (LDS atomics, accumulation in FP64) to the bin of
//                its diagonal in an LDS copy of the workgroup's grid window; the
//                window is then added to the gradient in FP64 (device atomics).
// The accumulation order inside a bin is not fixed: results agree to rounding,
// not bitwise, between runs.
#include <algorithm>

#include "common.h"
#include "mfma.h"

namespace prony {
namespace {

constexpr int kWaves = 4;
constexpr int kRows = kWaves * 16;
constexpr int kThreads = kWaves * 64;
constexpr int kHBlock = 16;          // h per MFMA output block (32 real columns)

struct AdjPlan {
    int d, n, N, m;
    int NR;        // (n+2)^d row-extended rows k'
    int cp;        // complex K (m) padded to a multiple of 8
    int ksteps;    // cp / 4
    int rf, rows;  // 16-row fragments per wave, rows k' per tile (64 rf)
    int kb, kc, sk, rt, nwg, win_cap, c0, gsize;
    size_t lds_bytes;
    size_t off_z, off_w, off_g, ws_bytes;
};

template <typename T>
__device__ __forceinline__ void adj_pack_body(const AdjPlan& P, const double2* __restrict__ U, int64_t u_rs,
                                              int64_t u_cs, const double* __restrict__ sigma,
                                              const double2* __restrict__ V, int64_t v_rs, int64_t v_cs,
                                              const double2* __restrict__ gS, pair_t<T>* __restrict__ zp,
                                              pair_t<T>* __restrict__ wp, int* __restrict__ gt,
                                              double2* __restrict__ gf, int section) {
    using T2 = pair_t<T>;
    const int stride = gridDim.x * blockDim.x;
    const int first = blockIdx.x * blockDim.x + threadIdx.x;
    const int kbp = P.sk * P.kc;
    if (section == 0) {
        // Z[k'][q] = sum over l (in order) of sum_i U[k'-e_l, i] gS_l[i,q] / sigma_q for
        // the l with k' - e_l in I_n; rows padded to whole tiles and columns to cp with zeros
        const int nz = P.rt * P.rows * P.cp;
        const int E = P.n + 2, Pn = P.n + 1;
        for (int e = first; e < nz; e += stride) {
            const int kr = e / P.cp, q = e - (e / P.cp) * P.cp;
            double re = 0.0, im = 0.0;
            if (kr < P.NR && q < P.m) {
                int dig[3] = {0, 0, 0};
                int rem = kr;
                for (int l = P.d - 1; l >= 0; --l) {
                    dig[l] = rem % E;
                    rem /= E;
                }
                for (int ell = 0; ell < P.d; ++ell) {
                    bool inside = dig[ell] >= 1;
                    int idx = 0;
                    for (int l = 0; l < P.d; ++l) {
                        const int coord = dig[l] - (l == ell ? 1 : 0);
                        inside = inside && coord <= P.n;
                        idx = idx * Pn + coord;
                    }
                    if (!inside) continue;
                    double zr = 0.0, zi = 0.0;
                    for (int i = 0; i < P.m; ++i) {
                        const double2 u = U[idx * u_rs + i * u_cs];
                        const double2 gv = gS[((size_t)ell * P.m + i) * P.m + q];
                        zr = fma(u.x, gv.x, fma(-u.y, gv.y, zr));
                        zi = fma(u.x, gv.y, fma(u.y, gv.x, zi));
                    }
                    re += zr;
                    im += zi;
                }
                const double s = sigma[q];
                re /= s;
                im /= s;
            }
            zp[e] = T2{(T)re, (T)im};
        }
    } else if (section == 1) {
        // W = conj(V) as (Re, Im) pairs, row q, column h
        const int nw = P.cp * kbp;
        for (int e = first; e < nw; e += stride) {
            const int q = e / kbp, hx = e - (e / kbp) * kbp;
            double wr = 0.0, wi = 0.0;
            if (hx < P.kb && q < P.m) {
                const double2 v = V[hx * v_rs + q * v_cs];
                wr = v.x;
                wi = -v.y;   // conj
            }
            wp[e] = T2{(T)wr, (T)wi};
        }
    } else {
        for (int hx = first; hx < kbp; hx += stride)
            gt[hx] = grid_offset_of_index(hx < P.kb ? hx : P.kb - 1, P.d, P.n);
        for (int p = first; p < P.gsize; p += stride) gf[p] = make_double2(0.0, 0.0);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void adjoint_pack(AdjPlan P, const double2* __restrict__ U, int64_t u_rs,
                                                    int64_t u_cs, const double* __restrict__ sigma,
                                                    const double2* __restrict__ V, int64_t v_rs, int64_t v_cs,
                                                    const double2* __restrict__ gS, pair_t<T>* __restrict__ zp,
                                                    pair_t<T>* __restrict__ wp, int* __restrict__ gt,
                                                    double2* __restrict__ gf) {
    adj_pack_body<T>(P, U, u_rs, u_cs, sigma, V, v_rs, v_cs, gS, zp, wp, gt, gf, blockIdx.y);
}

// Two 16-row fragments per wave where the rows of Z kept in registers allow it.
constexpr bool adj_rf2_supported(size_t tsize, int ks) { return ks <= (tsize == 4 ? 16 : 8); }

template <typename T>
struct AdjPtrs {
    const pair_t<T>* zp;
    const pair_t<T>* wp;
    const int* gtab;
    double2* gf;
};

// LDS: diagonal bins (2 win_cap doubles: LDS FP64 atomics measured several
// times faster than FP32 ones here, and the bins then add in FP64 for both
// precisions) | h' offsets (kc ints) | two staging
// buffers of one W block (cp rows x 16 pairs each).
__host__ __device__ inline size_t adj_bins_bytes(int win_cap) { return align_up(2 * sizeof(double) * (size_t)win_cap, 16); }
__host__ __device__ inline size_t adj_gt_bytes(int kc) { return align_up(4 * (size_t)kc, 16); }

template <typename T, int KS, int RF>
__device__ __forceinline__ void adjoint_body(const AdjPlan& P, const AdjPtrs<T>& ptr, const int L) {
    using T2 = pair_t<T>;
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    constexpr int kTileRows = kRows * RF;
    constexpr int cp = 4 * KS;              // padded complex K
    constexpr int kPairs = cp * kHBlock;          // W pairs of one h block
    constexpr int kBuf = kPairs + 1;              // staging buffer stride: the block and one spare slot
    constexpr int kStg = (kPairs + kThreads - 1) / kThreads;   // staged pairs per thread and block
    extern __shared__ __align__(16) unsigned char smem[];
    double* bins = reinterpret_cast<double*>(smem);
    int* gt = reinterpret_cast<int*>(smem + adj_bins_bytes(P.win_cap));
    T2* wst = reinterpret_cast<T2*>(smem + adj_bins_bytes(P.win_cap) + adj_gt_bytes(P.kc));

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, col = lane & 15;
    const int sk_i = L / P.rt, rt_i = L - (L / P.rt) * P.rt;
    const int k_first = rt_i * kTileRows;
    const int k_last = min(k_first + kTileRows - 1, P.NR - 1);
    const int h_first = sk_i * P.kc;
    const int h_last = min(h_first + P.kc, P.kb) - 1;
    const int lo = rowext_offset(k_first, P.d, P.n) - grid_offset_of_index(h_last, P.d, P.n) + P.c0;
    const int hi = rowext_offset(k_last, P.d, P.n) - grid_offset_of_index(h_first, P.d, P.n) + P.c0;
    const int W = hi - lo + 1;
    const int rowlen = P.sk * P.kc;
    const int nblk = P.kc / kHBlock;

    // W block hb: rows q < cp, 16 pairs from column h_first + 16 hb; thread tid
    // moves pairs e = tid + 256 u < cp 16 (row e / 16, pair e % 16). When the
    // block is not a whole number of rounds, the last round's other threads load
    // the block's last pair again (the loads stay unconditional, so the staging
    // registers stay registers) and write nothing.
    auto wsrc = [&](int u, int blk) {
        const int e = min(tid + u * kThreads, kPairs - 1);
        return ptr.wp + (size_t)(e >> 4) * rowlen + (e & 15) + h_first + kHBlock * blk;
    };
    constexpr int kTail = kPairs % kThreads;
    const bool tail_ok = kTail == 0 || tid < kTail;
    // LDS slot of staged pair u: its place in the block, or the buffer's spare slot
    // for the last round's idle threads (every thread writes: no branch)
    auto slot = [&](int u) { return u + 1 < kStg || tail_ok ? tid + u * kThreads : kPairs; };
    static_assert(kStg <= 2, "m <= 32: at most two staged pairs per thread");
    // two named registers rather than an array, which the compiler kept in scratch
    T2 stg0 = *wsrc(0, 0), stg1{};
    if constexpr (kStg > 1) stg1 = *wsrc(1, 0);
    for (int i = tid; i < 2 * W; i += kThreads) bins[i] = 0.0;
    for (int i = tid; i < P.kc; i += kThreads) gt[i] = ptr.gtab[min(h_first + i, h_last)];

    // A operand (rows of Z) for all K steps, kept in registers
    const int krow0 = k_first + 16 * RF * wave + col;
    T2 a[RF][KS];
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
        for (int s = 0; s < KS; ++s) a[f][s] = ptr.zp[(size_t)(krow0 + 16 * f) * cp + 4 * s + g];
    // diagonal bin base of the rows this lane's accumulator elements hold
    int gk[RF][4];
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            gk[f][r] = rowext_offset(min(k_first + 16 * RF * wave + 16 * f + M::row(g, r), P.NR - 1), P.d, P.n) +
                       P.c0 - lo;
    wst[slot(0)] = stg0;
    if constexpr (kStg > 1) wst[slot(1)] = stg1;
    __syncthreads();

    for (int hb = 0; hb < nblk; ++hb) {
        // next block's W (the last block fetches itself again) lands while the MFMAs run
        const int nxt = min(hb + 1, nblk - 1);
        stg0 = *wsrc(0, nxt);
        if constexpr (kStg > 1) stg1 = *wsrc(1, nxt);
        // three real products per complex product: P1 = Re z Re w, P2 = Im z Im w,
        // P3 = (Re z + Im z)(Re w + Im w); Re = P1 - P2, Im = P3 - P1 - P2
        const T2* wb = wst + (hb & 1) * kBuf + g * kHBlock + col;
        acc_t acc[RF][3];
#pragma unroll
        for (int f = 0; f < RF; ++f) acc[f][0] = acc[f][1] = acc[f][2] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const T2 b = wb[4 * s * kHBlock];
            const T bsum = b.x + b.y;
#pragma unroll
            for (int f = 0; f < RF; ++f) acc[f][0] = M::fma(a[f][s].x, b.x, acc[f][0]);
#pragma unroll
            for (int f = 0; f < RF; ++f) acc[f][1] = M::fma(a[f][s].y, b.y, acc[f][1]);
#pragma unroll
            for (int f = 0; f < RF; ++f) acc[f][2] = M::fma(a[f][s].x + a[f][s].y, bsum, acc[f][2]);
        }
        // element r of lane (g, col) of fragment f: row 16 f + row(g,r), column
        // h = 16 hb + col (rows past the last row of Z are zero rows: they add zeros)
        const int gh = gt[hb * kHBlock + col];
#pragma unroll
        for (int f = 0; f < RF; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const T p1 = acc[f][0][r], p2 = acc[f][1][r], p3 = acc[f][2][r];
                double* bin = &bins[2 * (gk[f][r] - gh)];
                atomicAdd(bin, (double)(p1 - p2));
                atomicAdd(bin + 1, (double)(p3 - p1 - p2));
            }
        // the other buffer was last read before the previous barrier
        wst[((hb + 1) & 1) * kBuf + slot(0)] = stg0;
        if constexpr (kStg > 1) wst[((hb + 1) & 1) * kBuf + slot(1)] = stg1;
        __syncthreads();
    }
    double* out = reinterpret_cast<double*>(ptr.gf + lo);
    for (int i = tid; i < 2 * W; i += kThreads) {
        const double v = bins[i];
        if (v != 0.0) unsafeAtomicAdd(&out[i], v);
    }
}

template <typename T, int KS, int RF>
__global__ __launch_bounds__(kThreads) void adjoint_tiles(AdjPlan P, AdjPtrs<T> ptr) {
    const int id = blockIdx.x;
    const int L = (P.nwg & 7) == 0 ? (id & 7) * (P.nwg >> 3) + (id >> 3) : id;
    adjoint_body<T, KS, RF>(P, ptr, L);
}

// One instance of a batched adjoint: its plan, packed operands, inputs and the
// offsets of its gS / gf blocks in the caller's concatenated buffers.
template <typename T>
struct AdjEntry {
    AdjPlan P;
    AdjPtrs<T> ptr;        // gf unused (taken from gf_all + gf_off)
    const double2* U;
    const double2* V;
    const double* sigma;
    int64_t gs_off, gf_off;   // complex elements
    int tile_begin;           // first workgroup of this instance within its class launch
};

template <typename T>
__global__ __launch_bounds__(256) void adjoint_pack_batched(const AdjEntry<T>* __restrict__ entries,
                                                            const double2* __restrict__ gS_all,
                                                            double2* __restrict__ gf_all) {
    const AdjEntry<T>& e = entries[blockIdx.z];
    const int m = e.P.m;
    adj_pack_body<T>(e.P, e.U, m, 1, e.sigma, e.V, m, 1, gS_all + e.gs_off, const_cast<pair_t<T>*>(e.ptr.zp),
                     const_cast<pair_t<T>*>(e.ptr.wp), const_cast<int*>(e.ptr.gtab), gf_all + e.gf_off, blockIdx.y);
}

template <typename T, int KS, int RF>
__global__ __launch_bounds__(kThreads) void adjoint_tiles_batched(const AdjEntry<T>* __restrict__ entries, int count,
                                                                  double2* __restrict__ gf_all) {
    const int id = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (entries[mid].tile_begin <= id)
            lo = mid;
        else
            hi = mid - 1;
    }
    const AdjEntry<T>& e = entries[lo];
    AdjPtrs<T> ptr = e.ptr;
    ptr.gf = gf_all + e.gf_off;
    adjoint_body<T, KS, RF>(e.P, ptr, id - e.tile_begin);
}

// A single adjoint aims at two workgroups per CU; a batch member splits its h
// range only into chunks of about 256 (long enough to amortise the window flush;
// the batch fills the GPU).
prony_status_t make_adj_plan(prony_handle_t h, int d, int n, int m, size_t tsize, AdjPlan& P, bool batched = false) {
    P = AdjPlan{};
    P.d = d;
    P.n = n;
    P.N = (int)ipow(n + 1, d);
    P.m = m;
    P.NR = (int)ipow(n + 2, d);
    P.cp = (int)align_up((size_t)m, 8);
    P.ksteps = P.cp / 4;
    P.kb = P.N;
    P.rf = adj_rf2_supported(tsize, P.ksteps) && P.NR > kRows ? 2 : 1;
    P.rows = kRows * P.rf;
    P.rt = (P.NR + P.rows - 1) / P.rows;
    P.c0 = grid_center(d, n);
    P.gsize = (int)ipow(2 * n + 2, d);
    const size_t staging = 2 * (2 * tsize) * ((size_t)P.cp * kHBlock + 1);
    const size_t budget = std::min<size_t>(h->lds_per_block, staging + 64 * 1024);
    const int target = batched ? P.rt * std::max(1, P.kb / 256) : 2 * h->num_cus;
    const int sk_target = std::max(1, target / P.rt);
    int kc = (int)align_up((size_t)((P.kb + sk_target - 1) / sk_target), kHBlock);
    kc = std::max(kc, std::min(128, (int)align_up((size_t)P.kb, kHBlock)));
    auto span = [&](int count, int len, bool rowext) {
        int best = 0;
        for (int s = 0; s < count; s += len) {
            const int e = std::min(s + len, count) - 1;
            const int a = rowext ? rowext_offset(s, d, n) : grid_offset_of_index(s, d, n);
            const int b = rowext ? rowext_offset(e, d, n) : grid_offset_of_index(e, d, n);
            best = std::max(best, b - a);
        }
        return best;
    };
    const int rowspan = span(P.NR, P.rows, true);
    for (;;) {
        const int win = rowspan + span(P.kb, kc, false) + 1;
        const size_t lds = adj_bins_bytes(win) + adj_gt_bytes(kc) + staging;
        if (lds <= budget) {
            P.kc = kc;
            P.sk = (P.kb + kc - 1) / kc;
            P.win_cap = win;
            P.lds_bytes = lds;
            break;
        }
        if (kc <= kHBlock) return fail(h, PRONY_ENOTSUP, "prony_build_S_adjoint: window does not fit in LDS");
        kc = (int)align_up((size_t)(kc / 2), kHBlock);
    }
    P.nwg = P.rt * P.sk;
    const size_t t2 = 2 * tsize;
    if ((int64_t)P.cp * P.sk * P.kc >= (int64_t(1) << 31))
        return fail(h, PRONY_ENOTSUP, "prony_build_S_adjoint: problem too large");
    size_t off = 0;
    P.off_z = off;
    off = align_up(off + t2 * (size_t)P.rt * P.rows * P.cp, 256);
    P.off_w = off;
    off = align_up(off + t2 * (size_t)P.cp * P.sk * P.kc, 256);
    P.off_g = off;
    off = align_up(off + 4 * (size_t)P.sk * P.kc, 256);
    P.ws_bytes = off;
    return PRONY_OK;
}

template <typename T, int KS, int RF>
prony_status_t launch_adj_tiles(prony_handle_t h, const AdjPlan& P, const AdjPtrs<T>& ptr) {
    if (P.lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&adjoint_tiles<T, KS, RF>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes);
        if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
    }
    ProfileScope prof(h, "adjoint_tiles");
    adjoint_tiles<T, KS, RF><<<P.nwg, kThreads, P.lds_bytes, h->stream>>>(P, ptr);
    return PRONY_OK;
}

template <typename T, int KS>
prony_status_t dispatch_adj_tiles(prony_handle_t h, const AdjPlan& P, const AdjPtrs<T>& ptr) {
    if constexpr (adj_rf2_supported(sizeof(T), KS))
        if (P.rf == 2) return launch_adj_tiles<T, KS, 2>(h, P, ptr);
    return launch_adj_tiles<T, KS, 1>(h, P, ptr);
}

template <typename T>
prony_status_t launch_adjoint(prony_handle_t h, const AdjPlan& P, const double* U, int64_t u_rs, int64_t u_cs,
                              const double* sigma, const double* V, int64_t v_rs, int64_t v_cs, const double* gS,
                              double* gf) {
    using T2 = pair_t<T>;
    prony_status_t st = ensure_workspace(h, P.ws_bytes);
    if (st != PRONY_OK) return st;
    unsigned char* ws = static_cast<unsigned char*>(h->ws);
    T2* zp = reinterpret_cast<T2*>(ws + P.off_z);
    T2* wp = reinterpret_cast<T2*>(ws + P.off_w);
    int* gt = reinterpret_cast<int*>(ws + P.off_g);
    const int64_t largest = std::max<int64_t>({(int64_t)P.rt * P.rows * P.cp, (int64_t)P.cp * P.sk * P.kc,
                                               (int64_t)P.gsize});
    const int blocks = (int)std::min<int64_t>((largest + 255) / 256, 2 * (int64_t)h->num_cus);
    {
        ProfileScope prof(h, "adjoint_pack");
        adjoint_pack<T><<<dim3(blocks, 3), 256, 0, h->stream>>>(
            P, reinterpret_cast<const double2*>(U), u_rs, u_cs, sigma, reinterpret_cast<const double2*>(V), v_rs,
            v_cs, reinterpret_cast<const double2*>(gS), zp, wp, gt, reinterpret_cast<double2*>(gf));
    }
    if ((st = check_launch(h, "adjoint_pack")) != PRONY_OK) return st;
    const AdjPtrs<T> ptr{zp, wp, gt, reinterpret_cast<double2*>(gf)};
    switch (P.ksteps) {
#define PRONY_ADJ_CASE(K) \
    case K:               \
        st = dispatch_adj_tiles<T, K>(h, P, ptr); \
        break;
        PRONY_ADJ_CASE(2)
        PRONY_ADJ_CASE(4)
        PRONY_ADJ_CASE(6)
        PRONY_ADJ_CASE(8)
#undef PRONY_ADJ_CASE
        default:
            return fail(h, PRONY_ENOTSUP, "prony_build_S_adjoint: m too large");
    }
    if (st != PRONY_OK) return st;
    return check_launch(h, "adjoint_tiles");
}

template <typename T, int KS>
prony_status_t launch_adj_batched_ks(prony_handle_t h, int rf, const AdjEntry<T>* entries, int count, int tiles,
                                     size_t lds, double2* gf) {
    if constexpr (adj_rf2_supported(sizeof(T), KS))
        if (rf == 2) {
            if (lds > 65536) {
                hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&adjoint_tiles_batched<T, KS, 2>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
            }
            ProfileScope prof(h, "adjoint_tiles_batched");
            adjoint_tiles_batched<T, KS, 2><<<tiles, kThreads, lds, h->stream>>>(entries, count, gf);
            return PRONY_OK;
        }
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&adjoint_tiles_batched<T, KS, 1>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
    }
    ProfileScope prof(h, "adjoint_tiles_batched");
    adjoint_tiles_batched<T, KS, 1><<<tiles, kThreads, lds, h->stream>>>(entries, count, gf);
    return PRONY_OK;
}

}  // namespace

struct AdjBatch {
    void* ws = nullptr;           // device AdjEntry<T>[count] (grouped by class), then operands
    int count = 0;
    int pack_x = 1;
    int64_t gs_elems = 0, gf_elems = 0;   // complex elements of the concatenated gS / gf
    struct ClassLaunch {
        int ks, rf, first, count, tiles;
        size_t lds;
    };
    std::vector<ClassLaunch> launches;
};

prony_status_t adj_batch_free(AdjBatch* a) {
    prony_status_t st = PRONY_OK;
    if (a->ws && hipFree(a->ws) != hipSuccess) st = PRONY_EHIP;
    delete a;
    return st;
}

namespace {

template <typename T>
prony_status_t adj_batch_build(prony_handle_t h, const prony_batch_s* B, AdjBatch* A) {
    using T2 = pair_t<T>;
    const int count = B->count;
    std::vector<AdjPlan> plans(count);
    std::vector<int64_t> gs_off(count), gf_off(count);
    for (int i = 0; i < count; ++i) {
        const prony_instance_t& x = B->inst[i];
        prony_status_t st = make_adj_plan(h, x.d, x.n, x.m, sizeof(T), plans[i], true);
        if (st != PRONY_OK) return fail(h, st, "instance " + std::to_string(i) + ": " + h->err);
        gs_off[i] = A->gs_elems;
        A->gs_elems += (int64_t)x.d * x.m * x.m;
        gf_off[i] = A->gf_elems;
        A->gf_elems += plans[i].gsize;
    }
    // classes by (K steps, fragments); inside a class, most workgroups first
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (plans[a].ksteps != plans[b].ksteps) return plans[a].ksteps < plans[b].ksteps;
        if (plans[a].rf != plans[b].rf) return plans[a].rf < plans[b].rf;
        return plans[a].nwg > plans[b].nwg;
    });
    size_t off = align_up(sizeof(AdjEntry<T>) * (size_t)count, 256);
    std::vector<size_t> base(count);
    for (int pos = 0; pos < count; ++pos) {
        base[pos] = off;
        off = align_up(off + plans[order[pos]].ws_bytes, 256);
    }
    hipError_t e = hipMalloc(&A->ws, off);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        A->ws = nullptr;
        return fail(h, PRONY_ENOMEM, std::string("batch adjoint workspace allocation failed: ") + hipGetErrorString(e));
    }
    unsigned char* w = static_cast<unsigned char*>(A->ws);
    std::vector<AdjEntry<T>> host(count);
    int first = 0;
    int64_t largest = 1;
    for (int pos = 0; pos < count; ++pos) {
        const int i = order[pos];
        const AdjPlan& P = plans[i];
        const prony_instance_t& x = B->inst[i];
        AdjEntry<T>& E = host[pos];
        E.P = P;
        E.ptr.zp = reinterpret_cast<const T2*>(w + base[pos] + P.off_z);
        E.ptr.wp = reinterpret_cast<const T2*>(w + base[pos] + P.off_w);
        E.ptr.gtab = reinterpret_cast<const int*>(w + base[pos] + P.off_g);
        E.ptr.gf = nullptr;
        E.U = reinterpret_cast<const double2*>(x.U);
        E.V = reinterpret_cast<const double2*>(x.V);
        E.sigma = x.sigma;
        E.gs_off = gs_off[i];
        E.gf_off = gf_off[i];
        const bool new_class = pos == 0 || plans[order[pos - 1]].ksteps != P.ksteps ||
                               plans[order[pos - 1]].rf != P.rf;
        if (new_class) {
            A->launches.push_back({P.ksteps, P.rf, pos, 0, 0, 0});
            first = 0;
        }
        auto& cl = A->launches.back();
        E.tile_begin = first;
        first += P.nwg;
        cl.count += 1;
        cl.tiles = first;
        cl.lds = std::max(cl.lds, P.lds_bytes);
        largest = std::max<int64_t>({largest, (int64_t)P.rt * P.rows * P.cp, (int64_t)P.cp * P.sk * P.kc,
                                     (int64_t)P.gsize});
    }
    A->count = count;
    A->pack_x = (int)std::min<int64_t>((largest + 255) / 256, 64);
    e = hipMemcpyAsync(A->ws, host.data(), sizeof(AdjEntry<T>) * (size_t)count, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "batch adjoint work table upload");
    return PRONY_OK;
}

template <typename T>
prony_status_t adj_batch_launch(prony_handle_t h, const AdjBatch* A, const double* gS, double* gf) {
    const AdjEntry<T>* entries = static_cast<const AdjEntry<T>*>(A->ws);
    const double2* gs2 = reinterpret_cast<const double2*>(gS);
    double2* gf2 = reinterpret_cast<double2*>(gf);
    {
        ProfileScope prof(h, "adjoint_pack");
        adjoint_pack_batched<T><<<dim3(A->pack_x, 3, A->count), 256, 0, h->stream>>>(entries, gs2, gf2);
    }
    prony_status_t st = check_launch(h, "adjoint_pack_batched");
    if (st != PRONY_OK) return st;
    for (const auto& cl : A->launches) {
        switch (cl.ks) {
#define PRONY_ADJ_BCASE(K)                                                                              \
    case K:                                                                                             \
        st = launch_adj_batched_ks<T, K>(h, cl.rf, entries + cl.first, cl.count, cl.tiles, cl.lds, gf2); \
        break;
            PRONY_ADJ_BCASE(2)
            PRONY_ADJ_BCASE(4)
            PRONY_ADJ_BCASE(6)
            PRONY_ADJ_BCASE(8)
#undef PRONY_ADJ_BCASE
            default:
                return fail(h, PRONY_ENOTSUP, "prony_build_S_adjoint_batched: m too large");
        }
        if (st != PRONY_OK) return st;
        if ((st = check_launch(h, "adjoint_tiles_batched")) != PRONY_OK) return st;
    }
    return PRONY_OK;
}

}  // namespace

size_t adjoint_workspace_bytes(prony_handle_t h, int d, int n, int m) {
    size_t best = 0;
    for (size_t ts : {sizeof(float), sizeof(double)}) {
        AdjPlan P;
        if (make_adj_plan(h, d, n, m, ts, P) == PRONY_OK) best = std::max(best, P.ws_bytes);
    }
    return best;
}

}  // namespace prony

using namespace prony;

extern "C" prony_status_t prony_build_S_adjoint(prony_handle_t h, int d, int n, int m, const double* U,
                                                int64_t u_rs, int64_t u_cs, const double* sigma, const double* V,
                                                int64_t v_rs, int64_t v_cs, const double* gS, prony_prec_t prec,
                                                double* gf) {
    if (!h) return PRONY_EINVAL;
    prony_status_t st = check_dn(h, d, n);
    if (st != PRONY_OK) return st;
    const int64_t N = ipow(n + 1, d);
    if (m < 1 || m > N) return fail(h, PRONY_EINVAL, "prony_build_S_adjoint: m must be in 1..N");
    if (m > 32) return fail(h, PRONY_ENOTSUP, "prony_build_S_adjoint: m > 32 is not supported");
    if (!U || !V || !sigma || !gS || !gf) return fail(h, PRONY_EINVAL, "prony_build_S_adjoint: null pointer");
    if (u_rs < 1 || u_cs < 1 || v_rs < 1 || v_cs < 1)
        return fail(h, PRONY_EINVAL, "prony_build_S_adjoint: strides must be >= 1");
    if ((N - 1) * u_rs + (m - 1) * u_cs >= (int64_t(1) << 40) || (N - 1) * v_rs + (m - 1) * v_cs >= (int64_t(1) << 40))
        return fail(h, PRONY_EINVAL, "prony_build_S_adjoint: strides out of range");
    if (prec != PRONY_FP64 && prec != PRONY_FP32) return fail(h, PRONY_EINVAL, "prony_build_S_adjoint: bad precision");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    AdjPlan P;
    if (prec == PRONY_FP32) {
        if ((st = make_adj_plan(h, d, n, m, sizeof(float), P)) != PRONY_OK) return st;
        return launch_adjoint<float>(h, P, U, u_rs, u_cs, sigma, V, v_rs, v_cs, gS, gf);
    }
    if ((st = make_adj_plan(h, d, n, m, sizeof(double), P)) != PRONY_OK) return st;
    return launch_adjoint<double>(h, P, U, u_rs, u_cs, sigma, V, v_rs, v_cs, gS, gf);
}

extern "C" prony_status_t prony_build_S_adjoint_batched(prony_handle_t h, prony_batch_t B, const double* gS,
                                                        double* gf) {
    if (!h || !B) return PRONY_EINVAL;
    if (B->owner != h) return fail(h, PRONY_EINVAL, "prony_build_S_adjoint_batched: batch belongs to another handle");
    if (!gS || !gf) return fail(h, PRONY_EINVAL, "prony_build_S_adjoint_batched: null pointer");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    if (!B->adj) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(h->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return fail(h, PRONY_ECAPTURE,
                        "prony_build_S_adjoint_batched: the first call on a batch plans and allocates; "
                        "make it outside stream capture");
        AdjBatch* A = new (std::nothrow) AdjBatch();
        if (!A) return fail(h, PRONY_ENOMEM, "prony_build_S_adjoint_batched: out of host memory");
        const prony_status_t st = B->prec == PRONY_FP32 ? adj_batch_build<float>(h, B, A)
                                                        : adj_batch_build<double>(h, B, A);
        if (st != PRONY_OK) {
            (void)adj_batch_free(A);
            return st;
        }
        B->adj = A;
    }
    return B->prec == PRONY_FP32 ? adj_batch_launch<float>(h, B->adj, gS, gf)
                                 : adj_batch_launch<double>(h, B->adj, gS, gf);
}
