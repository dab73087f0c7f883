// Pencil matrices S_l = U^* T_l V Sigma^{-1} (Sec. 1, eq. generateSl) on MFMA.
//
// Formulation (row-extended). With k' = k + e_l, T_l[k,h] = f(k' - h), so the d
// products Y_l = T_l V are rows of ONE product of the row-extended Toeplitz matrix
// T_row[k',h] = f(k'-h), k' in {0..n+1}^d, h in I_n, with V itself:
//     Z = T_row V,   Y_l[k] = Z[k + e_l],
// and the U^* reduction of the pencil matrices becomes
//     U^* T_l V = sum_k' U_l[k']^* Z[k'],   U_l[k'] = U[k' - e_l]
// (zero where k' - e_l leaves I_n; U_0 = U for S_0). The MFMA work of the large
// product is that of one N x N by N x m product on (n+2)^d rows, not d of them;
// the d shifted copies of U enter only the m-row reduction of each tile.
// The complex product is run as a real one, in two forms of 16-column blocks.
// Pair form: every complex column q yields the real columns (Re, Im) and every
// complex T entry a contributes two MFMAs, one with Re(a) against (Re v, Im v)
// and one with Im(a) against (-Im v, Re v): two MFMAs per 8 complex columns.
// Three-product form: the complex columns are the MFMA columns and a v takes the
// three real products P1 = Re a Re v, P2 = Im a Im v, P3 = (Re a + Im a)(Re v +
// Im v), so Re(a v) = P1 - P2 and Im(a v) = P3 - P1 - P2: three MFMAs per 16
// complex columns. S-builds take ng three-product blocks for the first columns and
// a pair block for a remainder of at most 8 columns (m = 20: 16 + 4 columns, five
// MFMAs per K step and fragment instead of six), so that no shape needs more
// MFMAs than in either form alone. The second factor is packed once per call in
// that layout.
//
// Kernels:
//   pencil_pack         packs V (pair layout, or bfloat16 split planes), U in the
//                       row-extended layout (Re/Im pairs, zero rows where k' leaves
//                       I_n, zero guard rows in front so that every shift k' - e_l
//                       is a plain row offset) and the grid offsets G(h);
//   pencil_tiles        one workgroup = 64 rf rows k' x one chunk of h; the T_row
//                       tile is generated from a flat window of the sample grid
//                       staged in LDS, multiplied on MFMA (FP32 or FP64) against
//                       the packed V, then the reductions with the shifted U_l over
//                       the tile's rows run on MFMA as well and the m x (d m)
//                       partial is stored;
//   pencil_tiles_split  the same tile with both operands as three bfloat16 terms
//                       on the bf16 MFMA (FP32-accurate products);
//   pencil_finish       sums the partials of all workgroups in FP64 in a fixed
//                       order and applies Sigma^{-1} in FP64;
//   toeplitz_mm_tiles / toeplitz_mm_finish
//                       the product mode Y = T X or T^* X (h over I_n, no U^*);
//   toeplitz_mv         the same product with one column, on vector FMAs;
//   pencil_pack_batched / pencil_tiles_batched / pencil_tiles_queue /
//   pencil_finish_batched
//                       many instances: one launch per tile class, or one
//                       persistent launch over a queue of all tiles.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"
#include "mfma.h"
#include "reduce.h"

namespace prony {
namespace {

constexpr int kWaves = 4;               // waves per workgroup
constexpr int kRowsPerWave = 16;        // MFMA M dimension
constexpr int kRowsPerTile = kWaves * kRowsPerWave;
constexpr int kThreads = kWaves * 64;

// The K loop keeps operands of kDepth K steps (4 h' each) in flight; it reads
// up to kPrefetchRows h' past the end of a chunk (packed rows padded with zeros,
// offsets clamped to the chunk so that the reads stay inside the LDS window).
constexpr int kDepth = 4;
constexpr int kPrefetchRows = 4 * kDepth;

// 16-row fragments per wave (each B operand feeds RF times the MFMAs) that an
// instantiation supports: the accumulators of all fragments must fit the register
// file next to the operand ring. 1 always; 2 up to 8 (FP32) or 6 (FP64)
// accumulator blocks; 4 up to 4 (FP32, split bfloat16: 1 column block) or 2 (FP64).
// ng of the nb column blocks in the three-product form keep three accumulator
// blocks each; split tiles keep two per column block (Re a and Im a products).
constexpr bool rf_supported(size_t tsize, int nb, int rf, bool split = false, int ng = 0) {
    const int na = nb + 2 * ng;   // accumulator blocks per fragment (split: x 2)
    return rf == 1 || (rf == 2 && na <= (tsize == 4 ? 8 : 6)) ||
           (rf == 4 && na <= (split ? 1 : (tsize == 4 ? 4 : 2)));
}

// Whether the S-build epilogue stores Zr + Zi of its three-product blocks as a third
// LDS plane (when all planes of a tile of `rows` rows fit in 64 KiB).
__host__ __device__ constexpr bool z_sum_plane(size_t tsize, int nb, int ng, int rows) {
    return ng > 0 && (size_t)(2 * nb + ng) * rows * 16 * tsize <= 65536;
}

struct PencilPlan {
    int d, n, N, m;
    int mode;       // 0: S-build (row-extended k', shifted U^* epilogue); 1: product Y = T X
    int conj_grid;  // product mode: stage conj(f(-p)), i.e. multiply by T^* instead of T
    int split;      // 1: operands as three bfloat16 terms on the bf16 MFMA (T = float)
    int bbufs;      // split: LDS buffers of the staged B planes (2, or 1 when two do not fit)
    int ells;       // stacked matrices: d, or d + 1 with S_0
    int first_ell;  // 0 with S_0, else 1
    int C;          // complex columns of the result rows: ells * m (product: r)
    int CB;         // complex columns of the second operand V (or X): m
    int ng;         // leading column blocks in the three-product form (16 complex columns each)
    int nb;         // 16-wide column blocks of the second operand: ng three-product blocks, then
                    // pair blocks for the remaining columns (2 real columns per complex one)
    int nrp;        // 16 * nb
    int nrr;        // real columns of a product row: 32 per three-product block, 16 per pair block
    int mbi;        // 16-row blocks of the m output rows
    int NR;         // rows of the large product: (n+2)^d row-extended k' (product: N)
    int ug;         // zero guard rows in front of the packed U: (n+2)^(d-1), the largest shift
    int kb;         // N indices h of I_n (the K range)
    int kc;         // h per chunk (multiple of 16)
    int sk;         // chunks
    int rf;         // 16-row fragments per wave (1 or 2)
    int rows;       // rows k' per tile: 64 rf
    int rt;         // row tiles
    int nwg;        // rt * sk workgroups
    int win_cap;    // window capacity (complex elements)
    int wsum;       // three-product blocks: window entries (Re, Im, Re + Im, 0) instead of (Re, Im)
    int c0;         // grid offset of the origin shift
    size_t lds_bytes;
    // workspace offsets (bytes)
    size_t off_v, off_u, off_g, off_p, ws_bytes;
};


// Grid offset of the K index h of I_n.
__host__ __device__ inline int h_offset(const PencilPlan& P, int hx) { return grid_offset_of_index(hx, P.d, P.n); }

// Grid offset of row r of the large product: row-extended k' for the S-build,
// k of I_n for the product.
__host__ __device__ inline int row_offset(const PencilPlan& P, int r) {
    return P.mode ? grid_offset_of_index(r, P.d, P.n) : rowext_offset(r, P.d, P.n);
}

// Row-extended shift of e_l: (n+2)^(d-l) for l = 1..d, 0 for l = 0.
__host__ __device__ inline int rowext_shift(const PencilPlan& P, int ell) {
    if (ell <= 0) return 0;
    int s = 1;
    for (int l = ell; l < P.d; ++l) s *= P.n + 2;
    return s;
}

// Three-term bfloat16 split x = h + m + l (each term rounded to nearest; the
// subtractions are exact in FP32, so x - (h + m + l) is below 2^-24 |x|).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// 16-byte unit of the split operands (a native vector: copies stay in registers)
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
constexpr int kSplitK = 32;     // h' per K block of the bf16 MFMA (16x16x32)
constexpr int kSplitPlanes = 3; // stored B planes per K block: the Re-multiplier's h, m, l
__device__ __forceinline__ void split3(float x, unsigned short& h, unsigned short& m, unsigned short& l) {
    const __bf16 bh = (__bf16)x;
    float r = x - (float)bh;
    const __bf16 bm = (__bf16)r;
    r -= (float)bm;
    const __bf16 bl = (__bf16)r;
    h = __builtin_bit_cast(unsigned short, bh);
    m = __builtin_bit_cast(unsigned short, bm);
    l = __builtin_bit_cast(unsigned short, bl);
}

// Pair values of the second operand at (row hx, real column j): .x multiplies
// Re(a), .y multiplies Im(a); zero past the N rows and the CB columns. In the
// three-product blocks (j < 16 ng) j is the complex column and the pair is (Re v, Im v).
__device__ __forceinline__ double2 pair_of(const PencilPlan& P, const double2* __restrict__ V, int64_t v_rs,
                                           int64_t v_cs, int hx, int j) {
    const int g16 = 16 * P.ng;
    const int c = j < g16 ? j : g16 + ((j - g16) >> 1);
    double vr = 0.0, vi = 0.0;
    if (hx < P.kb && c < P.CB) {
        const double2 v = V[hx * v_rs + c * v_cs];
        vr = v.x;
        vi = v.y;
    }
    if (j < g16) return make_double2(vr, vi);   // three-product block: complex column c as it is
    return ((j - g16) & 1) ? make_double2(vi, vr) : make_double2(vr, -vi);
}

// Split packing of the second operand: per K block of 32 h', per plane p (the
// h, m, l terms of the Re-multiplier .x of the pair layout) and real column j, the 32
// bfloat16 values of rows h' = 32 kblk .. 32 kblk + 31, ordered so that element t
// of MFMA lane group g is h' = 32 kblk + 4 t + g (interleaved: the four lane groups
// then read neighbouring window entries, which keeps the LDS reads free of bank
// conflicts); a thread makes the eight rows of one lane group (16 bytes per plane).
// The Im-multiplier is not stored: .y of column j is -.x of column j + 1 (j even)
// or .x of column j - 1 (j odd); the tile kernel multiplies Im a by the .x planes
// into a second accumulator and applies that lane exchange once after its K loop.
__device__ __forceinline__ void pack_split(const PencilPlan& P, const double2* __restrict__ V, int64_t v_rs,
                                           int64_t v_cs, u32x4* __restrict__ vp16, int first, int stride) {
    const int nunits = (P.sk * P.kc / kSplitK) * P.nrp * 4;
    for (int i = first; i < nunits; i += stride) {
        const int t8 = i & 3, rest = i >> 2;
        const int kblk = rest / P.nrp, j = rest - (rest / P.nrp) * P.nrp;
        unsigned short w[kSplitPlanes][8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const double2 pr = pair_of(P, V, v_rs, v_cs, kblk * kSplitK + 4 * t + t8, j);
            split3((float)pr.x, w[0][t], w[1][t], w[2][t]);
        }
#pragma unroll
        for (int p = 0; p < kSplitPlanes; ++p) {
            u32x4 u;
            u.x = w[p][0] | ((unsigned)w[p][1] << 16);
            u.y = w[p][2] | ((unsigned)w[p][3] << 16);
            u.z = w[p][4] | ((unsigned)w[p][5] << 16);
            u.w = w[p][6] | ((unsigned)w[p][7] << 16);
            vp16[((size_t)(kblk * kSplitPlanes + p) * P.nrp + j) * 4 + t8] = u;
        }
    }
}

// Packs, per call: (y = 0) the second factor (V, or X of the product) in the pair
// layout, rows h padded with zeros to sk*kc + kPrefetchRows; (y = 1) the (Re U,
// Im U) pairs in the row-extended layout: ug zero guard rows, then row k' of
// {0..n+1}^d (padded to whole tiles) holding U[k'] where k' lies in I_n and zero
// elsewhere, columns padded to 16*mbi, so that U_l[k'] = U[k' - e_l] is the packed
// row ug + k' - shift(e_l); (y = 2) the grid offsets G(h). All index arithmetic
// fits in 32 bits (checked by the host plan).
template <typename T>
__device__ __forceinline__ void pack_body(const PencilPlan& P, const double2* __restrict__ U, int64_t u_rs,
                                          int64_t u_cs, const double2* __restrict__ V, int64_t v_rs, int64_t v_cs,
                                          pair_t<T>* __restrict__ vp, pair_t<T>* __restrict__ up,
                                          int* __restrict__ gt, int section) {
    using T2 = pair_t<T>;
    const int kbp = P.sk * P.kc + kPrefetchRows;
    const int stride = gridDim.x * blockDim.x;
    const int first = blockIdx.x * blockDim.x + threadIdx.x;
    if (section == 0 && P.split) {
        pack_split(P, V, v_rs, v_cs, reinterpret_cast<u32x4*>(vp), first, stride);
    } else if (section == 0) {
        const int nv = kbp * P.nrp;
        for (int i = first; i < nv; i += stride) {
            const int hx = i / P.nrp;
            const int j = i - hx * P.nrp;
            // (Re a) multiplies the first member, (Im a) the second.
            const double2 pr = pair_of(P, V, v_rs, v_cs, hx, j);
            vp[i] = T2{(T)pr.x, (T)pr.y};
        }
    } else if (section == 1) {
        if (P.mode) return;   // the product has no U^* epilogue
        const int mup = P.mbi * 16;
        const int nu = (P.ug + P.rt * P.rows) * mup;
        const int E = P.n + 2, Pn = P.n + 1;
        for (int r = first; r < nu; r += stride) {
            const int kr = r / mup - P.ug;   // row-extended index k'
            const int col = r - (r / mup) * mup;
            double ur = 0.0, ui = 0.0;
            if (kr >= 0 && kr < P.NR && col < P.m) {
                int rem = kr, idx = 0, scale = 1;
                bool inside = true;
                for (int l = P.d - 1; l >= 0; --l) {
                    const int qq = rem / E;
                    const int coord = rem - qq * E;
                    rem = qq;
                    inside = inside && coord <= P.n;
                    idx += coord * scale;
                    scale *= Pn;
                }
                if (inside) {
                    const double2 u = U[idx * u_rs + col * u_cs];
                    ur = u.x;
                    ui = u.y;
                }
            }
            up[r] = T2{(T)ur, (T)ui};
        }
    } else {
        for (int hx = first; hx < kbp; hx += stride) gt[hx] = h_offset(P, hx < P.kb ? hx : P.kb - 1);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void pencil_pack(PencilPlan P, const double2* __restrict__ U, int64_t u_rs,
                                                   int64_t u_cs, const double2* __restrict__ V, int64_t v_rs,
                                                   int64_t v_cs, pair_t<T>* __restrict__ vp, pair_t<T>* __restrict__ up,
                                                   int* __restrict__ gt) {
    pack_body<T>(P, U, u_rs, u_cs, V, v_rs, v_cs, vp, up, gt, blockIdx.y);
}


// Output o = i*C + c of the summed m x (ells m) block: S_l(i, q) = sum / sigma_q.
__device__ __forceinline__ void store_s(const PencilPlan& P, const double* __restrict__ sigma,
                                        double2* __restrict__ S, int o, double re, double im) {
    const int i = o / P.C, c = o - (o / P.C) * P.C;
    const int li = c / P.m, q = c - li * P.m;
    const double sq = sigma[q];
    S[((size_t)li * P.m + i) * P.m + q] = make_double2(re / sq, im / sq);
}

// Device pointers of one S-build: inputs, packed operands and reduction scratch.
template <typename T>
struct TilePtrs {
    const double2* grid;
    const pair_t<T>* vp;
    const pair_t<T>* up;
    const int* gtab;
    pair_t<T>* part;
    const double* sigma;
    double2* S;
};

// One workgroup tile: rows kRows rt_i .. +kRows-1 of the large product (row-extended
// k' for the S-build, k of I_n for the product) against chunk sk_i of the indices h
// of I_n, where L = sk_i * rt + rt_i. See the file comment for the formulation.
// NG: the first NG of the NB column blocks are in the three-product form (S-build
// tiles, FP32/FP64 operands); each keeps three accumulator blocks per fragment
// (P1, P2, P3 at cb, NG + cb, 2 NG + cb) and pair block pb is at 3 NG + pb.
template <typename T, int NB, int RF, int MODE, bool SPLIT = false, int NG = 0>
__device__ __forceinline__ void tile_body(const PencilPlan& P, const TilePtrs<T>& ptr, const int L) {
    static_assert(!SPLIT || sizeof(T) == 4, "the split operands accumulate in FP32");
    static_assert(NG == 0 || !SPLIT, "three-product form: FP32/FP64 operands");
    static_assert(NG >= 0 && NG <= NB, "three-product blocks come first");
    constexpr int NP = NB - NG;                   // pair blocks
    constexpr int NA = 3 * NG + NP;               // accumulator blocks per fragment
    using T2 = pair_t<T>;
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    const double2* __restrict__ grid = ptr.grid;
    const T2* __restrict__ vp = ptr.vp;
    const T2* __restrict__ up = ptr.up;
    const int* __restrict__ gtab = ptr.gtab;
    T2* __restrict__ part = ptr.part;
    constexpr int kRows = kRowsPerTile * RF;   // rows k of the tile; RF 16-row fragments per wave

    extern __shared__ __align__(16) unsigned char smem[];
    // Phase 1 (K loop): grid window + h' offsets. Phase 2 (U^* reduction): the
    // same bytes hold the tile's rows of Z (S-build).
    // window entries: complex<T>, with three-product blocks and P.wsum (Re, Im,
    // Re + Im, 0), or for split operands 16 bytes (Re h | Im h, Re m | Im m,
    // Re l | Im l, 0) as bfloat16 pairs
    typedef T vec4_t __attribute__((ext_vector_type(4)));
    const bool wide = !SPLIT && NG > 0 && P.wsum;
    const int entry = SPLIT ? 16 : (wide ? (int)sizeof(vec4_t) : (int)sizeof(T2));
    T2* win = reinterpret_cast<T2*>(smem);
    vec4_t* win4 = reinterpret_cast<vec4_t*>(smem);
    u32x4* win16 = reinterpret_cast<u32x4*>(smem);
    int* gt = reinterpret_cast<int*>(smem + align_up((size_t)entry * P.win_cap, 16));
    T* zpl = reinterpret_cast<T*>(smem);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, col = lane & 15;
    const bool odd = lane & 1;
    const int sk_i = L / P.rt, rt_i = L - (L / P.rt) * P.rt;

    const int k_first = rt_i * kRows;
    const int k_last = min(k_first + kRows - 1, P.NR - 1);
    const int h_first = sk_i * P.kc;
    const int h_last = min(h_first + P.kc, P.kb) - 1;
    const int lo = row_offset(P, k_first) - h_offset(P, h_last) + P.c0;
    const int hi = row_offset(P, k_last) - h_offset(P, h_first) + P.c0;
    const int W = hi - lo + 1;
    // T^* X multiplies by the Toeplitz matrix of g(p) = conj(f(-p)): grid offsets
    // are affine in p, so g at offset o is conj(f at 2 c0 - o).
    const bool reflect = MODE == 1 && P.conj_grid;

    // Stage the window (converted to T) and the h' offsets, kStage loads per
    // thread in flight. The offsets are stored transposed per lane group:
    // gt[g * stride + s] = G(h' = h_first + 4 s + g) (in bytes: G times the window
    // entry size), so one 16-byte LDS read gives a lane the offsets of four
    // consecutive K steps.
    constexpr int kStage = 8;
    const int ngt = SPLIT ? P.kc : P.kc + kPrefetchRows;
    const int gstride = ngt >> 2;
    for (int base = 0; base < max(W, ngt); base += kStage * kThreads) {
        double2 v[kStage];
        int o[kStage];
#pragma unroll
        for (int j = 0; j < kStage; ++j) {
            const int w = base + j * kThreads + tid;
            if (w < W) v[j] = grid[reflect ? 2 * P.c0 - (lo + w) : lo + w];
            if (w < ngt) o[j] = gtab[min(h_first + w, h_last)];
        }
#pragma unroll
        for (int j = 0; j < kStage; ++j) {
            const int w = base + j * kThreads + tid;
            if constexpr (SPLIT) {
                if (w < W) {
                    unsigned short rh, rm, rl, ih, im, il;
                    split3((float)v[j].x, rh, rm, rl);
                    split3((float)v[j].y, ih, im, il);
                    win16[w] = u32x4{rh | ((unsigned)ih << 16), rm | ((unsigned)im << 16), rl | ((unsigned)il << 16), 0u};
                }
                // per K block, h' = 4 t + g at 8 g + t: a lane reads its 8 offsets as two int4
                if (w < ngt) gt[(w & ~31) | ((w & 3) << 3) | ((w & 31) >> 2)] = o[j] * entry;   // bytes
            } else {
                if (w < W) {
                    const T x = (T)v[j].x, y = reflect ? -(T)v[j].y : (T)v[j].y;
                    if (wide)
                        win4[w] = vec4_t{x, y, x + y, T(0)};
                    else
                        win[w] = T2{x, y};
                }
                if (w < ngt) gt[(w & 3) * gstride + (w >> 2)] = o[j] * entry;   // bytes
            }
        }
    }
    // Split operands: the six B planes of one K block (32 h') are staged in LDS
    // (two buffers, or one); the four 16-byte units of a column are XOR-swizzled by
    // bits 1..2 of the column, the pattern under which a ds_read_b128 of 16 columns
    // x 4 lane groups runs without bank conflicts on gfx950 (measured).
    u32x4* bst = reinterpret_cast<u32x4*>(smem + align_up((size_t)entry * P.win_cap, 16) +
                                          align_up(4 * ((size_t)P.kc + kPrefetchRows + 16), 16));
    const int bunits = kSplitPlanes * P.nrp * 4;  // 16-byte units of one K block
    const u32x4* bsrc = reinterpret_cast<const u32x4*>(vp) + (size_t)(h_first / kSplitK) * bunits;
    auto bslot = [&](int e) {
        const int row = e >> 2;                   // plane * nrp + column j
        return (row << 2) | ((e & 3) ^ (((row - (row / P.nrp) * P.nrp) >> 1) & 3));
    };
    if constexpr (SPLIT)
        for (int e = tid; e < bunits; e += kThreads) bst[bslot(e)] = bsrc[e];
    __syncthreads();

    // Rows of this wave: k_first + 16 (RF wave + f) + col for fragment f (rows past
    // the last read the last row's offsets; their results are discarded).
    const int krow0 = k_first + kRowsPerWave * RF * wave + col;
    // window offsets of the fragments' rows as LDS byte addresses, with the staged
    // h' offsets in bytes, so that an A address is one subtraction
    typedef T vec2_t __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const vec2_t lds_t2;
    const int lds_base = (int)(size_t)(__attribute__((address_space(3))) unsigned char*)smem;
    int gk[RF];
#pragma unroll
    for (int f = 0; f < RF; ++f) {
        gk[f] = row_offset(P, min(krow0 + kRowsPerWave * f, P.NR - 1)) + P.c0 - lo;
        gk[f] = gk[f] * entry + lds_base;
    }

    acc_t acc[RF][NA];
    // split operands: the Im(a) products against the same (Re-multiplier) B planes,
    // combined with acc through a lane-pair swap after the K loop
    acc_t acc2[RF][SPLIT ? NB : 1];
#pragma unroll
    for (int f = 0; f < RF; ++f) {
#pragma unroll
        for (int cb = 0; cb < NA; ++cb) acc[f][cb] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int cb = 0; cb < (SPLIT ? NB : 1); ++cb) acc2[f][cb] = acc_t{0, 0, 0, 0};
    }

    // K loop over this chunk, 4 h' per step (lane group g takes h' = 4 ks + g).
    // Operands rotate through kDepth register buffers: while the MFMAs of step
    // ks run, the loads of steps ks+1 .. ks+kDepth-1 are in flight. Every B
    // operand feeds the RF fragments of the wave.
    const T2* vrow = vp + (size_t)(h_first + g) * P.nrp + col;
    // 4 packed rows per K step; the row length is 16 NB pairs for every FP32/FP64
    // tile (a compile-time stride lets the steps of a loop iteration share one
    // address with immediate offsets)
    constexpr size_t kstride = (size_t)4 * 16 * NB;
    const int nks = P.kc >> 2;
    const int4* gq = reinterpret_cast<const int4*>(gt + g * gstride);
    T2 a[kDepth][RF];
    T as4[kDepth][RF];   // Re + Im of the A entries (wide window entries)
    T2 b[kDepth][NB];
    typedef __attribute__((address_space(3))) const vec4_t lds_t4;
    // wc: std::integral_constant<bool, wide window entries>
    auto load_a = [&](auto wc, T2* dst, T* sdst, int off) {
#pragma unroll
        for (int f = 0; f < RF; ++f) {
            if constexpr (decltype(wc)::value) {
                const vec4_t e = *(lds_t4*)(size_t)(unsigned)(gk[f] - off);
                dst[f] = T2{e.x, e.y};
                sdst[f] = e.z;
            } else {
                const vec2_t e = *(lds_t2*)(size_t)(unsigned)(gk[f] - off);
                dst[f] = T2{e.x, e.y};
            }
        }
    };
    auto load_b = [&](T2* dst, int step) {
        const T2* src = vrow + (size_t)step * kstride;
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) dst[cb] = src[cb * 16];
    };
    auto mma_x = [&](const T2* av, const T2* bv) {
#pragma unroll
        for (int f = 0; f < RF; ++f)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) acc[f][cb] = M::fma(av[f].x, bv[cb].x, acc[f][cb]);
    };
    auto mma_y = [&](const T2* av, const T2* bv) {
#pragma unroll
        for (int f = 0; f < RF; ++f)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) acc[f][cb] = M::fma(av[f].y, bv[cb].y, acc[f][cb]);
    };
    // One K step of the ring: the prefetches of a later step (A offset `off` into
    // slot ad, B step `bs` into slot bd), then the MFMAs of the current slot. With
    // many MFMAs per step (FP32, NB RF >= 12) the B prefetch goes between the Re and
    // Im halves, which measured 6-11 % faster there and 3 % slower for 5 x 2.
    constexpr bool kSplitLoads = sizeof(T) == 4 && NB * RF >= 12 && NG == 0;
    // With three-product blocks: P1 += Re a Re v, P2 += Im a Im v, P3 += (Re a +
    // Im a)(Re v + Im v) for those, the pair MFMAs for the rest; the Re-multiplier
    // MFMAs of every block first, so that dependent MFMAs sit apart.
    auto mma_g = [&](auto wc, const T2* av, const T* avs, const T2* bv) {
        // the operand sums first, as one group: a VALU operation between this wave's
        // MFMAs leaves the matrix core idle for about its latency (measured); the A
        // sums come with the window entries where they are staged
        T bsum[NG > 0 ? NG : 1], asum[RF];
#pragma unroll
        for (int cb = 0; cb < NG; ++cb) bsum[cb] = bv[cb].x + bv[cb].y;
#pragma unroll
        for (int f = 0; f < RF; ++f) asum[f] = decltype(wc)::value ? avs[f] : av[f].x + av[f].y;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int f = 0; f < RF; ++f) {
#pragma unroll
            for (int cb = 0; cb < NG; ++cb) acc[f][cb] = M::fma(av[f].x, bv[cb].x, acc[f][cb]);
#pragma unroll
            for (int pb = 0; pb < NP; ++pb) acc[f][3 * NG + pb] = M::fma(av[f].x, bv[NG + pb].x, acc[f][3 * NG + pb]);
        }
#pragma unroll
        for (int f = 0; f < RF; ++f) {
#pragma unroll
            for (int cb = 0; cb < NG; ++cb) acc[f][NG + cb] = M::fma(av[f].y, bv[cb].y, acc[f][NG + cb]);
#pragma unroll
            for (int pb = 0; pb < NP; ++pb) acc[f][3 * NG + pb] = M::fma(av[f].y, bv[NG + pb].y, acc[f][3 * NG + pb]);
        }
#pragma unroll
        for (int f = 0; f < RF; ++f) {
#pragma unroll
            for (int cb = 0; cb < NG; ++cb) acc[f][2 * NG + cb] = M::fma(asum[f], bsum[cb], acc[f][2 * NG + cb]);
        }
    };
    auto ring_step = [&](auto wc, T2* ad, T* asd, int off, T2* bd, int bs, const T2* av, const T* avs,
                         const T2* bv) {
        load_a(wc, ad, asd, off);
        if constexpr (NG > 0) {
            load_b(bd, bs);
            __builtin_amdgcn_sched_barrier(0);
            mma_g(wc, av, avs, bv);
        } else if constexpr (kSplitLoads) {
            __builtin_amdgcn_sched_barrier(0);
            mma_x(av, bv);
            __builtin_amdgcn_sched_barrier(0);
            load_b(bd, bs);
            __builtin_amdgcn_sched_barrier(0);
            mma_y(av, bv);
        } else {
            load_b(bd, bs);
            __builtin_amdgcn_sched_barrier(0);
            mma_x(av, bv);
            mma_y(av, bv);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    if constexpr (SPLIT) {
        constexpr int kVecB = (kSplitPlanes * 16 * NB * 4 + kThreads - 1) / kThreads;
        const int nkb = P.kc / kSplitK;
        const int swz = (col >> 1) & 3;
        typedef __attribute__((address_space(3))) const u32x4 lds_u4;
        auto mfma = [](const bf16x8& x, const bf16x8& y, acc_t c) {
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
        };
        // A terms of block kb for every fragment: element t of lane group g is
        // h' = 32 kb + 4 t + g. The window and the offsets stay in LDS for the whole
        // chunk, so with one fragment per wave the next block's terms are read and
        // assembled while this block's MFMAs run (two register sets, swapped by
        // unrolling the block loop by two; measured 3 % faster on c1 at the same
        // register count). With two or more fragments the second set would take the
        // kernel past 256 registers and halve the waves per SIMD (c2: 1.5x slower).
        constexpr bool kPipeA = RF == 1;
        typedef bf16x8 aterms_t[RF][3];
        auto load_split_a = [&](int kb, aterms_t& ar, aterms_t& ai) {
            const int4 o0 = *reinterpret_cast<const int4*>(gt + kSplitK * kb + 8 * g);
            const int4 o1 = *reinterpret_cast<const int4*>(gt + kSplitK * kb + 8 * g + 4);
            const int offs[8] = {o0.x, o0.y, o0.z, o0.w, o1.x, o1.y, o1.z, o1.w};
#pragma unroll
            for (int f = 0; f < RF; ++f) {
                u32x4 e[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) e[t] = *(lds_u4*)(size_t)(unsigned)(gk[f] - offs[t]);
                unsigned re[3][4], im[3][4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    // byte permutes of {hi : lo}: low halves (Re) and high halves (Im)
                    const u32x4 lo = e[2 * k], hi = e[2 * k + 1];
                    re[0][k] = __builtin_amdgcn_perm(hi.x, lo.x, 0x05040100u);
                    im[0][k] = __builtin_amdgcn_perm(hi.x, lo.x, 0x07060302u);
                    re[1][k] = __builtin_amdgcn_perm(hi.y, lo.y, 0x05040100u);
                    im[1][k] = __builtin_amdgcn_perm(hi.y, lo.y, 0x07060302u);
                    re[2][k] = __builtin_amdgcn_perm(hi.z, lo.z, 0x05040100u);
                    im[2][k] = __builtin_amdgcn_perm(hi.z, lo.z, 0x07060302u);
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    ar[f][q] = __builtin_bit_cast(bf16x8, u32x4{re[q][0], re[q][1], re[q][2], re[q][3]});
                    ai[f][q] = __builtin_bit_cast(bf16x8, u32x4{im[q][0], im[q][1], im[q][2], im[q][3]});
                }
            }
        };
        // One K block with the A terms (ar, ai); with kPipeA loads the next block's
        // into (nar, nai), else its own into (ar, ai) first.
        // The buffer count is a compile-time constant of each loop copy: a barrier
        // under a run-time condition sends the staging registers to scratch.
        auto kblock = [&](auto two_buffers, int kb, aterms_t& ar, aterms_t& ai, aterms_t& nar, aterms_t& nai) {
            constexpr bool kTwo = decltype(two_buffers)::value;
            const int nxt = min(kb + 1, nkb - 1);
            u32x4 stg[kVecB];
#pragma unroll
            for (int u = 0; u < kVecB; ++u) stg[u] = bsrc[(size_t)nxt * bunits + min(tid + u * kThreads, bunits - 1)];
            __builtin_amdgcn_sched_barrier(0);   // issue the next block's loads before this block's MFMAs
            if constexpr (!kPipeA) load_split_a(kb, ar, ai);
            const u32x4* bb = bst + (kTwo ? (kb & 1) * bunits : 0);
            // With 4 or more column blocks the B planes of block cb + 1 are read before
            // the MFMAs of block cb (measured 3-6 % faster on 8 and 12 blocks, neutral
            // on 5, 1 % slower on 2).
            constexpr bool kPrefetchB = NB >= 4;
            u32x4 xb[kSplitPlanes], xn[kSplitPlanes];
            if constexpr (kPrefetchB) {
#pragma unroll
                for (int pl = 0; pl < kSplitPlanes; ++pl) xb[pl] = bb[((pl * P.nrp + col) << 2) | (g ^ swz)];
            }
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                if constexpr (kPrefetchB) {
                    if (cb + 1 < NB) {
#pragma unroll
                        for (int pl = 0; pl < kSplitPlanes; ++pl)
                            xn[pl] = bb[((pl * P.nrp + 16 * (cb + 1) + col) << 2) | (g ^ swz)];
                    }
                    __builtin_amdgcn_sched_barrier(0);
                } else {
#pragma unroll
                    for (int pl = 0; pl < kSplitPlanes; ++pl) xb[pl] = bb[((pl * P.nrp + 16 * cb + col) << 2) | (g ^ swz)];
                }
                bf16x8 b[kSplitPlanes];
#pragma unroll
                for (int pl = 0; pl < kSplitPlanes; ++pl) b[pl] = __builtin_bit_cast(bf16x8, xb[pl]);
                // the six products of the three-term splits above 2^-24 (h h, h m, m h, h l, l h,
                // m m), of Re a into acc and of Im a into acc2, alternating
#pragma unroll
                for (int f = 0; f < RF; ++f) {
                    acc_t c = acc[f][cb], c2 = acc2[f][cb];
                    c = mfma(ar[f][2], b[0], c);
                    c2 = mfma(ai[f][2], b[0], c2);
                    c = mfma(ar[f][0], b[2], c);
                    c2 = mfma(ai[f][0], b[2], c2);
                    c = mfma(ar[f][1], b[1], c);
                    c2 = mfma(ai[f][1], b[1], c2);
                    c = mfma(ar[f][1], b[0], c);
                    c2 = mfma(ai[f][1], b[0], c2);
                    c = mfma(ar[f][0], b[1], c);
                    c2 = mfma(ai[f][0], b[1], c2);
                    c = mfma(ar[f][0], b[0], c);
                    c2 = mfma(ai[f][0], b[0], c2);
                    acc[f][cb] = c;
                    acc2[f][cb] = c2;
                }
                // the next block's A terms behind the first column block's MFMAs
                if constexpr (kPipeA) {
                    if (cb == 0) load_split_a(nxt, nar, nai);
                }
                if constexpr (kPrefetchB) {
#pragma unroll
                    for (int pl = 0; pl < kSplitPlanes; ++pl) xb[pl] = xn[pl];
                }
            }
            // with two buffers the other one was last read before the previous barrier;
            // with one, every wave must be done with it first
            if constexpr (!kTwo) __syncthreads();
            u32x4* wb = bst + (kTwo ? ((kb + 1) & 1) * bunits : 0);
#pragma unroll
            for (int u = 0; u < kVecB; ++u) wb[bslot(min(tid + u * kThreads, bunits - 1))] = stg[u];
            __syncthreads();
        };
        auto kloop = [&](auto two_buffers) {
            aterms_t a0r, a0i, a1r, a1i;
            if constexpr (kPipeA) {
                load_split_a(0, a0r, a0i);
                int kb = 0;
                for (; kb + 1 < nkb; kb += 2) {
                    kblock(two_buffers, kb, a0r, a0i, a1r, a1i);
                    kblock(two_buffers, kb + 1, a1r, a1i, a0r, a0i);
                }
                if (kb < nkb) kblock(two_buffers, kb, a0r, a0i, a1r, a1i);
            } else {
                for (int kb = 0; kb < nkb; ++kb) kblock(two_buffers, kb, a0r, a0i, a1r, a1i);
            }
        };
        if (P.bbufs == 2)
            kloop(std::integral_constant<bool, true>{});
        else
            kloop(std::integral_constant<bool, false>{});
        // The B planes hold the Re-multipliers only (lane column j: Re v for even j,
        // Im v for odd j, of complex column j / 2): acc2 holds Im a times them, so the
        // pair result is Re = acc - acc2 of the odd neighbour (Im a Im v) on even
        // lanes and Im = acc + acc2 of the even neighbour (Im a Re v) on odd lanes.
#pragma unroll
        for (int f = 0; f < RF; ++f)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const T y = swap_lane_pair(acc2[f][cb][r]);
                    acc[f][cb][r] += odd ? y : -y;
                }
    } else {
    // The prologue issues the ring's first three steps in the order the loop body
    // issues them (step by step, A then B), pinned by sched_barrier: the wait
    // counters of the loop header merge this path with the back edge, and an
    // order that differs there makes the header wait for every load in flight
    // instead of the oldest step's.
    // one copy of the loop per window entry form (a uniform branch before it)
    auto kloop_pairs = [&](auto wc) {
    int4 gc = gq[0];
    load_a(wc, a[0], as4[0], gc.x);
    load_b(b[0], 0);
    __builtin_amdgcn_sched_barrier(0);
    load_a(wc, a[1], as4[1], gc.y);
    load_b(b[1], 1);
    __builtin_amdgcn_sched_barrier(0);
    load_a(wc, a[2], as4[2], gc.z);
    load_b(b[2], 2);
    __builtin_amdgcn_sched_barrier(0);
    // sched_barrier keeps the compiler from sinking the prefetches next to their use.
    for (int ks = 0; ks < nks; ks += kDepth) {
        const int4 gn = gq[(ks >> 2) + 1];
        ring_step(wc, a[3], as4[3], gc.w, b[3], ks + 3, a[0], as4[0], b[0]);
        ring_step(wc, a[0], as4[0], gn.x, b[0], ks + 4, a[1], as4[1], b[1]);
        ring_step(wc, a[1], as4[1], gn.y, b[1], ks + 5, a[2], as4[2], b[2]);
        ring_step(wc, a[2], as4[2], gn.z, b[2], ks + 6, a[3], as4[3], b[3]);
        gc = gn;
    }
    };
    if constexpr (NG > 0) {
        if (wide)
            kloop_pairs(std::integral_constant<bool, true>{});
        else
            kloop_pairs(std::integral_constant<bool, false>{});
    } else {
        kloop_pairs(std::integral_constant<bool, false>{});
    }
    }

    if constexpr (NG > 0) {
        // three-product blocks: Re Z = P1 - P2 at block cb, Im Z = P3 - P1 - P2 at NG + cb
#pragma unroll
        for (int f = 0; f < RF; ++f)
#pragma unroll
            for (int cb = 0; cb < NG; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const T p1 = acc[f][cb][r], p2 = acc[f][NG + cb][r], p3 = acc[f][2 * NG + cb][r];
                    acc[f][cb][r] = p1 - p2;
                    acc[f][NG + cb][r] = p3 - p1 - p2;
                }
    }
    if constexpr (MODE == 1) {
        // Product: this chunk's part of Y = T X for the wave's rows, summed over
        // chunks by the finishing launch, as rows of nrr real columns with complex
        // column c at (2c, 2c + 1): a three-product block's lane col holds column
        // 16 cb + col (Re and Im from two blocks), a pair block's lane col real
        // column 32 NG + 16 pb + col. No barrier: the window is not reused.
        T* yp = reinterpret_cast<T*>(part) + ((size_t)sk_i * P.rt * P.rows + k_first + kRowsPerWave * RF * wave) * P.nrr;
#pragma unroll
        for (int f = 0; f < RF; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T* yr = yp + (size_t)(kRowsPerWave * f + M::row(g, r)) * P.nrr;
#pragma unroll
                for (int cb = 0; cb < NG; ++cb) {
                    yr[2 * (16 * cb + col)] = acc[f][cb][r];
                    yr[2 * (16 * cb + col) + 1] = acc[f][NG + cb][r];
                }
#pragma unroll
                for (int pb = 0; pb < NP; ++pb) yr[32 * NG + 16 * pb + col] = acc[f][3 * NG + pb][r];
            }
        return;
    }

    // Rows past the last row of the product (padding of the last row tile) hold
    // copies of that row's sums; they must not meet the shifted U_l rows below.
    const int wrow0 = k_first + kRowsPerWave * RF * wave;
    if (wrow0 + kRowsPerWave * RF > P.NR) {
#pragma unroll
        for (int f = 0; f < RF; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (wrow0 + kRowsPerWave * f + M::row(g, r) >= P.NR)
#pragma unroll
                    for (int cb = 0; cb < NA; ++cb) acc[f][cb][r] = T(0);
    }

    // Reductions with the shifted U_l. Item (ib, l) is the 16 x m block
    // e(i, c) = sum over the tile's rows k' of conj(U_l[k'][16 ib + i]) Z[k'][c], with
    // U_l[k'] = packed U row ug + k' - shift(e_l); items are numbered block-major.
    // The waves first store their rows of Z in LDS (the window is dead by then) as
    // the MFMA's second operands, in planes of one 16-column slot per column block
    // laid out as [K step s][slot][row 4 s + k][column], so that a read is 64
    // consecutive elements: three-product blocks as Zr, Zi and (where the LDS
    // allows) Zr + Zi; pair blocks lane-ready, [Zr | Zi] and [Zi | -Zr] (lane column
    // n is complex column n / 2 of the block, real part for even n, imaginary part
    // for odd n). Then each wave runs the MFMAs of its units: the items wave,
    // wave + 4, ... over all kRows / 4 K steps of the tile, and, when 1 or 2 items
    // are left over after the multiples of 4, one of the rs = 4 / (items mod 4)
    // parts of a left-over item's K steps (at most one per group of steps), so that
    // no wave idles; the parts are added in part order through LDS before the store.
    // The first operand (lane (k, i) of step s: U_l[4 s + k][16 ib + i]) comes in
    // groups of GS steps, two groups in flight in two register sets. The loads are
    // unconditional (clamped to the wave's last group and to the last item) and the
    // first two are issued before the barrier, so that their latency overlaps the
    // other waves' K loops and every path to a group's MFMAs has the same loads in
    // flight. Three-product blocks: conj(U) Z as Q1 = Ur Zr, Q2 = Ui Zi,
    // Q3 = (Ur - Ui)(Zr + Zi), Re = Q1 + Q2, Im = Q3 - Q1 + Q2. Pair blocks:
    // Ur [Zr | Zi] + Ui [Zi | -Zr].
    constexpr int KS = kRows / 4;                                   // K steps over the tile's rows
    constexpr int kGroup = (int)(128 / sizeof(T2));                 // 128 bytes of operands per lane
    constexpr int GS = KS / 2 < kGroup ? KS / 2 : kGroup;           // steps per group
    constexpr int NGR = KS / GS;                                    // groups per item (2, 4 or 8)
    static_assert(MODE == 1 || 2 * kRows * 16 * NB * sizeof(T) <= 65536, "Z planes above 64 KiB");
    constexpr bool kZs = z_sum_plane(sizeof(T), NB, NG, kRows);   // Zr + Zi stored
    T* const zre = zpl;
    T* const zim = zpl + KS * NB * 64;
    T* const zsm = zpl + 2 * KS * NB * 64;   // [s][three-product block][k][column]
    // packed U row length: 16 mbi pairs (mbi = NB for FP32/FP64 S-builds, checked by
    // the planner; a compile-time stride lets the U loads use immediate offsets)
    const int mup = SPLIT ? P.mbi * 16 : 16 * NB;
    const int items = P.mbi * P.ells;
    constexpr int kLgr = __builtin_ctz(NGR);
    const int rem = items & 3;
    const int lrs = rem == 1 || rem == 2 ? min(rem == 2 ? 1 : 2, kLgr) : 0;   // log2 of the parts per tail item
    const int lgpu = kLgr - lrs;                                              // log2 of the groups per part
    const int nfull = lrs ? items - rem : items;                              // items taken whole
    const int nwhole = nfull > wave ? (nfull - wave + kWaves - 1) / kWaves : 0;
    const bool has_part = lrs > 0 && wave < (rem << lrs);
    const int total = (nwhole << kLgr) + (has_part ? 1 << lgpu : 0);
    const int xlast = max(total, 1) - 1;
    const T2* ubase = up + (size_t)(P.ug + k_first + g) * mup + col;
    // The wave's x-th group: whole items wave, wave + 4, ... first, then part
    // wave & (rs - 1) of tail item nfull + (wave >> lrs).
    auto unit_at = [&](int x, int& it, int& grp) {
        const int xw = x - (nwhole << kLgr);
        if (xw < 0) {
            it = wave + kWaves * (x >> kLgr);
            grp = x & (NGR - 1);
        } else {
            it = nfull + (wave >> lrs);
            grp = ((wave & ((1 << lrs) - 1)) << lgpu) | xw;
        }
    };
    auto load_g = [&](T2 (&u)[GS], int x) {
        int it, grp;
        unit_at(min(x, xlast), it, grp);
        it = min(it, items - 1);
        const int ib = it / P.ells, li = it - ib * P.ells;
        const T2* src = ubase + (ptrdiff_t)(4 * GS * grp - rowext_shift(P, li + P.first_ell)) * mup + ib * 16;
#pragma unroll
        for (int s = 0; s < GS; ++s) u[s] = src[(size_t)(4 * s) * mup];
    };
    T2 ua[GS], ub[GS];
    // the K loop's last steps prefetched operands nobody reads; let them land
    // before these registers are written
    __builtin_amdgcn_s_waitcnt(0x0F70);
    load_g(ua, 0);
    load_g(ub, 1);
    __syncthreads();   // the window is dead from here on; its bytes become the Z planes
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = kRowsPerWave * (RF * wave + f) + M::row(g, r);   // row of the tile
            const int zo = (t >> 2) * NB * 64 + (t & 3) * 16;
#pragma unroll
            for (int cb = 0; cb < NG; ++cb) {
                zre[zo + cb * 64 + col] = acc[f][cb][r];
                zim[zo + cb * 64 + col] = acc[f][NG + cb][r];
                if constexpr (kZs) zsm[(t >> 2) * NG * 64 + (t & 3) * 16 + cb * 64 + col] = acc[f][cb][r] + acc[f][NG + cb][r];
            }
#pragma unroll
            for (int pb = 0; pb < NP; ++pb) {
                const T y = acc[f][3 * NG + pb][r];   // Zr (even col) or Zi (odd col) of complex column col / 2
                zre[zo + (NG + pb) * 64 + col] = y;
                zim[zo + (NG + pb) * 64 + (col ^ 1)] = odd ? y : -y;
            }
        }
    __syncthreads();

    // Accumulators in two sets, [0] for even and [1] for odd K steps, and the two
    // products of a pair block in two of them, so that the MFMAs issued back to back
    // are independent (a single 16-row block per item has no fragments to alternate).
    constexpr int NGa = NG > 0 ? NG : 1, NPa = NP > 0 ? NP : 1;
    constexpr int NV = 8 * NG + 4 * NP;   // result values of a unit per lane
    acc_t e1[2][NGa], e2[2][NGa], e3[2][NGa], epr[2][NPa], epi[2][NPa];
    T res[NV];   // unit result: (Re, Im) of the three-product blocks' rows, then the pair values
    T* const out = reinterpret_cast<T*>(part + (size_t)L * P.m * P.C);
    // output row 16 ib + row(g, r), lane column col
    auto store_item = [&](int it) {
        const int ib = it / P.ells, li = it - ib * P.ells;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * ib + M::row(g, r);
            if (i >= P.m) continue;
            T* orow = out + 2 * ((size_t)i * P.C + li * P.m);
#pragma unroll
            for (int cb = 0; cb < NG; ++cb) {
                const int c = 16 * cb + col;
                if (c < P.m) reinterpret_cast<T2*>(orow)[c] = T2{res[8 * cb + 2 * r], res[8 * cb + 2 * r + 1]};
            }
#pragma unroll
            for (int pb = 0; pb < NP; ++pb) {
                const int c = 16 * NG + 8 * pb + (col >> 1);
                if (c < P.m) orow[2 * c + (col & 1)] = res[8 * NG + 4 * pb + r];
            }
        }
    };
    auto group = [&](const T2 (&u)[GS], int x) {
        int it, grp;
        unit_at(x, it, grp);
        const bool whole = x < (nwhole << kLgr);
        const int lg = whole ? kLgr : lgpu;   // log2 of the unit's groups
        const int gi = grp & ((1 << lg) - 1);
        if (gi == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int cb = 0; cb < NG; ++cb) e1[h][cb] = e2[h][cb] = e3[h][cb] = acc_t{0, 0, 0, 0};
#pragma unroll
                for (int pb = 0; pb < NP; ++pb) epr[h][pb] = epi[h][pb] = acc_t{0, 0, 0, 0};
            }
        }
        // second operands of step s (plane 0, plane 1 and, three-product blocks,
        // the sum), read one step ahead
        constexpr int NGa2 = NG > 0 ? NG : 1;
        auto zread = [&](int s, T (&zr)[NB], T (&zi)[NB], T (&zz)[NGa2]) {
            const int zs = (GS * grp + s) * NB * 64 + lane;
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                zr[cb] = zre[zs + cb * 64];
                zi[cb] = zim[zs + cb * 64];
            }
#pragma unroll
            for (int cb = 0; cb < NG; ++cb) zz[cb] = kZs ? zsm[(GS * grp + s) * NG * 64 + lane + cb * 64] : T(0);
        };
        auto step = [&](int s, const T (&zr)[NB], const T (&zi)[NB], const T (&zz)[NGa2]) {
            const T ur = u[s].x, ui = u[s].y;
            const int h = s & 1;
#pragma unroll
            for (int cb = 0; cb < NG; ++cb) {
                e1[h][cb] = M::fma(ur, zr[cb], e1[h][cb]);
                e2[h][cb] = M::fma(ui, zi[cb], e2[h][cb]);
                e3[h][cb] = M::fma(ur - ui, kZs ? zz[cb] : zr[cb] + zi[cb], e3[h][cb]);
            }
#pragma unroll
            for (int pb = 0; pb < NP; ++pb) {
                epr[h][pb] = M::fma(ur, zr[NG + pb], epr[h][pb]);
                epi[h][pb] = M::fma(ui, zi[NG + pb], epi[h][pb]);
            }
        };
        T zra[NB], zia[NB], zza[NGa2], zrb[NB], zib[NB], zzb[NGa2];
        // (the scheduling barriers keep the reads ahead of the previous step's MFMAs)
        zread(0, zra, zia, zza);
#pragma unroll
        for (int s = 0; s < GS; s += 2) {   // GS is even
            zread(s + 1, zrb, zib, zzb);
            __builtin_amdgcn_sched_barrier(0);
            step(s, zra, zia, zza);
            if (s + 2 < GS) zread(s + 2, zra, zia, zza);
            __builtin_amdgcn_sched_barrier(0);
            step(s + 1, zrb, zib, zzb);
        }
        if (gi == (1 << lg) - 1) {   // the unit is complete
#pragma unroll
            for (int r = 0; r < 4; ++r) {
#pragma unroll
                for (int cb = 0; cb < NG; ++cb) {
                    const T q1 = e1[0][cb][r] + e1[1][cb][r], q2 = e2[0][cb][r] + e2[1][cb][r];
                    const T q3 = e3[0][cb][r] + e3[1][cb][r];
                    res[8 * cb + 2 * r] = q1 + q2;
                    res[8 * cb + 2 * r + 1] = q3 - q1 + q2;
                }
#pragma unroll
                for (int pb = 0; pb < NP; ++pb)
                    res[8 * NG + 4 * pb + r] = (epr[0][pb][r] + epr[1][pb][r]) + (epi[0][pb][r] + epi[1][pb][r]);
            }
            if (whole) store_item(it);
        }
    };
    for (int x = 0; x < total; x += 2) {
        group(ua, x);
        load_g(ua, x + 2);
        __builtin_amdgcn_sched_barrier(0);
        if (x + 1 == total) break;
        group(ub, x + 1);
        load_g(ub, x + 3);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lrs > 0) {
        // tail items: parts 1.. go through LDS (the Z planes are free once every
        // wave is past its MFMAs) and part 0 adds them in part order and stores
        const int pt = wave & ((1 << lrs) - 1);
        __syncthreads();
        if (pt > 0 && has_part) {
#pragma unroll
            for (int v = 0; v < NV; ++v) zpl[((wave - 1) * NV + v) * 64 + lane] = res[v];
        }
        __syncthreads();
        if (pt == 0 && has_part) {
            for (int q = 1; q < (1 << lrs); ++q)
#pragma unroll
                for (int v = 0; v < NV; ++v) res[v] += zpl[((wave + q - 1) * NV + v) * 64 + lane];
            store_item(nfull + (wave >> lrs));
        }
    }
}
template <typename T, int NB, int RF, int NG>
__global__ __launch_bounds__(kThreads) void pencil_tiles(PencilPlan P, TilePtrs<T> ptr) {
    const int id = blockIdx.x;
    const int L = (P.nwg & 7) == 0 ? (id & 7) * (P.nwg >> 3) + (id >> 3) : id;
    tile_body<T, NB, RF, 0, false, NG>(P, ptr, L);
}

// S-build tiles with split operands (FP32-accurate products on the bf16 MFMA).
template <int NB, int RF>
__global__ __launch_bounds__(kThreads) void pencil_tiles_split(PencilPlan P, TilePtrs<float> ptr) {
    const int id = blockIdx.x;
    const int L = (P.nwg & 7) == 0 ? (id & 7) * (P.nwg >> 3) + (id >> 3) : id;
    tile_body<float, NB, RF, 0, true>(P, ptr, L);
}

// Y = T X (or T^* X) for a block of columns: tiles of the product, partial
// over the K chunks (summed by toeplitz_mm_finish).
template <typename T, int NB, int RF, int NG>
__global__ __launch_bounds__(kThreads) void toeplitz_mm_tiles(PencilPlan P, TilePtrs<T> ptr) {
    const int id = blockIdx.x;
    const int L = (P.nwg & 7) == 0 ? (id & 7) * (P.nwg >> 3) + (id >> 3) : id;
    tile_body<T, NB, RF, 1, false, NG>(P, ptr, L);
}

// Y[k, c] = sum over chunks s (in order) of the partial real columns 2c, 2c+1, FP64.
template <typename T>
__global__ __launch_bounds__(256) void toeplitz_mm_finish(PencilPlan P, const T* __restrict__ part,
                                                         double2* __restrict__ Y, int64_t ldy) {
    const int o = blockIdx.x * 256 + threadIdx.x;
    if (o >= P.N * P.C) return;
    const int k = o / P.C, c = o - (o / P.C) * P.C;
    const size_t slab = (size_t)P.rt * P.rows * P.nrr;
    const T* src = part + (size_t)k * P.nrr + 2 * c;
    double re = 0.0, im = 0.0;
    for (int s2 = 0; s2 < P.sk; ++s2) {
        re += (double)src[s2 * slab];
        im += (double)src[s2 * slab + 1];
    }
    Y[(size_t)k * ldy + c] = make_double2(re, im);
}

// Product with one column, y = T x or T^* x (Lanczos steps): vector FMAs instead of
// the MFMA tiles, which would use 2 of their 16 columns. Same plan, packing and
// partial-row layout as toeplitz_mm_tiles: a workgroup stages its tile's window and
// its chunk's h offsets and x values in LDS; thread t accumulates row t mod R of the
// tile (R = 64 rf rows) over the t / R-th of S contiguous shares of the chunk
// (S = 256 / R), the S shares are added in order through LDS, and
// toeplitz_mm_finish sums the chunks.
template <typename T>
__global__ __launch_bounds__(kThreads) void toeplitz_mv(PencilPlan P, TilePtrs<T> ptr) {
    using T2 = pair_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int id = blockIdx.x;
    const int L = (P.nwg & 7) == 0 ? (id & 7) * (P.nwg >> 3) + (id >> 3) : id;
    const int sk_i = L / P.rt, rt_i = L - (L / P.rt) * P.rt;
    const int k_first = rt_i * P.rows;
    const int k_last = min(k_first + P.rows - 1, P.NR - 1);
    const int h_first = sk_i * P.kc;
    const int h_last = min(h_first + P.kc, P.kb) - 1;
    const int nh = h_last - h_first + 1;
    const int lo = row_offset(P, k_first) - h_offset(P, h_last) + P.c0;
    const int hi = row_offset(P, k_last) - h_offset(P, h_first) + P.c0;
    const int W = hi - lo + 1;
    // T^* multiplies by the Toeplitz matrix of conj(f(-p)): offsets reflected about c0
    const bool reflect = P.conj_grid;
    T2* win = reinterpret_cast<T2*>(smem);
    int* go = reinterpret_cast<int*>(smem + align_up(sizeof(T2) * (size_t)P.win_cap, 16));
    T2* xs = reinterpret_cast<T2*>(smem + align_up(sizeof(T2) * (size_t)P.win_cap, 16) + align_up(4 * (size_t)P.kc, 16));
    T2* red = xs + P.kc;   // one partial sum per thread
    const int tid = threadIdx.x;
    // kStage loads per thread in flight
    constexpr int kStage = 8;
    for (int base = 0; base < max(W, nh); base += kStage * kThreads) {
        double2 v[kStage];
        int o[kStage];
        T2 p[kStage];
#pragma unroll
        for (int j = 0; j < kStage; ++j) {
            const int w = base + j * kThreads + tid;
            if (w < W) v[j] = ptr.grid[reflect ? 2 * P.c0 - (lo + w) : lo + w];
            if (w < nh) {
                o[j] = ptr.gtab[h_first + w];
                p[j] = ptr.vp[(size_t)(h_first + w) * P.nrp];   // pair column 0: (Re x, -Im x)
            }
        }
#pragma unroll
        for (int j = 0; j < kStage; ++j) {
            const int w = base + j * kThreads + tid;
            if (w < W) win[w] = T2{(T)v[j].x, reflect ? -(T)v[j].y : (T)v[j].y};
            if (w < nh) {
                go[w] = o[j];
                xs[w] = T2{p[j].x, -p[j].y};
            }
        }
    }
    __syncthreads();
    const int R = P.rows, S = kThreads / P.rows;   // R is a multiple of 64: sub is uniform per wave
    const int r = tid % R, sub = tid / R;
    const int gk = row_offset(P, min(k_first + r, P.NR - 1)) + P.c0 - lo;
    // share sub: a contiguous range of the chunk. Along a line of I_n the h offset
    // grows by one, so the window index of the next h is one lower; after a line's
    // last h it is read from the offsets (one read per line instead of per h).
    const int per = (nh + S - 1) / S;
    const int w0 = __builtin_amdgcn_readfirstlane(min(sub * per, nh));
    const int w1 = __builtin_amdgcn_readfirstlane(min(w0 + per, nh));
    T re = 0, im = 0;
    // runs of consecutive h along one line: window indices pos, pos - 1, ...
    for (int w = w0, j = (h_first + w0) % (P.n + 1); w < w1; j = 0) {
        const int run = min(P.n + 1 - j, w1 - w);
        const int pos = gk - go[w];
#pragma unroll 8
        for (int t = 0; t < run; ++t) {
            const T2 a = win[pos - t];
            const T2 x = xs[w + t];
            re = fma(a.x, x.x, re);
            re = fma(-a.y, x.y, re);
            im = fma(a.x, x.y, im);
            im = fma(a.y, x.x, im);
        }
        w += run;
    }
    red[tid] = T2{re, im};
    __syncthreads();
    if (sub == 0 && k_first + r <= k_last) {
        T sr = red[r].x, si = red[r].y;
        for (int q = 1; q < S; ++q) {
            sr += red[q * R + r].x;
            si += red[q * R + r].y;
        }
        T* yp = reinterpret_cast<T*>(ptr.part) + ((size_t)sk_i * P.rt * P.rows + k_first + r) * P.nrr;
        yp[0] = sr;
        yp[1] = si;
    }
}

// One instance of a batch: its plan, its pointers and the first global tile
// index of the instance within its launch.
template <typename T>
struct BatchEntry {
    PencilPlan P;
    TilePtrs<T> ptr;
    const double2* U;
    const double2* V;
    int tile_begin;
};

// Packing for every instance of a batch: grid (x, 3, instances). The first
// thread also resets the work counter of the queue schedule (the tile launch
// follows on the same stream).
template <typename T>
__global__ __launch_bounds__(256) void pencil_pack_batched(const BatchEntry<T>* __restrict__ entries,
                                                           int* __restrict__ queue_counter) {
    if (queue_counter && (blockIdx.x | blockIdx.y | blockIdx.z | threadIdx.x) == 0) *queue_counter = 0;
    const BatchEntry<T>& e = entries[blockIdx.z];
    pack_body<T>(e.P, e.U, e.P.m, 1, e.V, e.P.m, 1, const_cast<pair_t<T>*>(e.ptr.vp),
                 const_cast<pair_t<T>*>(e.ptr.up), const_cast<int*>(e.ptr.gtab), blockIdx.y);
}

// Batched launch over the instances of one column-block class, ordered by
// decreasing work: workgroup `id` finds its instance by binary search over the
// tile offsets (the hardware dispatches workgroups in id order, so the longest
// tiles start first).
template <typename T, int NB, int RF, int NG>
__global__ __launch_bounds__(kThreads) void pencil_tiles_batched(const BatchEntry<T>* __restrict__ entries,
                                                                 int count) {
    const int id = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (entries[mid].tile_begin <= id)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchEntry<T>& e = entries[lo];
    tile_body<T, NB, RF, 0, false, NG>(e.P, e.ptr, id - e.tile_begin);
}

size_t lds_bytes_for(int win, int kc, size_t epi, size_t tsize, int split_nrp = 0, int bbufs = 2, bool wide = false) {
    const size_t entry = split_nrp ? 16 : (wide ? 4 : 2) * tsize;
    const size_t loop = align_up(entry * (size_t)win, 16) + align_up(4 * ((size_t)kc + kPrefetchRows + 16), 16) +
                        (split_nrp ? (size_t)bbufs * kSplitPlanes * split_nrp * 64 : 0);
    return align_up(std::max(loop, epi), 16);
}

// Largest G-span of the aligned runs of `len` consecutive indices (row tiles of
// I_n or of the row-extended set {0..n+1}^d, or chunks of I_n).
int max_span(int count, int len, int d, int n, bool rowext) {
    int best = 0;
    for (int s = 0; s < count; s += len) {
        const int e = std::min(s + len, count) - 1;
        const int a = rowext ? rowext_offset(s, d, n) : grid_offset_of_index(s, d, n);
        const int b = rowext ? rowext_offset(e, d, n) : grid_offset_of_index(e, d, n);
        best = std::max(best, b - a);
    }
    return best;
}

// Bytes of the packed second factor, the packed U, the offset table and the
// partial sums of a plan (the workspace sections, each aligned to 256 bytes).
struct PlanBytes {
    size_t v, u, g, p;
};
PlanBytes plan_bytes(const PencilPlan& P, size_t tsize) {
    const size_t t2 = 2 * tsize;
    PlanBytes b;
    if (P.split)   // three bfloat16 planes per K block, 32 values per (plane, column)
        b.v = align_up(((size_t)P.sk * P.kc / kSplitK) * kSplitPlanes * P.nrp * 64, 256);
    else
        b.v = align_up(t2 * ((size_t)P.sk * P.kc + kPrefetchRows) * P.nrp, 256);
    b.u = align_up(t2 * ((size_t)P.ug + (size_t)P.rt * P.rows) * P.mbi * 16, 256);
    b.g = align_up(4 * ((size_t)P.sk * P.kc + kPrefetchRows), 256);
    if (P.mode)   // partial Y rows of every chunk, real columns
        b.p = align_up(tsize * (size_t)P.sk * P.rt * P.rows * P.nrr, 256);
    else
        b.p = align_up(t2 * (size_t)P.nwg * P.m * P.C, 256);
    return b;
}

int tuned_target(prony_handle_t h, int d, int n, int m, int prec, int batched) {
    return tuned(h, d, n, m, prec, batched != 0).target;
}

int tuned_fragments(prony_handle_t h, int d, int n, int m, int prec, int batched) {
    return tuned(h, d, n, m, prec, batched != 0).fragments;
}

// target_wgs: workgroups the split of the h' range aims at (single instances
// fill the GPU with one launch; batch members use target 1, i.e. no split
// beyond what the LDS window imposes).
// mode 1 plans the product Y = T X of a block of m columns (h over I_n, no
// shifted copies, no U^* epilogue).
// rf_req: 16-row fragments per wave; 0 picks 2 where the instantiation allows it
// (and the product has more than one 64-row tile), 1, 2 or 4 ask for that count
// (the default when not supported for the column count).
// allow_gauss: S-builds take three-product blocks of 16 complex columns while more
// than 8 columns remain, then one pair block for the rest (per fragment and K step
// 3 MFMAs per three-product block and 2 per pair block: never more than either
// form alone, e.g. 5 instead of 6 at m = 20 and 6 instead of 8 at m = 30).
prony_status_t make_plan(prony_handle_t h, int d, int n, int m, bool with_s0, size_t tsize, PencilPlan& P,
                         int target_wgs = 0, int rf_req = 0, int mode = 0, bool split = false,
                         bool allow_gauss = false, int kal_req = 0) {
    P = PencilPlan{};
    P.d = d;
    P.n = n;
    P.N = (int)ipow(n + 1, d);
    P.m = m;
    P.mode = mode;
    P.split = split ? 1 : 0;
    P.ells = mode ? 1 : d + (with_s0 ? 1 : 0);
    P.first_ell = mode || with_s0 ? 0 : 1;
    P.C = P.ells * m;
    P.CB = m;
    P.ng = 0;
    if (!split && allow_gauss) {
        P.ng = m / 16;
        if (m - 16 * P.ng > 8) ++P.ng;
    }
    P.nb = P.ng + (2 * std::max(0, P.CB - 16 * P.ng) + 15) / 16;
    P.nrp = 16 * P.nb;
    P.nrr = 32 * P.ng + 16 * (P.nb - P.ng);
    P.mbi = mode ? 0 : (m + 15) / 16;
    // the FP32/FP64 S-build tiles take the packed U row length as 16 nb
    if (!mode && !split && P.mbi != P.nb) return fail(h, PRONY_ENOTSUP, "prony_build_S: unexpected column blocks");
    P.NR = mode ? P.N : (int)ipow(n + 2, d);
    P.ug = mode ? 0 : (int)ipow(n + 2, d - 1);
    P.kb = P.N;
    P.rf = rf_supported(tsize, P.nb, 2, split, P.ng) && P.NR > kRowsPerTile ? 2 : 1;
    if ((rf_req == 1 || rf_req == 2 || rf_req == 4) && rf_supported(tsize, P.nb, rf_req, split, P.ng))
        P.rf = rf_req;
    P.rows = kRowsPerTile * P.rf;
    P.rt = (P.NR + P.rows - 1) / P.rows;
    P.c0 = grid_center(d, n);

    // two workgroups per CU; the split kernel, which also stages B planes, may
    // take the whole LDS when its window does not fit otherwise. The S-build's
    // epilogue holds the tile's rows of Z as two planes of one 16-column slot per
    // column block, at most 64 KiB for every instantiated shape.
    size_t budget = std::min<size_t>(h->lds_per_block, 80 * 1024);
    const size_t epi = mode ? 0
                            : (size_t)(2 * P.nb + (z_sum_plane(tsize, P.nb, P.ng, P.rows) ? P.ng : 0)) * P.rows * 16 *
                                  tsize;
    P.bbufs = 2;
    const int target = target_wgs > 0 ? target_wgs : 4 * h->num_cus;
    const int sk_target = std::max(1, target / P.rt);
    // chunk granularity: K blocks of the MFMA loop, or kal_req (whole lines or planes of
    // I_n for the one-column product, whose windows are then the narrowest)
    const size_t kal = kal_req > 0 ? (size_t)kal_req : split ? kSplitK : 16;
    int kc = (int)align_up((size_t)((P.kb + sk_target - 1) / sk_target), kal);
    kc = std::max(kc, std::min(128, (int)align_up((size_t)P.kb, kal)));
    const int kc0 = kc;
    const int rowspan = max_span(P.NR, P.rows, d, n, !mode);
    for (;;) {
        const int colspan = max_span(P.kb, kc, d, n, false);
        const int win = rowspan + colspan + 1;
        size_t lds = lds_bytes_for(win, kc, epi, tsize, split ? P.nrp : 0, 2);
        if (split && lds > budget) {   // one B buffer (two barriers per K block) before smaller chunks
            P.bbufs = 1;
            lds = lds_bytes_for(win, kc, epi, tsize, P.nrp, 1);
        }
        if (lds <= budget) {
            P.kc = kc;
            P.sk = (P.kb + kc - 1) / kc;
            P.win_cap = win;
            P.lds_bytes = lds;
            break;
        }
        if (kc <= (int)kal) {
            if (split && budget < h->lds_per_block) {   // retry from the first chunk size
                budget = h->lds_per_block;
                kc = kc0;
                P.bbufs = 2;
                continue;
            }
            return fail(h, PRONY_ENOTSUP, "prony_build_S: sample window does not fit in LDS");
        }
        kc = (int)align_up((size_t)(kc / 2), kal);
        P.bbufs = 2;
    }
    // FP32 three-product S-build blocks: the sums Re + Im of the window entries
    // staged with them when the wider entries fit at this chunk size (one VALU
    // operation less per fragment and K step in the MFMA stream; measured slower
    // with FP64's 32-byte entries and in the product mode)
    if (!split && P.ng > 0 && tsize == 4 && !mode) {
        const size_t lw = lds_bytes_for(P.win_cap, P.kc, epi, tsize, 0, 2, true);
        if (lw <= budget) {
            P.wsum = 1;
            P.lds_bytes = lw;
        }
    }
    P.nwg = P.rt * P.sk;
    if (((int64_t)P.sk * P.kc + kPrefetchRows) * P.nrp >= (int64_t(1) << 31) ||
        (int64_t)P.nwg * P.m * P.C >= (int64_t(1) << 31) ||
        ((int64_t)P.ug + (int64_t)P.rt * P.rows) * P.mbi * 16 >= (int64_t(1) << 31) ||
        (int64_t)P.sk * P.rt * P.rows * P.nrr >= (int64_t(1) << 31))
        return fail(h, PRONY_ENOTSUP, "prony_build_S: problem too large for 32-bit tile indexing");
    const PlanBytes b = plan_bytes(P, tsize);
    P.off_v = 0;
    P.off_u = P.off_v + b.v;
    P.off_g = P.off_u + b.u;
    P.off_p = P.off_g + b.g;
    P.ws_bytes = P.off_p + b.p;
    return PRONY_OK;
}

// Sum of the workgroup partials (reduce.h) and Sigma^{-1}: S_l(i, q) = sum / sigma_q.
template <typename T>
__global__ __launch_bounds__(kFinishThreads) void pencil_finish(PencilPlan P, const pair_t<T>* __restrict__ part,
                                                                const double* __restrict__ sigma,
                                                                double2* __restrict__ S) {
    finish_rows(part, P.nwg, P.m * P.C, blockIdx.x * kFinishOuts,
                [&](int o, double re, double im) { store_s(P, sigma, S, o, re, im); });
}

// Same for every instance of a batch: grid (slices, instances).
template <typename T>
__global__ __launch_bounds__(kFinishThreads) void pencil_finish_batched(const BatchEntry<T>* __restrict__ entries) {
    const BatchEntry<T>& e = entries[blockIdx.y];
    const int tot = e.P.m * e.P.C;
    if ((int)blockIdx.x * kFinishOuts >= tot) return;
    finish_rows(e.ptr.part, e.P.nwg, tot, blockIdx.x * kFinishOuts,
                [&](int o, double re, double im) { store_s(e.P, e.ptr.sigma, e.ptr.S, o, re, im); });
}

template <typename T, int NB, int RF, int NG = 0>
prony_status_t launch_tiles(prony_handle_t h, const PencilPlan& P, const TilePtrs<T>& ptr) {
    if (P.lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pencil_tiles<T, NB, RF, NG>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes);
        if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
    }
    ProfileScope prof(h, "pencil_tiles");
    pencil_tiles<T, NB, RF, NG><<<P.nwg, kThreads, P.lds_bytes, h->stream>>>(P, ptr);
    return PRONY_OK;
}

template <typename T, int NB, int RF, int NG = 0>
prony_status_t launch_batched(prony_handle_t h, const BatchEntry<T>* entries, int count, int tiles, size_t lds,
                              hipStream_t stream) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pencil_tiles_batched<T, NB, RF, NG>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
    }
    ProfileScope prof(h, "pencil_tiles_batched", stream);
    pencil_tiles_batched<T, NB, RF, NG><<<tiles, kThreads, lds, stream>>>(entries, count);
    return PRONY_OK;
}

template <int NB, int RF>
prony_status_t launch_tiles_split(prony_handle_t h, const PencilPlan& P, const TilePtrs<float>& ptr) {
    if (P.lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pencil_tiles_split<NB, RF>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes);
        if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
    }
    ProfileScope prof(h, "pencil_tiles");
    pencil_tiles_split<NB, RF><<<P.nwg, kThreads, P.lds_bytes, h->stream>>>(P, ptr);
    return PRONY_OK;
}

// Column blocks of the S-build's second operand: 2m <= 64 real columns.
#define PRONY_NB_CASES(X) X(1) X(2) X(3) X(4)
// (blocks, three-product blocks) of the S-builds with three-product blocks, m <= 32:
// m = 9..16, 17..24, 25..32
#define PRONY_MIXED_CASES(X) X(1, 1) X(2, 1) X(2, 2)

// Work item of the queue schedule: a tile L of the instance at position `entry`
// of the batch's entry table.
struct WorkItem {
    int entry;
    int tile;
};

// One tile of any class: the instantiation is chosen per item from the
// instance's column blocks and row fragments.
template <typename T>
__device__ __forceinline__ void tile_of_class(const BatchEntry<T>& e, int L) {
    switch (e.P.ng * 16 + e.P.nb * 2 + e.P.rf - 1) {
        case 2:   // one pair block (m <= 8)
            tile_body<T, 1, 1, 0>(e.P, e.ptr, L);
            break;
        case 3:
            tile_body<T, 1, 2, 0>(e.P, e.ptr, L);
            break;
#define PRONY_QGCASE(NBV, NGV)                                                     \
    case NGV * 16 + NBV * 2:                                                       \
        tile_body<T, NBV, 1, 0, false, NGV>(e.P, e.ptr, L);                        \
        break;                                                                     \
    case NGV * 16 + NBV * 2 + 1:                                                   \
        if constexpr (rf_supported(sizeof(T), NBV, 2, false, NGV)) tile_body<T, NBV, 2, 0, false, NGV>(e.P, e.ptr, L); \
        break;
        PRONY_MIXED_CASES(PRONY_QGCASE)
#undef PRONY_QGCASE
        default:
            break;
    }
}

// Queue schedule of a batch: one persistent launch of as many workgroups as fit
// the device at once; each takes the next work item (all tiles of all
// instances, longest first) from a counter until the queue is empty. Bounded to
// two workgroups per CU: the union of the tile classes would take more registers.
template <typename T>
__global__ __launch_bounds__(kThreads, 2) void pencil_tiles_queue(const BatchEntry<T>* __restrict__ entries,
                                                               const WorkItem* __restrict__ items, int nitems,
                                                               int* __restrict__ counter) {
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        __syncthreads();   // every thread has read `next` (and left the previous tile's LDS)
        if (it >= nitems) break;
        const WorkItem w = items[it];
        tile_of_class<T>(entries[w.entry], w.tile);
    }
}

template <typename T>
prony_status_t dispatch_tiles(prony_handle_t h, const PencilPlan& P, const TilePtrs<T>& ptr) {
    if (P.ng) {   // three-product blocks (and a pair block), m <= 32
        switch (P.ng * 16 + P.nb) {
#define PRONY_GCASE(NBV, NGV)                                                   \
    case NGV * 16 + NBV:                                                        \
        if constexpr (rf_supported(sizeof(T), NBV, 4, false, NGV))              \
            if (P.rf == 4) return launch_tiles<T, NBV, 4, NGV>(h, P, ptr);      \
        if constexpr (rf_supported(sizeof(T), NBV, 2, false, NGV))              \
            if (P.rf == 2) return launch_tiles<T, NBV, 2, NGV>(h, P, ptr);      \
        return launch_tiles<T, NBV, 1, NGV>(h, P, ptr);
            PRONY_MIXED_CASES(PRONY_GCASE)
#undef PRONY_GCASE
            default:
                return fail(h, PRONY_ENOTSUP, "prony_build_S: too many columns");
        }
    }
    if constexpr (sizeof(T) == 4)
        if (P.split) {   // pair blocks only
            switch (P.nb) {
#define PRONY_CASE(NBV)                                                    \
    case NBV:                                                              \
        if constexpr (rf_supported(4, NBV, 4, true))                       \
            if (P.rf == 4) return launch_tiles_split<NBV, 4>(h, P, ptr);   \
        if constexpr (rf_supported(4, NBV, 2, true))                       \
            if (P.rf == 2) return launch_tiles_split<NBV, 2>(h, P, ptr);   \
        return launch_tiles_split<NBV, 1>(h, P, ptr);
                PRONY_NB_CASES(PRONY_CASE)
#undef PRONY_CASE
                default:
                    return fail(h, PRONY_ENOTSUP, "prony_build_S: too many columns");
            }
        }
    // without three-product blocks: one pair block (m <= 8)
    if (P.nb != 1) return fail(h, PRONY_ENOTSUP, "prony_build_S: unexpected column blocks");
    if (P.rf == 4) return launch_tiles<T, 1, 4>(h, P, ptr);
    if (P.rf == 2) return launch_tiles<T, 1, 2>(h, P, ptr);
    return launch_tiles<T, 1, 1>(h, P, ptr);
}

template <typename T>
prony_status_t dispatch_batched(prony_handle_t h, int nb, int rf, int ng, const BatchEntry<T>* entries, int count,
                                int tiles, size_t lds, hipStream_t stream) {
    if (ng) {
        switch (ng * 16 + nb) {
#define PRONY_GCASE(NBV, NGV)                                                                           \
    case NGV * 16 + NBV:                                                                                \
        if constexpr (rf_supported(sizeof(T), NBV, 2, false, NGV))                                      \
            if (rf == 2) return launch_batched<T, NBV, 2, NGV>(h, entries, count, tiles, lds, stream);  \
        return launch_batched<T, NBV, 1, NGV>(h, entries, count, tiles, lds, stream);
            PRONY_MIXED_CASES(PRONY_GCASE)
#undef PRONY_GCASE
            default:
                return fail(h, PRONY_ENOTSUP, "prony_build_S_batched: too many columns");
        }
    }
    // without three-product blocks: one pair block (m <= 8)
    if (nb != 1) return fail(h, PRONY_ENOTSUP, "prony_build_S_batched: unexpected column blocks");
    if (rf == 2) return launch_batched<T, 1, 2>(h, entries, count, tiles, lds, stream);
    return launch_batched<T, 1, 1>(h, entries, count, tiles, lds, stream);
}

// The three launches of one S-build with the packed operands and partial sums in
// the workspace at `ws` (P.ws_bytes bytes, owned by the caller of this function).
// Packing launch of one S-build: V pairs (or split planes), U_ext pairs and the
// G(h) table into the sections of `base` given by the plan's offsets.
template <typename T>
prony_status_t pack_operands(prony_handle_t h, const PencilPlan& P, unsigned char* base, const double* U,
                             int64_t u_rs, int64_t u_cs, const double* V, int64_t v_rs, int64_t v_cs) {
    using T2 = pair_t<T>;
    T2* vp = reinterpret_cast<T2*>(base + P.off_v);
    T2* up = reinterpret_cast<T2*>(base + P.off_u);
    int* gt = reinterpret_cast<int*>(base + P.off_g);
    const int64_t kbp = (int64_t)P.sk * P.kc + kPrefetchRows;
    const int64_t largest = std::max<int64_t>(kbp * P.nrp, ((int64_t)P.ug + (int64_t)P.rt * P.rows) * P.mbi * 16);
    const int pack_blocks = (int)std::min<int64_t>((largest + 255) / 256, 2 * (int64_t)h->num_cus);
    {
        ProfileScope prof(h, "pencil_pack");
        pencil_pack<T><<<dim3(pack_blocks, 3), 256, 0, h->stream>>>(
            P, reinterpret_cast<const double2*>(U), u_rs, u_cs, reinterpret_cast<const double2*>(V), v_rs, v_cs, vp,
            up, gt);
    }
    return check_launch(h, "pencil_pack");
}

// Tile and finishing launches of one S-build over packed operands at `base` (plan
// offsets) and partial rows at `part`.
template <typename T>
prony_status_t launch_tiles_finish(prony_handle_t h, const PencilPlan& P, const unsigned char* base,
                                   unsigned char* part_bytes, const double* f, const double* sigma, double* S) {
    using T2 = pair_t<T>;
    T2* part = reinterpret_cast<T2*>(part_bytes);
    const TilePtrs<T> ptr{reinterpret_cast<const double2*>(f), reinterpret_cast<const T2*>(base + P.off_v),
                          reinterpret_cast<const T2*>(base + P.off_u), reinterpret_cast<const int*>(base + P.off_g),
                          part, sigma, reinterpret_cast<double2*>(S)};
    prony_status_t st = dispatch_tiles<T>(h, P, ptr);
    if (st != PRONY_OK) return st;
    if ((st = check_launch(h, "pencil_tiles")) != PRONY_OK) return st;
    {
        ProfileScope prof(h, "pencil_finish");
        const int tot = P.m * P.C;
        pencil_finish<T><<<(tot + kFinishOuts - 1) / kFinishOuts, kFinishThreads, 0, h->stream>>>(
            P, part, sigma, reinterpret_cast<double2*>(S));
    }
    return check_launch(h, "pencil_finish");
}

template <typename T>
prony_status_t launch_pencil(prony_handle_t h, const PencilPlan& P, unsigned char* ws, const double* f,
                             const double* U, int64_t u_rs, int64_t u_cs, const double* sigma, const double* V,
                             int64_t v_rs, int64_t v_cs, double* S) {
    const prony_status_t st = pack_operands<T>(h, P, ws, U, u_rs, u_cs, V, v_rs, v_cs);
    if (st != PRONY_OK) return st;
    return launch_tiles_finish<T>(h, P, ws, ws + P.off_p, f, sigma, S);
}

template <typename T, int NB, int RF, int NG = 0>
prony_status_t launch_mm_tiles(prony_handle_t h, const PencilPlan& P, const TilePtrs<T>& ptr) {
    if (P.lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&toeplitz_mm_tiles<T, NB, RF, NG>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes);
        if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
    }
    ProfileScope prof(h, "toeplitz_mm_tiles");
    toeplitz_mm_tiles<T, NB, RF, NG><<<P.nwg, kThreads, P.lds_bytes, h->stream>>>(P, ptr);
    return PRONY_OK;
}


// (blocks, three-product blocks) of the products with three-product blocks, r <= 64
#define PRONY_MM_MIXED_CASES(X) X(1, 1) X(2, 1) X(2, 2) X(3, 2) X(3, 3) X(4, 3) X(4, 4)

template <typename T>
prony_status_t dispatch_mm(prony_handle_t h, const PencilPlan& P, const TilePtrs<T>& ptr) {
    if (P.ng) {
        switch (P.ng * 16 + P.nb) {
#define PRONY_GCASE(NBV, NGV)                                                    \
    case NGV * 16 + NBV:                                                         \
        if constexpr (rf_supported(sizeof(T), NBV, 2, false, NGV))               \
            if (P.rf == 2) return launch_mm_tiles<T, NBV, 2, NGV>(h, P, ptr);    \
        return launch_mm_tiles<T, NBV, 1, NGV>(h, P, ptr);
            PRONY_MM_MIXED_CASES(PRONY_GCASE)
#undef PRONY_GCASE
            default:
                return fail(h, PRONY_ENOTSUP, "prony_toeplitz_mm: too many columns");
        }
    }
    // without three-product blocks: one pair block (r <= 8)
    if (P.nb != 1) return fail(h, PRONY_ENOTSUP, "prony_toeplitz_mm: unexpected column blocks");
    if (P.rf == 2) return launch_mm_tiles<T, 1, 2>(h, P, ptr);
    return launch_mm_tiles<T, 1, 1>(h, P, ptr);
}

// LDS of toeplitz_mv under plan P: the window, the chunk's h offsets and x values,
// one partial sum per thread.
size_t mv_lds_bytes(const PencilPlan& P, size_t tsize) {
    return align_up(2 * tsize * (size_t)P.win_cap, 16) + align_up(4 * (size_t)P.kc, 16) +
           2 * tsize * ((size_t)P.kc + kThreads);
}

// Whether a product plan runs on toeplitz_mv (one column, rows per tile at most the
// threads of a workgroup, LDS within the device limit).
bool mv_fits(prony_handle_t h, const PencilPlan& P, size_t tsize) {
    return P.CB == 1 && P.rows <= kThreads && mv_lds_bytes(P, tsize) <= h->lds_per_block;
}

template <typename T>
prony_status_t launch_toeplitz_mm(prony_handle_t h, const PencilPlan& P, const double* f, const double* X,
                                  int64_t ldx, double* Y, int64_t ldy) {
    using T2 = pair_t<T>;
    prony_status_t st = ensure_workspace(h, P.ws_bytes);
    if (st != PRONY_OK) return st;
    unsigned char* ws = static_cast<unsigned char*>(h->ws);
    T2* vp = reinterpret_cast<T2*>(ws + P.off_v);
    int* gt = reinterpret_cast<int*>(ws + P.off_g);
    T2* part = reinterpret_cast<T2*>(ws + P.off_p);
    const int64_t kbp = (int64_t)P.sk * P.kc + kPrefetchRows;
    const int pack_blocks = (int)std::min<int64_t>((kbp * P.nrp + 255) / 256, 2 * (int64_t)h->num_cus);
    {
        ProfileScope prof(h, "pencil_pack");
        pencil_pack<T><<<dim3(pack_blocks, 3), 256, 0, h->stream>>>(
            P, nullptr, 0, 0, reinterpret_cast<const double2*>(X), ldx, 1, vp, nullptr, gt);
    }
    if ((st = check_launch(h, "pencil_pack")) != PRONY_OK) return st;
    const TilePtrs<T> ptr{reinterpret_cast<const double2*>(f), vp, nullptr, gt, part, nullptr, nullptr};
    // one column: the vector kernel on the same plan (window, h offsets and x of a
    // chunk, and one partial sum per thread, in LDS)
    const size_t mv_lds = mv_lds_bytes(P, sizeof(T));
    if (mv_fits(h, P, sizeof(T))) {
        if (mv_lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&toeplitz_mv<T>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)mv_lds);
            if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
        }
        {
            ProfileScope prof(h, "toeplitz_mv");
            toeplitz_mv<T><<<P.nwg, kThreads, mv_lds, h->stream>>>(P, ptr);
        }
        if ((st = check_launch(h, "toeplitz_mv")) != PRONY_OK) return st;
    } else {
        if (P.kc % 16) return fail(h, PRONY_ENOTSUP, "prony_toeplitz_mm: chunk not a multiple of 16");
        if ((st = dispatch_mm<T>(h, P, ptr)) != PRONY_OK) return st;
        if ((st = check_launch(h, "toeplitz_mm_tiles")) != PRONY_OK) return st;
    }
    {
        ProfileScope prof(h, "toeplitz_mm_finish");
        const int outs = P.N * P.C;
        toeplitz_mm_finish<T><<<(outs + 255) / 256, 256, 0, h->stream>>>(
            P, reinterpret_cast<const T*>(part), reinterpret_cast<double2*>(Y), ldy);
    }
    return check_launch(h, "toeplitz_mm_finish");
}

}  // namespace

// Workspace bytes of one build_S call of shape (d, n, m) under any plan the
// handle may choose (used by prony_reserve): every precision (the split-bfloat16
// plan included), with and without S_0, at the default target, every target the
// autotuner chooses from (1, 2, 3, 4 and 8 workgroups per compute unit) and the
// target registered for the shape.
size_t pencil_workspace_bytes(prony_handle_t h, int d, int n, int m) {
    size_t best = 0;
    const std::string saved = h->err;   // plans that do not fit only fail here
    for (int prec : {PRONY_FP64, PRONY_FP32, PRONY_BF16X3}) {
        const size_t ts = prec == PRONY_FP64 ? sizeof(double) : sizeof(float);
        const int targets[] = {0, h->num_cus, 2 * h->num_cus, 3 * h->num_cus, 4 * h->num_cus, 8 * h->num_cus,
                               tuned_target(h, d, n, m, prec, 0)};
        for (int s0 = 0; s0 < 2; ++s0)
            for (int tg : targets)
                for (int rf : {1, 2, 4}) {
                    PencilPlan P;
                    if (make_plan(h, d, n, m, s0 == 1, ts, P, tg, rf, 0, prec == PRONY_BF16X3, true) == PRONY_OK)
                        best = std::max(best, P.ws_bytes);
                }
    }
    h->err = saved;
    return best;
}

namespace {

// Fixed scratch of prony_build_S_noalloc: the packed operands and partial sums of
// one S-build, in device memory that the code object holds on every device the
// library runs on, until the process ends. Host code never uses this name as an
// address: the per-device address comes from hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of `scratch` on that device

}  // namespace

prony_status_t scratch_attach(prony_handle_t h) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(h->device);
    if (it != g_scratch_ptr.end()) {
        h->scratch = it->second;
        return PRONY_OK;
    }
    void* ptr = nullptr;   // the handle's device is current (prony_create)
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(h, PRONY_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[h->device] = ptr;
    h->scratch = ptr;
    return PRONY_OK;
}

namespace {

// Host-side validation shared by prony_build_S and prony_build_S_noalloc, and the
// plan of the call.
prony_status_t plan_build_S(prony_handle_t h, const char* who, int d, int n, int m, const double* f,
                            const double* U, int64_t u_rs, int64_t u_cs, const double* sigma, const double* V,
                            int64_t v_rs, int64_t v_cs, prony_prec_t prec, unsigned flags, double* S,
                            PencilPlan& P, bool plan_only = false) {
    prony_status_t st = check_dn(h, d, n);
    if (st != PRONY_OK) return st;
    const std::string w(who);
    const int64_t N = ipow(n + 1, d);
    if (m < 1 || m > N) return fail(h, PRONY_EINVAL, w + ": m must be in 1..N");
    if (m > 32) return fail(h, PRONY_ENOTSUP, w + ": m > 32 is not supported");
    if (!f || !U || !V || !sigma || !S) return fail(h, PRONY_EINVAL, w + ": null pointer");
    if (u_rs < 1 || u_cs < 1 || v_rs < 1 || v_cs < 1) return fail(h, PRONY_EINVAL, w + ": strides must be >= 1");
    if ((N - 1) * u_rs + (m - 1) * u_cs >= (int64_t(1) << 40) || (N - 1) * v_rs + (m - 1) * v_cs >= (int64_t(1) << 40))
        return fail(h, PRONY_EINVAL, w + ": strides out of range");
    if (prec != PRONY_FP64 && prec != PRONY_FP32 && prec != PRONY_BF16X3)
        return fail(h, PRONY_EINVAL, w + ": bad precision");
    if (flags & ~PRONY_WITH_S0) return fail(h, PRONY_EINVAL, w + ": unknown flag");
    if (h->device < 0 && !plan_only) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    const bool s0 = (flags & PRONY_WITH_S0) != 0;
    const size_t ts = prec == PRONY_FP64 ? sizeof(double) : sizeof(float);
    return make_plan(h, d, n, m, s0, ts, P, tuned_target(h, d, n, m, prec, 0), tuned_fragments(h, d, n, m, prec, 0),
                     0, prec == PRONY_BF16X3, true);
}

prony_status_t run_build_S(prony_handle_t h, const PencilPlan& P, unsigned char* ws, prony_prec_t prec,
                           const double* f, const double* U, int64_t u_rs, int64_t u_cs, const double* sigma,
                           const double* V, int64_t v_rs, int64_t v_cs, double* S) {
    if (prec == PRONY_FP64) return launch_pencil<double>(h, P, ws, f, U, u_rs, u_cs, sigma, V, v_rs, v_cs, S);
    return launch_pencil<float>(h, P, ws, f, U, u_rs, u_cs, sigma, V, v_rs, v_cs, S);
}

}  // namespace
}  // namespace prony

using namespace prony;

extern "C" prony_status_t prony_build_S(prony_handle_t h, int d, int n, int m, const double* f, const double* U,
                                        int64_t u_rs, int64_t u_cs, const double* sigma, const double* V,
                                        int64_t v_rs, int64_t v_cs, prony_prec_t prec, unsigned flags, double* S) {
    if (!h) return PRONY_EINVAL;
    PencilPlan P;
    prony_status_t st =
        plan_build_S(h, "prony_build_S", d, n, m, f, U, u_rs, u_cs, sigma, V, v_rs, v_cs, prec, flags, S, P);
    if (st != PRONY_OK) return st;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    if ((st = ensure_workspace(h, P.ws_bytes)) != PRONY_OK) return st;
    return run_build_S(h, P, static_cast<unsigned char*>(h->ws), prec, f, U, u_rs, u_cs, sigma, V, v_rs, v_cs, S);
}

extern "C" prony_status_t prony_build_S_plan(prony_handle_t h, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                             int* fragments, int* workgroups, int* chunk, size_t* workspace_bytes) {
    if (!h) return PRONY_EINVAL;
    // the plan does not read the arrays: stand-in pointers pass the null checks
    static const double dummy[2] = {0.0, 0.0};
    PencilPlan P;
    const prony_status_t st = plan_build_S(h, "prony_build_S_plan", d, n, m, dummy, dummy, 1, 1, dummy, dummy, 1, 1,
                                           prec, flags, const_cast<double*>(dummy), P, true);
    if (st != PRONY_OK) return st;
    if (fragments) *fragments = P.rf;
    if (workgroups) *workgroups = P.nwg;
    if (chunk) *chunk = P.kc;
    if (workspace_bytes) *workspace_bytes = P.ws_bytes;
    return PRONY_OK;
}

extern "C" prony_status_t prony_build_S_noalloc(prony_handle_t h, int d, int n, int m, const double* f,
                                                const double* U, int64_t u_rs, int64_t u_cs, const double* sigma,
                                                const double* V, int64_t v_rs, int64_t v_cs, prony_prec_t prec,
                                                unsigned flags, double* S) {
    if (!h) return PRONY_EINVAL;
    PencilPlan P;
    prony_status_t st = plan_build_S(h, "prony_build_S_noalloc", d, n, m, f, U, u_rs, u_cs, sigma, V, v_rs, v_cs,
                                     prec, flags, S, P);
    if (st != PRONY_OK) return st;
    if (P.ws_bytes > kScratchBytes)
        return fail(h, PRONY_ENOTSUP,
                    "prony_build_S_noalloc: the call needs " + std::to_string(P.ws_bytes) +
                        " bytes of scratch, more than the fixed " + std::to_string(kScratchBytes) +
                        " bytes per device; use prony_build_S");
    if (!h->scratch) return fail(h, PRONY_EHIP, "prony_build_S_noalloc: no scratch address for this device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    return run_build_S(h, P, static_cast<unsigned char*>(h->scratch), prec, f, U, u_rs, u_cs, sigma, V, v_rs,
                       v_cs, S);
}

// Prepared factors: the packed operands of one (U, sigma, V) under the plan that
// was current at creation, for repeated S-builds with other sample grids.
struct prony_factors_s {
    int device = -1;
    prony_prec_t prec = PRONY_FP64;
    PencilPlan P{};
    unsigned char* mem = nullptr;   // packed V | packed U | G table | sigma
    size_t off_sigma = 0;
};

extern "C" prony_status_t prony_factors_create(prony_handle_t h, int d, int n, int m, const double* U, int64_t u_rs,
                                               int64_t u_cs, const double* sigma, const double* V, int64_t v_rs,
                                               int64_t v_cs, prony_prec_t prec, unsigned flags,
                                               prony_factors_t* factors) {
    if (!h) return PRONY_EINVAL;
    if (!factors) return fail(h, PRONY_EINVAL, "prony_factors_create: null output pointer");
    *factors = nullptr;
    // the plan does not read the grid or the output: stand-ins pass the null checks
    static const double dummy[2] = {0.0, 0.0};
    PencilPlan P;
    prony_status_t st = plan_build_S(h, "prony_factors_create", d, n, m, dummy, U, u_rs, u_cs, sigma, V, v_rs, v_cs,
                                     prec, flags, const_cast<double*>(dummy), P);
    if (st != PRONY_OK) return st;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(h->stream, &cs);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(h, PRONY_ECAPTURE, "prony_factors_create allocates device memory; create factors before capture");
    prony_factors_s* F = new (std::nothrow) prony_factors_s;
    if (!F) return fail(h, PRONY_ENOMEM, "prony_factors_create: out of host memory");
    F->device = h->device;
    F->prec = prec;
    F->P = P;
    F->off_sigma = P.off_p;   // the packed sections end where the partial rows would start
    e = hipMalloc(reinterpret_cast<void**>(&F->mem), F->off_sigma + align_up(sizeof(double) * (size_t)m, 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete F;
        return fail(h, PRONY_ENOMEM, std::string("prony_factors_create: hipMalloc failed: ") + hipGetErrorString(e));
    }
    st = prec == PRONY_FP64 ? pack_operands<double>(h, P, F->mem, U, u_rs, u_cs, V, v_rs, v_cs)
                            : pack_operands<float>(h, P, F->mem, U, u_rs, u_cs, V, v_rs, v_cs);
    if (st == PRONY_OK) {
        e = hipMemcpyAsync(F->mem + F->off_sigma, sigma, sizeof(double) * (size_t)m, hipMemcpyDeviceToDevice,
                           h->stream);
        if (e != hipSuccess) st = hip_fail(h, e, "hipMemcpyAsync(sigma)");
    }
    if (st != PRONY_OK) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(F->mem);
        delete F;
        return st;
    }
    *factors = F;
    return PRONY_OK;
}

extern "C" prony_status_t prony_build_S_factors(prony_handle_t h, prony_factors_t F, const double* f, double* S) {
    if (!h) return PRONY_EINVAL;
    if (!F || !f || !S) return fail(h, PRONY_EINVAL, "prony_build_S_factors: null pointer");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    if (F->device != h->device)
        return fail(h, PRONY_EINVAL, "prony_build_S_factors: the factors belong to another device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    const PencilPlan& P = F->P;
    prony_status_t st = ensure_workspace(h, P.ws_bytes - P.off_p);
    if (st != PRONY_OK) return st;
    const double* sigma = reinterpret_cast<const double*>(F->mem + F->off_sigma);
    unsigned char* part = static_cast<unsigned char*>(h->ws);
    if (F->prec == PRONY_FP64) return launch_tiles_finish<double>(h, P, F->mem, part, f, sigma, S);
    return launch_tiles_finish<float>(h, P, F->mem, part, f, sigma, S);
}

extern "C" prony_status_t prony_factors_info(prony_factors_t F, int* d, int* n, int* m, prony_prec_t* prec,
                                             unsigned* flags) {
    if (!F) return PRONY_EINVAL;
    if (d) *d = F->P.d;
    if (n) *n = F->P.n;
    if (m) *m = F->P.m;
    if (prec) *prec = F->prec;
    if (flags) *flags = F->P.first_ell == 0 ? PRONY_WITH_S0 : 0u;
    return PRONY_OK;
}

extern "C" prony_status_t prony_factors_destroy(prony_factors_t F) {
    if (!F) return PRONY_EINVAL;
    prony_status_t st = PRONY_OK;
    {
        DeviceGuard g(F->device);
        if (!g.ok || hipFree(F->mem) != hipSuccess) {
            (void)hipGetLastError();
            st = PRONY_EHIP;
        }
    }
    delete F;
    return st;
}

extern "C" prony_status_t prony_reserve(prony_handle_t h, int d_max, int n_max, int m_max) {
    if (!h) return PRONY_EINVAL;
    prony_status_t st = check_dn(h, d_max, n_max);
    if (st != PRONY_OK) return st;
    if (m_max < 1 || m_max > 64) return fail(h, PRONY_EINVAL, "prony_reserve: m_max must be in 1..64");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    // The plans are sized at the largest m; over n, the largest plans come from the
    // top of the range (the operands grow with n, the partial sums with the target),
    // so the last 16 values of n are planned.
    size_t need = 0;
    for (int d = 1; d <= d_max; ++d)
        for (int n = std::max(1, n_max - 15); n <= n_max; ++n) {
            const int m = (int)std::min<int64_t>(m_max, ipow(n + 1, d));
            if (m <= 32) {
                need = std::max(need, pencil_workspace_bytes(h, d, n, m));
                need = std::max(need, adjoint_workspace_bytes(h, d, n, m));
            }
            need = std::max(need, coeffs_workspace_bytes(d, n, m));
        }
    return ensure_workspace(h, need);
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

namespace prony {
namespace {

template <typename T>
prony_status_t batch_build(prony_handle_t h, int count, const prony_instance_t* inst, prony_batch_s* B) {
    using T2 = pair_t<T>;
    std::vector<PencilPlan> plans(count);
    for (int i = 0; i < count; ++i) {
        const prony_instance_t& x = inst[i];
        const std::string who = "instance " + std::to_string(i) + ": ";
        if (x.d < 1 || x.d > 3 || x.n < 1) return fail(h, PRONY_EINVAL, who + "bad d or n");
        if (ipow(2 * (int64_t)x.n + 2, x.d) > (int64_t(1) << 30))
            return fail(h, PRONY_ENOTSUP, who + "sample grid larger than 2^30 points");
        const int64_t N = ipow(x.n + 1, x.d);
        if (x.m < 1 || x.m > N) return fail(h, PRONY_EINVAL, who + "m must be in 1..N");
        if (x.m > 32) return fail(h, PRONY_ENOTSUP, who + "m > 32 is not supported");
        if (!x.f || !x.U || !x.sigma || !x.V || !x.S) return fail(h, PRONY_EINVAL, who + "null pointer");
        // batch members: split into the tuned number of chunks (default 1)
        const TuneEntry te = tuned(h, x.d, x.n, x.m, sizeof(T) == 4 ? PRONY_FP32 : PRONY_FP64, true);
        // fragments: the tuned 1 or 2 where supported, else the default (never 4:
        // the queue kernel instantiates 1 and 2); a first plan gives the row tiles
        // that the chunk count multiplies
        const int rf_req = te.fragments == 1 || te.fragments == 2 ? te.fragments : 0;
        PencilPlan probe;
        prony_status_t st = make_plan(h, x.d, x.n, x.m, false, sizeof(T), probe, 1, rf_req, 0, false, true);
        if (st == PRONY_OK)
            st = make_plan(h, x.d, x.n, x.m, false, sizeof(T), plans[i], std::max(1, te.target) * probe.rt, probe.rf,
                           0, false, true);
        if (st != PRONY_OK) return fail(h, st, who + h->err);
    }
    // classes by (product form, column-block count, row fragments); inside a class,
    // longest tiles first
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (plans[a].ng != plans[b].ng) return plans[a].ng < plans[b].ng;
        if (plans[a].nb != plans[b].nb) return plans[a].nb < plans[b].nb;
        if (plans[a].rf != plans[b].rf) return plans[a].rf < plans[b].rf;
        return (int64_t)plans[a].kc * plans[a].rf > (int64_t)plans[b].kc * plans[b].rf;
    });
    // work items of the queue schedule (FP32): every tile of every instance,
    // longest first; tiles of one instance stay in L order
    size_t nitems = 0;
    for (int i = 0; i < count; ++i) nitems += (size_t)plans[i].nwg;
    if (nitems > (size_t)INT32_MAX) return fail(h, PRONY_ENOTSUP, "prony_batch_create: too many tiles");
    // workspace layout: entries, queue counter, work items, then per instance vp | up | gt | part
    const size_t off_counter = align_up(sizeof(BatchEntry<T>) * (size_t)count, 256);
    const size_t off_items = off_counter + 256;
    size_t off = align_up(off_items + sizeof(WorkItem) * nitems, 256);
    std::vector<BatchEntry<T>> host(count);
    std::vector<size_t> base(count);
    for (int pos = 0; pos < count; ++pos) {
        base[pos] = off;
        off += plans[order[pos]].ws_bytes;
    }
    void* ws = nullptr;
    hipError_t e = hipMalloc(&ws, off);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, PRONY_ENOMEM, std::string("batch workspace allocation failed: ") + hipGetErrorString(e));
    }
    B->ws = ws;
    B->ws_bytes = off;
    unsigned char* w = static_cast<unsigned char*>(ws);
    int first = 0;
    int largest = 1;
    for (int pos = 0; pos < count; ++pos) {
        const int i = order[pos];
        const PencilPlan& P = plans[i];
        const prony_instance_t& x = inst[i];
        unsigned char* o = w + base[pos];
        BatchEntry<T>& E = host[pos];
        E.P = P;
        E.ptr.grid = reinterpret_cast<const double2*>(x.f);
        E.ptr.vp = reinterpret_cast<const T2*>(o + P.off_v);
        E.ptr.up = reinterpret_cast<const T2*>(o + P.off_u);
        E.ptr.gtab = reinterpret_cast<const int*>(o + P.off_g);
        E.ptr.part = reinterpret_cast<T2*>(o + P.off_p);
        E.ptr.sigma = x.sigma;
        E.ptr.S = reinterpret_cast<double2*>(x.S);
        E.U = reinterpret_cast<const double2*>(x.U);
        E.V = reinterpret_cast<const double2*>(x.V);
        const PencilPlan* prev = pos == 0 ? nullptr : &plans[order[pos - 1]];
        const bool new_class = !prev || prev->ng != P.ng || prev->nb != P.nb || prev->rf != P.rf;
        if (new_class) {
            B->launches.push_back({P.nb, P.rf, P.ng, pos, 0, 0, 0, 0.0});
            first = 0;
        }
        auto& cl = B->launches.back();
        E.tile_begin = first;
        first += P.nwg;
        cl.count += 1;
        cl.tiles = first;
        cl.lds = std::max(cl.lds, P.lds_bytes);
        cl.work += (double)P.nwg * P.kc * P.rf * (2 * P.nb + P.ng);   // MFMAs per K step and fragment
        const int64_t big = std::max<int64_t>(((int64_t)P.sk * P.kc + kPrefetchRows) * P.nrp,
                                              ((int64_t)P.ug + (int64_t)P.rt * P.rows) * P.mbi * 16);
        largest = (int)std::max<int64_t>(largest, (big + 255) / 256);
    }
    B->pack_x = std::min(largest, 64);
    for (int i = 0; i < count; ++i)
        B->finish_x = std::max(B->finish_x, (plans[i].m * plans[i].C + kFinishOuts - 1) / kFinishOuts);
    B->entries = ws;
    std::vector<WorkItem> items;
    items.reserve(nitems);
    std::vector<int> by_cost(count);
    for (int pos = 0; pos < count; ++pos) by_cost[pos] = pos;
    auto cost = [&](int pos) {
        return (int64_t)host[pos].P.kc * host[pos].P.rf * (2 * host[pos].P.nb + host[pos].P.ng);
    };
    std::stable_sort(by_cost.begin(), by_cost.end(), [&](int a, int b) { return cost(a) > cost(b); });
    for (int pos : by_cost)
        for (int L = 0; L < host[pos].P.nwg; ++L) items.push_back({pos, L});
    B->queue_counter = w + off_counter;
    B->queue_items = w + off_items;
    B->queue_n = (int)nitems;
    B->queue_lds = 0;
    for (int pos = 0; pos < count; ++pos) B->queue_lds = std::max(B->queue_lds, host[pos].P.lds_bytes);
    // resident workgroups per CU: LDS (dynamic + the kernel's 16 static bytes), and
    // at most 2 (the kernel is bounded to 256 registers, 2 waves per SIMD)
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(2, h->lds_per_block / (B->queue_lds + 16)));
    B->queue_grid = (int)std::min<size_t>(nitems, (size_t)per_cu * h->num_cus);
    // class launches by default: each class's own kernel keeps as many workgroups
    // resident as its registers and LDS allow, and the lanes overlap the classes'
    // tails (measured faster than the merged queue kernel on the 512-instance mix);
    // the queue stays selectable for FP32 batches
    B->schedule = PRONY_SCHEDULE_CLASSES;
    e = hipMemcpyAsync(ws, host.data(), sizeof(BatchEntry<T>) * (size_t)count, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w + off_items, items.data(), sizeof(WorkItem) * nitems, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "batch work table upload");
    return PRONY_OK;
}

template <typename T>
prony_status_t batch_launch(prony_handle_t h, prony_batch_s* B) {
    const BatchEntry<T>* entries = static_cast<const BatchEntry<T>*>(B->entries);
    const bool queue = B->schedule == PRONY_SCHEDULE_QUEUE;
    int* counter = queue ? static_cast<int*>(B->queue_counter) : nullptr;
    {
        ProfileScope prof(h, "pencil_pack");
        pencil_pack_batched<T><<<dim3(B->pack_x, 3, B->count), 256, 0, h->stream>>>(entries, counter);
    }
    prony_status_t st = check_launch(h, "pencil_pack_batched");
    if (st != PRONY_OK) return st;
    if (queue) {
        if constexpr (sizeof(T) == 4) {
            if (B->queue_lds > 65536) {
                hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pencil_tiles_queue<T>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)B->queue_lds);
                if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
            }
            {
                ProfileScope prof(h, "pencil_tiles_batched");
                pencil_tiles_queue<T><<<B->queue_grid, kThreads, B->queue_lds, h->stream>>>(
                    entries, static_cast<const WorkItem*>(B->queue_items), B->queue_n, counter);
            }
            if ((st = check_launch(h, "pencil_tiles_queue")) != PRONY_OK) return st;
            ProfileScope prof(h, "pencil_finish");
            pencil_finish_batched<T><<<dim3(B->finish_x, B->count), kFinishThreads, 0, h->stream>>>(entries);
            return check_launch(h, "pencil_finish_batched");
        } else {
            return fail(h, PRONY_ENOTSUP, "prony_build_S_batched: the queue schedule is FP32 only");
        }
    }
    // The class launches are independent: they run on the handle's stream and up
    // to kAux auxiliary streams (forked after the packing launch, joined before
    // the finishing launch), each class on the lane with the least work so far
    // (largest classes first), so that the tails of the classes overlap.
    const int nl = h->aux_ready ? std::min<int>(1 + prony_handle_s::kAux, (int)B->launches.size()) : 1;
    hipError_t e = hipSuccess;
    if (nl > 1) {
        e = hipEventRecord(h->fork, h->stream);
        for (int a = 0; a + 1 < nl && e == hipSuccess; ++a) e = hipStreamWaitEvent(h->aux[a], h->fork, 0);
        if (e != hipSuccess) return hip_fail(h, e, "batch fork");
    }
    std::vector<int> by_work(B->launches.size());
    for (size_t c = 0; c < by_work.size(); ++c) by_work[c] = (int)c;
    std::stable_sort(by_work.begin(), by_work.end(),
                     [&](int a, int b) { return B->launches[a].work > B->launches[b].work; });
    double load[1 + prony_handle_s::kAux] = {};
    for (int c : by_work) {
        const auto& cl = B->launches[c];
        int lane = 0;
        for (int l = 1; l < nl; ++l)
            if (load[l] < load[lane]) lane = l;
        load[lane] += cl.work;
        hipStream_t s = lane == 0 ? h->stream : h->aux[lane - 1];
        st = dispatch_batched<T>(h, cl.nb, cl.rf, cl.ng, entries + cl.first, cl.count, cl.tiles, cl.lds, s);
        if (st != PRONY_OK) return st;
        if ((st = check_launch(h, "pencil_tiles_batched")) != PRONY_OK) return st;
    }
    if (nl > 1) {
        for (int a = 0; a + 1 < nl && e == hipSuccess; ++a) {
            e = hipEventRecord(h->join[a], h->aux[a]);
            if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->join[a], 0);
        }
        if (e != hipSuccess) return hip_fail(h, e, "batch join");
    }
    {
        ProfileScope prof(h, "pencil_finish");
        pencil_finish_batched<T><<<dim3(B->finish_x, B->count), kFinishThreads, 0, h->stream>>>(entries);
    }
    return check_launch(h, "pencil_finish_batched");
}

}  // namespace
}  // namespace prony

extern "C" prony_status_t prony_batch_create(prony_handle_t h, int count, const prony_instance_t* instances,
                                             prony_prec_t prec, prony_batch_t* batch) {
    if (!h || !batch) return PRONY_EINVAL;
    *batch = nullptr;
    if (count < 1 || count > 65535 || !instances)
        return fail(h, PRONY_EINVAL, "prony_batch_create: count must be in 1..65535");
    if (prec != PRONY_FP64 && prec != PRONY_FP32) return fail(h, PRONY_EINVAL, "prony_batch_create: bad precision");
    if (h->device < 0) {
        // validate only
        for (int i = 0; i < count; ++i) {
            const prony_instance_t& x = instances[i];
            const std::string who = "instance " + std::to_string(i) + ": ";
            if (x.d < 1 || x.d > 3 || x.n < 1) return fail(h, PRONY_EINVAL, who + "bad d or n");
            const int64_t N = ipow(x.n + 1, x.d);
            if (x.m < 1 || x.m > N) return fail(h, PRONY_EINVAL, who + "m must be in 1..N");
            if (x.m > 32) return fail(h, PRONY_ENOTSUP, who + "m > 32 is not supported");
            if (!x.f || !x.U || !x.sigma || !x.V || !x.S) return fail(h, PRONY_EINVAL, who + "null pointer");
        }
        return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    }
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    prony_status_t ast = ensure_aux(h);
    if (ast != PRONY_OK) return ast;
    prony_batch_s* B = new (std::nothrow) prony_batch_s();
    if (!B) return fail(h, PRONY_ENOMEM, "prony_batch_create: out of host memory");
    B->owner = h;
    B->count = count;
    B->prec = prec;
    B->inst.assign(instances, instances + count);
    const prony_status_t st = prec == PRONY_FP32 ? batch_build<float>(h, count, instances, B)
                                                 : batch_build<double>(h, count, instances, B);
    if (st != PRONY_OK) {
        if (B->ws) (void)hipFree(B->ws);
        delete B;
        return st;
    }
    *batch = B;
    return PRONY_OK;
}

extern "C" prony_status_t prony_batch_destroy(prony_batch_t B) {
    if (!B) return PRONY_EINVAL;
    prony_status_t st = PRONY_OK;
    if (B->ws || B->adj) {
        DeviceGuard g(B->owner->device);
        if (hipStreamSynchronize(B->owner->stream) != hipSuccess) st = PRONY_EHIP;
        if (B->ws && hipFree(B->ws) != hipSuccess) st = PRONY_EHIP;
        if (B->adj && adj_batch_free(B->adj) != PRONY_OK) st = PRONY_EHIP;
    }
    delete B;
    return st;
}

extern "C" prony_status_t prony_batch_set_schedule(prony_batch_t B, int schedule) {
    if (!B) return PRONY_EINVAL;
    prony_handle_t h = B->owner;
    if (schedule != PRONY_SCHEDULE_QUEUE && schedule != PRONY_SCHEDULE_CLASSES)
        return fail(h, PRONY_EINVAL, "prony_batch_set_schedule: unknown schedule");
    if (schedule == PRONY_SCHEDULE_QUEUE && B->prec != PRONY_FP32)
        return fail(h, PRONY_ENOTSUP, "prony_batch_set_schedule: the queue schedule is FP32 only");
    B->schedule = schedule;
    return PRONY_OK;
}

extern "C" prony_status_t prony_build_S_batched(prony_handle_t h, prony_batch_t B) {
    if (!h || !B) return PRONY_EINVAL;
    if (B->owner != h) return fail(h, PRONY_EINVAL, "prony_build_S_batched: batch belongs to another handle");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    return B->prec == PRONY_FP32 ? batch_launch<float>(h, B) : batch_launch<double>(h, B);
}

extern "C" prony_status_t prony_graph_capture(prony_handle_t h, prony_batch_t B, void** graph_exec) {
    if (!h || !B || !graph_exec) return PRONY_EINVAL;
    *graph_exec = nullptr;
    if (B->owner != h) return fail(h, PRONY_EINVAL, "prony_graph_capture: batch belongs to another handle");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamCreateWithFlags");
    // the captured stream must first see everything already queued on the handle's stream
    hipStream_t user = h->stream;
    e = hipStreamSynchronize(user);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(h, e, "hipStreamSynchronize");
    }
    const std::string saved_prof = h->prof_kernel;
    h->prof_kernel.clear();     // no event records inside the graph
    h->stream = cap;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    prony_status_t st = PRONY_OK;
    if (e != hipSuccess) {
        st = hip_fail(h, e, "hipStreamBeginCapture");
    } else {
        st = prony_build_S_batched(h, B);
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (st == PRONY_OK && e2 != hipSuccess) st = hip_fail(h, e2, "hipStreamEndCapture");
    }
    h->stream = user;
    h->prof_kernel = saved_prof;
    (void)hipStreamDestroy(cap);
    if (st != PRONY_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
    *graph_exec = exec;
    return PRONY_OK;
}

extern "C" prony_status_t prony_graph_launch(prony_handle_t h, void* graph_exec) {
    if (!h || !graph_exec) return PRONY_EINVAL;
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    hipError_t e = hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
    return PRONY_OK;
}

extern "C" prony_status_t prony_graph_destroy(void* graph_exec) {
    if (!graph_exec) return PRONY_EINVAL;
    return hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec)) == hipSuccess ? PRONY_OK : PRONY_EHIP;
}

namespace prony {

TuneKey tune_key(int d, int n, int m, int prec, bool batched, bool bucket) {
    if (!bucket) return std::make_tuple(0, d, n, m, prec, batched ? 1 : 0);
    const int64_t N = ipow(n + 1, d);
    int lg = 0;
    while ((int64_t(2) << lg) <= N) ++lg;   // floor(log2 N)
    return std::make_tuple(1, d, lg, (m + 7) / 8, prec, batched ? 1 : 0);
}

TuneEntry tuned(prony_handle_t h, int d, int n, int m, int prec, bool batched) {
    TuneEntry e;
    const auto it = h->tune.find(tune_key(d, n, m, prec, batched, false));
    if (it != h->tune.end()) e = it->second;
    if (e.target == 0 || e.fragments == 0) {
        const auto jt = h->tune.find(tune_key(d, n, m, prec, batched, true));
        if (jt != h->tune.end()) {
            if (e.target == 0) e.target = jt->second.target;
            if (e.fragments == 0) e.fragments = jt->second.fragments;
        }
    }
    return e;
}

}  // namespace prony

extern "C" prony_status_t prony_tune_set_tile(prony_handle_t h, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                              int fragments, int target_wgs) {
    if (!h) return PRONY_EINVAL;
    if (d < 1 || d > 3 || n < 1 || m < 1 || m > 32) return fail(h, PRONY_EINVAL, "prony_tune_set: bad shape");
    if (ipow(2 * (int64_t)n + 2, d) > (int64_t(1) << 30)) return fail(h, PRONY_EINVAL, "prony_tune_set: bad shape");
    if (flags & ~(PRONY_TUNE_BATCHED | PRONY_TUNE_BUCKET)) return fail(h, PRONY_EINVAL, "prony_tune_set: unknown flag");
    const bool batched = (flags & PRONY_TUNE_BATCHED) != 0;
    if (prec != PRONY_FP64 && prec != PRONY_FP32 && !(prec == PRONY_BF16X3 && !batched))
        return fail(h, PRONY_EINVAL, "prony_tune_set: bad precision");
    if (target_wgs < 0 || target_wgs > (1 << 20)) return fail(h, PRONY_EINVAL, "prony_tune_set: bad target");
    if (!(fragments == 0 || fragments == 1 || fragments == 2 || (fragments == 4 && !batched)))
        return fail(h, PRONY_EINVAL, "prony_tune_set_tile: fragments must be 0, 1, 2 or 4 (batch members: 0, 1, 2)");
    const TuneKey key = tune_key(d, n, m, (int)prec, batched, (flags & PRONY_TUNE_BUCKET) != 0);
    if (target_wgs == 0 && fragments == 0)
        h->tune.erase(key);
    else
        h->tune[key] = TuneEntry{target_wgs, fragments};
    return PRONY_OK;
}

extern "C" prony_status_t prony_tune_set(prony_handle_t h, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                         int target_wgs) {
    if (!h) return PRONY_EINVAL;
    int fragments = 0;
    if (d >= 1 && d <= 3 && n >= 1 && m >= 1 && ipow(2 * (int64_t)n + 2, d) <= (int64_t(1) << 30)) {
        const auto it = h->tune.find(tune_key(d, n, m, (int)prec, (flags & PRONY_TUNE_BATCHED) != 0,
                                              (flags & PRONY_TUNE_BUCKET) != 0));
        if (it != h->tune.end()) fragments = it->second.fragments;   // keep the entry's tile shape
    }
    return prony_tune_set_tile(h, d, n, m, prec, flags, fragments, target_wgs);
}

extern "C" prony_status_t prony_toeplitz_mm(prony_handle_t h, int d, int n, int adjoint, const double* f, int r,
                                            const double* X, int64_t ldx, prony_prec_t prec, double* Y,
                                            int64_t ldy) {
    if (!h) return PRONY_EINVAL;
    prony_status_t st = check_dn(h, d, n);
    if (st != PRONY_OK) return st;
    if (adjoint != 0 && adjoint != 1) return fail(h, PRONY_EINVAL, "prony_toeplitz_mm: adjoint must be 0 or 1");
    if (r < 1 || r > 64) return fail(h, PRONY_EINVAL, "prony_toeplitz_mm: r must be in 1..64");
    if (ldx < r || ldy < r) return fail(h, PRONY_EINVAL, "prony_toeplitz_mm: leading dimensions must be >= r");
    if (!f || !X || !Y) return fail(h, PRONY_EINVAL, "prony_toeplitz_mm: null pointer");
    if (prec != PRONY_FP64 && prec != PRONY_FP32) return fail(h, PRONY_EINVAL, "prony_toeplitz_mm: bad precision");
    const int64_t N = ipow(n + 1, d);
    if ((N - 1) * ldx + r >= (int64_t(1) << 40) || (N - 1) * ldy + r >= (int64_t(1) << 40))
        return fail(h, PRONY_EINVAL, "prony_toeplitz_mm: leading dimensions out of range");
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    PencilPlan P;
    const size_t ts = prec == PRONY_FP32 ? sizeof(float) : sizeof(double);
    // one column (toeplitz_mv): eight workgroups per CU, whose smaller windows let more
    // of them share a CU (d = 3, n = 20: 75 -> 57 us per product against four), and
    // chunks of whole planes of I_n (d >= 3) or whole lines (d = 2)
    const int target = r == 1 ? 8 * h->num_cus : 0;
    const int kal = r == 1 && d >= 2 ? (int)ipow(n + 1, d >= 3 ? d - 1 : 1) : 0;
    st = make_plan(h, d, n, r, false, ts, P, target, 0, 1, false, true, kal);
    if (kal > 0 && (st != PRONY_OK || !mv_fits(h, P, ts)))   // chunks of multiples of 16 instead
        st = make_plan(h, d, n, r, false, ts, P, target, 0, 1, false, true);
    if (st != PRONY_OK) return st;
    P.conj_grid = adjoint;
    return prec == PRONY_FP32 ? launch_toeplitz_mm<float>(h, P, f, X, ldx, Y, ldy)
                              : launch_toeplitz_mm<double>(h, P, f, X, ldx, Y, ldy);
}
