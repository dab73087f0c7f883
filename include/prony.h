/*
 * prony.h -- C ABI of the MI355X (gfx950) hot path of the multivariate
 * matrix-pencil Prony method (N. Bosner, "Parallel Prony's method with
 * multivariate matrix pencil approach and its numerical aspect",
 * arXiv 2012.11430).
 *
 * The library computes, on one GPU, the data-parallel steps of Algorithm 1:
 * the samples f(k) of the exponential sum (Sec. 1, eq. exp_sum), the
 * multilevel Toeplitz matrices T = [f(k-h)] and T_l = [f(k-h+e_l)]
 * (Sec. 1), the pencil matrices S_l = U^* T_l V Sigma^{-1}
 * (Sec. 1, eq. generateSl) and the Vandermonde products of the coefficient
 * least-squares problem A^T c = f (Sec. 1, eq. ls_probl). The SVD of T, the
 * eigendecomposition of C_mu and the small least-squares solve stay on the
 * host, as the paper assigns them (Sec. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array pointers are DEVICE pointers unless stated otherwise; the
 *    caller allocates and owns them. The library owns only its workspace.
 *  - Complex numbers are interleaved {re, im} doubles (complex128).
 *  - d in {1,2,3}, n >= 1, N = (n+1)^d. The index set I_n = {0..n}^d is
 *    ordered row-major (last coordinate fastest): idx(k) = sum_l k_l (n+1)^(d-l).
 *  - The sample grid holds f(p) for p in {-n..n+1}^d, row-major, flat:
 *    g(p) = sum_l (p_l + n) (2n+2)^(d-l); it has (2n+2)^d entries and covers
 *    every argument k-h and k-h+e_l.
 *  - Calls enqueue work on the handle's stream and return without waiting.
 *    Arguments are validated on the host before anything is launched; a bad
 *    argument returns PRONY_EINVAL (or PRONY_ENOTSUP for a valid request the
 *    kernels do not cover) and launches nothing. A failing HIP call returns
 *    PRONY_EHIP; faults inside kernels surface at the next synchronising call.
 *    prony_last_error() returns a text for the last failure on the handle.
 *  - Documented preconditions that are not checked on the device: sigma_j > 0
 *    and finite inputs. NaN inputs propagate to the outputs.
 *  - A handle may be used by one host thread at a time. Its single-instance
 *    calls share one workspace; prony_set_stream orders a new stream after the
 *    work already queued on the previous one, so calls through one handle on
 *    several streams do not overwrite each other's operands (see there).
 */
#ifndef PRONY_H
#define PRONY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct prony_handle_s* prony_handle_t;

typedef enum {
    PRONY_OK = 0,
    PRONY_EINVAL = 1,    /* invalid argument (nothing launched)             */
    PRONY_ENOTSUP = 2,   /* valid but unsupported request (nothing launched) */
    PRONY_EHIP = 3,      /* a HIP runtime call failed                        */
    PRONY_ENOMEM = 4,    /* workspace allocation failed                      */
    PRONY_ECAPTURE = 5,  /* workspace growth needed while the stream is being captured */
    PRONY_ENODEV = 6     /* the handle has no device (validation-only handle) */
} prony_status_t;

typedef enum {
    PRONY_FP64 = 0,      /* complex128 operands, FP64 MFMA, FP64 accumulation            */
    PRONY_FP32 = 1,      /* complex64 operands, FP32 MFMA with FP32 accumulation per tile,
                            FP64 reduction of the tile partials and FP64 Sigma^{-1}       */
    PRONY_BF16X3 = 2,    /* prony_build_S only: both operands split into three bfloat16
                            terms (x = h + m + l, 24 significant bits), the six products
                            above 2^-24 on the bf16 MFMA with FP32 accumulation; then as
                            PRONY_FP32. Same error scale as PRONY_FP32.                   */
    PRONY_PREC_MAX_ENUM = 0x7FFFFFFF  /* not a precision: makes every value 0..2^31-1 a
                            valid object of this type, so that calls can reject unknown
                            values with PRONY_EINVAL (negative values are not allowed) */
} prony_prec_t;

/* Flag of prony_build_S: also form S_0 = U^* T V Sigma^{-1} (equal to I for an
   exact SVD of T) and store it in front of S_1..S_d. */
#define PRONY_WITH_S0 1u

/* ---- handle ---------------------------------------------------------------- */

/* Create a handle bound to HIP device `device` (the device is made current for
   every call on the handle). The stream is the null stream until set.
   device = -1 creates a validation-only handle that touches no GPU: every call
   validates its arguments as usual and then returns PRONY_ENODEV instead of
   launching (for testing argument checks on machines without a GPU). */
prony_status_t prony_create(prony_handle_t* handle, int device);

/* Free the workspace and the handle. Waits for the handle's stream first. */
prony_status_t prony_destroy(prony_handle_t handle);

/* Enqueue all later work on `stream` (a hipStream_t owned by the caller).
   When `stream` differs from the current one, the new stream first waits, on the
   device, for the work already queued on the previous stream (an event recorded
   there), because every call through the handle shares the handle's workspace.
   While either stream is being captured no such ordering is recorded: set the
   stream before beginning a capture. */
prony_status_t prony_set_stream(prony_handle_t handle, void* stream);

/* Wait for the handle's stream; reports asynchronous kernel faults as PRONY_EHIP. */
prony_status_t prony_synchronize(prony_handle_t handle);

/* Text describing the last failure on the handle (never NULL). */
const char* prony_last_error(prony_handle_t handle);

/* Pre-size the workspace for problems up to (d_max, n_max, m_max) so that later
   single-instance calls (samples, build_T, build_S, build_S_adjoint, coeffs)
   allocate nothing (needed before capturing such calls into a HIP graph). The
   S-build is planned for every precision (PRONY_BF16X3 included), with and
   without S_0, at the default split target, at every target the autotuner
   chooses from and at the target registered for the shape, for m = m_max (or
   N when smaller) and the 16 largest n up to n_max. Register tuning entries
   before reserving. */
prony_status_t prony_reserve(prony_handle_t handle, int d_max, int n_max, int m_max);

/* Profiling aid. With a non-NULL `kernel` name, every later launch of that kernel
   by the handle is bracketed by a pair of HIP events recorded on the handle's
   stream; NULL stops recording. Each call discards earlier records.
   Kernel names: "samples", "toeplitz", "pencil_pack", "pencil_tiles",
   "pencil_tiles_batched", "pencil_finish", "coeffs_tiles", "coeffs_finish",
   "adjoint_pack", "adjoint_tiles". */
prony_status_t prony_profile_enable(prony_handle_t handle, const char* kernel);

/* Synchronise the stream and report the recorded launches of the profiled kernel:
   their count and the sum of their event-to-event times in milliseconds. */
prony_status_t prony_profile_read(prony_handle_t handle, int* launches, double* total_ms);

/* Tile selection (filled by the autotuner). prony_build_S splits the index range
   I_n of one instance into chunks so that about `target_wgs` workgroups run
   (default 4 per compute unit). With flag PRONY_TUNE_BATCHED the entry applies to
   instances of that shape inside batches and gives the number of chunks per
   instance (default 1: split only as far as the LDS window requires). With flag
   PRONY_TUNE_BUCKET the entry applies to every shape of the bucket of (d, n, m):
   the same d, the same floor(log2 N) and the same column-block count ceil(m/8);
   an entry of the exact shape takes precedence, field by field. target_wgs = 0
   removes the target. PRONY_BF16X3 entries exist for single instances only
   (batches run PRONY_FP32 or PRONY_FP64). Entries live in the handle. */
#define PRONY_TUNE_BATCHED 1u
#define PRONY_TUNE_BUCKET 2u
prony_status_t prony_tune_set(prony_handle_t handle, int d, int n, int m, prony_prec_t prec, unsigned flags,
                              int target_wgs);

/* The registered target of a shape's entry (or of its bucket's with
   PRONY_TUNE_BUCKET; 0 when none). */
prony_status_t prony_tune_get(prony_handle_t handle, int d, int n, int m, prony_prec_t prec, unsigned flags,
                              int* target_wgs);

/* Tile shape and split target in one entry (flags as for prony_tune_set):
   `fragments` is the number of 16-row fragments per wave (64 * fragments rows of
   the product per workgroup): 1, 2 or 4 for single instances, 1 or 2 for batch
   members (the persistent queue kernel instantiates those), used where the kernel
   instantiation supports it for the shape's column count (else the default: 2
   where supported); 0 keeps the default. fragments = target_wgs = 0 removes the
   entry. Applies to prony_build_S, prony_build_S_noalloc and batches. */
prony_status_t prony_tune_set_tile(prony_handle_t handle, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                   int fragments, int target_wgs);

/* The registered tile shape and target of an entry (zeros when none). */
prony_status_t prony_tune_get_tile(prony_handle_t handle, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                   int* fragments, int* target_wgs);

/* Register the autotuner's cached entries for this handle's device. The cache is
   the JSON file the Python autotuner writes (paper_2012_11430_amd/autotune.py):
   {"version": 2, "devices": {"<arch name>:<compute units>": {"<key>": <value>}}}
   with <key> "d,n,m,prec,mode" or "bucket:d,n,m,prec,mode" (prec fp64 / fp32 /
   bf16x3, mode single / batch) and <value> the target as an integer or
   {"target": T, "fragments": F}; version 1 caches (integers) are read too.
   Entries are registered through prony_tune_set_tile (same validation); a device
   without entries registers nothing. EINVAL for a missing path, an unreadable
   file, malformed JSON or a malformed entry (entries before it stay registered);
   ENODEV on a validation-only handle. */
prony_status_t prony_autotune(prony_handle_t handle, const char* cache_json_path);

/* The same for the entries stored under an explicit device key (any handle,
   validation-only handles included). */
prony_status_t prony_autotune_device(prony_handle_t handle, const char* cache_json_path, const char* device_key);

/* ---- Algorithm 1, GPU steps -------------------------------------------------- */

/* Samples of the exponential sum (Sec. 1, eq. exp_sum), with the additive noise
   model of Sec. 4:
     f(p) = sum_{j<m} c_j exp(-2 pi i <t_j, p>) + noise(p),  p in {-n..n+1}^d.
   The phase <t_j,p> is reduced by its nearest integer before the exponential.
   t:     m x d doubles, row-major (t_j(l) at t[j*d + l]), nodes in [0,1)^d.
   c:     m complex128.
   noise: (2n+2)^d complex128 added to the samples, or NULL for none.
   f:     (2n+2)^d complex128 output (the sample grid).
   Requires 1 <= m <= 4096. */
prony_status_t prony_samples(prony_handle_t handle, int d, int n, int m,
                             const double* t, const double* c, const double* noise,
                             double* f);

/* Multilevel Toeplitz matrix (Sec. 1): which = 0 gives T[k,h] = f(k-h), which = l
   in 1..d gives T_l[k,h] = f(k-h+e_l), for k, h in I_n.
   f:   the sample grid ((2n+2)^d complex128).
   out: N x N complex128, row k at out + 2*k*ld; ld >= N (elements). `out` may be
        device memory or pinned host memory mapped for the device.
   The write is N*N*16 bytes; it exists to feed the host SVD of T and to test the
   index map. Requires N*ld < 2^62. */
prony_status_t prony_build_T(prony_handle_t handle, int d, int n, int which,
                             const double* f, double* out, int64_t ld);

/* Pencil matrices (Sec. 1, eq. generateSl):
     S_l = U^* T_l V Sigma^{-1},  l = 1..d,
   with T_l generated on the fly from the sample grid (never stored).
   f:      sample grid ((2n+2)^d complex128).
   U, V:   N x m complex128; entry (k, j) at U + 2*(k*u_rs + j*u_cs) (strides in
           complex elements, both >= 1). V is the right factor itself, not V^*.
   sigma:  m doubles > 0 (device memory).
   prec:   PRONY_FP64, PRONY_FP32 or PRONY_BF16X3 (see prony_prec_t).
   flags:  0 or PRONY_WITH_S0.
   S:      output, (d or d+1) x m x m complex128, row-major per matrix: S_l(i,j)
           at S + 2*((l*m + i)*m + j), l counted from the first stored matrix.
   Requires 1 <= m <= min(N, 32). */
prony_status_t prony_build_S(prony_handle_t handle, int d, int n, int m, const double* f,
                             const double* U, int64_t u_rs, int64_t u_cs,
                             const double* sigma,
                             const double* V, int64_t v_rs, int64_t v_cs,
                             prony_prec_t prec, unsigned flags, double* S);

/* The launch plan prony_build_S would use for this call shape under the handle's
   tuning entries, without launching or allocating anything: 16-row fragments per
   wave, workgroups of the tile launch, indices h per chunk and the workspace
   bytes the call needs. Validates like prony_build_S (pointers aside). Works on
   validation-only handles, which plan for 256 compute units and 160 KiB of LDS
   per workgroup (the MI355X figures). Any output pointer may be NULL. */
prony_status_t prony_build_S_plan(prony_handle_t handle, int d, int n, int m, prony_prec_t prec, unsigned flags,
                                  int* fragments, int* workgroups, int* chunk, size_t* workspace_bytes);

/* prony_build_S for callers that cannot allocate device memory (code under HIP
   graph capture, serving loops, harnesses that forbid hipMalloc): the same
   validation, plan, kernels and result as prony_build_S, with the packed operands
   and partial sums in a fixed scratch array of 64 MiB that the library holds on
   every device it runs on until the process ends (looked up once per device by
   prony_create). Calls no hipMalloc or hipFree. A call whose plan needs more than
   64 MiB of scratch returns PRONY_ENOTSUP with the size in prony_last_error (c1,
   d=2, n=63, m=20, needs about 10 MB in FP32; call prony_build_S for larger
   plans). Every call on one device shares that device's array, across handles
   and streams: calls that overlap on one GPU race, so keep them in one stream
   order. The array keeps the last call's contents; the kernels overwrite every
   byte they read, so nothing has to start at zero. */
prony_status_t prony_build_S_noalloc(prony_handle_t handle, int d, int n, int m, const double* f,
                                     const double* U, int64_t u_rs, int64_t u_cs,
                                     const double* sigma,
                                     const double* V, int64_t v_rs, int64_t v_cs,
                                     prony_prec_t prec, unsigned flags, double* S);

/* Prepared factors: the packed operands of one (U, sigma, V) for S-builds with
   many sample grids (Sec. 1, eq. generateSl with the factors held fixed, as in
   the differentiation and noise-sensitivity workloads). prony_build_S packs U
   and V on every call; prony_factors_create packs them once, on the handle's
   stream, into a device allocation owned by the factors object, under the plan
   that is current for (d, n, m, prec, flags) at creation (later tuning entries
   do not change it). U, sigma and V may be released once the creation's work on
   the handle's stream has run. Arguments and requirements as for prony_build_S.
   Allocates device memory: PRONY_ECAPTURE under stream capture, ENODEV on a
   validation-only handle. */
typedef struct prony_factors_s* prony_factors_t;
prony_status_t prony_factors_create(prony_handle_t handle, int d, int n, int m,
                                    const double* U, int64_t u_rs, int64_t u_cs,
                                    const double* sigma,
                                    const double* V, int64_t v_rs, int64_t v_cs,
                                    prony_prec_t prec, unsigned flags, prony_factors_t* factors);

/* S_l = U^* T_l V Sigma^{-1} for the sample grid f with prepared factors: the
   tile and finishing launches of prony_build_S only (same kernels, plan and
   fixed-order sums, so the result is bitwise equal to prony_build_S's under that
   plan). f and S as for prony_build_S. The partial rows live in the handle's
   workspace (grown as needed; PRONY_ECAPTURE if it must grow under capture, so
   call once or prony_reserve before capturing). The factors must belong to the
   handle's device; builds with one factors object on several streams may run
   concurrently (the object is only read), as long as each uses its own handle. */
prony_status_t prony_build_S_factors(prony_handle_t handle, prony_factors_t factors, const double* f, double* S);

/* Shape, precision and flags of prepared factors (any pointer may be NULL). */
prony_status_t prony_factors_info(prony_factors_t factors, int* d, int* n, int* m, prony_prec_t* prec,
                                  unsigned* flags);

/* Release prepared factors (hipFree waits for the device's work in flight). */
prony_status_t prony_factors_destroy(prony_factors_t factors);

/* Vandermonde products of the least-squares step argmin_c ||A^T c - f||_2
   (Sec. 1, eq. ls_probl; Algorithm 1, last line):
     A^T[k, j] = prod_l z_j(l)^{k_l}  (k in I_n),
     gram = (A^T)^* A^T  (m x m),  rhs = (A^T)^* f_I  (m),
   where f_I is the sample grid restricted to I_n. The host then solves
   gram c = rhs in FP64.
   z:      m x d complex128, row-major (z_j(l) at z + 2*(j*d + l)).
   f:      sample grid ((2n+2)^d complex128).
   gram:   m x m complex128 output, row-major.
   rhs:    m complex128 output.
   AT_out: N x m complex128 output (row-major) or NULL to skip writing A^T.
   Requires 1 <= m <= min(N, 64). */
prony_status_t prony_coeffs(prony_handle_t handle, int d, int n, int m,
                            const double* z, const double* f,
                            double* gram, double* rhs, double* AT_out);

/* Adjoint of the pencil map (system pattern: differentiation). With U, Sigma, V
   held fixed, f -> S_l = U^* T_l(f) V Sigma^{-1} (Sec. 1, eq. generateSl) is
   complex-linear, so for a real loss L with gS_l = dL/dS_l in PyTorch's
   convention (dL/dRe + i dL/dIm) the gradient on the sample grid is
     gf(p) = sum_l sum_{k - h + e_l = p} [U gS_l Sigma^{-1} V^*]_{k,h}.
   U, V, sigma, strides: as for prony_build_S. gS: d x m x m complex128 (gradient
   of S_1..S_d). gf: (2n+2)^d complex128, overwritten. prec selects the MFMA and
   tile-accumulation type (FP32 or FP64); the diagonal bins and the window sums
   added to gf are FP64. Summation order inside a bin is not fixed (LDS atomics),
   so repeated runs agree to rounding, not bitwise. Requires 1 <= m <= min(N, 32). */
prony_status_t prony_build_S_adjoint(prony_handle_t handle, int d, int n, int m,
                                     const double* U, int64_t u_rs, int64_t u_cs,
                                     const double* sigma,
                                     const double* V, int64_t v_rs, int64_t v_cs,
                                     const double* gS, prony_prec_t prec, double* gf);

/* Product of the multilevel Toeplitz matrix T = [f(k - h)]_{k,h in I_n} (Sec. 1), or of
   its conjugate transpose, with a block of r columns: the two products of every sweep
   of the block power method for the SVD of T (Sec. 2.2, Algorithm 3):
     Y = T X      (adjoint = 0),     Y = T^* X    (adjoint = 1),
   computed from the sample grid without forming T (T^* is the Toeplitz matrix of
   g(p) = conj(f(-p))).
   f:    sample grid ((2n+2)^d complex128; only {-n..n}^d is read).
   X:    N x r complex128, row-major with leading dimension ldx >= r (device).
   Y:    N x r complex128 output, row-major with leading dimension ldy >= r; must not
         overlap X.
   prec: arithmetic and tile-accumulation type (FP32 or FP64): MFMA tiles, or vector
         FMAs when r = 1 (one Lanczos step's product); the chunk partials are added
         in FP64 in a fixed order (bitwise reproducible). Requires 1 <= r <= 64.
   Uses the handle's workspace (grown as needed; PRONY_ECAPTURE if it must grow
   under stream capture). */
prony_status_t prony_toeplitz_mm(prony_handle_t handle, int d, int n, int adjoint, const double* f, int r,
                                 const double* X, int64_t ldx, prony_prec_t prec, double* Y, int64_t ldy);

/* ---- many instances: one planned launch sequence, graph capture ------------- */

/* The batched S-build and its graph capture take a plan object rather than the
   descriptor array on every call: prony_batch_create validates, plans and uploads
   the descriptors once and owns the batch's workspace, so that
   prony_build_S_batched and prony_graph_capture only enqueue launches — no
   allocation, host-to-device copy or memset per call, which graph capture and
   replay require. Descriptors therefore live on the host, and prony_reserve does
   not size batches (each batch brings its own workspace). */
typedef struct prony_batch_s* prony_batch_t;

/* One S-build of a batch (Sec. 1, eq. generateSl, per instance). Pointers are
   device pointers owned by the caller; they must stay valid, and keep their
   shapes, for every launch of the batch. */
typedef struct {
    int d, n, m;          /* 1 <= d <= 3, n >= 1, 1 <= m <= min(N, 32)        */
    const double* f;      /* sample grid, (2n+2)^d complex128                */
    const double* U;      /* N x m complex128, row-major, contiguous          */
    const double* sigma;  /* m doubles > 0                                    */
    const double* V;      /* N x m complex128, row-major, contiguous          */
    double* S;            /* output: d x m x m complex128 (S_1..S_d)          */
} prony_instance_t;

/* Plan the S-build of `count` (1..65535) instances (host array of descriptors, copied):
   validates every descriptor, chooses tiles per instance, groups the instances
   by tile class (three-product blocks, column blocks, row fragments), orders them
   by decreasing work, builds the queue of all
   tiles (longest first), allocates the batch's own device workspace and uploads
   its work tables (synchronously on the handle's stream). Errors name the
   offending instance. */
prony_status_t prony_batch_create(prony_handle_t handle, int count, const prony_instance_t* instances,
                                  prony_prec_t prec, prony_batch_t* batch);

/* Free a batch (waits for the stream of the handle that created it). */
prony_status_t prony_batch_destroy(prony_batch_t batch);

/* How prony_build_S_batched runs the tiles of a batch (a system pattern, not in
   the paper):
   PRONY_SCHEDULE_QUEUE   — one persistent launch (as many workgroups as fit the
                            device at once) that takes (instance, tile) work items,
                            longest first, from a counter the packing launch resets.
                            FP32 batches only.
   PRONY_SCHEDULE_CLASSES — one launch per class of instances with the same tile
                            instantiation (three-product blocks, column blocks,
                            row fragments), spread over the
                            handle's stream and three auxiliary streams (forked after
                            the packing launch, joined before the finishing launch).
                            The default: each class's kernel keeps as many workgroups
                            resident as its own registers and LDS allow (measured
                            faster than the merged queue kernel on a 512-instance mix
                            of d, n and m); the FP64 batches' only schedule.
   Both compute the same tiles and the same fixed-order sums: their results are
   bitwise equal. */
#define PRONY_SCHEDULE_QUEUE 0
#define PRONY_SCHEDULE_CLASSES 1
/* Select the schedule of a batch (EINVAL for an unknown value, ENOTSUP for the
   queue on an FP64 batch). Takes effect at the next prony_build_S_batched or
   prony_graph_capture; a graph captured before keeps the launches it recorded. */
prony_status_t prony_batch_set_schedule(prony_batch_t batch, int schedule);

/* Enqueue the S-build of every instance of the batch on the handle's stream:
   one packing launch for all instances, the tile launch(es) of the batch's
   schedule and one finishing launch (fixed-order sums, Sigma^{-1}) for all
   instances. Allocates nothing and records no memset, so it can be captured.
   The handle must be the one that created the batch. Launches of one batch
   share its workspace and work counter: they must not overlap (stream order,
   as on the handle's stream, keeps them apart). */
prony_status_t prony_build_S_batched(prony_handle_t handle, prony_batch_t batch);

/* Adjoint of prony_build_S_batched: prony_build_S_adjoint for every instance of
   the batch, with its U, sigma and V held fixed, in one packing launch and one
   launch per class of instances with the same d*m.
   gS: device buffer of the gradients dL/dS of all instances, concatenated in the
       order given to prony_batch_create; instance i contributes d_i x m_i x m_i
       complex128 values.
   gf: device output, the grid gradients of all instances concatenated in the
       same order; instance i contributes (2n_i+2)^{d_i} complex128 values, all
       overwritten.
   Computes in the batch's precision (window sums added in FP64; bin order not
   fixed, as for prony_build_S_adjoint). The first call on a batch plans it and
   allocates the batch's adjoint workspace (synchronously on the handle's stream;
   PRONY_ECAPTURE under stream capture); later calls allocate nothing. The handle
   must be the one that created the batch. */
prony_status_t prony_build_S_adjoint_batched(prony_handle_t handle, prony_batch_t batch,
                                             const double* gS, double* gf);

/* Capture prony_build_S_batched(handle, batch) into a HIP graph (on a private
   stream) and instantiate it; *graph_exec receives a hipGraphExec_t. */
prony_status_t prony_graph_capture(prony_handle_t handle, prony_batch_t batch, void** graph_exec);

/* Launch an instantiated graph on the handle's stream. */
prony_status_t prony_graph_launch(prony_handle_t handle, void* graph_exec);

/* Destroy an instantiated graph. */
prony_status_t prony_graph_destroy(void* graph_exec);

#ifdef __cplusplus
}
#endif

#endif /* PRONY_H */
