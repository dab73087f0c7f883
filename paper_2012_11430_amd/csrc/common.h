// Internal declarations shared by the translation units of libprony.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "prony.h"

namespace prony {
// A tuning entry: split target (single instances: workgroups to aim at; batch
// members: chunks of the h range) and 16-row fragments per wave; 0 = default.
struct TuneEntry {
    int target = 0;
    int fragments = 0;
};
// (bucket, d, n or floor(log2 N), m or ceil(m/8), prec, batched)
using TuneKey = std::tuple<int, int, int, int, int, int>;
}  // namespace prony

struct prony_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    void* ws = nullptr;          // device workspace owned by the handle
    size_t ws_bytes = 0;
    int num_cus = 256;           // MI355X figures for validation-only handles;
    size_t lds_per_block = 163840;   // device handles read their device's
    std::string err;
    // tuning entries of exact shapes and of shape buckets (see prony_tune_set)
    std::map<prony::TuneKey, prony::TuneEntry> tune;
    // profiling: events around launches of one named kernel
    std::string prof_kernel;
    std::vector<hipEvent_t> prof_events;   // pool, pairs (start, stop)
    size_t prof_used = 0;                  // events in use (2 per launch)
    // auxiliary streams (default priority) and fork/join events for launches
    // that are independent of each other (the class launches of a batch)
    static constexpr int kAux = 3;
    hipStream_t aux[kAux] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kAux] = {};
    bool aux_ready = false;
    // orders the previous stream's work before the next stream's on a stream change
    hipEvent_t order = nullptr;
    // device address of the fixed scratch array of prony_build_S_noalloc on this
    // handle's device (looked up once per device when the handle is created)
    void* scratch = nullptr;
};

namespace prony {

prony_status_t fail(prony_handle_t h, prony_status_t st, const std::string& msg);
prony_status_t hip_fail(prony_handle_t h, hipError_t e, const char* what);

// Make the handle's device current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Grow the workspace to at least `bytes`. Returns PRONY_ECAPTURE when growth is
// needed while the handle's stream is being captured.
prony_status_t ensure_workspace(prony_handle_t h, size_t bytes);

// Brackets one kernel launch with profiling events when the handle profiles `name`.
class ProfileScope {
  public:
    ProfileScope(prony_handle_t h, const char* name, hipStream_t stream = nullptr);
    ~ProfileScope();
  private:
    prony_handle_t h_;
    hipStream_t stream_ = nullptr;
    hipEvent_t stop_ = nullptr;
};

// Look up (once per device, with the handle's device current) the device address
// of the fixed scratch array used by prony_build_S_noalloc and keep it in the handle.
prony_status_t scratch_attach(prony_handle_t h);

// Create the auxiliary streams and events (outside stream capture).
prony_status_t ensure_aux(prony_handle_t h);

// Launch-error check after a kernel launch.
prony_status_t check_launch(prony_handle_t h, const char* what);

inline int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace bytes of one prony_build_S / prony_coeffs call (largest precision/flag).
size_t pencil_workspace_bytes(prony_handle_t h, int d, int n, int m);
size_t coeffs_workspace_bytes(int d, int n, int m);
size_t adjoint_workspace_bytes(prony_handle_t h, int d, int n, int m);

// Adjoint state of a batch (planned on the first batched adjoint call; adjoint.hip).
struct AdjBatch;
prony_status_t adj_batch_free(AdjBatch* a);

// Key of a tuning entry: the exact shape, or its bucket (same d, floor(log2 N) and
// column-block count ceil(m/8)).
TuneKey tune_key(int d, int n, int m, int prec, bool batched, bool bucket);
// The entry that applies to a shape: each field from the exact entry, else from
// the bucket entry (0 when neither has it).
TuneEntry tuned(prony_handle_t h, int d, int n, int m, int prec, bool batched);

// Common argument validation for (d, n): 1 <= d <= 3, n >= 1, sizes within int32.
prony_status_t check_dn(prony_handle_t h, int d, int n);

// ---- index maps (Sec. 1: I_n = {0..n}^d row-major; grid {-n..n+1}^d row-major) ----

// Flat grid offset G(k) = sum_l k_l (2n+2)^(d-l) of the point k in I_n with
// row-major index idx (base n+1).
__host__ __device__ inline int grid_offset_of_index(int idx, int d, int n) {
    const int P = n + 1, Q = 2 * n + 2;
    int g = 0, scale = 1;
    for (int l = d - 1; l >= 0; --l) {
        const int q = idx / P;
        g += (idx - q * P) * scale;
        idx = q;
        scale *= Q;
    }
    return g;
}

// Grid offset of the origin shift: c0 = G((n,..,n)), so that f(k-h+e) sits at
// G(k) - G(h) + c0 + G(e).
__host__ __device__ inline int grid_center(int d, int n) {
    const int Q = 2 * n + 2;
    int g = 0;
    for (int l = 0; l < d; ++l) g = g * Q + n;
    return g;
}

// Grid stride s_l = (2n+2)^(d-l) of unit vector e_l, l = 1..d (0 for l = 0).
__host__ __device__ inline int grid_shift(int d, int n, int ell) {
    if (ell <= 0) return 0;
    const int Q = 2 * n + 2;
    int s = 1;
    for (int l = ell; l < d; ++l) s *= Q;
    return s;
}

}  // namespace prony

// A planned batch of S-builds (pencil.hip) and, once used, its adjoint state.
struct prony_batch_s {
    prony_handle_t owner = nullptr;
    int count = 0;
    prony_prec_t prec = PRONY_FP64;
    std::vector<prony_instance_t> inst;   // descriptors in the caller's order
    void* ws = nullptr;           // entries + per-instance operands and scratch
    size_t ws_bytes = 0;
    void* entries = nullptr;      // device BatchEntry<T>[count], grouped by class
    int pack_x = 1;               // pack blocks per (instance, section)
    int finish_x = 1;             // finishing workgroups per instance (largest instance)
    struct ClassLaunch {
        int nb, rf, ng, first, count, tiles;
        size_t lds;
        double work;   // sum of nwg * kc over the class (MFMA work, up to a factor)
    };
    std::vector<ClassLaunch> launches;
    // queue schedule (FP32): one persistent launch over all tiles, longest first
    int schedule = PRONY_SCHEDULE_CLASSES;
    void* queue_counter = nullptr;   // device int, reset by the packing launch
    void* queue_items = nullptr;     // device WorkItem[queue_n]
    int queue_n = 0;
    int queue_grid = 0;
    size_t queue_lds = 0;
    prony::AdjBatch* adj = nullptr;
};
