// Handle, stream, workspace and error reporting of libprony.
#include <cstdio>
#include <new>

#include "common.h"

namespace prony {

prony_status_t fail(prony_handle_t h, prony_status_t st, const std::string& msg) {
    if (h) h->err = msg;
    return st;
}

prony_status_t hip_fail(prony_handle_t h, hipError_t e, const char* what) {
    return fail(h, PRONY_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

prony_status_t check_launch(prony_handle_t h, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, what);
    return PRONY_OK;
}

prony_status_t check_dn(prony_handle_t h, int d, int n) {
    if (d < 1 || d > 3) return fail(h, PRONY_EINVAL, "d must be 1, 2 or 3");
    if (n < 1) return fail(h, PRONY_EINVAL, "n must be >= 1");
    // keep (2n+2)^d and N^2 index arithmetic inside the 32/64-bit ranges used
    if (ipow(2 * (int64_t)n + 2, d) > (int64_t(1) << 30))
        return fail(h, PRONY_ENOTSUP, "sample grid larger than 2^30 points");
    return PRONY_OK;
}

prony_status_t ensure_workspace(prony_handle_t h, size_t bytes) {
    if (bytes <= h->ws_bytes) return PRONY_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(h->stream, &cs);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(h, PRONY_ECAPTURE, "workspace must grow during stream capture; call prony_reserve first");
    if (h->ws) {
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
        e = hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
        if (e != hipSuccess) return hip_fail(h, e, "hipFree");
    }
    const size_t grow = align_up(bytes + bytes / 4, size_t(1) << 20);
    e = hipMalloc(&h->ws, grow);
    if (e != hipSuccess) {
        h->ws = nullptr;
        (void)hipGetLastError();
        return fail(h, PRONY_ENOMEM, std::string("hipMalloc of workspace failed: ") + hipGetErrorString(e));
    }
    h->ws_bytes = grow;
    return PRONY_OK;
}

static hipEvent_t next_event(prony_handle_t h) {
    if (h->prof_used == h->prof_events.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->prof_events.push_back(e);
    }
    return h->prof_events[h->prof_used++];
}

ProfileScope::ProfileScope(prony_handle_t h, const char* name, hipStream_t stream)
    : h_(h), stream_(stream ? stream : h->stream) {
    if (h->prof_kernel.empty() || h->prof_kernel != name) return;
    hipEvent_t start = next_event(h);
    hipEvent_t stop = next_event(h);
    if (!start || !stop) return;
    if (hipEventRecord(start, stream_) != hipSuccess) return;
    stop_ = stop;
}

ProfileScope::~ProfileScope() {
    if (stop_) (void)hipEventRecord(stop_, stream_);
}

prony_status_t ensure_aux(prony_handle_t h) {
    if (h->aux_ready) return PRONY_OK;
    hipError_t e = hipEventCreateWithFlags(&h->fork, hipEventDisableTiming);
    for (int a = 0; a < prony_handle_s::kAux && e == hipSuccess; ++a) {
        e = hipStreamCreateWithFlags(&h->aux[a], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join[a], hipEventDisableTiming);
    }
    if (e != hipSuccess) return hip_fail(h, e, "auxiliary stream setup");
    h->aux_ready = true;
    return PRONY_OK;
}

}  // namespace prony

using namespace prony;

extern "C" prony_status_t prony_profile_enable(prony_handle_t h, const char* kernel) {
    if (!h) return PRONY_EINVAL;
    h->prof_kernel = kernel ? kernel : "";
    h->prof_used = 0;
    return PRONY_OK;
}

extern "C" prony_status_t prony_profile_read(prony_handle_t h, int* launches, double* total_ms) {
    if (!h || !launches || !total_ms) return PRONY_EINVAL;
    *launches = 0;
    *total_ms = 0.0;
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    for (size_t i = 0; i + 1 < h->prof_used; i += 2) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, h->prof_events[i], h->prof_events[i + 1]);
        if (e != hipSuccess) return hip_fail(h, e, "hipEventElapsedTime");
        *total_ms += ms;
        *launches += 1;
    }
    return PRONY_OK;
}

extern "C" prony_status_t prony_create(prony_handle_t* handle, int device) {
    if (!handle) return PRONY_EINVAL;
    *handle = nullptr;
    if (device == -1) {
        prony_handle_s* h = new (std::nothrow) prony_handle_s();
        if (!h) return PRONY_ENOMEM;
        h->device = -1;
        *handle = h;
        return PRONY_OK;
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return PRONY_EHIP;
    if (device < 0 || device >= count) return PRONY_EINVAL;
    prony_handle_s* h = new (std::nothrow) prony_handle_s();
    if (!h) return PRONY_ENOMEM;
    h->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        h->num_cus = prop.multiProcessorCount;
        h->lds_per_block = prop.sharedMemPerBlock;
    }
    prony_status_t st = PRONY_OK;
    {
        DeviceGuard g(device);
        if (!g.ok) {
            st = PRONY_EHIP;
        } else if (hipEventCreateWithFlags(&h->order, hipEventDisableTiming) != hipSuccess) {
            h->order = nullptr;
            st = PRONY_EHIP;
        } else {
            st = scratch_attach(h);
        }
    }
    if (st != PRONY_OK) {
        if (h->order) (void)hipEventDestroy(h->order);
        delete h;
        return st;
    }
    *handle = h;
    return PRONY_OK;
}

extern "C" prony_status_t prony_destroy(prony_handle_t h) {
    if (!h) return PRONY_EINVAL;
    if (h->device < 0) {
        delete h;
        return PRONY_OK;
    }
    DeviceGuard g(h->device);
    prony_status_t st = PRONY_OK;
    if (h->ws) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) st = PRONY_EHIP;
        if (hipFree(h->ws) != hipSuccess) st = PRONY_EHIP;
    }
    for (hipEvent_t e : h->prof_events) (void)hipEventDestroy(e);
    for (int a = 0; a < prony_handle_s::kAux; ++a) {
        if (h->aux[a]) {
            if (hipStreamSynchronize(h->aux[a]) != hipSuccess) st = PRONY_EHIP;
            (void)hipStreamDestroy(h->aux[a]);
        }
        if (h->join[a]) (void)hipEventDestroy(h->join[a]);
    }
    if (h->fork) (void)hipEventDestroy(h->fork);
    if (h->order) (void)hipEventDestroy(h->order);
    delete h;
    return st;
}

// Every call through a handle shares its workspace. On a change of stream the new
// stream waits (on the device, through an event) for the work already queued on the
// previous one, so a call on the new stream cannot overwrite operands or partial
// sums that a kernel still running on the old stream reads. Under stream capture
// (of either stream) no ordering is recorded: set the stream before capturing.
extern "C" prony_status_t prony_set_stream(prony_handle_t h, void* stream) {
    if (!h) return PRONY_EINVAL;
    hipStream_t next = reinterpret_cast<hipStream_t>(stream);
    if (next == h->stream || h->device < 0 || !h->order) {
        h->stream = next;
        return PRONY_OK;
    }
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PRONY_EHIP, "hipSetDevice failed");
    hipStreamCaptureStatus a = hipStreamCaptureStatusNone, b = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(h->stream, &a);
    if (e == hipSuccess) e = hipStreamIsCapturing(next, &b);
    if (e != hipSuccess) {
        // a query refused because some capture is in progress: treat as capturing
        (void)hipGetLastError();
        a = hipStreamCaptureStatusActive;
    }
    if (a == hipStreamCaptureStatusNone && b == hipStreamCaptureStatusNone) {
        e = hipEventRecord(h->order, h->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(next, h->order, 0);
        if (e != hipSuccess) return hip_fail(h, e, "stream ordering");
    }
    h->stream = next;
    return PRONY_OK;
}

extern "C" prony_status_t prony_synchronize(prony_handle_t h) {
    if (!h) return PRONY_EINVAL;
    if (h->device < 0) return fail(h, PRONY_ENODEV, "validation-only handle has no device");
    DeviceGuard g(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    return PRONY_OK;
}

extern "C" const char* prony_last_error(prony_handle_t h) {
    if (!h) return "invalid handle";
    return h->err.c_str();
}
