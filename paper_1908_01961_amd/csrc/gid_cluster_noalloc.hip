// gid_cluster_frame_noalloc: the chromaticity clustering of gid_cluster_frame
// with its device scratch in a fixed device array instead of a per-call
// allocation, for callers that cannot allocate (graph capture, serving loops,
// harnesses that forbid hipMalloc).  The kernels and the host-side clustering
// are gid_cluster_frame's own (gid_cluster.hip); only the scratch differs.
//
// The array lives for the whole process on every device the library runs on.
// Its address on a device is taken once, with that device current, by
// hipGetSymbolAddress; host code uses only that address (the array's name on
// the host is a stand-in, not a device pointer).  Calls on one device share the
// array: every value a call reads it has written first in the same call, so
// nothing is cleared, and calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gid.h"

namespace gidc {
gid_status run(const float* frame, int W, int H, int k_max, double merge_dist, hipStream_t s, uint8_t* ids,
               double* colors, double* centres_out, int32_t* k_out, char* scratch);
gid_status check_args(const float* frame, int W, int H, int k_max, double merge_dist, const uint8_t* ids,
                      const double* colors, const int32_t* k_out);
}  // namespace gidc

namespace {

__device__ __align__(256) char scratch[GID_CLUSTER_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
char* g_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up once per device,
// with the device current); nullptr if the lookup fails.
char* scratch_on(int dev) {
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_ptr[dev] = static_cast<char*>(p);
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" gid_status gid_cluster_frame_noalloc(const float* frame_dev, int32_t width, int32_t height, int32_t k_max,
                                                double merge_dist, void* hip_stream, uint8_t* ids_dev,
                                                double* colors_host, double* centres_host, int32_t* k_out) {
    gid_status st = gidc::check_args(frame_dev, width, height, k_max, merge_dist, ids_dev, colors_host, k_out);
    if (st != GID_OK) return st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GID_ERR_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return GID_ERR_UNSUPPORTED;
    char* ptr = scratch_on(dev);
    if (!ptr) return GID_ERR_HIP;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    st = gidc::run(frame_dev, width, height, k_max, merge_dist, s, ids_dev, colors_host, centres_host, k_out, ptr);
    (void)hipStreamSynchronize(s);
    return st;
}
