// Reflectance correction of a misclustered region by sparsity (Sec. 5.2.2):
// every base colour is tried as the region's reflectance, each candidate frame
// is decomposed in full, and the colour whose indirect layers are sparsest over
// the region (the illumination sparsity term of Sec. 6.2) is kept.
//
// The K candidate decompositions are one batch of K contexts advanced together
// through shared launches (gid_batch_*): the same frame, K id maps that differ
// only inside the region.  Two small kernels build the candidate id maps and
// sum sum_{k>=1} |T_k| over the region of each candidate's layers (FP64,
// per-workgroup partials summed in index order, so the result is reproducible).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gid.h"

namespace {

constexpr int CR_THREADS = 256;
constexpr int CR_MAXWG = 1024;

__global__ __launch_bounds__(CR_THREADS) void k_candidate_ids(const uint8_t* ids, const uint8_t* region,
                                                                long long npx, int j, uint8_t* out) {
    for (long long i = (long long)blockIdx.x * CR_THREADS + threadIdx.x; i < npx; i += (long long)gridDim.x * CR_THREADS)
        out[i] = region[i] ? (uint8_t)j : ids[i];
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Per-workgroup sum over the region of sum_{k=1..K} |T_k|; layers hold R_r,
// R_g, R_b, T_0 .. T_K.
__global__ __launch_bounds__(CR_THREADS) void k_region_sparsity(const float* layers, const uint8_t* region,
                                                                  long long npx, int K, double* part) {
    __shared__ double sh[CR_THREADS / 64];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * CR_THREADS + threadIdx.x; i < npx; i += (long long)gridDim.x * CR_THREADS) {
        if (!region[i]) continue;
        for (int k = 1; k <= K; ++k) acc += fabs((double)layers[(long long)(3 + k) * npx + i]);
    }
    const double w = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_sum_partials(const double* part, int n, double* out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int w = 0; w < n; ++w) s += part[w];
    *out = s;
}

struct Resources {
    std::vector<gid_ctx*> ctx;
    gid_batch* batch = nullptr;
    void* mem = nullptr;
    ~Resources() {
        if (batch) (void)gid_batch_destroy(batch);
        for (gid_ctx* c : ctx) (void)gid_destroy(c);
        if (mem) (void)hipFree(mem);
    }
};

}  // namespace

extern "C" gid_status gid_correct_region(const gid_params* params, int32_t width, int32_t height,
                                         const float* frame_dev, const uint8_t* ids_dev, const uint8_t* region_dev,
                                         const double* colors_host, void* hip_stream, uint8_t* ids_out_dev,
                                         double* sparsity_host, int32_t* best_out) {
    if (!params || !frame_dev || !ids_dev || !region_dev || !colors_host || !ids_out_dev || !sparsity_host || !best_out)
        return GID_ERR_INVALID_ARG;
    if (width < 2 || height < 2 || (long long)width * height > (1LL << 28)) return GID_ERR_INVALID_ARG;
    const int K = params->K;
    if (K < 1 || K > 16) return GID_ERR_INVALID_ARG;
    gid_params prm = *params;
    prm.record_energy = 0;      // a batch runs without per-half-step energies
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const long long npx = (long long)width * height;
    const int nwg = (int)std::min<long long>(CR_MAXWG, (npx + CR_THREADS - 1) / CR_THREADS);
    Resources r;
    // device memory: K candidate id maps, K layer sets, partials, K sums
    const size_t ids_bytes = (size_t)npx, lay_bytes = sizeof(float) * (size_t)(K + 4) * npx;
    const size_t o_ids = 0, o_lay = (o_ids + ids_bytes * K + 255) & ~(size_t)255;
    const size_t o_part = o_lay + lay_bytes * K, o_sum = o_part + sizeof(double) * CR_MAXWG;
    if (hipMalloc(&r.mem, o_sum + sizeof(double) * 16) != hipSuccess) return GID_ERR_OUT_OF_MEMORY;
    char* base = static_cast<char*>(r.mem);
    std::vector<const float*> frames(K, frame_dev);
    std::vector<const uint8_t*> cids(K);
    std::vector<float*> lays(K);
    for (int j = 0; j < K; ++j) {
        gid_ctx* c = nullptr;
        gid_status st = gid_create(&prm, width, height, hip_stream, &c);
        if (st != GID_OK) return st;
        r.ctx.push_back(c);
        if ((st = gid_set_base_colors(c, colors_host)) != GID_OK) return st;
        uint8_t* cid = reinterpret_cast<uint8_t*>(base + o_ids + ids_bytes * j);
        k_candidate_ids<<<nwg, CR_THREADS, 0, s>>>(ids_dev, region_dev, npx, j, cid);
        cids[j] = cid;
        lays[j] = reinterpret_cast<float*>(base + o_lay + lay_bytes * j);
    }
    if (hipGetLastError() != hipSuccess) return GID_ERR_HIP;
    gid_status st = gid_batch_create(r.ctx.data(), K, &r.batch);
    if (st != GID_OK) return st;
    if ((st = gid_batch_decompose(r.batch, frames.data(), cids.data(), lays.data())) != GID_OK) return st;
    if ((st = gid_batch_synchronize(r.batch, nullptr)) != GID_OK) return st;
    double* part = reinterpret_cast<double*>(base + o_part);
    double* sums = reinterpret_cast<double*>(base + o_sum);
    for (int j = 0; j < K; ++j) {
        k_region_sparsity<<<nwg, CR_THREADS, 0, s>>>(lays[j], region_dev, npx, K, part);
        k_sum_partials<<<1, 64, 0, s>>>(part, nwg, sums + j);
    }
    if (hipGetLastError() != hipSuccess) return GID_ERR_HIP;
    double h[16];
    if (hipMemcpyAsync(h, sums, sizeof(double) * K, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GID_ERR_HIP;
    int best = 0;
    for (int j = 0; j < K; ++j) {
        sparsity_host[j] = (double)prm.lambda.i_sparsity * h[j];
        if (sparsity_host[j] < sparsity_host[best]) best = j;
    }
    if (hipMemcpyAsync(ids_out_dev, cids[best], ids_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GID_ERR_HIP;
    *best_out = best;
    return GID_OK;
}
