// Base-colour initialisation by chromaticity clustering (Sec. 5.1): a histogram
// of the first frame's chromaticity with 10 partitions per axis (device), weighted
// k-means on the bin mid-points with merging of close centres (host: at most
// 1000 bins, independent of the frame size), then every pixel assigned to its
// nearest centre and the mean RGB of each cluster (device).
//
// Readings (the paper leaves them open): |I| is the channel mean, so each
// chromaticity component of a non-negative colour lies in [0, 3] and falls in
// partition floor(10 C / 3) (clamped to 0..9); pixels darker than 1e-6 are
// white.  k-means is seeded with the most populated bin and then the non-empty
// bin farthest from the seeds (ties: lowest bin), Lloyd iterations run until the
// assignment repeats (at most 100); merging joins the smaller of the closest
// pair below the threshold into the larger (ties: the higher index joins) and
// recomputes its centre from the joint bins; a cluster left without pixels is
// dropped and the pixels assigned again.  Every discrete decision is taken in
// FP64 with squared distances d0 d0 + d1 d1 + d2 d2 evaluated left to right
// without contraction, on the device and on the host alike.
//
// Scratch: per-workgroup partial histograms and colour sums, at most
// GID_CLUSTER_SCRATCH_BYTES.  gid_cluster_frame allocates it per call;
// gid_cluster_frame_noalloc uses a fixed device array instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "gid.h"

#pragma clang fp contract(off)

namespace gidc {

constexpr int BINS = 10;
constexpr int NBIN = BINS * BINS * BINS;
constexpr int NSLOT = NBIN + 1;          // the last slot counts non-finite pixels
constexpr int THREADS = 256;
constexpr int MAXWG = 512;               // workgroups of a clustering launch (grid-stride)
constexpr int CKMAX = 16;
constexpr int MAX_LLOYD = 100;
constexpr double C_MAX = 3.0;
constexpr double FLOOR = 1e-6;

// Scratch layout (bytes): partial histograms, then the reduced histogram, then
// per-workgroup colour sums, then the reduced colour sums.
constexpr size_t OFF_HPART = 0;
constexpr size_t OFF_HIST = OFF_HPART + sizeof(unsigned) * (size_t)MAXWG * NSLOT;
constexpr size_t OFF_CPART = (OFF_HIST + sizeof(unsigned long long) * NSLOT + 255) & ~(size_t)255;
constexpr size_t OFF_CSUM = OFF_CPART + sizeof(double) * (size_t)MAXWG * CKMAX * 4;
constexpr size_t SCRATCH_BYTES = OFF_CSUM + sizeof(double) * CKMAX * 4;
static_assert(SCRATCH_BYTES <= GID_CLUSTER_SCRATCH_BYTES, "the declared scratch bound covers the layout");

__device__ __forceinline__ void chroma(float f0, float f1, float f2, double* C) {
    const double v0 = f0, v1 = f1, v2 = f2;
    const double m = (v0 + v1 + v2) / 3.0;
    if (m >= FLOOR) {
        C[0] = v0 / m;
        C[1] = v1 / m;
        C[2] = v2 / m;
    } else {
        C[0] = C[1] = C[2] = 1.0;
    }
}

__device__ __forceinline__ int part_of(double c) {
    const double j = floor(c * (double)BINS / C_MAX);
    return j < 0.0 ? 0 : (j > (double)(BINS - 1) ? BINS - 1 : (int)j);
}

// Per-workgroup histogram in LDS (integer counts: the totals do not depend on
// the order of the atomic increments), written as one partial row per workgroup.
__global__ __launch_bounds__(THREADS) void k_hist(const float* I, long long npx, unsigned* part) {
    __shared__ unsigned h[NSLOT];
    for (int j = threadIdx.x; j < NSLOT; j += THREADS) h[j] = 0u;
    __syncthreads();
    for (long long i = (long long)blockIdx.x * THREADS + threadIdx.x; i < npx; i += (long long)gridDim.x * THREADS) {
        const float f0 = I[i], f1 = I[npx + i], f2 = I[2 * npx + i];
        int slot;
        if (!isfinite(f0) || !isfinite(f1) || !isfinite(f2)) {
            slot = NBIN;
        } else {
            double C[3];
            chroma(f0, f1, f2, C);
            slot = (part_of(C[0]) * BINS + part_of(C[1])) * BINS + part_of(C[2]);
        }
        atomicAdd(&h[slot], 1u);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < NSLOT; j += THREADS) part[(size_t)blockIdx.x * NSLOT + j] = h[j];
}

__global__ __launch_bounds__(THREADS) void k_hist_reduce(const unsigned* part, int nwg, unsigned long long* hist) {
    const int j = blockIdx.x * THREADS + threadIdx.x;
    if (j >= NSLOT) return;
    unsigned long long s = 0;
    for (int w = 0; w < nwg; ++w) s += part[(size_t)w * NSLOT + j];
    hist[j] = s;
}

struct Centres {
    double c[CKMAX][3];
    int k;
};

// Nearest centre of every pixel's chromaticity (ties: the lowest index).
__global__ __launch_bounds__(THREADS) void k_assign(const float* I, long long npx, Centres cs, uint8_t* ids) {
    for (long long i = (long long)blockIdx.x * THREADS + threadIdx.x; i < npx; i += (long long)gridDim.x * THREADS) {
        double C[3];
        chroma(I[i], I[npx + i], I[2 * npx + i], C);
        double best = INFINITY;
        int arg = 0;
        for (int j = 0; j < cs.k; ++j) {
            const double d0 = C[0] - cs.c[j][0], d1 = C[1] - cs.c[j][1], d2 = C[2] - cs.c[j][2];
            const double d = d0 * d0 + d1 * d1 + d2 * d2;
            if (d < best) {
                best = d;
                arg = j;
            }
        }
        ids[i] = (uint8_t)arg;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums of R, G, B and the pixel count of cluster blockIdx.y over this
// workgroup's pixels (wavefront butterfly, then the four wavefronts in order).
__global__ __launch_bounds__(THREADS) void k_colour_sums(const float* I, long long npx, const uint8_t* ids,
                                                          double* part) {
    __shared__ double sh[4][THREADS / 64];
    const int j = blockIdx.y;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * THREADS + threadIdx.x; i < npx; i += (long long)gridDim.x * THREADS) {
        if (ids[i] != j) continue;
        acc[0] += (double)I[i];
        acc[1] += (double)I[npx + i];
        acc[2] += (double)I[2 * npx + i];
        acc[3] += 1.0;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int v = 0; v < 4; ++v) {
        const double s = wave_sum(acc[v]);
        if (lane == 0) sh[v][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int v = threadIdx.x;
        part[((size_t)blockIdx.x * CKMAX + j) * 4 + v] = (sh[v][0] + sh[v][1]) + (sh[v][2] + sh[v][3]);
    }
}

__global__ void k_colour_reduce(const double* part, int nwg, int k, double* out) {
    const int t = threadIdx.x;
    if (t >= 4 * k) return;
    double s = 0.0;
    for (int w = 0; w < nwg; ++w) s += part[(size_t)w * CKMAX * 4 + t];
    out[t] = s;
}

// ------------------------------------------------------------------ host side

struct Vec3 {
    double v[3];
};

double d2(const Vec3& a, const Vec3& b) {
    const double d0 = a.v[0] - b.v[0], d1 = a.v[1] - b.v[1], d2_ = a.v[2] - b.v[2];
    return d0 * d0 + d1 * d1 + d2_ * d2_;
}

Vec3 midpoint(int b) {
    const int j[3] = {b / (BINS * BINS), (b / BINS) % BINS, b % BINS};
    Vec3 m;
    for (int c = 0; c < 3; ++c) m.v[c] = ((double)j[c] + 0.5) * C_MAX / (double)BINS;
    return m;
}

// Weighted mean of the mid-points of the bins with cl[b] == j (bin order).
bool weighted_mean(const unsigned long long* hist, const int* nz, int nnz, const int* cl, int j, Vec3* out) {
    double s[3] = {0.0, 0.0, 0.0};
    unsigned long long w = 0;
    for (int t = 0; t < nnz; ++t) {
        if (cl[t] != j) continue;
        const Vec3 m = midpoint(nz[t]);
        const double wf = (double)hist[nz[t]];
        for (int c = 0; c < 3; ++c) s[c] = s[c] + wf * m.v[c];
        w += hist[nz[t]];
    }
    if (w == 0) return false;
    for (int c = 0; c < 3; ++c) out->v[c] = s[c] / (double)w;
    return true;
}

// Seeds, Lloyd iterations and merging on the histogram; returns the number of
// centres (<= k_max) and fills cen.
int cluster_histogram(const unsigned long long* hist, int k_max, double merge_dist, Vec3* cen) {
    int nz[NBIN], cl[NBIN], prev[NBIN];
    int nnz = 0;
    for (int b = 0; b < NBIN; ++b)
        if (hist[b]) nz[nnz++] = b;
    if (nnz == 0) return 0;
    // farthest-point seeds
    int seeds[CKMAX];
    int ns = 0;
    {
        int first = nz[0];
        for (int t = 1; t < nnz; ++t)
            if (hist[nz[t]] > hist[first]) first = nz[t];
        seeds[ns++] = first;
        while (ns < k_max) {
            int best = -1;
            double best_d = 0.0;
            for (int t = 0; t < nnz; ++t) {
                const Vec3 m = midpoint(nz[t]);
                double d = INFINITY;
                for (int s = 0; s < ns; ++s) {
                    const double e = d2(m, midpoint(seeds[s]));
                    if (e < d) d = e;
                }
                if (d > best_d) {
                    best = nz[t];
                    best_d = d;
                }
            }
            if (best < 0) break;
            seeds[ns++] = best;
        }
    }
    int k = ns;
    for (int j = 0; j < k; ++j) cen[j] = midpoint(seeds[j]);
    // Lloyd iterations
    bool have_prev = false;
    for (int it = 0; it < MAX_LLOYD; ++it) {
        for (int t = 0; t < nnz; ++t) {
            const Vec3 m = midpoint(nz[t]);
            int arg = 0;
            double best = d2(m, cen[0]);
            for (int j = 1; j < k; ++j) {
                const double e = d2(m, cen[j]);
                if (e < best) {
                    best = e;
                    arg = j;
                }
            }
            cl[t] = arg;
        }
        if (have_prev && std::memcmp(cl, prev, sizeof(int) * nnz) == 0) break;
        std::memcpy(prev, cl, sizeof(int) * nnz);
        have_prev = true;
        for (int j = 0; j < k; ++j) {
            Vec3 m;
            if (weighted_mean(hist, nz, nnz, cl, j, &m)) cen[j] = m;
        }
    }
    // merging of close centres
    for (;;) {
        int pa = -1, pb = -1;
        double best = 0.0;
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b) {
                const double d = std::sqrt(d2(cen[a], cen[b]));
                if (d < merge_dist && (pa < 0 || d < best)) {
                    pa = a;
                    pb = b;
                    best = d;
                }
            }
        if (pa < 0) break;
        unsigned long long wa = 0, wb = 0;
        for (int t = 0; t < nnz; ++t) {
            if (cl[t] == pa) wa += hist[nz[t]];
            if (cl[t] == pb) wb += hist[nz[t]];
        }
        const int keep = wa >= wb ? pa : pb, drop = wa >= wb ? pb : pa;
        for (int t = 0; t < nnz; ++t)
            if (cl[t] == drop) cl[t] = keep;
        Vec3 m;
        if (weighted_mean(hist, nz, nnz, cl, keep, &m)) cen[keep] = m;
        for (int j = drop; j + 1 < k; ++j) cen[j] = cen[j + 1];
        for (int t = 0; t < nnz; ++t)
            if (cl[t] > drop) cl[t] -= 1;
        k -= 1;
    }
    return k;
}

gid_status run(const float* frame, int W, int H, int k_max, double merge_dist, hipStream_t s, uint8_t* ids,
               double* colors, double* centres_out, int32_t* k_out, char* scratch) {
    const long long npx = (long long)W * H;
    const int nwg = (int)std::min<long long>(MAXWG, (npx + THREADS - 1) / THREADS);
    unsigned* hpart = reinterpret_cast<unsigned*>(scratch + OFF_HPART);
    unsigned long long* dhist = reinterpret_cast<unsigned long long*>(scratch + OFF_HIST);
    double* cpart = reinterpret_cast<double*>(scratch + OFF_CPART);
    double* csum = reinterpret_cast<double*>(scratch + OFF_CSUM);
    k_hist<<<nwg, THREADS, 0, s>>>(frame, npx, hpart);
    k_hist_reduce<<<(NSLOT + THREADS - 1) / THREADS, THREADS, 0, s>>>(hpart, nwg, dhist);
    if (hipGetLastError() != hipSuccess) return GID_ERR_HIP;
    unsigned long long hist[NSLOT];
    if (hipMemcpyAsync(hist, dhist, sizeof(hist), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GID_ERR_HIP;
    if (hist[NBIN] != 0) return GID_ERR_NUMERIC;
    Vec3 cen[CKMAX];
    int k = cluster_histogram(hist, k_max, merge_dist, cen);
    double sums[CKMAX * 4];
    for (;;) {
        Centres cs;
        cs.k = k;
        for (int j = 0; j < k; ++j)
            for (int c = 0; c < 3; ++c) cs.c[j][c] = cen[j].v[c];
        k_assign<<<nwg, THREADS, 0, s>>>(frame, npx, cs, ids);
        k_colour_sums<<<dim3(nwg, k), THREADS, 0, s>>>(frame, npx, ids, cpart);
        k_colour_reduce<<<1, 64, 0, s>>>(cpart, nwg, k, csum);
        if (hipGetLastError() != hipSuccess) return GID_ERR_HIP;
        if (hipMemcpyAsync(sums, csum, sizeof(double) * 4 * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return GID_ERR_HIP;
        int kk = 0;
        for (int j = 0; j < k; ++j)
            if (sums[4 * j + 3] > 0.0) cen[kk++] = cen[j];
        if (kk == k) break;
        k = kk;      // a centre without pixels is dropped; assign again
    }
    for (int j = 0; j < k; ++j) {
        for (int c = 0; c < 3; ++c) colors[3 * j + c] = sums[4 * j + c] / sums[4 * j + 3];
        if (centres_out)
            for (int c = 0; c < 3; ++c) centres_out[3 * j + c] = cen[j].v[c];
    }
    *k_out = k;
    return GID_OK;
}

gid_status check_args(const float* frame, int W, int H, int k_max, double merge_dist, const uint8_t* ids,
                      const double* colors, const int32_t* k_out) {
    if (!frame || !ids || !colors || !k_out) return GID_ERR_INVALID_ARG;
    if (W < 1 || H < 1 || (long long)W * H > (1LL << 28)) return GID_ERR_INVALID_ARG;
    if (k_max < 1 || k_max > CKMAX) return GID_ERR_INVALID_ARG;
    if (!(merge_dist >= 0.0) || !std::isfinite(merge_dist)) return GID_ERR_INVALID_ARG;
    return GID_OK;
}

}  // namespace gidc

extern "C" gid_status gid_cluster_frame(const float* frame_dev, int32_t width, int32_t height, int32_t k_max,
                                        double merge_dist, void* hip_stream, uint8_t* ids_dev, double* colors_host,
                                        double* centres_host, int32_t* k_out) {
    using namespace gidc;
    gid_status st = check_args(frame_dev, width, height, k_max, merge_dist, ids_dev, colors_host, k_out);
    if (st != GID_OK) return st;
    char* scratch = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&scratch), SCRATCH_BYTES) != hipSuccess) return GID_ERR_OUT_OF_MEMORY;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    st = run(frame_dev, width, height, k_max, merge_dist, s, ids_dev, colors_host, centres_host, k_out, scratch);
    // the kernels are done: run() ends with a stream synchronisation, or failed before its launches completed
    (void)hipStreamSynchronize(s);
    (void)hipFree(scratch);
    return st;
}
