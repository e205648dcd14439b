// Re-synthesis of frames from their layers for the live applications of
// Sec. 8.4 (recolouring, colour keying, colour-spill suppression):
//   I'_c(x) = R_c(x) s_{id(x),c} (T_0(x) + sum_{k=1..K} g_k b'_{k,c} T_k(x)),
// the image-formation model of Sec. 4 with edited base colours b', a gain g_k
// per indirect layer (0 drops a colour's spill) and a per-cluster reflectance
// scale s.  A streaming kernel: each thread reads K + 4 layer planes (and the
// id) of four consecutive pixels with 16-byte loads where the planes allow it,
// and writes three output planes; the coefficients g_k b'_k and s travel in
// the kernel arguments.  Bound by HBM bandwidth: (K + 7) * 4 (+ 1 with ids)
// bytes per pixel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>

#include "gid.h"

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_KMAX = 16;
constexpr int RS_MAXWG = 4096;

struct ResynthArgs {
    float coef[RS_KMAX][3];     // g_k b'_{k,c}
    float scale[RS_KMAX][3];    // s_{j,c}
    long long npx;
    int K;
    int use_scale;
};

template <int K>
__device__ __forceinline__ void pixel(const ResynthArgs& ra, const float* R, const float* T, int id, float* out) {
    float S[3] = {T[0], T[0], T[0]};
#pragma unroll
    for (int k = 1; k <= K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) S[c] = fmaf(ra.coef[k - 1][c], T[k], S[c]);
    // ids outside [0, K) keep their reflectance
    const bool sc = ra.use_scale && id < K;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = (sc ? R[c] * ra.scale[sc ? id : 0][c] : R[c]) * S[c];
}

// VEC: four pixels per thread with 16-byte loads (npx a multiple of 4 and
// 16-byte aligned planes); otherwise one pixel per thread.
template <int K, bool VEC>
__global__ __launch_bounds__(RS_THREADS) void k_resynth(const float* L, const uint8_t* ids, float* out,
                                                        const ResynthArgs ra) {
    constexpr int N = K + 4;
    const long long np = ra.npx;
    if (VEC) {
        const long long nq = np >> 2;
        for (long long q = (long long)blockIdx.x * RS_THREADS + threadIdx.x; q < nq;
             q += (long long)gridDim.x * RS_THREADS) {
            float4 lv[N];
#pragma unroll
            for (int v = 0; v < N; ++v) lv[v] = reinterpret_cast<const float4*>(L + v * np)[q];
            uchar4 id4 = make_uchar4(0, 0, 0, 0);
            if (ra.use_scale) id4 = reinterpret_cast<const uchar4*>(ids)[q];
            const int idv[4] = {id4.x, id4.y, id4.z, id4.w};
            float o[4][3];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float Rv[3], Tv[K + 1];
#pragma unroll
                for (int c = 0; c < 3; ++c) Rv[c] = (&lv[c].x)[e];
#pragma unroll
                for (int k = 0; k <= K; ++k) Tv[k] = (&lv[3 + k].x)[e];
                pixel<K>(ra, Rv, Tv, idv[e], o[e]);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                reinterpret_cast<float4*>(out + c * np)[q] = make_float4(o[0][c], o[1][c], o[2][c], o[3][c]);
        }
    } else {
        for (long long i = (long long)blockIdx.x * RS_THREADS + threadIdx.x; i < np;
             i += (long long)gridDim.x * RS_THREADS) {
            float Rv[3], Tv[K + 1], o[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) Rv[c] = L[c * np + i];
#pragma unroll
            for (int k = 0; k <= K; ++k) Tv[k] = L[(3 + k) * np + i];
            pixel<K>(ra, Rv, Tv, ra.use_scale ? ids[i] : 0, o);
#pragma unroll
            for (int c = 0; c < 3; ++c) out[c * np + i] = o[c];
        }
    }
}

template <int K>
void launch_k(bool vec, int nwg, hipStream_t s, const float* L, const uint8_t* ids, float* out, const ResynthArgs& ra) {
    if (vec)
        k_resynth<K, true><<<nwg, RS_THREADS, 0, s>>>(L, ids, out, ra);
    else
        k_resynth<K, false><<<nwg, RS_THREADS, 0, s>>>(L, ids, out, ra);
}

template <int... Ks>
void launch_any(int K, bool vec, int nwg, hipStream_t s, const float* L, const uint8_t* ids, float* out,
                const ResynthArgs& ra, std::integer_sequence<int, Ks...>) {
    ((K == Ks + 1 ? launch_k<Ks + 1>(vec, nwg, s, L, ids, out, ra) : void()), ...);
}

}  // namespace

extern "C" gid_status gid_resynthesize(const float* layers_dev, int32_t width, int32_t height, int32_t K,
                                       const double* b_new_host, const float* gain_host, const uint8_t* ids_dev,
                                       const float* refl_scale_host, void* hip_stream, float* out_dev) {
    if (!layers_dev || !b_new_host || !out_dev) return GID_ERR_INVALID_ARG;
    if (width < 1 || height < 1 || (long long)width * height > (1LL << 28)) return GID_ERR_INVALID_ARG;
    if (K < 1 || K > RS_KMAX) return GID_ERR_INVALID_ARG;
    if ((refl_scale_host != nullptr) != (ids_dev != nullptr)) return GID_ERR_INVALID_ARG;
    ResynthArgs ra{};
    ra.npx = (long long)width * height;
    ra.K = K;
    ra.use_scale = refl_scale_host != nullptr;
    for (int k = 0; k < K; ++k) {
        const double g = gain_host ? (double)gain_host[k] : 1.0;
        for (int c = 0; c < 3; ++c) {
            const double bv = b_new_host[3 * k + c];
            if (!std::isfinite(bv) || !std::isfinite(g)) return GID_ERR_INVALID_ARG;
            ra.coef[k][c] = (float)(g * bv);
            ra.scale[k][c] = ra.use_scale ? refl_scale_host[3 * k + c] : 1.0f;
        }
    }
    const bool vec = (ra.npx % 4) == 0 && (reinterpret_cast<uintptr_t>(layers_dev) % 16) == 0 &&
                     (reinterpret_cast<uintptr_t>(out_dev) % 16) == 0 &&
                     (!ids_dev || (reinterpret_cast<uintptr_t>(ids_dev) % 4) == 0);
    const long long work = vec ? ra.npx / 4 : ra.npx;
    const int nwg = (int)std::max(1LL, std::min<long long>(RS_MAXWG, (work + RS_THREADS - 1) / RS_THREADS));
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    launch_any(K, vec, nwg, s, layers_dev, ids_dev, out_dev, ra, std::make_integer_sequence<int, RS_KMAX>{});
    return hipGetLastError() == hipSuccess ? GID_OK : GID_ERR_HIP;
}
