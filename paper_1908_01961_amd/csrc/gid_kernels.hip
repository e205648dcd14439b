// HIP kernels of libgid for gfx950: the per-frame precompute, the layer step
// (Gauss-Newton build, matrix-free J^T J matvec, PCG update), the apply +
// base-colour sums, the small FP64 base-colour solve, the FP64 energy and the
// output pass.
//
// Execution model: one thread per pixel.  A workgroup is 256 threads = four
// wavefronts; it covers a tile of 64 columns x (4 * ppt) rows, each wavefront one
// row of 64 pixels, so every plane access is a 256-byte coalesced row segment.
// Tiles are handed to workgroups XCD-aware: the hardware deals workgroup i to XCD
// i % 8, and logical_block() gives each XCD a contiguous band of tiles so that
// the halo rows a tile shares with its vertical neighbours stay in that XCD's L2.
//
// Grids are persistent-style: at most a few workgroups per CU, each owning a
// contiguous chunk of tiles, so a launch produces at most ~1024 partial sums.
//
// Precision: unknowns and PCG vectors are FP32; every dot product, alpha, beta,
// base-colour sum, the 3K x 3K solve and the energy are FP64.  Reductions are
// deterministic and need no atomics or cache-maintenance fences (which serialise
// badly across eight L2s): a workgroup reduces its pixels (wavefront butterfly,
// then the four wavefronts in fixed order) and stores one partial per value with
// a plain store; the consuming kernel -- the next launch in the stream, so the
// partials are visible -- sums them in index order in every workgroup that needs
// the scalar, each workgroup computing the identical total.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "gid_internal.h"

namespace gid {
namespace {

__device__ __forceinline__ int logical_block() {
    const int per = gridDim.x >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 256 threads; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* sh4) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
}

__device__ __forceinline__ double* site_ptr(const Args& a, int site) {
    return a.partials + (long long)site * a.part_stride;
}

// Store this workgroup's nv values (every thread holds them) as partials of a site.
__device__ __forceinline__ void publish(const Args& a, int site, const double* vals, int nv) {
    double* p = site_ptr(a, site);
    if ((int)threadIdx.x < nv) p[(long long)threadIdx.x * gridDim.x + blockIdx.x] = vals[threadIdx.x];
}

// Total of value v of a site produced by a launch of nb workgroups; every
// thread gets the same result, summed in a fixed order.
__device__ __forceinline__ double site_total(const Args& a, int site, int v, int nb, double* sh4) {
    const double* p = site_ptr(a, site) + (long long)v * nb;
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += NTHREADS) s += p[i];
    return block_sum(s, sh4);
}

// PCG inner-product sites: <r, z> after PCG iteration i lives in site rz_site(i);
// iteration -1 is the Gauss-Newton build.
__device__ __forceinline__ int rz_site(int i) { return (i & 1) ? R_RZB : R_RZA; }

// Visit every pixel of this workgroup's contiguous chunk of tiles: f(x, y, i).
template <typename F>
__device__ __forceinline__ void for_each_pixel(const Args& a, F&& f) {
    const int lb = logical_block();
    const int t0 = (int)(((long long)lb * a.ntiles) / gridDim.x);
    const int t1 = (int)(((long long)(lb + 1) * a.ntiles) / gridDim.x);
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int rows = TYW * a.ppt;
    for (int tile = t0; tile < t1; ++tile) {
        const int x = (tile % a.ntx) * TX + lx;
        if (x >= a.W) continue;
        const int ybase = (tile / a.ntx) * rows + ly;
        for (int j = 0; j < a.ppt; ++j) {
            const int y = ybase + TYW * j;
            if (y >= a.H) break;
            f(x, y, (long long)y * a.W + x);
        }
    }
}

__device__ __forceinline__ bool lead_thread() { return blockIdx.x == 0 && threadIdx.x == 0; }

// Basis with the white illuminant first, and the basis minus its channel mean.
template <int K>
struct Basis {
    float B[K + 1][3];
    float Bc[K + 1][3];
    __device__ __forceinline__ void load(const float* bf) {
        B[0][0] = B[0][1] = B[0][2] = 1.0f;
        Bc[0][0] = Bc[0][1] = Bc[0][2] = 0.0f;
#pragma unroll
        for (int k = 1; k <= K; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) B[k][c] = bf[(k - 1) * 3 + c];
            const float mu = (B[k][0] + B[k][1] + B[k][2]) * (1.0f / 3.0f);
#pragma unroll
            for (int c = 0; c < 3; ++c) Bc[k][c] = B[k][c] - mu;
        }
    }
};

// IRLS weight of the reflectance-gradient sparsity term at a pixel from its
// forward differences (the norm over both directions and all channels).
__device__ __forceinline__ float w_rsparsity(const float* r0, bool hr, const float* rr, bool hd,
                                             const float* rd, const Lam& L) {
    float s = 0.0f;
    if (hr) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = rr[c] - r0[c];
            s += d * d;
        }
    }
    if (hd) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = rd[c] - r0[c];
            s += d * d;
        }
    }
    const float nrm = sqrtf(s) + L.eps_irls;
    return (L.p == 1.0f) ? 1.0f / nrm : powf(nrm, L.p - 2.0f);
}

__device__ __forceinline__ float w_pair(float a, float b, float eps) { return 1.0f / (fabsf(b - a) + eps); }

__device__ __forceinline__ void load3(const float* base, long long ps, long long i, float* v) {
    v[0] = base[i];
    v[1] = base[ps + i];
    v[2] = base[2 * ps + i];
}

// Lambda-scaled weights of the four reflectance-gradient pairs touching pixel
// (x, y): right and down use the pixel's own weight, left and up the weights of
// the left and upper neighbours.  Zero where the pair does not exist.
__device__ __forceinline__ void rsparsity_pairs(const Args& a, int x, int y, long long i, float wr[4]) {
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    const bool hr = x + 1 < W, hd = y + 1 < H, hl = x > 0, hu = y > 0;
    float r0[3], rr[3] = {0, 0, 0}, rd[3] = {0, 0, 0}, rl[3] = {0, 0, 0}, ru[3] = {0, 0, 0};
    load3(a.u, ps, i, r0);
    if (hr) load3(a.u, ps, i + 1, rr);
    if (hd) load3(a.u, ps, i + W, rd);
    if (hl) load3(a.u, ps, i - 1, rl);
    if (hu) load3(a.u, ps, i - W, ru);
    const float lr = a.lam.rs;
    const float wself = (hr || hd) ? lr * w_rsparsity(r0, hr, rr, hd, rd, a.lam) : 0.0f;
    wr[0] = hr ? wself : 0.0f;
    wr[1] = hd ? wself : 0.0f;
    if (hl) {
        float rld[3] = {0, 0, 0};
        const bool ld = y + 1 < H;
        if (ld) load3(a.u, ps, i - 1 + W, rld);
        wr[2] = lr * w_rsparsity(rl, true, r0, ld, rld, a.lam);
    } else {
        wr[2] = 0.0f;
    }
    if (hu) {
        float rur[3] = {0, 0, 0};
        const bool ur = x + 1 < W;
        if (ur) load3(a.u, ps, i - W + 1, rur);
        wr[3] = lr * w_rsparsity(ru, ur, rur, true, r0, a.lam);
    } else {
        wr[3] = 0.0f;
    }
}

// p of the current PCG iteration at plane element j: the stored p0 for the first
// iteration, z + beta p_old afterwards (recomputed identically by every reader).
__device__ __forceinline__ float p_at(const Args& a, long long j, double beta) {
    if (a.iter == 0) return a.pold[j];
    const float z = a.res[j] * a.minv[j];
    return (float)((double)z + beta * (double)a.pold[j]);
}

// --------------------------------------------------------------- input scan

// Count non-finite frame values and cluster ids outside [0, K); any hit makes the
// rest of the frame's kernels no-ops so the solver state is left unchanged.
__global__ __launch_bounds__(NTHREADS) void k_scan(Args a) {
    __shared__ double sh4[4];
    const long long ps = a.ps;
    double bad = 0.0;
    for_each_pixel(a, [&](int x, int y, long long i) {
        float v[3];
        load3(a.in_frame, ps, i, v);
        if (!isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2])) bad += 1.0;
        if ((int)a.in_ids[i] >= a.K) bad += 1.0;
    });
    const double vals[1] = {block_sum(bad, sh4)};
    publish(a, R_SCAN, vals, 1);
}

// ----------------------------------------------------------------- precompute

__device__ __forceinline__ void chroma64(const float* I, long long ps, long long i, double floor_, double* C) {
    const double v0 = I[i], v1 = I[ps + i], v2 = I[2 * ps + i];
    const double m = (v0 + v1 + v2) / 3.0;
    if (m >= floor_) {
        C[0] = v0 / m;
        C[1] = v1 / m;
        C[2] = v2 / m;
    } else {
        C[0] = C[1] = C[2] = 1.0;
    }
}

__device__ __forceinline__ double cdist(const double* a, const double* b) {
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return sqrt((d0 * d0 + d1 * d1) + d2 * d2);
}

template <int K>
__global__ __launch_bounds__(NTHREADS) void k_precompute(Args a) {
    __shared__ double sh4[4];
    // input check of the scan (every workgroup computes the same total)
    const double bad = site_total(a, R_SCAN, 0, gridDim.x, sh4);
    if (lead_thread()) a.scal[S_BADIN] = bad;
    if (bad != 0.0) return;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    const double floor_ = a.lam.cfloor;
    const float* F = a.in_frame;
    for_each_pixel(a, [&](int x, int y, long long i) {
        float Iv[3];
        load3(F, ps, i, Iv);
        a.I[i] = Iv[0];
        a.I[ps + i] = Iv[1];
        a.I[2 * ps + i] = Iv[2];
        const uint8_t id = a.in_ids[i];
        a.ids[i] = id;
        double C[3], Cn[3];
        chroma64(F, ps, i, floor_, C);
        double dC = 0.0;
        if (x + 1 < W) { chroma64(F, ps, i + 1, floor_, Cn); dC = fmax(dC, cdist(Cn, C)); }
        if (x > 0)     { chroma64(F, ps, i - 1, floor_, Cn); dC = fmax(dC, cdist(C, Cn)); }
        if (y + 1 < H) { chroma64(F, ps, i + W, floor_, Cn); dC = fmax(dC, cdist(Cn, C)); }
        if (y > 0)     { chroma64(F, ps, i - W, floor_, Cn); dC = fmax(dC, cdist(C, Cn)); }
        a.wsr[i] = (float)(1.0 - exp(-(double)a.lam.rk * dC));
        float gsum = 0.0f, tr0 = 0.0f, tr1 = 0.0f, tr2 = 0.0f;
        if (a.temporal) {
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = y + dy;
                if (yy < 0 || yy >= H) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = x + dx;
                    if (xx < 0 || xx >= W) continue;
                    const long long jj = (long long)yy * W + xx;
                    chroma64(a.Iprev, ps, jj, floor_, Cn);
                    if (cdist(C, Cn) < a.lam.gate) {
                        gsum += 1.0f;
                        tr0 += a.rprev[jj];
                        tr1 += a.rprev[ps + jj];
                        tr2 += a.rprev[2 * ps + jj];
                    }
                }
            }
        }
        a.tg[i] = gsum;
        a.tg[ps + i] = tr0;
        a.tg[2 * ps + i] = tr1;
        a.tg[3 * ps + i] = tr2;
        if (a.first) {
            const double* b = a.b64 + 3 * id;
            a.u[i] = a.lnb[3 * id];
            a.u[ps + i] = a.lnb[3 * id + 1];
            a.u[2 * ps + i] = a.lnb[3 * id + 2];
            const double mI = ((double)Iv[0] + (double)Iv[1] + (double)Iv[2]) / 3.0;
            const double mR = (b[0] + b[1] + b[2]) / 3.0;
            a.u[3 * ps + i] = (float)fmin(fmax(mI / mR, 0.0), 4.0);
#pragma unroll
            for (int k = 1; k <= K; ++k) a.u[(3 + k) * ps + i] = 0.01f;
        }
    });
}

// ------------------------------------------------------------------ GN build

template <int K>
__global__ __launch_bounds__(NTHREADS) void k_gn_build(Args a) {
    constexpr int N = K + 4;
    __shared__ double sh4[4];
    if (a.scal[S_BADIN] != 0.0) return;
    Basis<K> bs;
    bs.load(a.bf);
    const Lam L = a.lam;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    double acc = 0.0;
    for_each_pixel(a, [&](int x, int y, long long i) {
        float r[3], T[K + 1], Iv[3];
        load3(a.u, ps, i, r);
#pragma unroll
        for (int k = 0; k <= K; ++k) T[k] = a.u[(3 + k) * ps + i];
        load3(a.I, ps, i, Iv);
        const int id = a.ids[i];
        const float w = a.wsr[i];
        float R[3], S[3], e[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R[c] = expf(r[c]);
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k <= K; ++k) s += bs.B[k][c] * T[k];
            S[c] = s;
            e[c] = Iv[c] - R[c] * s;
        }
        float g[N], M[N];
        const float gs = a.temporal ? a.tg[i] : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float RS = R[c] * S[c];
            const float tgr = a.temporal ? a.tg[(1 + c) * ps + i] : 0.0f;
            g[c] = L.data * RS * e[c] - L.cl * (r[c] - a.lnb[3 * id + c]) - L.rc * (gs * r[c] - tgr);
            M[c] = L.data * RS * RS + L.cl + L.rc * gs;
        }
        const float mS = (S[0] + S[1] + S[2]) * (1.0f / 3.0f);
        float md[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) md[c] = S[c] - mS;
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            float gd = 0.0f, Md = 0.0f, gm = 0.0f, Mm = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float RB = R[c] * bs.B[k][c];
                gd += RB * e[c];
                Md += RB * RB;
                gm += bs.Bc[k][c] * md[c];
                Mm += bs.Bc[k][c] * bs.Bc[k][c];
            }
            const float at = fabsf(T[k]);
            const float wis = (k > 0) ? L.is / (at + L.eps_irls) : 0.0f;
            const float wnn = (T[k] > 0.0f) ? 0.0f : L.nn / (at + L.eps_nn);
            g[3 + k] = L.data * gd - L.mo * w * gm - (wis + wnn) * T[k];
            M[3 + k] = L.data * Md + L.mo * w * Mm + wis + wnn;
        }
        // reflectance sparsity stencil
        {
            float wr[4];
            rsparsity_pairs(a, x, y, i, wr);
            const long long nb[4] = {i + 1, i + W, i - 1, i - W};
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                if (wr[d] == 0.0f) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) g[c] -= wr[d] * (r[c] - a.u[c * ps + nb[d]]);
#pragma unroll
                for (int c = 0; c < 3; ++c) M[c] += wr[d];
            }
        }
        // smoothness stencil, one layer at a time
        {
            const bool hv[4] = {x + 1 < W, y + 1 < H, x > 0, y > 0};
            const long long nb[4] = {i + 1, i + W, i - 1, i - W};
#pragma unroll
            for (int k = 0; k <= K; ++k) {
                const float* Tk = a.u + (3 + k) * ps;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if (!hv[d]) continue;
                    const float tn = Tk[nb[d]];
                    const float ws = L.sm * w_pair(T[k], tn, L.eps_irls);
                    g[3 + k] -= ws * (T[k] - tn);
                    M[3 + k] += ws;
                }
            }
        }
        if (a.debug) {
#pragma unroll
            for (int v = 0; v < N; ++v) {
                a.out[v * ps + i] = g[v];
                a.out2[v * ps + i] = M[v];
            }
        } else {
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const float mi = 1.0f / M[v];
                const float z = g[v] * mi;
                a.res[v * ps + i] = g[v];
                a.minv[v * ps + i] = mi;
                a.pnew[v * ps + i] = z;
                a.delta[v * ps + i] = 0.0f;
                acc += (double)g[v] * (double)z;
            }
        }
    });
    if (a.debug) return;
    const double vals[1] = {block_sum(acc, sh4)};
    publish(a, rz_site(-1), vals, 1);
    if (lead_thread()) a.scal[S_STOP] = 0.0;
}

// ---------------------------------------------------------------- PCG matvec

template <int K>
__global__ __launch_bounds__(NTHREADS) void k_matvec(Args a) {
    constexpr int N = K + 4;
    __shared__ double sh4[4];
    if (!a.debug && (a.scal[S_STOP] != 0.0 || a.scal[S_BADIN] != 0.0)) return;   // uniform over the grid
    Basis<K> bs;
    bs.load(a.bf);
    const Lam L = a.lam;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    double beta = 0.0;
    if (!a.debug && a.iter > 0) {
        // beta of the previous iteration from the last two <r, z> totals
        const double rz_now = site_total(a, rz_site(a.iter - 1), 0, gridDim.x, sh4);
        const double rz_before = site_total(a, rz_site(a.iter - 2), 0, gridDim.x, sh4);
        if (lead_thread()) a.scal[S_RZ_LOG + (a.gn & 63)] = rz_now;
        if (rz_now == 0.0) {      // converged exactly: the rest of the layer step is a no-op
            if (lead_thread()) a.scal[S_STOP] = 1.0;
            return;
        }
        beta = rz_now / rz_before;
    }
    Args ad = a;
    if (a.debug) {               // apply J^T J to a caller vector
        ad.iter = 0;
        ad.pold = const_cast<float*>(a.pdebug);
    }
    double acc = 0.0;
    for_each_pixel(a, [&](int x, int y, long long i) {
        float p[N], q[N];
#pragma unroll
        for (int v = 0; v < N; ++v) p[v] = p_at(ad, v * ps + i, beta);
        float r[3], T[K + 1];
        load3(a.u, ps, i, r);
#pragma unroll
        for (int k = 0; k <= K; ++k) T[k] = a.u[(3 + k) * ps + i];
        float R[3], S[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R[c] = expf(r[c]);
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k <= K; ++k) s += bs.B[k][c] * T[k];
            S[c] = s;
        }
        // data term block
        float ac[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float s = S[c] * p[c];
#pragma unroll
            for (int k = 0; k <= K; ++k) s += bs.B[k][c] * p[3 + k];
            ac[c] = R[c] * s;
        }
        const float gs = a.temporal ? a.tg[i] : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) q[c] = L.data * R[c] * S[c] * ac[c] + (L.cl + L.rc * gs) * p[c];
        // monochrome block
        const float w = a.wsr[i];
        float m[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float s = 0.0f;
#pragma unroll
            for (int k = 1; k <= K; ++k) s += bs.Bc[k][c] * p[3 + k];
            m[c] = s;
        }
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            float sd = 0.0f, sm = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sd += R[c] * bs.B[k][c] * ac[c];
                sm += bs.Bc[k][c] * m[c];
            }
            const float at = fabsf(T[k]);
            const float wis = (k > 0) ? L.is / (at + L.eps_irls) : 0.0f;
            const float wnn = (T[k] > 0.0f) ? 0.0f : L.nn / (at + L.eps_nn);
            q[3 + k] = L.data * sd + L.mo * w * sm + (wis + wnn) * p[3 + k];
        }
        // reflectance sparsity stencil
        {
            float wr[4];
            rsparsity_pairs(a, x, y, i, wr);
            const long long nb[4] = {i + 1, i + W, i - 1, i - W};
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                if (wr[d] == 0.0f) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) q[c] += wr[d] * (p[c] - p_at(ad, c * ps + nb[d], beta));
            }
        }
        // smoothness stencil
        {
            const bool hv[4] = {x + 1 < W, y + 1 < H, x > 0, y > 0};
            const long long nb[4] = {i + 1, i + W, i - 1, i - W};
#pragma unroll
            for (int k = 0; k <= K; ++k) {
                const float* Tk = a.u + (3 + k) * ps;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if (!hv[d]) continue;
                    const float ws = L.sm * w_pair(T[k], Tk[nb[d]], L.eps_irls);
                    q[3 + k] += ws * (p[3 + k] - p_at(ad, (3 + k) * ps + nb[d], beta));
                }
            }
        }
        if (a.debug) {
#pragma unroll
            for (int v = 0; v < N; ++v) a.out[v * ps + i] = q[v];
        } else {
#pragma unroll
            for (int v = 0; v < N; ++v) {
                a.q[v * ps + i] = q[v];
                if (a.iter > 0) a.pnew[v * ps + i] = p[v];
                acc += (double)p[v] * (double)q[v];
            }
        }
    });
    if (a.debug) return;
    const double vals[1] = {block_sum(acc, sh4)};
    publish(a, R_PQ, vals, 1);
}

// ---------------------------------------------------------------- PCG update

template <int K>
__global__ __launch_bounds__(NTHREADS) void k_update(Args a) {
    constexpr int N = K + 4;
    __shared__ double sh4[4];
    if (a.scal[S_STOP] != 0.0 || a.scal[S_BADIN] != 0.0) return;
    const long long ps = a.ps;
    const double pq = site_total(a, R_PQ, 0, gridDim.x, sh4);
    const double rz = site_total(a, rz_site(a.iter - 1), 0, gridDim.x, sh4);
    if (!(pq > 0.0) || !isfinite(pq)) {       // breakdown guard: no update, layer step ends
        if (lead_thread()) {
            a.scal[S_STOP] = 1.0;
            a.scal[S_BREAKDOWNS] += 1.0;
            a.scal[S_RZ_LOG + (a.gn & 63)] = rz;
        }
        return;
    }
    const double alpha = rz / pq;
    double acc = 0.0;
    for_each_pixel(a, [&](int x, int y, long long i) {
#pragma unroll
        for (int v = 0; v < N; ++v) {
            const long long e = v * ps + i;
            const float p = a.pnew[e];
            const float dn = (float)((double)a.delta[e] + alpha * (double)p);
            const float rn = (float)((double)a.res[e] - alpha * (double)a.q[e]);
            a.delta[e] = dn;
            a.res[e] = rn;
            acc += (double)rn * (double)(rn * a.minv[e]);
        }
    });
    const double vals[1] = {block_sum(acc, sh4)};
    publish(a, rz_site(a.iter), vals, 1);
}

// ---------------------------------------------------- apply + base-colour sums

constexpr int BS_BATCH = 128;   // pixels staged in LDS per round

template <int K>
__global__ __launch_bounds__(NTHREADS) void k_apply_bsum(Args a) {
    constexpr int N = K + 4;
    constexpr int NV = 3 * (K + 1);                  // per pixel: R_c T_k (k = 1..K) and R_c e_c
    constexpr int GS = (3 * K <= 32) ? 32 : 64;      // threads per pixel group
    constexpr int NG = NTHREADS / GS;
    __shared__ double stage[BS_BATCH * NV];
    __shared__ double red[NG * 3 * K * (K + 1)];
    __shared__ double sh4[4];
    if (a.scal[S_BADIN] != 0.0) return;
    if (a.log_rz && a.scal[S_STOP] == 0.0) {
        // <r, z> after the last PCG iteration (site of iteration pcg_iters - 1)
        const double rz = site_total(a, rz_site(a.iter), 0, a.nblocks, sh4);
        if (lead_thread()) a.scal[S_RZ_LOG + (a.gn & 63)] = rz;
    }
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    // this workgroup's contiguous chunk of tiles (XCD-aware)
    const int lb = logical_block();
    const int t0 = (int)(((long long)lb * a.ntiles) / gridDim.x);
    const int t1 = (int)(((long long)(lb + 1) * a.ntiles) / gridDim.x);
    const int grp = threadIdx.x / GS, lane = threadIdx.x % GS;
    const bool owner = lane < 3 * K;
    const int oc = owner ? lane / K : 0, ok = owner ? lane % K : 0;
    double acc[K + 1];
#pragma unroll
    for (int l = 0; l <= K; ++l) acc[l] = 0.0;
    double B64[K][3];
    if (a.refine) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) B64[k][c] = a.b64[3 * k + c];
    }
    const int rows = TYW * a.ppt;
    const int tile_px = TX * rows;
    for (int tile = t0; tile < t1; ++tile) {
        const int tx = tile % a.ntx, ty = tile / a.ntx;
        for (int base = 0; base < tile_px; base += BS_BATCH) {
            // stage: threads 0..BS_BATCH-1 each own one pixel of the batch
            if (threadIdx.x < BS_BATCH) {
                const int lp = base + threadIdx.x;
                const int x = tx * TX + (lp % TX), y = ty * rows + lp / TX;
                double* sv = stage + threadIdx.x * NV;
                if (x < W && y < H) {
                    const long long i = (long long)y * W + x;
                    float uv[N];
#pragma unroll
                    for (int v = 0; v < N; ++v) {
                        const long long e = v * ps + i;
                        if (a.add_delta) {
                            uv[v] = a.u[e] + a.delta[e];
                            a.u[e] = uv[v];
                        } else {
                            uv[v] = a.u[e];
                        }
                    }
                    if (a.refine) {
                        double R[3], S[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            R[c] = exp((double)uv[c]);
                            double s = (double)uv[3];
#pragma unroll
                            for (int k = 0; k < K; ++k) s += B64[k][c] * (double)uv[4 + k];
                            S[c] = s;
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const double ec = (double)a.I[c * ps + i] - R[c] * S[c];
#pragma unroll
                            for (int k = 0; k < K; ++k) sv[c * (K + 1) + k] = R[c] * (double)uv[4 + k];
                            sv[c * (K + 1) + K] = ec;
                        }
                    }
                } else if (a.refine) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) sv[v] = 0.0;
                }
            }
            if (!a.refine) continue;
            __syncthreads();
            if (owner) {
                for (int px = grp; px < BS_BATCH; px += NG) {
                    const double* sv = stage + px * NV + oc * (K + 1);
                    const double vk = sv[ok];
#pragma unroll
                    for (int l = 0; l <= K; ++l)
                        if (l >= ok) acc[l] += vk * sv[l];
                }
            }
            __syncthreads();
        }
    }
    if (!a.refine) return;
    // combine the pixel groups, then publish this workgroup's sums
    if (owner) {
#pragma unroll
        for (int l = 0; l <= K; ++l) red[(grp * 3 * K + lane) * (K + 1) + l] = acc[l];
    }
    __syncthreads();
    const int nb = gridDim.x;
    const int nsum = bstep_nsums(K);
    double* part = a.partials + (long long)R_BS * a.part_stride;
    for (int e = threadIdx.x; e < 3 * K * (K + 1); e += NTHREADS) {
        const int jj = e / (K + 1), l = e % (K + 1);
        const int c = jj / K, k = jj % K;
        if (l < K && l < k) continue;
        double s = 0.0;
        for (int g = 0; g < NG; ++g) s += red[(g * 3 * K + jj) * (K + 1) + l];
        int idx;
        if (l < K) idx = c * (K * (K + 1) / 2) + (k * K - k * (k - 1) / 2) + (l - k);
        else       idx = 3 * K * (K + 1) / 2 + c * K + k;
        part[(long long)idx * nb + lb] = s;
    }
    (void)nsum;
}

// -------------------------------------------------------- base-colour solve

// One workgroup: reduce the per-workgroup sums, assemble the 3K x 3K system of
// the base-colour step, solve it by FP64 Cholesky, apply the guards, update b.
template <int K>
__global__ __launch_bounds__(1024) void k_bsolve(Args a, int nb) {
    constexpr int NA = 3 * K * (K + 1) / 2;
    constexpr int NS = NA + 3 * K;
    constexpr int NN = 3 * K;
    __shared__ double sums[NS];
    __shared__ double Hm[NN][NN + 1];
    __shared__ double gv[NN];
    __shared__ double piv_ok;
    if (a.scal[S_BADIN] != 0.0) return;
    const double* part = a.partials + (long long)R_BS * a.part_stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int e = wave; e < NS; e += nw) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += part[(long long)e * nb + b];
        s = wave_sum(s);
        if (lane == 0) sums[e] = s * (double)a.lam.data;
    }
    __syncthreads();
    if (a.debug) {   // publish the raw sums for single-step access
        for (int e = threadIdx.x; e < NS; e += blockDim.x) a.bsum[e] = sums[e];
        return;
    }
    const double npix = (double)a.W * (double)a.H;
    const double lir = a.lam.ir, lcr = a.lam.cr;
    for (int e = threadIdx.x; e < NN * NN; e += blockDim.x) {
        const int row = e / NN, col = e % NN;
        const int k = row / 3, c = row % 3, l = col / 3, c2 = col % 3;
        double v = 0.0;
        if (c == c2) {
            const int kk = k < l ? k : l, ll = k < l ? l : k;
            v = sums[c * (K * (K + 1) / 2) + (kk * K - kk * (kk - 1) / 2) + (ll - kk)] / npix;
        }
        if (row == col) v += lir + (a.cr_literal ? lcr : 0.0);
        Hm[row][col] = v;
    }
    __syncthreads();
    if (threadIdx.x < NN) {
        const int row = threadIdx.x, k = row / 3, c = row % 3;
        const double dtot = a.b64[3 * k + c] - a.binit64[3 * k + c];
        double g = sums[NA + c * K + k] / npix - lir * dtot;
        if (a.cr_literal) g -= lcr * dtot;
        gv[row] = g;
    }
    __syncthreads();
    if (!a.cr_literal && threadIdx.x < K) {
        // chromaticity regulariser, linearised at b_k, anchored at the initial estimate
        const int k = threadIdx.x;
        double b[3], b0[3], C[3], C0[3];
        for (int c = 0; c < 3; ++c) { b[c] = a.b64[3 * k + c]; b0[c] = a.binit64[3 * k + c]; }
        const double m = (b[0] + b[1] + b[2]) / 3.0, m0 = (b0[0] + b0[1] + b0[2]) / 3.0;
        const double fl = a.lam.cfloor;
        for (int c = 0; c < 3; ++c) {
            C[c] = m >= fl ? b[c] / m : 1.0;
            C0[c] = m0 >= fl ? b0[c] / m0 : 1.0;
        }
        double J[3][3];
        for (int i2 = 0; i2 < 3; ++i2)
            for (int j2 = 0; j2 < 3; ++j2) J[i2][j2] = ((i2 == j2 ? 1.0 : 0.0) - C[i2] / 3.0) / m;
        for (int i2 = 0; i2 < 3; ++i2) {
            for (int j2 = 0; j2 < 3; ++j2) {
                double s = 0.0;
                for (int r2 = 0; r2 < 3; ++r2) s += J[r2][i2] * J[r2][j2];
                Hm[3 * k + i2][3 * k + j2] += lcr * s;
            }
            double s = 0.0;
            for (int r2 = 0; r2 < 3; ++r2) s += J[r2][i2] * (C[r2] - C0[r2]);
            gv[3 * k + i2] -= lcr * s;
        }
    }
    __syncthreads();
    // Cholesky H = L L^T in place (lower triangle), column by column
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i2 = 0; i2 < NN; ++i2) tr += Hm[i2][i2];
        piv_ok = tr;
    }
    __syncthreads();
    const double trace = piv_ok;
    __syncthreads();
    if (threadIdx.x == 0) piv_ok = 1.0;
    __syncthreads();
    for (int jc = 0; jc < NN; ++jc) {
        if (threadIdx.x == 0) {
            double d = Hm[jc][jc];
            for (int kk = 0; kk < jc; ++kk) d -= Hm[jc][kk] * Hm[jc][kk];
            if (!(d > 1e-12 * trace)) { piv_ok = 0.0; d = 1.0; }
            Hm[jc][jc] = sqrt(d);
        }
        __syncthreads();
        const int i2 = jc + 1 + (int)threadIdx.x;
        if (i2 < NN) {
            double s = Hm[i2][jc];
            for (int kk = 0; kk < jc; ++kk) s -= Hm[i2][kk] * Hm[jc][kk];
            Hm[i2][jc] = s / Hm[jc][jc];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double y[NN], db[NN];
        for (int i2 = 0; i2 < NN; ++i2) {
            double s = gv[i2];
            for (int kk = 0; kk < i2; ++kk) s -= Hm[i2][kk] * y[kk];
            y[i2] = s / Hm[i2][i2];
        }
        for (int i2 = NN - 1; i2 >= 0; --i2) {
            double s = y[i2];
            for (int kk = i2 + 1; kk < NN; ++kk) s -= Hm[kk][i2] * db[kk];
            db[i2] = s / Hm[i2][i2];
        }
        bool ok = piv_ok != 0.0;
        double nbv[NN];
        for (int i2 = 0; i2 < NN; ++i2) {
            nbv[i2] = a.b64[i2] + db[i2];
            if (!isfinite(nbv[i2]) || !(nbv[i2] > 1e-4)) ok = false;
        }
        if (ok) {
            for (int i2 = 0; i2 < NN; ++i2) {
                a.b64[i2] = nbv[i2];
                a.bf[i2] = (float)nbv[i2];
                const double lg = log(nbv[i2]);
                a.lnb64[i2] = lg;
                a.lnb[i2] = (float)lg;
            }
            a.scal[S_BACCEPT] = 1.0;
        } else {
            a.scal[S_BACCEPT] = 0.0;
            a.scal[S_BREJECT] += 1.0;
        }
    }
}

// --------------------------------------------------------------- FP64 energy

template <int K>
__global__ __launch_bounds__(NTHREADS) void k_energy(Args a) {
    __shared__ double sh4[4];
    if (a.scal[S_BADIN] != 0.0) return;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    double e[NTERMS];
#pragma unroll
    for (int v = 0; v < NTERMS; ++v) e[v] = 0.0;
    const double p = a.lam.p;
    const double fl = a.lam.cfloor;
    double Bk[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) Bk[k][c] = a.b64[3 * k + c];
    for_each_pixel(a, [&](int x, int y, long long i) {
        double r[3], T[K + 1];
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = a.u[c * ps + i];
#pragma unroll
        for (int k = 0; k <= K; ++k) T[k] = a.u[(3 + k) * ps + i];
        const int id = a.ids[i];
        double S[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double s = T[0];
#pragma unroll
            for (int k = 0; k < K; ++k) s += Bk[k][c] * T[k + 1];
            S[c] = s;
            const double d = (double)a.I[c * ps + i] - exp(r[c]) * s;
            e[0] += d * d;
            const double dc = r[c] - a.lnb64[3 * id + c];
            e[1] += dc * dc;
        }
        // reflectance-gradient norm (forward differences)
        double g2 = 0.0;
        const bool hr = x + 1 < W, hd = y + 1 < H;
        if (hr) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { const double d = (double)a.u[c * ps + i + 1] - r[c]; g2 += d * d; }
        }
        if (hd) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { const double d = (double)a.u[c * ps + i + W] - r[c]; g2 += d * d; }
        }
        const double gn = sqrt(g2);
        e[2] += (p == 1.0) ? gn : ((gn > 0.0) ? pow(gn, p) : 0.0);
        if (a.temporal) {
            double C[3], Cn[3];
            chroma64(a.I, ps, i, fl, C);
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = y + dy;
                if (yy < 0 || yy >= H) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = x + dx;
                    if (xx < 0 || xx >= W) continue;
                    const long long jj = (long long)yy * W + xx;
                    chroma64(a.Iprev, ps, jj, fl, Cn);
                    if (cdist(C, Cn) < a.lam.gate) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const double d = r[c] - (double)a.rprev[c * ps + jj];
                            e[3] += d * d;
                        }
                    }
                }
            }
        }
        const double mS = (S[0] + S[1] + S[2]) / 3.0;
        double md = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) md += (S[c] - mS) * (S[c] - mS);
        e[4] += (double)a.wsr[i] * md;
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            if (k > 0) e[5] += fabs(T[k]);
            if (hr) e[6] += fabs((double)a.u[(3 + k) * ps + i + 1] - T[k]);
            if (hd) e[6] += fabs((double)a.u[(3 + k) * ps + i + W] - T[k]);
            e[7] += fmax(-T[k], 0.0);
        }
    });
    const Lam L = a.lam;
    const double lam[NTERMS] = {L.data, L.cl, L.rs, L.rc, L.mo, L.is, L.sm, L.nn};
    double vals[NTERMS];
#pragma unroll
    for (int v = 0; v < NTERMS; ++v) vals[v] = block_sum(e[v] * lam[v], sh4);
    publish(a, R_EN, vals, NTERMS);
}

// One workgroup: total the energy partials of the preceding k_energy launch
// (nb workgroups) into an energy-log slot.
__global__ __launch_bounds__(NTHREADS) void k_energy_finish(Args a, int nb) {
    __shared__ double sh4[4];
    if (a.scal[S_BADIN] != 0.0) return;
    double tot[NTERMS];
    for (int v = 0; v < NTERMS; ++v) tot[v] = site_total(a, R_EN, v, nb, sh4);
    if (threadIdx.x == 0) {
        double* slot = a.elog + (long long)a.slot * ELOG_STRIDE;
        double s = 0.0;
        for (int v = 0; v < NTERMS; ++v) {
            slot[1 + v] = tot[v];
            s += tot[v];
        }
        slot[0] = s;
    }
}

// -------------------------------------------------------------------- output

template <int K>
__global__ __launch_bounds__(NTHREADS) void k_output(Args a) {
    constexpr int N = K + 4;
    if (a.scal[S_BADIN] != 0.0) return;
    const long long ps = a.ps;
    for_each_pixel(a, [&](int x, int y, long long i) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float r = a.u[c * ps + i];
            if (a.out) a.out[c * ps + i] = expf(r);
            a.rprev[c * ps + i] = r;
            a.Iprev[c * ps + i] = a.I[c * ps + i];
        }
        if (a.out) {
#pragma unroll
            for (int v = 3; v < N; ++v) a.out[v * ps + i] = a.u[v * ps + i];
        }
    });
}

__global__ void k_reset_frame(Args a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        a.scal[S_BREAKDOWNS] = 0.0;
        a.scal[S_BREJECT] = 0.0;
        a.scal[S_STOP] = 0.0;
        a.scal[S_BADIN] = 0.0;
        for (int g = 0; g < 64; ++g) a.scal[S_RZ_LOG + g] = 0.0;
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

namespace {
// Call fn(std::integral_constant<int, K>) for the runtime K (1..KMAX).
template <typename Fn>
hipError_t with_K(int K, Fn&& fn) {
    switch (K) {
        case 1: fn(std::integral_constant<int, 1>{}); break;
        case 2: fn(std::integral_constant<int, 2>{}); break;
        case 3: fn(std::integral_constant<int, 3>{}); break;
        case 4: fn(std::integral_constant<int, 4>{}); break;
        case 5: fn(std::integral_constant<int, 5>{}); break;
        case 6: fn(std::integral_constant<int, 6>{}); break;
        case 7: fn(std::integral_constant<int, 7>{}); break;
        case 8: fn(std::integral_constant<int, 8>{}); break;
        case 9: fn(std::integral_constant<int, 9>{}); break;
        case 10: fn(std::integral_constant<int, 10>{}); break;
        case 11: fn(std::integral_constant<int, 11>{}); break;
        case 12: fn(std::integral_constant<int, 12>{}); break;
        case 13: fn(std::integral_constant<int, 13>{}); break;
        case 14: fn(std::integral_constant<int, 14>{}); break;
        case 15: fn(std::integral_constant<int, 15>{}); break;
        case 16: fn(std::integral_constant<int, 16>{}); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

#define GID_TILED_LAUNCHER(NAME)                                                              \
    hipError_t launch_##NAME(const Args& a, hipStream_t s) {                                  \
        return with_K(a.K, [&](auto kc) {                                                     \
            constexpr int KK = decltype(kc)::value;                                           \
            hipLaunchKernelGGL(k_##NAME<KK>, dim3(a.nblocks), dim3(NTHREADS), 0, s, a);       \
        });                                                                                   \
    }

GID_TILED_LAUNCHER(precompute)
GID_TILED_LAUNCHER(gn_build)
GID_TILED_LAUNCHER(matvec)
GID_TILED_LAUNCHER(update)
GID_TILED_LAUNCHER(energy)
GID_TILED_LAUNCHER(output)

hipError_t launch_apply_bsum(const Args& a, int nblocks_bs, hipStream_t s) {
    return with_K(a.K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        hipLaunchKernelGGL(k_apply_bsum<KK>, dim3(nblocks_bs), dim3(NTHREADS), 0, s, a);
    });
}

hipError_t launch_bsolve(const Args& a, int nblocks_bs, hipStream_t s) {
    return with_K(a.K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        hipLaunchKernelGGL(k_bsolve<KK>, dim3(1), dim3(1024), 0, s, a, nblocks_bs);
    });
}

hipError_t launch_energy_finish(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(NTHREADS), 0, s, a, a.nblocks);
    return hipGetLastError();
}

hipError_t launch_scan(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_scan, dim3(a.nblocks), dim3(NTHREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reset_frame(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_frame, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace gid
