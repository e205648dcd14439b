// HIP kernels of libgid for gfx950: the per-frame precompute, the layer step
// (Gauss-Newton build, one launch per PCG iteration: vector updates and the
// matrix-free J^T J product fused, one reduction per iteration), the apply +
// base-colour sums, the small FP64 base-colour solve, the FP64 energy and the
// output pass.
//
// Execution model: one thread per pixel.  A workgroup is 256 threads = four
// wavefronts; it covers a tile of 64 columns x (4 * ppt) rows, each wavefront one
// row of 64 pixels, so every plane access is a 256-byte coalesced row segment.
// Tiles are handed to workgroups XCD-aware: the hardware deals workgroup i to XCD
// i % 8, and xcd_order() gives each XCD a contiguous band of tiles so that the
// halo rows a tile shares with its vertical neighbours stay in that XCD's L2.
//
// Grids are persistent-style: at most 2048 workgroups, each owning every m-th
// tile of its XCD's band (one tile each while the frame has at most 2048
// tiles), so a launch produces at most 2048 partial sums.
// Every kernel is a body over (clip descriptor, launch context, step); a
// single-clip launch runs it over its whole grid, a batched launch runs it for
// several clips of uneven size in one grid, each workgroup finding its clip
// from a prefix table.  The clips of a batched launch here share K (one launch
// per K), so every kernel is compiled for exactly its K and keeps that K's
// register allocation and occupancy; gid_kernels_table.inc builds the kernels
// that take a whole batch of mixed K in one launch.
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

// Position of a workgroup within its clip's launch: lb is the XCD-aware logical
// index among the clip's nb workgroups (nb a multiple of 8, and the clip's first
// workgroup index a multiple of 8, so workgroup lb runs on XCD j % 8 where j is
// its index within the clip).
struct Lc {
    int lb, nb;
};

__device__ __forceinline__ int xcd_order(int j, int nb) { return (j & 7) * (nb >> 3) + (j >> 3); }

// Tiles of a workgroup.  XCD x (workgroups x m .. x m + m - 1 in xcd_order, with
// m = nb / 8) owns the contiguous band of tiles [x ntiles / 8, (x + 1) ntiles / 8)
// in row-major tile order; its workgroups take the band's tiles round-robin
// (tile c0, c0 + m, ...), so the workgroups in flight on one XCD work on
// neighbouring tiles and share their halo lines through that XCD's L2.  With one
// tile per workgroup this is lb itself.  (Dealing each workgroup a vertical run
// of tiles instead, so that a workgroup reuses the halo rows of its previous
// tile, measured 6% slower per PCG iteration at 1920x1080 K=10.)
// nb is a multiple of 8 (every per-pixel grid is).
struct TileSet {
    int c0, c1, step;    // tiles c0, c0 + step, ... below c1 (row-major index)
};

__device__ __forceinline__ TileSet tiles_of(const Args& a, const Lc& lc) {
    const int m = lc.nb >> 3, x = lc.lb / m, jl = lc.lb - x * m;
    TileSet s;
    s.c0 = (int)(((long long)x * a.ntiles) >> 3) + jl;
    s.c1 = (int)(((long long)(x + 1) * a.ntiles) >> 3);
    s.step = m;
    return s;
}

// Tile coordinates of tile l.  When a launch gives its workgroups 4 tiles or more
// each (s.step is the workgroups per XCD), the tiles are numbered in vertical
// strips of 4 tile columns (the last strip holds the ntx % 4 columns left over),
// each strip row by row, so that the tiles an XCD has in flight (a contiguous
// range of numbers) form a compact block and a tile's upper neighbour was started
// a few tiles before it; otherwise row by row.  Same box, same run: at 1920x1080
// K = 10 (10.5 tiles per workgroup) the PCG iteration takes 258.3 us in strips
// against 261.0 us row by row (strips of 2 columns 276 us, of 8 264.5 us, a wider
// last strip 263.0 us); at 640x480 K = 6 (1.25 tiles per workgroup) 36.8 us in
// strips against 35.4 us row by row.
constexpr int TSTRIP = 4;
__device__ __forceinline__ void tile_xy(const Args& a, const TileSet& s, int l, int& tx, int& ty) {
    if (a.ntiles < 32 * s.step) {
        tx = l % a.ntx;
        ty = l / a.ntx;
        return;
    }
    const int full = a.nty * TSTRIP, st = l / full, x0 = st * TSTRIP;
    const int ws = a.ntx - x0 < TSTRIP ? a.ntx - x0 : TSTRIP;
    const int rem = l - st * full;
    ty = rem / ws;
    tx = x0 + rem - ty * ws;
}

__device__ __forceinline__ Lc whole_grid() { return Lc{xcd_order((int)blockIdx.x, (int)gridDim.x), (int)gridDim.x}; }

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
__device__ __forceinline__ void publish(const Args& a, const Lc& lc, int site, const double* vals, int nv) {
    double* p = site_ptr(a, site);
    if ((int)threadIdx.x < nv) p[(long long)threadIdx.x * lc.nb + lc.lb] = vals[threadIdx.x];
}

// Total of value v of a site produced by a launch of nb workgroups; every
// thread gets the same result, summed in a fixed order.
// The loads are unrolled up to the largest launch (nb <= NB_TUNE_MAX) and issued
// unconditionally (index clamped, value masked), so no branch separates them and
// they are all in flight together.
constexpr int SITE_LOADS = NB_TUNE_MAX / NTHREADS;

__device__ __forceinline__ double masked_load(const double* p, int i, int n) {
    const double x = p[i < n ? i : n - 1];
    return i < n ? x : 0.0;
}

__device__ __forceinline__ double site_total(const Args& a, int site, int v, int nb, double* sh4) {
    const double* p = site_ptr(a, site) + (long long)v * nb;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < SITE_LOADS; ++j) s += masked_load(p, (int)threadIdx.x + j * NTHREADS, nb);
    return block_sum(s, sh4);
}

// Totals of the first NV values of a site, every partial load issued before the
// first block reduction.
template <int NV>
__device__ __forceinline__ void site_totals(const Args& a, int site, int nb, double* sh4, double* out) {
    const double* p = site_ptr(a, site);
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        s[v] = 0.0;
#pragma unroll
        for (int j = 0; j < SITE_LOADS; ++j) s[v] += masked_load(p + (long long)v * nb, (int)threadIdx.x + j * NTHREADS, nb);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = block_sum(s[v], sh4);
}

// NV sums over the 256 threads with one pair of barriers (sh: 4 NV doubles);
// every thread gets the results, combined in the order block_sum uses.
template <int NV>
__device__ __forceinline__ void block_sums(double* v, double* sh) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) sh[(threadIdx.x >> 6) * NV + j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = (sh[j] + sh[NV + j]) + (sh[2 * NV + j] + sh[3 * NV + j]);
}

// PCG vectors of iteration i (ping-pong by parity; the build writes p0 = z0 into
// the even p buffer).
__device__ __forceinline__ int pcg_site(int i) { return (i & 1) ? R_PCGB : R_PCGA; }
// (both fields are read and the values selected, so that a descriptor held in
// registers is never addressed through a selected field address)
__device__ __forceinline__ float* pick(int i, float* even, float* odd) { return (i & 1) ? odd : even; }
__device__ __forceinline__ float* p_buf(const Args& a, int i) { return pick(i, a.pA, a.pB); }
__device__ __forceinline__ float* z_buf(const Args& a, int i) { return pick(i, a.zA, a.zB); }
__device__ __forceinline__ float* q_buf(const Args& a, int i) { return pick(i, a.qA, a.qB); }

// The step length of PCG iteration i and the preconditioned residual norm that
// follows it, from the sums the iteration published:
//   alpha_i = <r_i, z_i> / <p_i, q_i>,
//   <r_i+1, z_i+1> = <r_i, z_i> - 2 alpha_i <q_i, z_i> + alpha_i^2 <q_i, M^-1 q_i>
// (r_i+1 = r_i - alpha_i q_i, z = M^-1 r), so the next iteration's beta needs no
// reduction of its own.  ok is false on breakdown (<p, q> not positive or not finite).
struct PcgScalars {
    double rz, alpha, rz_next;
    bool ok;
};
// sh: 4 doubles, or with WIDE 4 PV_N doubles (all four totals reduced behind one
// pair of barriers; the same sums, combined in the same order)
template <bool WIDE = false>
__device__ __forceinline__ PcgScalars pcg_scalars(const Args& a, int i, int nb, double* sh) {
    double t[PV_N];
    if (WIDE) {
        const double* p = site_ptr(a, pcg_site(i));
#pragma unroll
        for (int v = 0; v < PV_N; ++v) {
            t[v] = 0.0;
#pragma unroll
            for (int j = 0; j < SITE_LOADS; ++j) t[v] += masked_load(p + (long long)v * nb, (int)threadIdx.x + j * NTHREADS, nb);
        }
        block_sums<PV_N>(t, sh);
    } else {
        site_totals<PV_N>(a, pcg_site(i), nb, sh, t);
    }
    PcgScalars s;
    s.rz = t[PV_RZ];
    s.ok = t[PV_PQ] > 0.0 && isfinite(t[PV_PQ]);
    s.alpha = s.ok ? s.rz / t[PV_PQ] : 0.0;
    s.rz_next = s.rz - 2.0 * s.alpha * t[PV_QZ] + s.alpha * s.alpha * t[PV_QMQ];
    return s;
}

// Visit every pixel of this workgroup's tiles: f(x, y, i).
template <typename F>
__device__ __forceinline__ void for_each_pixel(const Args& a, const Lc& lc, F&& f) {
    const TileSet tset = tiles_of(a, lc);
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int rows = TYW * a.ppt;
    for (int tile = tset.c0; tile < tset.c1; tile += tset.step) {
        int tx, ty;
        tile_xy(a, tset, tile, tx, ty);
        const int x = tx * TX + lx;
        if (x >= a.W) continue;
        const int ybase = ty * rows + ly;
        for (int j = 0; j < a.ppt; ++j) {
            const int y = ybase + TYW * j;
            if (y >= a.H) break;
            f(x, y, (long long)y * a.W + x);
        }
    }
}

__device__ __forceinline__ bool lead_thread(const Lc& lc) { return lc.lb == 0 && threadIdx.x == 0; }

// Nothing left to do in this frame: its input was rejected, or it reached its
// energy target (uniform over the grid: both flags change only between launches).
__device__ __forceinline__ bool frame_idle(const Args& a) { return a.scal[S_BADIN] != 0.0 || a.scal[S_DONE] != 0.0; }

// Basis with the white illuminant first, and the basis minus its channel mean.
// Both come from device tables with uniform addresses, so they live in scalar
// registers (the base-colour solve and the colour upload maintain the tables).
template <int K>
struct Basis {
    float B[K + 1][3];
    float Bc[K + 1][3];
    __device__ __forceinline__ void load(const float* bf, const float* bcf) {
        B[0][0] = B[0][1] = B[0][2] = 1.0f;
        Bc[0][0] = Bc[0][1] = Bc[0][2] = 0.0f;
#pragma unroll
        for (int k = 1; k <= K; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                B[k][c] = bf[(k - 1) * 3 + c];
                Bc[k][c] = bcf[(k - 1) * 3 + c];
            }
        }
    }
};

// Reciprocal of an IRLS denominator |x| + eps (always >= eps > 0): the hardware
// reciprocal, within 1 ulp.
__device__ __forceinline__ float rcp_pos(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float w_pair(float a, float b, float eps) { return rcp_pos(fabsf(b - a) + eps); }

// Value of a double held by lane `src` of the wavefront (src uniform).
__device__ __forceinline__ double rdlane(double v, int src) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ void load3(const float* base, long long ps, long long i, float* v) {
    v[0] = base[i];
    v[1] = base[ps + i];
    v[2] = base[2 * ps + i];
}

// --------------------------------------------------------------- input scan

// Count non-finite frame values and cluster ids outside [0, K); any hit makes the
// rest of the frame's kernels no-ops so the solver state is left unchanged.
__device__ __forceinline__ void scan_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    double* sh4 = reinterpret_cast<double*>(smem);
    // the frame's scalar bookkeeping starts from zero (no workgroup of this pass reads it)
    if (lead_thread(lc)) {
        a.scal[S_BREAKDOWNS] = 0.0;
        a.scal[S_BREJECT] = 0.0;
        a.scal[S_STOP] = 0.0;
        a.scal[S_BADIN] = 0.0;
        a.scal[S_DONE] = 0.0;
        a.scal[S_GN_DONE] = 0.0;
        for (int g = 0; g < 64; ++g) a.scal[S_RZ_LOG + g] = 0.0;
    }
    const long long ps = a.ps;
    double bad = 0.0;
    for_each_pixel(a, lc, [&](int x, int y, long long i) {
        float v[3];
        load3(a.in_frame, ps, i, v);
        if (!isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2])) bad += 1.0;
        if (a.in_ids && (int)a.in_ids[i] >= a.K) bad += 1.0;
    });
    const double vals[1] = {block_sum(bad, sh4)};
    publish(a, lc, R_SCAN, vals, 1);
}

// ----------------------------------------------------------------- precompute

// Chromaticity of a pixel in FP64: its colour over its channel mean, or
// (1, 1, 1) where the mean is below the floor.
__device__ __forceinline__ void chroma64v(float f0, float f1, float f2, double floor_, double* C) {
    const double v0 = f0, v1 = f1, v2 = f2;
    const double m = (v0 + v1 + v2) / 3.0;
    if (m >= floor_) {
        C[0] = v0 / m;
        C[1] = v1 / m;
        C[2] = v2 / m;
    } else {
        C[0] = C[1] = C[2] = 1.0;
    }
}

// The 3 x 3 window of the previous frame around (x, y) in row-major order: the
// previous frame's colours and final r at each in-frame position (ok[w]).
// Loads are unconditional (off-frame positions read the centre pixel) so all
// of them are in flight together.
struct Window3 {
    float I[9][3], r[9][3];
    bool ok[9];
};
__device__ __forceinline__ void load_window3(const Args& a, int x, int y, long long i, Window3& w) {
    const long long ps = a.ps;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int yy = y + k / 3 - 1, xx = x + k % 3 - 1;
        w.ok[k] = yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
        const long long jj = w.ok[k] ? (long long)yy * a.W + xx : i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w.I[k][c] = a.Iprev[c * ps + jj];
            w.r[k][c] = a.rprev[c * ps + jj];
        }
    }
}

__device__ __forceinline__ double cdist(const double* a, const double* b) {
#pragma clang fp contract(off)
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return sqrt((d0 * d0 + d1 * d1) + d2 * d2);
}

// SplitMix64 output for state x (Steele, Lea and Flood, 2014).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Spatial pairs of the consistency prior (Sec. 6.1: every pixel tied to randomly
// sampled pixels of a small window under a chromaticity gate).  Reading: the
// edges to the eight neighbours, each owned by one pixel in one of four forward
// directions d (right, down-right, down, down-left); an edge is sampled when the
// top bit of SplitMix64((seed << 32) | (4 owner + d)) is zero and active when the
// two chromaticities are closer than the gate.  Bit b of a pixel's mask is its
// edge to neighbour b: b < 4 its own forward edges, b >= 4 the edges the left,
// up-left, up and up-right neighbours own (direction b - 4).
__constant__ int SP_DX[8] = {1, 1, 0, -1, -1, -1, 0, 1};
__constant__ int SP_DY[8] = {0, 1, 1, 1, 0, -1, -1, -1};

// Index of the colour chromaticity nearest to C: squared L2 distance formed
// d0 d0 + d1 d1 + d2 d2 left to right without contraction, ties to the lowest index.
template <int K>
__device__ __forceinline__ int nearest_colour(const double* C, const double (*Cb)[3]) {
#pragma clang fp contract(off)
    double best = INFINITY;
    int arg = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double d0 = C[0] - Cb[k][0], d1 = C[1] - Cb[k][1], d2 = C[2] - Cb[k][2];
        const double d = d0 * d0 + d1 * d1 + d2 * d2;
        if (d < best) {
            best = d;
            arg = k;
        }
    }
    return arg;
}

template <int K>
__device__ __forceinline__ void precompute_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    double* sh4 = reinterpret_cast<double*>(smem);
    // input check of the scan (every workgroup computes the same total)
    const double bad = site_total(a, R_SCAN, 0, lc.nb, sh4);
    if (lead_thread(lc)) a.scal[S_BADIN] = bad;
    if (bad != 0.0) return;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    const double floor_ = a.lam.cfloor;
    const float* F = a.in_frame;
    // without caller ids: the base colour of nearest chromaticity (Sec. 5.1's
    // assignment rule against the current colours)
    double Cb[K][3];
    if (!a.in_ids) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double* b = a.b64 + 3 * k;
            const double m = (b[0] + b[1] + b[2]) / 3.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) Cb[k][c] = b[c] / m;
        }
    }
    for_each_pixel(a, lc, [&](int x, int y, long long i) {
        float Iv[3];
        load3(F, ps, i, Iv);
        a.I[i] = Iv[0];
        a.I[ps + i] = Iv[1];
        a.I[2 * ps + i] = Iv[2];
        double C[3], Cn[3];
        chroma64v(Iv[0], Iv[1], Iv[2], floor_, C);
        uint8_t id;
        if (a.in_ids) {
            id = a.in_ids[i];
        } else {
            id = (uint8_t)nearest_colour<K>(C, Cb);
        }
        a.ids[i] = id;
        // the four neighbours (right, left, down, up), loaded unconditionally
        const bool hn[4] = {x + 1 < W, x > 0, y + 1 < H, y > 0};
        const long long jn[4] = {hn[0] ? i + 1 : i, hn[1] ? i - 1 : i, hn[2] ? i + W : i, hn[3] ? i - W : i};
        float Fn[4][3];
#pragma unroll
        for (int d = 0; d < 4; ++d) load3(F, ps, jn[d], Fn[d]);
        double dC = 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (!hn[d]) continue;
            chroma64v(Fn[d][0], Fn[d][1], Fn[d][2], floor_, Cn);
            dC = fmax(dC, (d & 1) ? cdist(C, Cn) : cdist(Cn, C));
        }
        a.wsr[i] = (float)(1.0 - exp(-(double)a.lam.rk * dC));
        float gsum = 0.0f, tr0 = 0.0f, tr1 = 0.0f, tr2 = 0.0f;
        unsigned gmask = 0;   // bit k: window position k is a temporal pair
        if (a.temporal) {
            Window3 w;
            load_window3(a, x, y, i, w);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                chroma64v(w.I[k][0], w.I[k][1], w.I[k][2], floor_, Cn);
                if (w.ok[k] && cdist(C, Cn) < a.lam.gate) {
                    gsum += 1.0f;
                    tr0 += w.r[k][0];
                    tr1 += w.r[k][1];
                    tr2 += w.r[k][2];
                    gmask |= 1u << k;
                }
            }
        }
        a.tg[i] = gsum;
        a.tg[ps + i] = tr0;
        a.tg[2 * ps + i] = tr1;
        a.tg[3 * ps + i] = tr2;
        a.tg[4 * ps + i] = (float)gmask;   // exact: below 2^9
        if (a.spatial) {
            unsigned smask = 0;
            for (int nb = 0; nb < 8; ++nb) {
                const int xx = x + SP_DX[nb], yy = y + SP_DY[nb];
                if (xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
                const long long j = (long long)yy * W + xx;
                const unsigned long long owner = (unsigned long long)(nb < 4 ? i : j);
                const unsigned long long key = ((unsigned long long)a.spatial_seed << 32) | (4ull * owner + (nb & 3));
                if (splitmix64(key) >> 63) continue;
                float Fj[3];
                load3(F, ps, j, Fj);
                chroma64v(Fj[0], Fj[1], Fj[2], floor_, Cn);
                if (cdist(C, Cn) < a.lam.gate) smask |= 1u << nb;
            }
            a.tg[5 * ps + i] = (float)smask;   // exact: below 2^8
        }
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

// ------------------------------------------------------- halo-staged tiles

// The stencil kernels (GN build, PCG iteration) stage a 66 x 6 halo'd tile of every
// plane they read into LDS with one load phase, then read neighbours from LDS.
constexpr int HW = TX + 2;          // halo'd tile width
constexpr int HH = TYW + 2;         // halo'd tile height (tiles of 64 x 4 pixels)
constexpr int HN = HW * HH;

// IRLS weight of the reflectance-gradient term at halo'd-tile index li, from
// the forward differences that exist (the norm over both directions and all
// channels).  Ul holds the three r planes.
__device__ __forceinline__ float w_rs_lds(const float* Ul, int li, bool hr, bool hd, const Lam& L) {
    float s = 0.0f;
    if (hr) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = Ul[c * HN + li + 1] - Ul[c * HN + li];
            s += d * d;
        }
    }
    if (hd) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = Ul[c * HN + li + HW] - Ul[c * HN + li];
            s += d * d;
        }
    }
    const float nrm = sqrtf(s) + L.eps_irls;
    return (L.p == 1.0f) ? rcp_pos(nrm) : powf(nrm, L.p - 2.0f);
}

// Lambda-scaled weights of the four reflectance-gradient pairs touching the
// pixel (right, down, left, up); zero where the pair does not exist.
__device__ __forceinline__ void rs_pairs_lds(const Args& a, const float* Ul, int li, int x, int y, float wr[4]) {
    const int W = a.W, H = a.H;
    const bool hr = x + 1 < W, hd = y + 1 < H, hl = x > 0, hu = y > 0;
    const float lr = a.lam.rs;
    const float ws = (hr || hd) ? lr * w_rs_lds(Ul, li, hr, hd, a.lam) : 0.0f;
    wr[0] = hr ? ws : 0.0f;
    wr[1] = hd ? ws : 0.0f;
    wr[2] = hl ? lr * w_rs_lds(Ul, li - 1, true, hd, a.lam) : 0.0f;
    wr[3] = hu ? lr * w_rs_lds(Ul, li - HW, hr, true, a.lam) : 0.0f;
}

// Reflectance R = exp(r) and shading S_c = sum_k b_kc T_k of a pixel (Sec. 4),
// the sum as an explicit FMA chain so every kernel forms it identically.
template <int K>
__device__ __forceinline__ void refl_shading(const float* r, const float* T, const Basis<K>& bs, float* R, float* S) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        R[c] = expf(r[c]);
        float sum = 0.0f;
#pragma unroll
        for (int k = 0; k <= K; ++k) sum = fmaf(bs.B[k][c], T[k], sum);
        S[c] = sum;
    }
}

// IRLS weights of the unary layer terms (Sec. 6.4): indirect sparsity (k >= 1)
// and non-negativity (0 for T > 0, else lambda / (|T| + eps)).
__device__ __forceinline__ float w_unary(float T, int k, const Lam& L) {
    const float at = fabsf(T);
    const float wis = (k > 0) ? L.is * rcp_pos(at + L.eps_irls) : 0.0f;
    const float wnn = (T > 0.0f) ? 0.0f : L.nn * rcp_pos(at + L.eps_nn);
    return wis + wnn;
}

// Jacobi diagonal diag(J^T J) of a pixel without its stencil terms: data,
// clustering, temporal pairs, monochromaticity and the unary layer terms.
// Every operation is rounded on its own (no contraction), and the stencil
// terms are added with __fadd_rn, so that the build and the PCG iteration,
// which both rebuild the diagonal from the staged unknowns, agree bit for bit.
template <int K>
__device__ __forceinline__ void diag_unary(const float* R, const float* S, const float* T, float w, float gs,
                                           const Basis<K>& bs, const Lam& L, float* M) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float RS = __fmul_rn(R[c], S[c]);
        M[c] = __fadd_rn(__fadd_rn(__fmul_rn(__fmul_rn(L.data, RS), RS), L.cl), __fmul_rn(L.rc, gs));
    }
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        float Md = 0.0f, Mm = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float RB = __fmul_rn(R[c], bs.B[k][c]);
            Md = __fadd_rn(Md, __fmul_rn(RB, RB));
            Mm = __fadd_rn(Mm, __fmul_rn(bs.Bc[k][c], bs.Bc[k][c]));
        }
        M[3 + k] = __fadd_rn(__fadd_rn(__fmul_rn(L.data, Md), __fmul_rn(__fmul_rn(L.mo, w), Mm)), w_unary(T[k], k, L));
    }
}

// Spatial consistency partners of a pixel from its active-pair mask: adds
// their number to n and their values of the three r-like planes staged at
// V (r for the right-hand side, p for the product) to s.
__device__ __forceinline__ void spatial_partners(const float* V, int li, unsigned mask, float& n, float* s) {
    const int off[8] = {1, HW + 1, HW, HW - 1, -1, -HW - 1, -HW, -HW + 1};
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) {
        if (!((mask >> nb) & 1u)) continue;
        n += 1.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += V[c * HN + li + off[nb]];
    }
}

// ------------------------------------------------------------------ GN build

template <int K>
__device__ __forceinline__ void gn_build_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    constexpr int N = K + 4;
    double* sh4 = reinterpret_cast<double*>(smem);
    float* Ul = reinterpret_cast<float*>(smem + 32);
    if (frame_idle(a)) return;
    Basis<K> bs;
    bs.load(a.bf, a.bcf);
    const Lam L = a.lam;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int li = (ly + 1) * HW + lx + 1;
    const int off[4] = {1, HW, -1, -HW};
    const TileSet tset = tiles_of(a, lc);
    double acc = 0.0;
    for (int tile = tset.c0; tile < tset.c1; tile += tset.step) {
        int tx, ty;
        tile_xy(a, tset, tile, tx, ty);
        const int x0 = tx * TX, y0 = ty * TYW;
        const int x = x0 + lx, y = y0 + ly;
        const bool own_in = x < W && y < H;
        const long long i = own_in ? (long long)y * W + x : 0;   // off-frame: read pixel 0, unused
        // every load of the tile in one batch: the own pixel's per-pixel data, then
        // the two elements of the 66 x 6 unknowns tile this thread stages (the second
        // only for the first 140 threads; off-frame elements read pixel 0, masked)
        float Iv[3];
        load3(a.I, ps, i, Iv);
        const int id = a.ids[i];
        const float w = a.wsr[i];
        float gs = 0.0f, tgr[3] = {0.0f, 0.0f, 0.0f};
        if (a.temporal) {
            gs = a.tg[i];
#pragma unroll
            for (int c = 0; c < 3; ++c) tgr[c] = a.tg[(1 + c) * ps + i];
        }
        const unsigned smask = a.spatial ? (unsigned)a.tg[5 * ps + i] : 0u;
        const int e1 = (int)threadIdx.x + NTHREADS;
        const bool has1 = e1 < HN;
        long long gi[2];
        bool gin[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int idx = h == 0 ? (int)threadIdx.x : (has1 ? e1 : 0);
            const int gx = x0 + idx % HW - 1, gy = y0 + idx / HW - 1;
            gin[h] = gx >= 0 && gx < W && gy >= 0 && gy < H;
            gi[h] = gin[h] ? (long long)gy * W + gx : 0;
        }
        float uv0[N], uv1[N];
#pragma unroll
        for (int v = 0; v < N; ++v) {
            uv0[v] = a.u[v * ps + gi[0]];
            uv1[v] = a.u[v * ps + gi[1]];
        }
        __builtin_amdgcn_sched_barrier(0);   // every load issued before the first store
#pragma unroll
        for (int v = 0; v < N; ++v) Ul[v * HN + threadIdx.x] = gin[0] ? uv0[v] : 0.0f;
        if (has1) {
#pragma unroll
            for (int v = 0; v < N; ++v) Ul[v * HN + e1] = gin[1] ? uv1[v] : 0.0f;
        }
        __syncthreads();
        if (own_in) {
            const bool hv[4] = {x + 1 < W, y + 1 < H, x > 0, y > 0};
            float r[3], T[K + 1];
#pragma unroll
            for (int c = 0; c < 3; ++c) r[c] = Ul[c * HN + li];
#pragma unroll
            for (int k = 0; k <= K; ++k) T[k] = Ul[(3 + k) * HN + li];
            float R[3], S[3], e[3];
            refl_shading<K>(r, T, bs, R, S);
#pragma unroll
            for (int c = 0; c < 3; ++c) e[c] = Iv[c] - R[c] * S[c];
            float g[N], M[N];
            // consistency pairs: their count and the sum of the partners' r (temporal
            // partners from the previous frame, spatial ones from the staged tile)
            if (a.spatial) spatial_partners(Ul, li, smask, gs, tgr);
            diag_unary<K>(R, S, T, w, gs, bs, L, M);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float RS = R[c] * S[c];
                g[c] = L.data * RS * e[c] - L.cl * (r[c] - a.lnb[3 * id + c]) - L.rc * (gs * r[c] - tgr[c]);
            }
            const float mS = (S[0] + S[1] + S[2]) * (1.0f / 3.0f);
            float md[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) md[c] = S[c] - mS;
#pragma unroll
            for (int k = 0; k <= K; ++k) {
                float gd = 0.0f, gm = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float RB = R[c] * bs.B[k][c];
                    gd += RB * e[c];
                    gm += bs.Bc[k][c] * md[c];
                }
                g[3 + k] = L.data * gd - L.mo * w * gm - w_unary(T[k], k, L) * T[k];
            }
            // reflectance sparsity stencil
            float wr[4];
            rs_pairs_lds(a, Ul, li, x, y, wr);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    g[c] -= wr[d] * (r[c] - Ul[c * HN + li + off[d]]);
                    M[c] = __fadd_rn(M[c], wr[d]);
                }
            }
            // smoothness stencil
#pragma unroll
            for (int k = 0; k <= K; ++k) {
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if (!hv[d]) continue;
                    const float tn = Ul[(3 + k) * HN + li + off[d]];
                    const float ws = L.sm * w_pair(T[k], tn, L.eps_irls);
                    g[3 + k] -= ws * (T[k] - tn);
                    M[3 + k] = __fadd_rn(M[3 + k], ws);
                }
            }
            if (st.debug) {
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    a.out[v * ps + i] = g[v];
                    a.out2[v * ps + i] = M[v];
                }
            } else {
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    // the PCG iterations rebuild M from the unknowns, bit for bit, so it is not stored
                    const float mi = 1.0f / M[v];
                    const float z = g[v] * mi;
                    a.pA[v * ps + i] = z;   // x0 = 0 is not stored: iteration 1 starts from zero
                    acc += (double)g[v] * (double)z;
                }
            }
        }
        __syncthreads();
    }
    if (st.debug) return;
    const double vals[1] = {block_sum(acc, sh4)};
    publish(a, lc, R_RZ0, vals, 1);
    if (lead_thread(lc)) a.scal[S_STOP] = 0.0;
}

// ------------------------------------------------------------ PCG iteration

// One Jacobi-PCG iteration i of the layer step per launch, the standard
// recurrence rearranged so that it needs one grid-wide reduction per iteration
// and carried in preconditioned form (z = M^-1 r and M^-1 q are stored instead
// of r and q, so the halo needs no M^-1):
//   i > 0: alpha_{i-1}, beta_{i-1} from the sums of iteration i-1, then
//          x += alpha p_{i-1},  z_i = z_{i-1} - alpha M^-1 q_{i-1},
//          p_i = z_i + beta p_{i-1};
//   all:   q_i = A p_i (J^T W J applied matrix-free from the unknowns), M^-1 q_i
//          stored, and the sums <p_i, q_i>, <q_i, z_i>, <q_i, M^-1 q_i>,
//          <r_i, z_i> (r_i = z_i / M^-1).
// The vector updates are FP32 (the two axpys through FP64, rounded once); p_i
// is recomputed identically on the one-pixel halo of the tile, so the staged
// search direction needs no separate pass.  z0 = p0 is the build's p0.  The last
// iteration's x update is applied by the apply pass.  Debug launches apply A to
// a caller vector.
constexpr int NHALO = 2 * HW + 2 * TYW;   // halo elements of a 64 x 4 tile
static_assert(NHALO <= NTHREADS, "one halo element per thread");

// X1: iteration 1, whose x starts from x0 = 0 (the build stores no x0, so the
// iteration neither reads x nor depends on what the buffer holds).
template <int K, bool X1 = false>
__device__ __forceinline__ void pcg_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    constexpr int N = K + 4;
    double* shr = reinterpret_cast<double*>(smem);             // 4 PV_N doubles
    float* Ul = reinterpret_cast<float*>(smem + 32 * PV_N);    // unknowns (r planes, then T planes)
    float* Pl = Ul + N * HN;                                   // search direction p_i
    // colour basis first: loaded before this kernel's first store, it stays in
    // scalar registers
    Basis<K> bs;
    bs.load(a.bf, a.bcf);
    const bool dbg = st.debug != 0;
    if (!dbg && (a.scal[S_STOP] != 0.0 || frame_idle(a))) return;   // uniform over the grid
    const int it = st.iter;
    const bool first = dbg || it == 0;
    double alpha = 0.0;
    float betaf = 0.0f;
    if (!first) {
        const PcgScalars ps_ = pcg_scalars<true>(a, it - 1, lc.nb, shr);
        if (!ps_.ok) {     // breakdown guard: iteration it-1 is not applied, the layer step ends
            if (lead_thread(lc)) {
                a.scal[S_STOP] = (double)(it + 1);
                a.scal[S_BREAKDOWNS] += 1.0;
                a.scal[S_RZ_LOG + (st.gn & 63)] = ps_.rz;
            }
            return;
        }
        alpha = ps_.alpha;
        if (lead_thread(lc)) a.scal[S_RZ_LOG + (st.gn & 63)] = ps_.rz_next;
        // a residual norm that rounding drove to zero or below restarts the
        // directions (p = z)
        betaf = ps_.rz_next > 0.0 ? (float)(ps_.rz_next / ps_.rz) : 0.0f;
    }
    const float* pdbg = a.pdebug;
    const float* pold = dbg ? pdbg : p_buf(a, first ? 0 : it - 1);
    const float* zold = it <= 1 ? p_buf(a, 0) : z_buf(a, it - 1);     // z0 = p0
    const float* qold = q_buf(a, it - 1);                        // M^-1 q of iteration it-1
    float* pcur = p_buf(a, it);
    float* zcur = z_buf(a, it);
    float* const out = a.out;
    float* qcur = dbg ? out : q_buf(a, it);
    const Lam L = a.lam;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int li = (ly + 1) * HW + lx + 1;
    const int off[4] = {1, HW, -1, -HW};
    // this thread's halo element: the rows above and below the tile, then the
    // left and right columns
    const int ht = (int)threadIdx.x;
    const int hrow = ht < HW ? 0 : (ht < 2 * HW ? TYW + 1 : 1 + ((ht - 2 * HW) >> 1));
    const int hcol = ht < 2 * HW ? ht % HW : (((ht - 2 * HW) & 1) ? HW - 1 : 0);
    const TileSet tset = tiles_of(a, lc);
    double acc[PV_N];
#pragma unroll
    for (int v = 0; v < PV_N; ++v) acc[v] = 0.0;
    for (int tile = tset.c0; tile < tset.c1; tile += tset.step) {
        int tx, ty;
        tile_xy(a, tset, tile, tx, ty);
        const int x0 = tx * TX, y0 = ty * TYW;
        const int x = x0 + lx, y = y0 + ly;
        const bool own_in = x < W && y < H;
        const long long i = (long long)y * W + x;
        // own pixel: unknowns, then the vector updates of this iteration.  Loads
        // are unconditional (an off-frame pixel reads pixel 0 and is masked), and
        // the mode test sits outside the plane loops, so every load of a loop is
        // in flight before the first use.
        const long long io = own_in ? i : 0;
        {
            float uv[N];
#pragma unroll
            for (int v = 0; v < N; ++v) uv[v] = a.u[v * ps + io];
            __builtin_amdgcn_sched_barrier(0);   // every load issued before the first store
#pragma unroll
            for (int v = 0; v < N; ++v) Ul[v * HN + li] = own_in ? uv[v] : 0.0f;
        }
        // z of the own pixel, held through the stencil for the iteration's sums
        float zk[N];
        if (dbg || first) {
            float pv[N];
#pragma unroll
            for (int v = 0; v < N; ++v) pv[v] = pold[v * ps + io];
#pragma unroll
            for (int v = 0; v < N; ++v) {
                zk[v] = dbg ? 0.0f : pv[v];            // z0 = p0
                Pl[v * HN + li] = own_in ? pv[v] : 0.0f;
            }
        } else {
            float po[N], zv[N], qv[N], xv[N];
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const long long j = v * ps + io;
                po[v] = pold[j];
                zv[v] = zold[j];
                qv[v] = qold[j];
                xv[v] = X1 ? 0.0f : a.delta[j];
            }
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const float z = (float)((double)zv[v] - alpha * (double)qv[v]);
                zk[v] = z;
                const float p = fmaf(betaf, po[v], z);
                xv[v] = (float)((double)xv[v] + alpha * (double)po[v]);
                po[v] = p;
                Pl[v * HN + li] = own_in ? p : 0.0f;
            }
            if (own_in) {
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    const long long j = v * ps + i;
                    a.delta[j] = xv[v];
                    zcur[j] = zk[v];
                    pcur[j] = po[v];
                }
            }
        }
        // halo element: unknowns and p only (kept apart from the own pixel's
        // loads, which the scheduler would otherwise interleave past the registers)
        __builtin_amdgcn_sched_barrier(0);
        if (ht < NHALO) {
            const int gx = x0 + hcol - 1, gy = y0 + hrow - 1;
            const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
            const long long gi = in ? (long long)gy * W + gx : 0;
            const int e = hrow * HW + hcol;
            // every load of the element in one batch
            if (first) {
                float uv[N], pv[N];
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    uv[v] = a.u[v * ps + gi];
                    pv[v] = pold[v * ps + gi];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    Ul[v * HN + e] = in ? uv[v] : 0.0f;
                    Pl[v * HN + e] = in ? pv[v] : 0.0f;
                }
            } else {
                float uv[N], po[N], zv[N], qv[N];
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    const long long j = v * ps + gi;
                    uv[v] = a.u[j];
                    po[v] = pold[j];
                    zv[v] = zold[j];
                    qv[v] = qold[j];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    const float z = (float)((double)zv[v] - alpha * (double)qv[v]);
                    Ul[v * HN + e] = in ? uv[v] : 0.0f;
                    Pl[v * HN + e] = in ? fmaf(betaf, po[v], z) : 0.0f;
                }
            }
        }
        __syncthreads();
        if (own_in) {
            const bool hv[4] = {x + 1 < W, y + 1 < H, x > 0, y > 0};
            float p[N], q[N], T[K + 1], R[3], S[3], rv[3];
#pragma unroll
            for (int v = 0; v < N; ++v) p[v] = Pl[v * HN + li];
#pragma unroll
            for (int k = 0; k <= K; ++k) T[k] = Ul[(3 + k) * HN + li];
#pragma unroll
            for (int c = 0; c < 3; ++c) rv[c] = Ul[c * HN + li];
            refl_shading<K>(rv, T, bs, R, S);
            // data term block
            float ac[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float sum = S[c] * p[c];
#pragma unroll
                for (int k = 0; k <= K; ++k) sum += bs.B[k][c] * p[3 + k];
                ac[c] = R[c] * sum;
            }
            float gs = a.temporal ? a.tg[i] : 0.0f;
            float psum[3] = {0.0f, 0.0f, 0.0f};
            if (a.spatial) spatial_partners(Pl, li, (unsigned)a.tg[5 * ps + i], gs, psum);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                q[c] = L.data * R[c] * S[c] * ac[c] + (L.cl + L.rc * gs) * p[c] - L.rc * psum[c];
            // monochrome block and unary layer terms
            const float w = a.wsr[i];
            // Jacobi diagonal, rebuilt as the build formed it (no M^-1 plane is read)
            float M[N];
            diag_unary<K>(R, S, T, w, gs, bs, L, M);
            float m[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float sum = 0.0f;
#pragma unroll
                for (int k = 1; k <= K; ++k) sum += bs.Bc[k][c] * p[3 + k];
                m[c] = sum;
            }
#pragma unroll
            for (int k = 0; k <= K; ++k) {
                float sd = 0.0f, sm = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sd += R[c] * bs.B[k][c] * ac[c];
                    sm += bs.Bc[k][c] * m[c];
                }
                q[3 + k] = L.data * sd + L.mo * w * sm + w_unary(T[k], k, L) * p[3 + k];
            }
            // reflectance sparsity stencil
            float wr[4];
            rs_pairs_lds(a, Ul, li, x, y, wr);
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    q[c] += wr[d] * (p[c] - Pl[c * HN + li + off[d]]);
                    M[c] = __fadd_rn(M[c], wr[d]);
                }
            // smoothness stencil (one layer at a time: unrolling it makes the
            // compiler hoist every layer's LDS reads and double the registers)
#pragma unroll 1
            for (int k = 0; k <= K; ++k) {
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if (!hv[d]) continue;
                    const float ws = L.sm * w_pair(T[k], Ul[(3 + k) * HN + li + off[d]], L.eps_irls);
                    q[3 + k] += ws * (p[3 + k] - Pl[(3 + k) * HN + li + off[d]]);
                    M[3 + k] = __fadd_rn(M[3 + k], ws);
                }
            }
            if (dbg) {
#pragma unroll
                for (int v = 0; v < N; ++v) qcur[v * ps + i] = q[v];
            } else {
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    const float mq = q[v] * (1.0f / M[v]);   // M^-1 q, what the next iteration reads
                    qcur[v * ps + i] = mq;
                    acc[PV_PQ] += (double)p[v] * (double)q[v];
                    acc[PV_QZ] += (double)q[v] * (double)zk[v];
                    acc[PV_QMQ] += (double)q[v] * (double)mq;
                    acc[PV_RZ] += (double)(zk[v] * M[v]) * (double)zk[v];   // r = M z
                }
            }
        }
        __syncthreads();
    }
    if (dbg) return;
    block_sums<PV_N>(acc, shr);
    if (threadIdx.x == 0) {
        double* part = site_ptr(a, pcg_site(it));
#pragma unroll
        for (int v = 0; v < PV_N; ++v) part[(long long)v * lc.nb + lc.lb] = acc[v];
    }
}

// ---------------------------------------------------- apply + base-colour sums

constexpr int BS_BATCH = NTHREADS;   // pixels staged in LDS per round (one per thread)
constexpr int BS_STRIDE = BS_BATCH + 1;   // padded row: rows of one pixel fall in different banks

template <int K>
__device__ __forceinline__ void apply_bsum_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    constexpr int N = K + 4;
    // pixel groups of 3K owner threads (one per Gram row (c, k)), as many as fit a
    // wavefront, so that few lanes idle
    constexpr int GPW = 64 / (3 * K);                 // groups per wavefront
    constexpr int NG = (NTHREADS / 64) * GPW;
    // per staged pixel: R_c and the data residual e_c in FP64, T_k (k >= 1) in FP32
    double* sh4 = reinterpret_cast<double*>(smem);
    double (*Rs)[BS_STRIDE] = reinterpret_cast<double (*)[BS_STRIDE]>(smem + 32);
    double (*Es)[BS_STRIDE] = reinterpret_cast<double (*)[BS_STRIDE]>(smem + 32 + 3 * BS_STRIDE * 8);
    double* red = reinterpret_cast<double*>(smem + 32 + 6 * BS_STRIDE * 8);
    float (*Ts)[BS_STRIDE] = reinterpret_cast<float (*)[BS_STRIDE]>(smem + 32 + 6 * BS_STRIDE * 8 +
                                                                      NG * 3 * K * (K + 1) * 8);
    if (frame_idle(a)) return;
    // x += alpha p of the last PCG iteration (st.iter), applied with the layer step
    // u += x; without PCG iterations x is zero and <r0, z0> is logged
    double alpha = 0.0;
    bool pend = false;
    const double stop0 = a.scal[S_STOP];
    if (st.add_delta && stop0 == 0.0) {
        if (st.iter >= 0) {
            const PcgScalars ps_ = pcg_scalars(a, st.iter, a.nblocks, sh4);
            pend = ps_.ok;
            alpha = ps_.alpha;
            if (lead_thread(lc)) {
                if (!ps_.ok) {   // breakdown guard: the iteration is not applied
                    a.scal[S_STOP] = (double)(st.iter + 2);
                    a.scal[S_BREAKDOWNS] += 1.0;
                }
                if (st.log_rz) a.scal[S_RZ_LOG + (st.gn & 63)] = ps_.ok ? ps_.rz_next : ps_.rz;
            }
        } else if (st.log_rz) {
            const double rz = site_total(a, R_RZ0, 0, a.nblocks, sh4);
            if (lead_thread(lc)) a.scal[S_RZ_LOG + (st.gn & 63)] = rz;
        }
    }
    const float* plast = p_buf(a, st.iter < 0 ? 0 : st.iter);
    // x is in memory once iteration 1 has run its update (x0 = 0 is never
    // stored).  A stop value is 1 + the iteration whose launch refused the update
    // before it (the apply pass counting as iteration P), so 3 or more means
    // iteration 1 ran; every workgroup takes the same decision, whether or not it
    // saw this kernel's own guard.
    const bool xstored = stop0 == 0.0 ? st.iter >= 1 : stop0 >= 3.0;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    // this workgroup's tiles (XCD-aware)
    const TileSet tset = tiles_of(a, lc);
    const int wl = (int)threadIdx.x & 63, wg_in = wl / (3 * K);
    const int grp = ((int)threadIdx.x >> 6) * GPW + wg_in, lane = wl % (3 * K);
    const bool owner = wg_in < GPW;
    const int oc = owner ? lane / K : 0, ok = owner ? lane % K : 0;
    double acc[K + 1];
#pragma unroll
    for (int l = 0; l <= K; ++l) acc[l] = 0.0;
    // the FP64 colours are read where they are used (uniform loads, reissued per
    // batch): held through the tile loop they would take 6K registers
    const double* __restrict__ b64 = a.b64;
    const int rows = TYW * a.ppt;
    const int tile_px = TX * rows;
    for (int tile = tset.c0; tile < tset.c1; tile += tset.step) {
        int tx, ty;
        tile_xy(a, tset, tile, tx, ty);
        for (int base = 0; base < tile_px; base += BS_BATCH) {
            // stage: every thread owns one pixel of the batch
            const int lp = base + threadIdx.x;
            const int x = tx * TX + (lp % TX), y = ty * rows + lp / TX;
            const int sp = threadIdx.x;
            if (x < W && y < H) {
                const long long i = (long long)y * W + x;
                float uv[N], Iv[3];
                if (st.add_delta) {
                    // every load of the pixel in one batch, ahead of the u stores, which
                    // the compiler may not move them past
                    float xv[N], pv[N];
#pragma unroll
                    for (int v = 0; v < N; ++v) {
                        uv[v] = a.u[v * ps + i];
                        xv[v] = a.delta[v * ps + i];
                        pv[v] = plast[v * ps + i];
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) Iv[c] = a.I[c * ps + i];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int v = 0; v < N; ++v) xv[v] = xstored ? xv[v] : 0.0f;
#pragma unroll
                    for (int v = 0; v < N; ++v) {
                        const float x = pend ? (float)((double)xv[v] + alpha * (double)pv[v]) : xv[v];
                        uv[v] = uv[v] + x;
                        a.u[v * ps + i] = uv[v];
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < N; ++v) uv[v] = a.u[v * ps + i];
#pragma unroll
                    for (int c = 0; c < 3; ++c) Iv[c] = a.I[c * ps + i];
                }
                if (st.refine) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double R = exp((double)uv[c]);
                        double S = (double)uv[3];
#pragma unroll
                        for (int k = 0; k < K; ++k) S += b64[3 * k + c] * (double)uv[4 + k];
                        Rs[c][sp] = R;
                        Es[c][sp] = (double)Iv[c] - R * S;
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k) Ts[k][sp] = uv[4 + k];
                }
            } else if (st.refine) {
#pragma unroll
                for (int c = 0; c < 3; ++c) Rs[c][sp] = Es[c][sp] = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) Ts[k][sp] = 0.0f;
            }
            if (!st.refine) continue;
            __syncthreads();
            if (owner) {
                // the whole row k of the Gram block, branch-free so every LDS read of a
                // pixel is in flight at once; entries l < k are discarded at the end
#pragma unroll 2
                for (int px = grp; px < BS_BATCH; px += NG) {
                    const double Rc = Rs[oc][px];
                    float tl[K];
#pragma unroll
                    for (int l = 0; l < K; ++l) tl[l] = Ts[l][px];
                    const double vk = Rc * (double)Ts[ok][px];
                    const double ec = Es[oc][px];
#pragma unroll
                    for (int l = 0; l < K; ++l) acc[l] += vk * (Rc * (double)tl[l]);
                    acc[K] += vk * ec;
                }
            }
            __syncthreads();
        }
    }
    if (!st.refine) return;
    // combine the pixel groups, then publish this workgroup's sums
    if (owner) {
#pragma unroll
        for (int l = 0; l <= K; ++l) red[(grp * 3 * K + lane) * (K + 1) + l] = acc[l];
    }
    __syncthreads();
    const int nb = lc.nb;
    double* part = a.partials + (long long)R_BS * a.part_stride;
    for (int e = threadIdx.x; e < 3 * K * (K + 1); e += NTHREADS) {
        const int jj = e / (K + 1), l = e % (K + 1);
        const int c = jj / K, k = jj % K;
        if (l < K && l < k) continue;
        double sum = 0.0;
        for (int g = 0; g < NG; ++g) sum += red[(g * 3 * K + jj) * (K + 1) + l];
        int idx;
        if (l < K) idx = c * (K * (K + 1) / 2) + (k * K - k * (k - 1) / 2) + (l - k);
        else       idx = 3 * K * (K + 1) / 2 + c * K + k;
        part[(long long)idx * nb + lc.lb] = sum;
    }
}

// ------------------------------------------------------------ colour tables

// Derive the FP32 colours, ln b (FP64 and FP32) and b minus its channel mean
// from the FP64 colours, one wavefront with lane i owning colour entry i
// (3K <= 48 < 64); bval is that lane's FP64 colour.  The only place these
// tables are computed, so a state restored from a checkpoint reproduces them
// bit for bit.
__device__ void colour_tables_to(int K, int lane, double bval, float* bfo, double* lnb64o, float* lnbo, float* bcfo) {
    const int nn = 3 * K;
    const float bf = (float)bval;
    const int k3 = 3 * (lane / 3);
    const float b0 = __shfl(bf, k3, 64), b1 = __shfl(bf, k3 + 1, 64), b2 = __shfl(bf, k3 + 2, 64);
    if (lane < nn) {
        bfo[lane] = bf;
        const double lg = log(bval);
        lnb64o[lane] = lg;
        lnbo[lane] = (float)lg;
        const float mu = (b0 + b1 + b2) * (1.0f / 3.0f);
        bcfo[lane] = bf - mu;
    }
}

__device__ __forceinline__ void colour_tables_wave(const Args& a, int lane, double bval) {
    colour_tables_to(a.K, lane, bval, a.bf, a.lnb64, a.lnb, a.bcf);
}

__device__ __forceinline__ void tables_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    const int lane = (int)threadIdx.x;
    if (lane < 64) colour_tables_wave(a, lane, lane < 3 * a.K ? a.b64[lane] : 1.0);
}

// ------------------------------------------------- learned warm-start judge

// Candidate colours b + db from the network's head and their tables; flags
// whether every component is admissible.  One wavefront.
__device__ __forceinline__ void cand_tables_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    const int lane = (int)threadIdx.x;
    if (lane >= 64) return;
    const bool act = lane < 3 * a.K;
    const double bval = act ? a.b64[lane] + (double)a.dbc[lane] : 1.0;
    const bool bad = act && (!isfinite(bval) || !(bval > 1e-4));
    const bool ok = __ballot(bad) == 0;
    if (act) a.b64c[lane] = bval;
    colour_tables_to(a.K, lane, ok ? bval : 1.0, a.bfc, a.lnb64c, a.lnbc, a.bcfc);
    if (lane == 0) a.scal[S_CAND_OK] = ok ? 1.0 : 0.0;
}

// Keep the network's prediction as the frame's start when its energy is finite
// and lower than the energy at the previous frame's result (and its colours are
// admissible); otherwise leave the state alone.  Every workgroup takes the same
// decision from the two logged totals and copies its own pixels.
__device__ __forceinline__ void judge_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    const double e_prev = a.elog[(long long)JUDGE_PREV_SLOT * ELOG_STRIDE];
    const double e_net = a.elog[(long long)JUDGE_NET_SLOT * ELOG_STRIDE];
    const bool use = a.scal[S_BADIN] == 0.0 && a.scal[S_CAND_OK] != 0.0 && isfinite(e_net) && e_net < e_prev;
    if (lead_thread(lc)) a.scal[S_LEARNED] = use ? 1.0 : 0.0;
    if (!use) return;
    const int n = a.K + 4;
    const long long ps = a.ps;
    for_each_pixel(a, lc, [&](int x, int y, long long i) {
        for (int v = 0; v < n; ++v) a.u[v * ps + i] = a.ucand[v * ps + i];
    });
    if (lc.lb == 0 && threadIdx.x < 64) {
        const int lane = (int)threadIdx.x;
        const bool act = lane < 3 * a.K;
        const double bval = act ? a.b64c[lane] : 1.0;
        if (act) a.b64[lane] = bval;
        colour_tables_wave(a, lane, bval);
    }
}

// -------------------------------------------------------- base-colour solve

// Eight wavefronts: enough to keep the partial loads in flight, and two per SIMD
// leave the solving wavefront registers for a 48 x 48 factor without spilling.
constexpr int BSOLVE_THREADS = 512;

// One workgroup: reduce the per-workgroup sums, assemble the 3K x 3K system of
// the base-colour step, solve it by FP64 Cholesky, apply the guards, update b.
// The base-colour sums from the apply pass's per-workgroup partials, one sum per
// wavefront (four per workgroup; workgroup g of a clip takes sums 4g .. 4g + 3):
// every partial of a sum in one unrolled batch of masked loads (nb <= NB_BS_MAX =
// 64 NCH), then the wavefront butterfly, so each sum is reduced in a fixed order.
// The totals (times lambda_data) go to a.bsum, where the solve reads them.
constexpr int BSR_WAVES = NTHREADS / 64;
template <int K> constexpr int bsum_groups() { return (3 * K * (K + 1) / 2 + 3 * K + BSR_WAVES - 1) / BSR_WAVES; }

template <int K>
__device__ __forceinline__ void bsum_reduce_body(const Args& a, int g) {
    constexpr int NS = 3 * K * (K + 1) / 2 + 3 * K;
    constexpr int NCH = NB_BS_MAX / 64;
    if (frame_idle(a)) return;
    const int lane = threadIdx.x & 63, e = g * BSR_WAVES + (int)(threadIdx.x >> 6);
    if (e >= NS) return;
    const int nb = a.nb_bs;
    const double* row = a.partials + (long long)R_BS * a.part_stride + (long long)e * nb;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NCH; ++j) s += masked_load(row, lane + 64 * j, nb);
    const double t = wave_sum(s);
    if (lane == 0) a.bsum[e] = t * (double)a.lam.data;
}

template <int K>
__device__ __forceinline__ void bsolve_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    constexpr int NA = 3 * K * (K + 1) / 2;
    constexpr int NS = NA + 3 * K;
    constexpr int NN = 3 * K;
    double* sums = reinterpret_cast<double*>(smem);
    double (*Hm)[NN + 1] = reinterpret_cast<double (*)[NN + 1]>(smem + 8 * NS);
    double* gv = reinterpret_cast<double*>(smem + 8 * (NS + NN * (NN + 1)));
    if (frame_idle(a)) return;
    // the sums, reduced from the apply pass's partials by the reduction kernel
    // launched just before (many workgroups while this one solves)
    for (int e = threadIdx.x; e < NS; e += blockDim.x) sums[e] = a.bsum[e];
    __syncthreads();
    if (st.debug) return;   // the raw sums stay published for single-step access
    const double npix = a.bstep_sum ? 1.0 : (double)a.W * (double)a.H;
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
    // H = L L^T and the two triangular solves on one wavefront, in registers:
    // lane i holds row i of H (then of L) and entry i of the right-hand side;
    // column values travel by readlane, so no step waits on LDS.
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    const bool act = lane < NN;
    double h[NN];
#pragma unroll
    for (int k = 0; k < NN; ++k) h[k] = act ? Hm[lane][k] : 0.0;
    double g = act ? gv[lane] : 0.0;
    double trace = 0.0;
#pragma unroll
    for (int k = 0; k < NN; ++k) trace += Hm[k][k];
    bool ok = true;
    // right-looking Cholesky: column j, then the trailing lower triangle; lane j
    // keeps 1 / L_jj so that the substitutions multiply instead of divide
    double rinv = 1.0;
#pragma unroll
    for (int j = 0; j < NN; ++j) {
        double d = rdlane(h[j], j);
        if (!(d > 1e-12 * trace)) { ok = false; d = 1.0; }
        const double ljj = sqrt(d);
        const double r = 1.0 / ljj;
        const double lij = h[j] * r;
        if (lane == j) rinv = r;
        h[j] = (lane == j) ? ljj : (lane > j ? lij : h[j]);
#pragma unroll
        for (int k = j + 1; k < NN; ++k) {
            const double lkj = rdlane(lij, k);
            if (lane >= k) h[k] -= lij * lkj;
        }
    }
    // L y = g: lane j finishes y_j, every later lane i subtracts L_ij y_j (its own h[j])
#pragma unroll
    for (int j = 0; j < NN; ++j) {
        const double yj = rdlane(g * rinv, j);
        g = (lane == j) ? yj : (lane > j ? g - h[j] * yj : g);
    }
    // L^T x = y: lane i needs column i of L (L_ji for j > i), transposed once
    // through LDS (the Gram matrix's space, no longer needed)
    if (act) {
#pragma unroll
        for (int k = 0; k < NN; ++k)
            if (k <= lane) Hm[lane][k] = h[k];
    }
    __threadfence_block();
    double lt[NN];
#pragma unroll
    for (int j = 0; j < NN; ++j) lt[j] = (act && j > lane) ? Hm[j][lane] : 0.0;
#pragma unroll
    for (int j = NN - 1; j >= 0; --j) {
        const double xj = rdlane(g * rinv, j);
        g = (lane == j) ? xj : (lane < j ? g - lt[j] * xj : g);
    }
    // guards: a non-positive pivot, or a colour that would leave (1e-4, inf)
    const double bold = act ? a.b64[lane] : 1.0;
    const double bnew = bold + g;
    const bool bad = act && (!isfinite(bnew) || !(bnew > 1e-4));
    ok = ok && __ballot(bad) == 0;
    if (ok) {
        if (act) a.b64[lane] = bnew;
        colour_tables_wave(a, lane, bnew);
    }
    if (lane == 0) {
        if (ok) {
            a.scal[S_BACCEPT] = 1.0;
        } else {
            a.scal[S_BACCEPT] = 0.0;
            a.scal[S_BREJECT] += 1.0;
        }
    }
}

// --------------------------------------------------------------- FP64 energy

template <int K>
__device__ __forceinline__ void energy_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    double* sh4 = reinterpret_cast<double*>(smem);
    if (frame_idle(a)) return;
    const long long ps = a.ps;
    const int W = a.W, H = a.H;
    double e[NTERMS];
#pragma unroll
    for (int v = 0; v < NTERMS; ++v) e[v] = 0.0;
    const double p = a.lam.p;
    double Bk[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) Bk[k][c] = a.b64[3 * k + c];
    for_each_pixel(a, lc, [&](int x, int y, long long i) {
        constexpr int N = K + 4;
        // the pixel and its right and lower neighbours (loaded unconditionally,
        // the centre standing in for a missing neighbour)
        const bool hr = x + 1 < W, hd = y + 1 < H;
        const long long ir = hr ? i + 1 : i, id_ = hd ? i + W : i;
        float uc[N], ur[N], ud[N], Ic[3];
#pragma unroll
        for (int v = 0; v < N; ++v) {
            uc[v] = a.u[v * ps + i];
            ur[v] = a.u[v * ps + ir];
            ud[v] = a.u[v * ps + id_];
        }
        load3(a.I, ps, i, Ic);
        double r[3], T[K + 1];
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = uc[c];
#pragma unroll
        for (int k = 0; k <= K; ++k) T[k] = uc[3 + k];
        const int id = a.ids[i];
        double S[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double s = T[0];
#pragma unroll
            for (int k = 0; k < K; ++k) s += Bk[k][c] * T[k + 1];
            S[c] = s;
            const double d = (double)Ic[c] - exp(r[c]) * s;
            e[0] += d * d;
            const double dc = r[c] - a.lnb64[3 * id + c];
            e[1] += dc * dc;
        }
        // reflectance-gradient norm (forward differences)
        double g2 = 0.0;
        if (hr) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { const double d = (double)ur[c] - r[c]; g2 += d * d; }
        }
        if (hd) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { const double d = (double)ud[c] - r[c]; g2 += d * d; }
        }
        const double gn = sqrt(g2);
        e[2] += (p == 1.0) ? gn : ((gn > 0.0) ? pow(gn, p) : 0.0);
        if (a.temporal) {
            // the frame's pairs as the precompute pass found them (same gate test)
            const unsigned gmask = (unsigned)a.tg[4 * ps + i];
            float rp[9][3];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int yy = y + k / 3 - 1, xx = x + k % 3 - 1;
                const bool ok = yy >= 0 && yy < H && xx >= 0 && xx < W;
                const long long jj = ok ? (long long)yy * W + xx : i;
#pragma unroll
                for (int c = 0; c < 3; ++c) rp[k][c] = a.rprev[c * ps + jj];
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                if ((gmask >> k) & 1u) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double d = r[c] - (double)rp[k][c];
                        e[3] += d * d;
                    }
                }
            }
        }
        if (a.spatial) {
            // the pixel's own (forward) spatial pairs, so every pair counts once
            const unsigned smask = (unsigned)a.tg[5 * ps + i];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                if (!((smask >> nb) & 1u)) continue;
                const long long jj = (long long)(y + SP_DY[nb]) * W + (x + SP_DX[nb]);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double d = r[c] - (double)a.u[c * ps + jj];
                    e[3] += d * d;
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
            if (hr) e[6] += fabs((double)ur[3 + k] - T[k]);
            if (hd) e[6] += fabs((double)ud[3 + k] - T[k]);
            e[7] += fmax(-T[k], 0.0);
        }
    });
    const Lam L = a.lam;
    const double lam[NTERMS] = {L.data, L.cl, L.rs, L.rc, L.mo, L.is, L.sm, L.nn};
    double vals[NTERMS];
#pragma unroll
    for (int v = 0; v < NTERMS; ++v) vals[v] = block_sum(e[v] * lam[v], sh4);
    publish(a, lc, R_EN, vals, NTERMS);
}

// One workgroup: total the energy partials of the preceding k_energy launch
// (nb workgroups) into an energy-log slot.
__device__ __forceinline__ void energy_finish_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    const int nb = a.nblocks;
    double* sh4 = reinterpret_cast<double*>(smem);
    if (frame_idle(a)) return;
    double tot[NTERMS];
    site_totals<NTERMS>(a, R_EN, nb, sh4, tot);
    if (threadIdx.x == 0) {
        double* slot = a.elog + (long long)st.slot * ELOG_STRIDE;
        double s = 0.0;
        for (int v = 0; v < NTERMS; ++v) {
            slot[1 + v] = tot[v];
            s += tot[v];
        }
        slot[0] = s;
        if (st.check) {
            // energy-target mode: this outer iteration is done; its energy is
            // also the frame's final energy unless a later iteration runs
            double* fin = a.elog + (long long)ELOG_FINAL_SLOT * ELOG_STRIDE;
            for (int v = 0; v <= NTERMS; ++v) fin[v] = slot[v];
            a.scal[S_GN_DONE] = (double)(st.gn + 1);   // outer iterations run so far
            if (s <= a.scal[S_TARGET]) a.scal[S_DONE] = 1.0;
        }
    }
}

// -------------------------------------------------------------------- output

template <int K>
__device__ __forceinline__ void output_body(const Args& a, const Lc& lc, const Step& st, char* smem) {
    constexpr int N = K + 4;
    if (a.scal[S_BADIN] != 0.0) return;
    // the frame is over: single-step calls after it must not see its stop flag
    if (lead_thread(lc)) a.scal[S_DONE] = 0.0;
    const long long ps = a.ps;
    for_each_pixel(a, lc, [&](int x, int y, long long i) {
        // every load ahead of the stores, which the compiler may not move them past
        float uv[N], Iv[3];
#pragma unroll
        for (int v = 0; v < N; ++v) uv[v] = a.u[v * ps + i];
        load3(a.I, ps, i, Iv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.rprev[c * ps + i] = uv[c];
            a.Iprev[c * ps + i] = Iv[c];
        }
        if (a.out) {
#pragma unroll
            for (int c = 0; c < 3; ++c) a.out[c * ps + i] = expf(uv[c]);
#pragma unroll
            for (int v = 3; v < N; ++v) a.out[v * ps + i] = uv[v];
        }
    });
}

// --------------------------------------------------------- LDS footprints

constexpr size_t LDS_SMALL = 32;
template <int K> constexpr size_t lds_gn_build() { return 32 + sizeof(float) * (K + 4) * HN; }
template <int K> constexpr size_t lds_pcg() { return 32 * PV_N + sizeof(float) * 2 * (K + 4) * HN; }
template <int K> constexpr size_t lds_apply_bsum() {
    return 32 + 6 * BS_STRIDE * 8 + (NTHREADS / 64) * (64 / (3 * K)) * 3 * K * (K + 1) * 8 +
           sizeof(float) * K * BS_STRIDE;
}
template <int K> constexpr size_t lds_bsolve() {
    return 8 * (3 * K * (K + 1) / 2 + 3 * K + 3 * K * (3 * K + 1) + 3 * K);
}

// ------------------------------------------------------------------ wrappers

// Workgroup -> clip of a batched launch (wg: prefix of per-clip workgroup counts).
__device__ __forceinline__ int clip_index(const int* wg, int nclips) {
    int c = 0;
    while (c + 1 < nclips && (int)blockIdx.x >= wg[c + 1]) ++c;
    return c;
}

__device__ __forceinline__ Lc clip_grid(const int* wg, int c) {
    const int nb = wg[c + 1] - wg[c];
    return Lc{xcd_order((int)blockIdx.x - wg[c], nb), nb};
}

#define GID_PIXEL_KERNELS(NAME, ATTR, WG)                                                          \
    template <int K>                                                                               \
    __global__ __launch_bounds__(NTHREADS) ATTR(K) void k_##NAME(Args a, Step st) {                \
        extern __shared__ __align__(16) char smem[];                                               \
        NAME##_body<K>(a, whole_grid(), st, smem);                                                 \
    }                                                                                              \
    template <int KB>                                                                              \
    __global__ __launch_bounds__(NTHREADS) ATTR(KB) void kb_##NAME(const BatchArgs ba, Step st) {  \
        extern __shared__ __align__(16) char smem[];                                               \
        const int c = clip_index(ba.WG, ba.n);                                                     \
        NAME##_body<KB>(ba.a[c], clip_grid(ba.WG, c), st, smem);                                   \
    }

// Occupancy targets.  The PCG iteration's LDS tile limits a CU to lds_waves<K>()
// workgroups (one wavefront of each per SIMD).  For K <= 8 the allocator is held
// to that occupancy, at most six waves per SIMD for K <= 3 and five above (the
// registers that the PCG iteration holds through its stencil do not fit the 80 of
// six waves from K = 4 on); for larger K the natural allocation is kept.
template <int K> constexpr int lds_waves() {
    constexpr int w = (int)((160 * 1024) / lds_pcg<K>());
    return w > 8 ? 8 : (w < 1 ? 1 : w);
}
template <int K> constexpr int mv_waves() {
    constexpr int cap = K <= 3 ? 6 : 5;
    return K <= 8 ? (lds_waves<K>() < cap ? lds_waves<K>() : cap) : 1;
}
#define GID_NO_ATTR(T)
// energy: 170 VGPRs at K = 10 left two waves per SIMD, so the pixel grid's three
// workgroups per CU ran in one and a half waves of workgroups; held to three waves
// (168 VGPRs, no spills up to K = 10) it takes 73 us at 1920x1080 K = 10 (84 us
// before).  Larger K keep the compiler's allocation.  The precompute is not held:
// at three waves it spills from K = 8 on.
#define GID_W3_ATTR(T) __attribute__((amdgpu_waves_per_eu((T) <= 10 ? 3 : 1)))
#define GID_GN_ATTR(T) __attribute__((amdgpu_waves_per_eu(4)))
#define GID_MV_ATTR(T) __attribute__((amdgpu_waves_per_eu(mv_waves<T>())))

GID_PIXEL_KERNELS(precompute, GID_NO_ATTR, wg_pix)
GID_PIXEL_KERNELS(gn_build, GID_GN_ATTR, wg_pix)
GID_PIXEL_KERNELS(pcg, GID_MV_ATTR, wg_pix)
// iteration 1 (x starts from zero)
template <int K>
__global__ __launch_bounds__(NTHREADS) GID_MV_ATTR(K) void k_pcg1(Args a, Step st) {
    extern __shared__ __align__(16) char smem[];
    pcg_body<K, true>(a, whole_grid(), st, smem);
}
template <int KB>
__global__ __launch_bounds__(NTHREADS) GID_MV_ATTR(KB) void kb_pcg1(const BatchArgs ba, Step st) {
    extern __shared__ __align__(16) char smem[];
    const int c = clip_index(ba.wg_pix, ba.n);
    pcg_body<KB, true>(ba.a[c], clip_grid(ba.wg_pix, c), st, smem);
}
GID_PIXEL_KERNELS(apply_bsum, GID_NO_ATTR, wg_bs)
GID_PIXEL_KERNELS(energy, GID_W3_ATTR, wg_pix)
GID_PIXEL_KERNELS(output, GID_NO_ATTR, wg_pix)

__global__ __launch_bounds__(NTHREADS) void k_scan(Args a, Step st) {
    extern __shared__ __align__(16) char smem[];
    scan_body(a, whole_grid(), st, smem);
}
__global__ __launch_bounds__(NTHREADS) void kb_scan(const BatchArgs ba, Step st) {
    extern __shared__ __align__(16) char smem[];
    const int c = clip_index(ba.wg_pix, ba.n);
    scan_body(ba.a[c], clip_grid(ba.wg_pix, c), st, smem);
}

template <int K>
__global__ __launch_bounds__(NTHREADS) void k_bsum_reduce(Args a, Step st) {
    bsum_reduce_body<K>(a, (int)blockIdx.x);
}
// bsum_groups<KB>() workgroups per clip
template <int KB>
__global__ __launch_bounds__(NTHREADS) void kb_bsum_reduce(const BatchArgs ba, Step st) {
    constexpr int G = bsum_groups<KB>();
    bsum_reduce_body<KB>(ba.a[blockIdx.x / G], (int)(blockIdx.x % G));
}

// one workgroup per clip
template <int K>
__global__ __launch_bounds__(BSOLVE_THREADS) void k_bsolve(Args a, Step st) {
    extern __shared__ __align__(16) char smem[];
    bsolve_body<K>(a, Lc{0, 1}, st, smem);
}
template <int KB>
__global__ __launch_bounds__(BSOLVE_THREADS) void kb_bsolve(const BatchArgs ba, Step st) {
    extern __shared__ __align__(16) char smem[];
    bsolve_body<KB>(ba.a[blockIdx.x], Lc{0, 1}, st, smem);
}
__global__ __launch_bounds__(NTHREADS) void k_energy_finish(Args a, Step st) {
    extern __shared__ __align__(16) char smem[];
    energy_finish_body(a, Lc{0, 1}, st, smem);
}
__global__ __launch_bounds__(NTHREADS) void kb_energy_finish(const BatchArgs ba, Step st) {
    extern __shared__ __align__(16) char smem[];
    energy_finish_body(ba.a[blockIdx.x], Lc{0, 1}, st, smem);
}
__global__ void k_tables(Args a, Step st) { tables_body(a, Lc{0, 1}, st, nullptr); }
__global__ void k_cand_tables(Args a, Step st) { cand_tables_body(a, Lc{0, 1}, st, nullptr); }
__global__ __launch_bounds__(NTHREADS) void k_judge(Args a, Step st) { judge_body(a, whole_grid(), st, nullptr); }

}  // namespace

#ifndef GID_KERNELS_ONLY
// ------------------------------------------------------------------ launchers

namespace {
template <typename Fn>
hipError_t with_K(int K, Fn&& fn) {
    switch (K) {
#define GID_CASE(V) case V: fn(std::integral_constant<int, V>{}); break;
        GID_CASE(1) GID_CASE(2) GID_CASE(3) GID_CASE(4) GID_CASE(5) GID_CASE(6) GID_CASE(7) GID_CASE(8)
        GID_CASE(9) GID_CASE(10) GID_CASE(11) GID_CASE(12) GID_CASE(13) GID_CASE(14) GID_CASE(15) GID_CASE(16)
#undef GID_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_kernel(Kern k, const Args& a, const Step& st, hipStream_t s) {
    const dim3 blk(NTHREADS), grid(a.nblocks);
    switch (k) {
        case KN_SCAN:
            hipLaunchKernelGGL(k_scan, grid, blk, LDS_SMALL, s, a, st);
            return hipGetLastError();
        case KN_ENERGY_FINISH:
            hipLaunchKernelGGL(k_energy_finish, dim3(1), blk, LDS_SMALL, s, a, st);
            return hipGetLastError();
        case KN_CAND_TABLES:
            hipLaunchKernelGGL(k_cand_tables, dim3(1), dim3(64), 0, s, a, st);
            return hipGetLastError();
        case KN_JUDGE:
            hipLaunchKernelGGL(k_judge, dim3(a.nblocks), dim3(NTHREADS), 0, s, a, st);
            return hipGetLastError();
        case KN_TABLES:
            hipLaunchKernelGGL(k_tables, dim3(1), dim3(64), 0, s, a, st);
            return hipGetLastError();
        default:
            break;
    }
    return with_K(a.K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        switch (k) {
            case KN_PRECOMPUTE: hipLaunchKernelGGL(k_precompute<KK>, grid, blk, LDS_SMALL, s, a, st); break;
            case KN_GN_BUILD: hipLaunchKernelGGL(k_gn_build<KK>, grid, blk, lds_gn_build<KK>(), s, a, st); break;
            case KN_PCG:
                if (st.iter == 1 && !st.debug)
                    hipLaunchKernelGGL(k_pcg1<KK>, grid, blk, lds_pcg<KK>(), s, a, st);
                else
                    hipLaunchKernelGGL(k_pcg<KK>, grid, blk, lds_pcg<KK>(), s, a, st);
                break;
            case KN_APPLY_BSUM:
                hipLaunchKernelGGL(k_apply_bsum<KK>, dim3(a.nb_bs), blk, lds_apply_bsum<KK>(), s, a, st);
                break;
            case KN_BSOLVE:   // the sums' reduction, then the solve
                hipLaunchKernelGGL(k_bsum_reduce<KK>, dim3(bsum_groups<KK>()), blk, 0, s, a, st);
                hipLaunchKernelGGL(k_bsolve<KK>, dim3(1), dim3(BSOLVE_THREADS), lds_bsolve<KK>(), s, a, st);
                break;
            case KN_ENERGY: hipLaunchKernelGGL(k_energy<KK>, grid, blk, LDS_SMALL, s, a, st); break;
            case KN_OUTPUT: hipLaunchKernelGGL(k_output<KK>, grid, blk, LDS_SMALL, s, a, st); break;
            default: break;
        }
    });
}

hipError_t launch_batch(Kern k, const BatchGrid& g, const Step& st, hipStream_t s) {
    const dim3 blk(NTHREADS), gpix(g.total_pix), gbs(g.total_bs), gone(g.ba.n);
    switch (k) {
        case KN_SCAN:
            hipLaunchKernelGGL(kb_scan, gpix, blk, LDS_SMALL, s, g.ba, st);
            return hipGetLastError();
        case KN_ENERGY_FINISH:
            hipLaunchKernelGGL(kb_energy_finish, gone, blk, LDS_SMALL, s, g.ba, st);
            return hipGetLastError();
        default:
            break;
    }
    return with_K(g.k, [&](auto kc) {
        constexpr int KB = decltype(kc)::value;
        switch (k) {
            case KN_PRECOMPUTE:
                hipLaunchKernelGGL(kb_precompute<KB>, gpix, blk, LDS_SMALL, s, g.ba, st);
                break;
            case KN_GN_BUILD:
                hipLaunchKernelGGL(kb_gn_build<KB>, gpix, blk, lds_gn_build<KB>(), s, g.ba, st);
                break;
            case KN_PCG:
                if (st.iter == 1 && !st.debug)
                    hipLaunchKernelGGL(kb_pcg1<KB>, gpix, blk, lds_pcg<KB>(), s, g.ba, st);
                else
                    hipLaunchKernelGGL(kb_pcg<KB>, gpix, blk, lds_pcg<KB>(), s, g.ba, st);
                break;
            case KN_APPLY_BSUM:
                hipLaunchKernelGGL(kb_apply_bsum<KB>, gbs, blk, lds_apply_bsum<KB>(), s, g.ba, st);
                break;
            case KN_BSOLVE:
                hipLaunchKernelGGL(kb_bsum_reduce<KB>, dim3(g.ba.n * bsum_groups<KB>()), blk, 0, s, g.ba, st);
                hipLaunchKernelGGL(kb_bsolve<KB>, gone, dim3(BSOLVE_THREADS), lds_bsolve<KB>(), s, g.ba, st);
                break;
            case KN_ENERGY:
                hipLaunchKernelGGL(kb_energy<KB>, gpix, blk, LDS_SMALL, s, g.ba, st);
                break;
            case KN_OUTPUT:
                hipLaunchKernelGGL(kb_output<KB>, gpix, blk, LDS_SMALL, s, g.ba, st);
                break;
            default: break;
        }
    });
}

hipError_t launch_table(Kern k, const TableGrid& g, const Step& st, hipStream_t s) {
    if (g.n < 1 || g.n > TABLE_CLIPS_MAX || g.kmax < 1 || g.kmax > KMAX || (g.kmask >> (g.kmax + 1)) != 0)
        return hipErrorInvalidValue;
    if (g.kmax <= 4) return launch_table4(k, g, st, s);
    if (g.kmax <= 8) return launch_table8(k, g, st, s);
    if (g.kmax <= 12) return launch_table12(k, g, st, s);
    return launch_table16(k, g, st, s);
}

#endif  // GID_KERNELS_ONLY

}  // namespace gid
