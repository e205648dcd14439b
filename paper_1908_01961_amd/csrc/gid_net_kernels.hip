// Kernels of the learned warm start: a six-layer 3x3 convolutional network
// (32 channels, ReLU, BF16 weights and activations, FP32 accumulation) that
// predicts the change of the unknowns and of the base colours from one frame to
// the next.  The network is this project's own component; the paper names
// learned priors only as future work (Sec. 9).
//
// Every convolution is an implicit GEMM on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16): M = 16 pixels, N = 16 output channels, and the
// 32-long reduction is the 32 input channels of one filter tap, so a 3x3
// layer is 9 accumulating MFMAs per 16 x 16 output block.  Activations are
// stored pixel-major with 32 BF16 channels (64 bytes per pixel), which makes
// one 16-byte load per lane exactly one MFMA operand fragment:
//   A (16 x 32):  lane l holds row l % 16, k = 8 (l / 16) + j, j = 0..7
//   B (32 x 16):  lane l holds k = 8 (l / 16) + j, column l % 16
//   D (16 x 16):  lane l holds rows 4 (l / 16) + i, i = 0..3, column l % 16
// A wavefront covers a strip of 64 pixels of one row (four M blocks) and keeps
// the whole layer's B fragments (9 taps x N blocks) in registers; the four
// wavefronts of a workgroup share an LDS copy of their input rows.
//
// Reductions (pooling, loss, weight gradients) are deterministic: every
// wavefront or workgroup writes its own partial, a consumer sums them in index
// order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gid_net_internal.h"

namespace gidnet {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
    return z;
}

__device__ __forceinline__ bf16x8 load8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// Sum over the four lanes that share a D column (lanes c, c + 16, c + 32, c + 48).
__device__ __forceinline__ float col_sum(float v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------ convolution

// A tile's four rows (one per wavefront) read a 6-row x 66-pixel halo tile of
// the input, staged in LDS with coalesced 16-byte loads; every
// A fragment is then one conflict-free 128-bit LDS read (16 lanes cover 16
// consecutive pixels = 1 KiB).  MODE selects the epilogue at compile time.
constexpr int TROWS = CONV_ROWS + 2, TCOLS = STRIP + 2;

// Staged 16-byte elements of one tile, and per thread.
constexpr int NSE = TROWS * TCOLS * 4;
constexpr int SPT = (NSE + CONV_THREADS - 1) / CONV_THREADS;

// Issue the loads of tile t's staged input (off-frame elements are zero).
__device__ __forceinline__ void conv_stage_load(const ConvArgs& a, int t, int nsx, bf16x8* stg) {
    const int y0 = (t / nsx) * CONV_ROWS, x0 = (t % nsx) * STRIP;
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int e = (int)threadIdx.x + j * CONV_THREADS;
        const int q = e & 3, col = (e >> 2) % TCOLS, row = (e >> 2) / TCOLS;
        const int yy = y0 + row - 1, xx = x0 + col - 1;
        stg[j] = (e < NSE && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                     ? load8(a.in + ((long long)yy * a.W + xx) * C + 8 * q)
                     : zero8();
    }
}

__device__ __forceinline__ void conv_stage_store(__bf16 (*buf)[TCOLS][C], const bf16x8* stg) {
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int e = (int)threadIdx.x + j * CONV_THREADS;
        if (e >= NSE) continue;
        const int q = e & 3, col = (e >> 2) % TCOLS, row = (e >> 2) / TCOLS;
        *reinterpret_cast<bf16x8*>(&buf[row][col][8 * q]) = stg[j];
    }
}

// A resident workgroup takes tiles blockIdx.x, blockIdx.x + gridDim.x, ... and
// double-buffers their staged input: the next tile's loads are in flight while
// the current tile's MFMAs and epilogue run.  The weights are loaded once.
// Every tile's arithmetic and partial sums are those of one workgroup per tile.
template <int NB, int MODE>
__global__ __launch_bounds__(CONV_THREADS) void k_conv(ConvArgs a) {
    __shared__ __align__(16) __bf16 tiles[2][TROWS][TCOLS][C];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int W = a.W, H = a.H;
    const int nsx = (W + STRIP - 1) / STRIP;
    const int ntiles = nsx * ((H + CONV_ROWS - 1) / CONV_ROWS);
    bf16x8 bw[9][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bw[t][nb] = load8(a.w + ((t * C + nb * 16 + r16) * C + 8 * kq));
    bf16x8 stg[SPT];
    int t = blockIdx.x;
    if (t < ntiles) {
        conv_stage_load(a, t, nsx, stg);
        conv_stage_store(tiles[0], stg);
    }
    __syncthreads();
    for (int buf = 0; t < ntiles; t += gridDim.x, buf ^= 1) {
        const int tn = t + (int)gridDim.x;
        if (tn < ntiles) conv_stage_load(a, tn, nsx, stg);   // in flight through this tile
        __bf16 (*tile)[TCOLS][C] = tiles[buf];
        const long long wave_id = (long long)t * CONV_ROWS + wv;
        const int y0 = (t / nsx) * CONV_ROWS, x0 = (t % nsx) * STRIP;
        const int y = y0 + wv;
        const bool rowin = y < H;
        // masked gradient: the ReLU mask of the pixel this lane stores in the epilogue,
        // loaded now as four 16-byte loads (its latency hides behind the MFMAs)
        bf16x8 mk[4];
        if constexpr (MODE == M_MASK) {
            const int xp = x0 + lane;
            const bool in = rowin && xp < W;
            const long long px = in ? (long long)y * W + xp : 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) mk[q] = in ? load8(a.mask + px * C + 8 * q) : zero8();
        }
        float pool[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) pool[nb] = 0.0f;
        double lacc = 0.0;
        f32x4 acc[4][NB];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const bf16x8 av = *reinterpret_cast<const bf16x8*>(&tile[wv + dy][16 * m + r16 + dx][8 * kq]);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[dy * 3 + dx][nb], acc[m][nb], 0, 0, 0);
                }
        // epilogue: pixel x0 + 16 m + 4 kq + i, channel 16 nb + r16
        constexpr bool NHWC_OUT = MODE == M_RELU || MODE == M_LOSS || MODE == M_MASK;
        if constexpr (NHWC_OUT) {
            // values to BF16 in this wavefront's 64 x 32 block of the (no longer needed)
            // input tile, then each lane stores one pixel's 64 bytes with four 16-byte stores
            static_assert(NB == 2, "pixel-major outputs carry all 32 channels");
            __syncthreads();
            __bf16* blk = &tile[0][0][0] + wv * STRIP * C;
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int lp = 16 * m + 4 * kq + i, xp = x0 + lp;
                    const bool in = rowin && xp < W;
                    const long long px = (long long)y * W + xp;
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        const int o = 16 * nb + r16;
                        const float v = acc[m][nb][i];
                        __bf16 r;
                        if constexpr (MODE == M_RELU) {
                            r = (__bf16)fmaxf(v + a.bias[o], 0.0f);
                            if (in) pool[nb] += (float)r;
                        } else if constexpr (MODE == M_LOSS) {
                            float g = 0.0f;
                            if (in && o < a.nout) {
                                const float e = (v + a.bias[o]) - a.tgt[o * a.ps + px];
                                g = e * a.gscale;
                                lacc += (double)e * (double)e;
                            }
                            r = (__bf16)g;
                        } else {
                            const float sv = v + (a.addc ? a.addc[o] : 0.0f);
                            r = (__bf16)(in ? sv : 0.0f);   // masked below, per stored pixel
                        }
                        blk[lp * C + o] = r;
                    }
                }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int xp = x0 + lane;
            if (rowin && xp < W) {
                const long long px = (long long)y * W + xp;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bf16x8 v = *reinterpret_cast<const bf16x8*>(blk + lane * C + 8 * q);
                    if constexpr (MODE == M_MASK) {
#pragma unroll
                        for (int j = 0; j < 8; ++j)
                            if (!((float)mk[q][j] > 0.0f)) v[j] = (__bf16)0.0f;
                    }
                    *reinterpret_cast<bf16x8*>(a.out_b + px * C + 8 * q) = v;
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int o = 16 * nb + r16;
                    const int xb = x0 + 16 * m + 4 * kq;
                    if (!rowin) continue;
                    const long long pb = (long long)y * W + xb;
                    if constexpr (MODE == M_ADD) {
                        if (o >= a.nout) continue;
                        const float bo = a.bias[o];
                        if ((W & 3) == 0 && xb + 3 < W) {
                            const float4 up = *reinterpret_cast<const float4*>(a.uprev + o * a.ps + pb);
                            float4 r;
                            r.x = up.x + (acc[m][nb][0] + bo);
                            r.y = up.y + (acc[m][nb][1] + bo);
                            r.z = up.z + (acc[m][nb][2] + bo);
                            r.w = up.w + (acc[m][nb][3] + bo);
                            *reinterpret_cast<float4*>(a.out_f + o * a.ps + pb) = r;
                        } else {
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                if (xb + i < W) a.out_f[o * a.ps + pb + i] = a.uprev[o * a.ps + pb + i] + (acc[m][nb][i] + bo);
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (xb + i < W) a.out_f[(pb + i) * C + o] = acc[m][nb][i] + a.bias[o];
                    }
                }
            }
        }
        if constexpr (MODE == M_RELU) {
            if (a.pool_part) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const float s = col_sum(pool[nb]);
                    if (kq == 0) a.pool_part[wave_id * C + 16 * nb + r16] = s;
                }
                if (NB == 1 && kq == 0) a.pool_part[wave_id * C + 16 + r16] = 0.0f;
            }
        }
        if constexpr (MODE == M_LOSS) {
            if (a.loss_part) {
                const double s = wave_sum64(lacc);
                if (lane == 0) a.loss_part[wave_id] = s;
            }
        }
        // the next tile's input into the other buffer (last read before the previous
        // barrier); the barrier also ends this tile's use of its buffer
        if (tn < ntiles) conv_stage_store(tiles[buf ^ 1], stg);
        __syncthreads();
    }
}

// ------------------------------------------------------- weight gradients

// gW[o][c][tap] = sum_px gy[px][o] x[px + off(tap)][c]: the pixels are the
// MFMA reduction dimension.  A workgroup stages a 64-pixel row strip of gy and
// the matching 3 x 66 halo of x in LDS; wavefront w owns the 16 x 16 block
// (o block w / 2, c block w % 2) for all nine taps and accumulates over every
// strip the workgroup visits.
__global__ __launch_bounds__(CONV_THREADS) void k_wgrad(WgradArgs a) {
    __shared__ __bf16 xs[3][STRIP + 2][C];
    __shared__ __bf16 gs[STRIP][C];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    const int ob = wv >> 1, cb = wv & 1;
    const int W = a.W, H = a.H;
    const int nsx = (W + STRIP - 1) / STRIP;
    const int ntiles = nsx * H;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float gb = 0.0f;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int y = tile / nsx, x0 = (tile % nsx) * STRIP;
        for (int e = threadIdx.x; e < 3 * (STRIP + 2) * 4; e += CONV_THREADS) {
            const int q = e & 3, px = (e >> 2) % (STRIP + 2), row = (e >> 2) / (STRIP + 2);
            const int yy = y + row - 1, xx = x0 + px - 1;
            const bf16x8 v = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                                 ? load8(a.x + ((long long)yy * W + xx) * C + 8 * q)
                                 : zero8();
            *reinterpret_cast<bf16x8*>(&xs[row][px][8 * q]) = v;
        }
        {
            const int q = threadIdx.x & 3, px = threadIdx.x >> 2;
            const int xx = x0 + px;
            const bf16x8 v = xx < W ? load8(a.gy + ((long long)y * W + xx) * C + 8 * q) : zero8();
            *reinterpret_cast<bf16x8*>(&gs[px][8 * q]) = v;
        }
        __syncthreads();
#pragma unroll
        for (int ch = 0; ch < STRIP / 32; ++ch) {
            bf16x8 av;
#pragma unroll
            for (int j = 0; j < 8; ++j) av[j] = gs[ch * 32 + 8 * kq + j][ob * 16 + r16];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    bf16x8 bv;
#pragma unroll
                    for (int j = 0; j < 8; ++j) bv[j] = xs[dy][ch * 32 + 8 * kq + j + dx][cb * 16 + r16];
                    acc[dy * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[dy * 3 + dx], 0, 0, 0);
                }
        }
        if (cb == 0) {
#pragma unroll 4
            for (int px = kq * 16; px < kq * 16 + 16; ++px) gb += (float)gs[px][ob * 16 + r16];
        }
        __syncthreads();
    }
    float* part = a.gw_part + (long long)blockIdx.x * 9 * C * C;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) part[(t * C + ob * 16 + 4 * kq + i) * C + cb * 16 + r16] = acc[t][i];
    if (cb == 0) {
        const float s = col_sum(gb);
        if (kq == 0) a.gb_part[blockIdx.x * C + ob * 16 + r16] = s;
    }
}

// Sum the per-workgroup weight and bias gradients into the flat gradient (layout
// w[o][c][dy][dx], then b[o]).  A workgroup takes 64 entries of the partials' own
// layout (tap, o, c) -- the last workgroup the biases -- so that a wavefront's
// partial reads are contiguous; its 16 wavefronts sum 16 contiguous ranges of
// workgroups in order, and wavefront 0 adds the 16 range sums in order.  Entries
// beyond cin x cout of a narrower layer are skipped.
constexpr int WRED_WAVES = 16;
__global__ __launch_bounds__(64 * WRED_WAVES) void k_wgrad_reduce(const float* gw_part, const float* gb_part,
                                                                  int nparts, int cin, int cout, float* grad_w,
                                                                  float* grad_b) {
    constexpr int NE = 9 * C * C;
    __shared__ float red[WRED_WAVES][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool bias = (int)blockIdx.x * 64 >= NE;
    const int e = bias ? lane : (int)blockIdx.x * 64 + lane;
    const float* src = bias ? gb_part : gw_part;
    const long long stride = bias ? C : NE;
    const bool live = bias ? e < cout : true;
    const int p0 = (int)((long long)nparts * wv / WRED_WAVES), p1 = (int)((long long)nparts * (wv + 1) / WRED_WAVES);
    float s = 0.0f;
    if (live) {
#pragma unroll 8
        for (int p = p0; p < p1; ++p) s += src[(long long)p * stride + e];
    }
    red[wv][lane] = s;
    __syncthreads();
    if (wv != 0 || !live) return;
    float t = red[0][lane];
#pragma unroll
    for (int g = 1; g < WRED_WAVES; ++g) t += red[g][lane];
    if (bias) {
        grad_b[e] = t;
    } else {
        const int c = e % C, o = (e / C) % C, tap = e / (C * C);
        if (c < cin && o < cout) grad_w[(o * cin + c) * 9 + tap] = t;
    }
}

// ------------------------------------------------------------ head, loss

// First stage of the global average pool: workgroup g sums its contiguous range
// of the per-wavefront channel sums (FP64, fixed order) into stage[g][32].
__global__ __launch_bounds__(HEAD_THREADS) void k_pool_stage(const float* pool_part, long long nparts, int ngroups,
                                                            double* stage) {
    __shared__ double part[HEAD_THREADS];
    const int t = threadIdx.x, c = t % C, sub = t / C;
    constexpr int NSUB = HEAD_THREADS / C;
    const long long w0 = nparts * blockIdx.x / ngroups, w1 = nparts * (blockIdx.x + 1) / ngroups;
    double s = 0.0;
    for (long long w = w0 + sub; w < w1; w += NSUB) s += (double)pool_part[w * C + c];
    part[t] = s;
    __syncthreads();
    if (t < C) {
        double tot = 0.0;
        for (int k = 0; k < NSUB; ++k) tot += part[k * C + t];
        stage[(long long)blockIdx.x * C + t] = tot;
    }
}

// Global average pool of the layer-5 features and the linear colour head
// db = hw pooled + hb.  With train != 0 also the head's gradients for the loss
// 0.5 w_b mean((db - t_db)^2), the pooled-feature gradient spread over the
// pixels (addc = hw^T g_db / (H W)) and that loss term.
__global__ __launch_bounds__(HEAD_THREADS) void k_head(HeadArgs a) {
    __shared__ double part[HEAD_THREADS];
    __shared__ double pooled[C];
    __shared__ double db[3 * KMAX_NET];
    const int t = threadIdx.x;
    const int c = t % C, g = t / C;
    constexpr int NGRP = HEAD_THREADS / C;
    double s = 0.0;
    for (int w = g; w < a.nstage; w += NGRP) s += a.stage[(long long)w * C + c];
    part[t] = s;
    __syncthreads();
    if (t < C) {
        double tot = 0.0;
        for (int k = 0; k < NGRP; ++k) tot += part[k * C + t];
        pooled[t] = tot / a.npix;
        a.pooled[t] = (float)pooled[t];
    }
    __syncthreads();
    const int nb = 3 * a.K;
    if (t < nb) {
        double v = (double)a.hb[t];
        for (int k = 0; k < C; ++k) v += (double)a.hw[t * C + k] * pooled[k];
        db[t] = v;
        a.db[t] = (float)v;
    }
    __syncthreads();
    if (!a.train) return;
    if (t < nb) {
        const double e = db[t] - (double)a.tdb[t];
        const double gd = (double)a.wb * e / nb;
        a.grad_hb[t] = (float)gd;
        for (int k = 0; k < C; ++k) a.grad_hw[t * C + k] = (float)(gd * pooled[k]);
        part[t] = e * e;
    }
    __syncthreads();
    if (t < C) {
        double gp = 0.0;
        for (int j = 0; j < nb; ++j) gp += (double)a.hw[j * C + t] * ((double)a.wb * (db[j] - (double)a.tdb[j]) / nb);
        a.addc[t] = (float)(gp / a.npix);
    }
    if (t == 0) {
        double l = 0.0;
        for (int j = 0; j < nb; ++j) l += part[j];
        a.loss_db[0] = 0.5 * (double)a.wb * l / nb;
    }
}

// Sum of the per-wavefront squared errors of the layer outputs, in order.
__global__ __launch_bounds__(HEAD_THREADS) void k_loss_total(const double* loss_part, long long nparts, double scale,
                                                            const double* loss_db, double* out) {
    __shared__ double part[HEAD_THREADS];
    double s = 0.0;
    for (long long w = threadIdx.x; w < nparts; w += HEAD_THREADS) s += loss_part[w];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int k = 0; k < HEAD_THREADS; ++k) tot += part[k];
        out[0] = 0.5 * tot * scale + loss_db[0];
    }
}

// ------------------------------------------------------------ packing, Adam

// Network input: the frame (3 planes) and the previous unknowns (n planes),
// rounded to BF16, zero channels up to 32.
// One workgroup per 256 pixels: every channel plane is read with coalesced loads, each
// thread packs its pixel's 32 BF16 channels into LDS, and the workgroup's 16 KiB block
// is written out with contiguous 16-byte stores.
constexpr int PACK_PX = 256;

__global__ __launch_bounds__(PACK_PX) void k_pack_input(const float* frame, const float* u, int n, long long ps,
                                                        __bf16* out) {
    __shared__ __align__(16) __bf16 blk[PACK_PX][C];
    const long long p0 = (long long)blockIdx.x * PACK_PX;
    const long long px = p0 + threadIdx.x;
    const bool in = px < ps;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int ch = 8 * q + j;
            float f = 0.0f;
            if (in && ch < 3) f = frame[ch * ps + px];
            else if (in && ch < 3 + n) f = u[(ch - 3) * ps + px];
            v[j] = (__bf16)f;
        }
        *reinterpret_cast<bf16x8*>(&blk[threadIdx.x][8 * q]) = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = (int)threadIdx.x + PACK_PX * j;
        const long long pp = p0 + (e >> 2);
        if (pp < ps)
            *reinterpret_cast<bf16x8*>(out + pp * C + 8 * (e & 3)) =
                *reinterpret_cast<const bf16x8*>(&blk[e >> 2][8 * (e & 3)]);
    }
}

// BF16 copies of one layer's FP32 master weights for the forward pass
// (wf[tap][o][c]) and, flipped and transposed, for the input-gradient pass
// (wd[tap][c][o] = w[o][c][8 - tap]), plus the zero-padded FP32 bias.
__global__ void k_pack_layer(const float* w, const float* b, int cin, int cout, __bf16* wf, __bf16* wd,
                             float* bias) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * C * C) return;
    const int c = e % C, o = (e / C) % C, t = e / (C * C);
    const bool in = o < cout && c < cin;
    wf[e] = (__bf16)(in ? w[(o * cin + c) * 9 + t] : 0.0f);
    // input-gradient pass: its output channel (position o) is a forward input
    // channel, its reduction channel (position c) a forward output channel
    const bool in2 = c < cout && o < cin;
    wd[e] = (__bf16)(in2 ? w[(c * cin + o) * 9 + (8 - t)] : 0.0f);
    if (t == 0 && c == 0) bias[o] = o < cout ? b[o] : 0.0f;
}

__global__ void k_adam(float* p, float* m, float* v, const float* g, long long n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

// ------------------------------------------------------------ launchers

// Tiles of 4 rows x 64 pixels; one partial slot per wavefront of each tile.
int conv_grid(int W, int H) {
    return ((W + STRIP - 1) / STRIP) * ((H + CONV_ROWS - 1) / CONV_ROWS);
}

// Resident workgroups per compute unit of the convolution (two 6 x 66 x 32 BF16 tiles,
// 50.7 KB of LDS each, so three fit in 160 KB).
#ifndef CONV_WG_PER_CU
#define CONV_WG_PER_CU 2
#endif

static int conv_resident() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (!cus[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 0;
        cus[dev] = n;
    }
    return cus[dev] * CONV_WG_PER_CU;
}

hipError_t launch_conv(const ConvArgs& a, int nb, hipStream_t s) {
    const int ntiles = conv_grid(a.W, a.H);
    const int res = a.max_wg > 0 ? a.max_wg : conv_resident();
    if (res <= 0) return hipErrorInvalidDevice;
    if (ntiles <= 0) return hipSuccess;
    const dim3 grid(ntiles < res ? ntiles : res), blk(CONV_THREADS);
    // one output block only where nothing reads channels 16..31 of the output
    if (nb == 1 && a.mode != M_ADD) return hipErrorInvalidValue;
    switch (a.mode) {
        case M_RELU: hipLaunchKernelGGL((k_conv<2, M_RELU>), grid, blk, 0, s, a); break;
        case M_ADD:
            if (nb == 1) hipLaunchKernelGGL((k_conv<1, M_ADD>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_conv<2, M_ADD>), grid, blk, 0, s, a);
            break;
        case M_LOSS: hipLaunchKernelGGL((k_conv<2, M_LOSS>), grid, blk, 0, s, a); break;
        case M_MASK: hipLaunchKernelGGL((k_conv<2, M_MASK>), grid, blk, 0, s, a); break;
        default: hipLaunchKernelGGL((k_conv<2, M_RAW>), grid, blk, 0, s, a); break;
    }
    return hipGetLastError();
}

long long conv_waves(int W, int H) { return (long long)conv_grid(W, H) * CONV_ROWS; }

hipError_t launch_wgrad(const WgradArgs& a, int nparts, int cin, int cout, float* grad_w, float* grad_b,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_wgrad, dim3(nparts), dim3(CONV_THREADS), 0, s, a);
    // 9 C C / 64 workgroups of weight entries, then one of biases
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(9 * C * C / 64 + 1), dim3(64 * WRED_WAVES), 0, s, a.gw_part, a.gb_part,
                       nparts, cin, cout, grad_w, grad_b);
    return hipGetLastError();
}

hipError_t launch_head(const HeadArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_pool_stage, dim3(a.nstage), dim3(HEAD_THREADS), 0, s, a.pool_part, a.nparts, a.nstage,
                       a.stage);
    hipLaunchKernelGGL(k_head, dim3(1), dim3(HEAD_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_loss_total(const double* loss_part, long long nparts, double scale, const double* loss_db,
                             double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(HEAD_THREADS), 0, s, loss_part, nparts, scale, loss_db, out);
    return hipGetLastError();
}

hipError_t launch_pack_input(const float* frame, const float* u, int n, long long ps, __bf16* out, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((ps + PACK_PX - 1) / PACK_PX)), dim3(PACK_PX), 0, s, frame, u, n,
                       ps, out);
    return hipGetLastError();
}

hipError_t launch_pack_layer(const float* w, const float* b, int cin, int cout, __bf16* wf, __bf16* wd, float* bias,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_pack_layer, dim3((9 * C * C + 255) / 256), dim3(256), 0, s, w, b, cin, cout, wf, wd, bias);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, long long n, float lr, float b1, float b2,
                       float c1, float c2, float eps, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, c1, c2,
                       eps);
    return hipGetLastError();
}

}  // namespace gidnet
