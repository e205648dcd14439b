// Internal declarations shared by the warm-start network's kernels and host code.
#ifndef GID_NET_INTERNAL_H
#define GID_NET_INTERNAL_H

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gid.h"

namespace gidnet {

constexpr int C = 32;              // hidden channels; also the padded channel count of every activation
constexpr int NCONV = 6;
constexpr int KMAX_NET = 16;
constexpr int STRIP = 64;          // pixels of one row handled by a wavefront
constexpr int CONV_ROWS = 4;       // rows (wavefronts) per workgroup
constexpr int CONV_THREADS = 64 * CONV_ROWS;
constexpr int HEAD_THREADS = 256;

enum ConvMode { M_RELU = 0, M_ADD = 1, M_LOSS = 2, M_MASK = 3, M_RAW = 4 };

struct ConvArgs {
    const __bf16* in;        // H x W x 32 BF16
    const __bf16* w;         // packed [9][32 out][32 in] BF16
    const float* bias;       // [32] FP32 (zero-padded)
    int W, H;
    long long ps;            // W * H
    int mode, nout;          // nout: valid output channels (M_ADD, M_LOSS)
    __bf16* out_b;           // M_RELU, M_LOSS, M_MASK: H x W x 32 BF16
    float* out_f;            // M_ADD: nout planes; M_RAW: H x W x 32 FP32
    const float* uprev;      // M_ADD: planes added to the output
    const float* tgt;        // M_LOSS: target planes
    float gscale;            // M_LOSS: gradient scale 1 / (nout W H)
    double* loss_part;       // M_LOSS: per-wavefront sum of squared errors
    const __bf16* mask;      // M_MASK: activation whose positive entries pass
    const float* addc;       // M_MASK: per-channel term added before the mask (may be null)
    float* pool_part;        // M_RELU: per-wavefront channel sums (may be null)
    int max_wg;              // workgroups of the launch at most (0: the resident grid)
};

struct WgradArgs {
    const __bf16* x;         // layer input, H x W x 32
    const __bf16* gy;        // gradient of the layer output, H x W x 32
    int W, H;
    float* gw_part;          // [parts][9][32][32]
    float* gb_part;          // [parts][32]
};

constexpr int POOL_STAGES = 120;    // workgroups of the first pooling stage

struct HeadArgs {
    const float* pool_part;  // [nparts][32]
    long long nparts;
    double* stage;           // [nstage][32] first-stage sums
    int nstage;
    double npix;
    int K;
    const float* hw;         // [3K][32]
    const float* hb;         // [3K]
    float* pooled;           // [32] out
    float* db;               // [3K] out
    int train;
    const float* tdb;        // [3K] target
    float wb;
    float* grad_hw;
    float* grad_hb;
    float* addc;             // [32] out: pooled-feature gradient / (W H)
    double* loss_db;         // [1] out
};

hipError_t launch_conv(const ConvArgs& a, int nb, hipStream_t s);
long long conv_waves(int W, int H);
hipError_t launch_wgrad(const WgradArgs& a, int nparts, int cin, int cout, float* grad_w, float* grad_b,
                        hipStream_t s);
hipError_t launch_head(const HeadArgs& a, hipStream_t s);
hipError_t launch_loss_total(const double* loss_part, long long nparts, double scale, const double* loss_db,
                             double* out, hipStream_t s);
hipError_t launch_pack_input(const float* frame, const float* u, int n, long long ps, __bf16* out, hipStream_t s);
hipError_t launch_pack_layer(const float* w, const float* b, int cin, int cout, __bf16* wf, __bf16* wd, float* bias,
                             hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, long long n, float lr, float b1, float b2,
                       float c1, float c2, float eps, hipStream_t s);

}  // namespace gidnet

// Inference on a caller's stream: u_out = u + du, db (3K FP32) to db_dev when given.
hipError_t gidnet_forward_dev(gid_net* net, hipStream_t s, const float* frame, const float* u, float* u_out,
                              float* db_dev);
bool gidnet_matches(const gid_net* net, int K, int W, int H);

#endif
