// Host side of the learned warm start: the network object, its parameter
// layout, training step and inference, behind the C ABI of include/gid.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "gid.h"
#include "gid_net_internal.h"

using namespace gidnet;

struct gid_net {
    int K = 0, n = 0, cin = 0, W = 0, H = 0;
    long long ps = 0;
    hipStream_t stream = nullptr;
    int64_t nparam = 0;
    int lcin[NCONV] = {}, lcout[NCONV] = {};
    int64_t woff[NCONV] = {}, boff[NCONV] = {}, hwoff = 0, hboff = 0;
    float *P = nullptr, *Mo = nullptr, *Ve = nullptr, *G = nullptr;
    __bf16 *wf = nullptr, *wd = nullptr;
    float* bias = nullptr;
    __bf16* act[NCONV] = {};
    __bf16 *g0 = nullptr, *g1 = nullptr;
    float* pool_part = nullptr;
    double* loss_part = nullptr;
    long long nwaves = 0;
    float *pooled = nullptr, *db = nullptr, *tdb = nullptr, *addc = nullptr;
    double *loss_db = nullptr, *loss_tot = nullptr;
    double* stage = nullptr;
    int nstage = 0;
    float *gw_part = nullptr, *gb_part = nullptr;
    int nparts = 0;
    float* h_db = nullptr;
    double* h_loss = nullptr;
    int adam_t = 0;
    int conv_wg = 0;         // convolution workgroups at most (0: the resident grid)
    void* arena = nullptr;
    std::string err;
};

namespace {

constexpr int WGRAD_PARTS = 1024;   // four workgroups per CU: one per CU left the weight gradients latency-bound

gid_status nfail(gid_net* net, gid_status s, const std::string& msg) {
    if (net) net->err = msg;
    return s;
}

#define NET_HIP(net, expr)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return nfail(net, GID_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// Parameter layout (FP32, in this order): for each conv layer l = 0..5 its
// weights w[o][c][dy][dx] then bias b[o]; then the colour head hw[3K][32], hb[3K].
void layout(gid_net* net) {
    int64_t off = 0;
    for (int l = 0; l < NCONV; ++l) {
        net->lcin[l] = l == 0 ? net->cin : C;
        net->lcout[l] = l == NCONV - 1 ? net->n : C;
        net->woff[l] = off;
        off += (int64_t)net->lcout[l] * net->lcin[l] * 9;
        net->boff[l] = off;
        off += net->lcout[l];
    }
    net->hwoff = off;
    off += (int64_t)3 * net->K * C;
    net->hboff = off;
    off += 3 * net->K;
    net->nparam = off;
}

hipError_t pack_all(gid_net* net) {
    for (int l = 0; l < NCONV; ++l) {
        hipError_t e = launch_pack_layer(net->P + net->woff[l], net->P + net->boff[l], net->lcin[l], net->lcout[l],
                                         net->wf + (size_t)l * 9 * C * C, net->wd + (size_t)l * 9 * C * C,
                                         net->bias + l * C, net->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

ConvArgs conv_args(const gid_net* net, int l, const __bf16* in, int mode) {
    ConvArgs a{};
    a.in = in;
    a.w = net->wf + (size_t)l * 9 * C * C;
    a.bias = net->bias + l * C;
    a.W = net->W;
    a.H = net->H;
    a.ps = net->ps;
    a.mode = mode;
    a.nout = net->lcout[l];
    a.max_wg = net->conv_wg;
    return a;
}

// Layers 1..5 (ReLU) from the packed input in act[0]; pooled colour head.
hipError_t forward_trunk(gid_net* net, hipStream_t s, const float* frame, const float* u, int train) {
    hipError_t e = launch_pack_input(frame, u, net->n, net->ps, net->act[0], s);
    if (e != hipSuccess) return e;
    for (int l = 0; l < NCONV - 1; ++l) {
        ConvArgs a = conv_args(net, l, net->act[l], M_RELU);
        a.out_b = net->act[l + 1];
        if (l == NCONV - 2) a.pool_part = net->pool_part;
        if ((e = launch_conv(a, 2, s)) != hipSuccess) return e;
    }
    HeadArgs h{};
    h.pool_part = net->pool_part;
    h.nparts = net->nwaves;
    h.stage = net->stage;
    h.nstage = net->nstage;
    h.npix = (double)net->ps;
    h.K = net->K;
    h.hw = net->P + net->hwoff;
    h.hb = net->P + net->hboff;
    h.pooled = net->pooled;
    h.db = net->db;
    h.train = train;
    h.tdb = net->tdb;
    h.wb = 0.0f;
    h.grad_hw = net->G + net->hwoff;
    h.grad_hb = net->G + net->hboff;
    h.addc = net->addc;
    h.loss_db = net->loss_db;
    return launch_head(h, s);
}

// Forward with the loss at the output layer, then the backward pass into G.
hipError_t train_pass(gid_net* net, const float* frame, const float* u, const float* du_tgt, float wb) {
    hipStream_t s = net->stream;
    hipError_t e = launch_pack_input(frame, u, net->n, net->ps, net->act[0], s);
    if (e != hipSuccess) return e;
    for (int l = 0; l < NCONV - 1; ++l) {
        ConvArgs a = conv_args(net, l, net->act[l], M_RELU);
        a.out_b = net->act[l + 1];
        if (l == NCONV - 2) a.pool_part = net->pool_part;
        if ((e = launch_conv(a, 2, s)) != hipSuccess) return e;
    }
    HeadArgs h{};
    h.pool_part = net->pool_part;
    h.nparts = net->nwaves;
    h.stage = net->stage;
    h.nstage = net->nstage;
    h.npix = (double)net->ps;
    h.K = net->K;
    h.hw = net->P + net->hwoff;
    h.hb = net->P + net->hboff;
    h.pooled = net->pooled;
    h.db = net->db;
    h.train = 1;
    h.tdb = net->tdb;
    h.wb = wb;
    h.grad_hw = net->G + net->hwoff;
    h.grad_hb = net->G + net->hboff;
    h.addc = net->addc;
    h.loss_db = net->loss_db;
    if ((e = launch_head(h, s)) != hipSuccess) return e;
    // output layer: du and the loss gradient (BF16) in g0
    ConvArgs a = conv_args(net, NCONV - 1, net->act[NCONV - 1], M_LOSS);
    a.out_b = net->g0;
    a.tgt = du_tgt;
    a.gscale = (float)(1.0 / ((double)net->n * (double)net->ps));
    a.loss_part = net->loss_part;
    if ((e = launch_conv(a, 2, s)) != hipSuccess) return e;
    if ((e = launch_loss_total(net->loss_part, net->nwaves, 1.0 / ((double)net->n * (double)net->ps), net->loss_db,
                               net->loss_tot, s)) != hipSuccess)
        return e;
    // backward: layer l's weight gradient from (act[l], gy), then the input gradient
    // through the ReLU that produced act[l]
    __bf16* gy = net->g0;
    __bf16* gx = net->g1;
    for (int l = NCONV - 1; l >= 0; --l) {
        WgradArgs w{};
        w.x = net->act[l];
        w.gy = gy;
        w.W = net->W;
        w.H = net->H;
        w.gw_part = net->gw_part;
        w.gb_part = net->gb_part;
        if ((e = launch_wgrad(w, net->nparts, net->lcin[l], net->lcout[l], net->G + net->woff[l],
                              net->G + net->boff[l], s)) != hipSuccess)
            return e;
        if (l == 0) break;
        ConvArgs d{};
        d.in = gy;
        d.w = net->wd + (size_t)l * 9 * C * C;
        d.bias = nullptr;
        d.W = net->W;
        d.H = net->H;
        d.ps = net->ps;
        d.mode = M_MASK;
        d.nout = C;
        d.out_b = gx;
        d.mask = net->act[l];
        d.addc = (l == NCONV - 1) ? net->addc : nullptr;
        d.max_wg = net->conv_wg;
        if ((e = launch_conv(d, 2, s)) != hipSuccess) return e;
        __bf16* t = gy;
        gy = gx;
        gx = t;
    }
    return hipSuccess;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int64_t gid_net_num_params(int32_t K) {
    if (K < 1 || K > KMAX_NET) return -1;
    gid_net tmp;
    tmp.K = K;
    tmp.n = K + 4;
    tmp.cin = 3 + tmp.n;
    layout(&tmp);
    return tmp.nparam;
}

gid_status gid_net_create(int32_t K, int32_t width, int32_t height, void* hip_stream, gid_net** out) {
    if (!out || K < 1 || K > KMAX_NET || width < 1 || height < 1) return GID_ERR_INVALID_ARG;
    if (3 + K + 4 > C) return GID_ERR_UNSUPPORTED;
    *out = nullptr;
    gid_net* net = new gid_net();
    net->K = K;
    net->n = K + 4;
    net->cin = 3 + net->n;
    net->W = width;
    net->H = height;
    net->ps = (long long)width * height;
    net->stream = static_cast<hipStream_t>(hip_stream);
    layout(net);
    net->nwaves = conv_waves(width, height);
    const int nsx = (width + STRIP - 1) / STRIP;
    net->nparts = (int)std::max<long long>(1, std::min<long long>(WGRAD_PARTS, (long long)nsx * height));
    // one arena, 256-byte aligned pieces
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t np = (size_t)net->nparam;
    const size_t o_P = take(4 * np), o_M = take(4 * np), o_V = take(4 * np), o_G = take(4 * np);
    const size_t o_wf = take(2 * (size_t)NCONV * 9 * C * C), o_wd = take(2 * (size_t)NCONV * 9 * C * C);
    const size_t o_bias = take(4 * NCONV * C);
    size_t o_act[NCONV];
    for (int l = 0; l < NCONV; ++l) o_act[l] = take(2 * (size_t)net->ps * C);
    const size_t o_g0 = take(2 * (size_t)net->ps * C), o_g1 = take(2 * (size_t)net->ps * C);
    const size_t o_pool = take(4 * (size_t)net->nwaves * C);
    const size_t o_lp = take(8 * (size_t)net->nwaves);
    const size_t o_pooled = take(4 * C), o_db = take(4 * 3 * K), o_tdb = take(4 * 3 * K), o_addc = take(4 * C);
    const size_t o_ldb = take(8), o_ltot = take(8);
    net->nstage = (int)std::max<long long>(1, std::min<long long>(POOL_STAGES, net->nwaves));
    const size_t o_stage = take(8 * (size_t)net->nstage * C);
    const size_t o_gw = take(4 * (size_t)net->nparts * 9 * C * C), o_gb = take(4 * (size_t)net->nparts * C);
    char* base = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&base), off) != hipSuccess) {
        delete net;
        return GID_ERR_OUT_OF_MEMORY;
    }
    net->arena = base;
    net->P = reinterpret_cast<float*>(base + o_P);
    net->Mo = reinterpret_cast<float*>(base + o_M);
    net->Ve = reinterpret_cast<float*>(base + o_V);
    net->G = reinterpret_cast<float*>(base + o_G);
    net->wf = reinterpret_cast<__bf16*>(base + o_wf);
    net->wd = reinterpret_cast<__bf16*>(base + o_wd);
    net->bias = reinterpret_cast<float*>(base + o_bias);
    for (int l = 0; l < NCONV; ++l) net->act[l] = reinterpret_cast<__bf16*>(base + o_act[l]);
    net->g0 = reinterpret_cast<__bf16*>(base + o_g0);
    net->g1 = reinterpret_cast<__bf16*>(base + o_g1);
    net->pool_part = reinterpret_cast<float*>(base + o_pool);
    net->loss_part = reinterpret_cast<double*>(base + o_lp);
    net->pooled = reinterpret_cast<float*>(base + o_pooled);
    net->db = reinterpret_cast<float*>(base + o_db);
    net->tdb = reinterpret_cast<float*>(base + o_tdb);
    net->addc = reinterpret_cast<float*>(base + o_addc);
    net->loss_db = reinterpret_cast<double*>(base + o_ldb);
    net->loss_tot = reinterpret_cast<double*>(base + o_ltot);
    net->stage = reinterpret_cast<double*>(base + o_stage);
    net->gw_part = reinterpret_cast<float*>(base + o_gw);
    net->gb_part = reinterpret_cast<float*>(base + o_gb);
    if (hipMemsetAsync(base, 0, off, net->stream) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&net->h_db), 4 * 3 * K) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&net->h_loss), 8) != hipSuccess ||
        hipStreamSynchronize(net->stream) != hipSuccess) {
        gid_net_destroy(net);
        return GID_ERR_HIP;
    }
    *out = net;
    return GID_OK;
}

gid_status gid_net_destroy(gid_net* net) {
    if (!net) return GID_OK;
    (void)hipStreamSynchronize(net->stream);
    if (net->arena) (void)hipFree(net->arena);
    if (net->h_db) (void)hipHostFree(net->h_db);
    if (net->h_loss) (void)hipHostFree(net->h_loss);
    delete net;
    return GID_OK;
}

gid_status gid_net_set_params(gid_net* net, const float* host, int64_t count) {
    if (!net || !host || count != net->nparam) return nfail(net, GID_ERR_INVALID_ARG, "parameter count mismatch");
    NET_HIP(net, hipMemcpyAsync(net->P, host, 4 * (size_t)count, hipMemcpyHostToDevice, net->stream));
    NET_HIP(net, hipMemsetAsync(net->Mo, 0, 4 * (size_t)count, net->stream));
    NET_HIP(net, hipMemsetAsync(net->Ve, 0, 4 * (size_t)count, net->stream));
    net->adam_t = 0;
    NET_HIP(net, pack_all(net));
    NET_HIP(net, hipStreamSynchronize(net->stream));
    return GID_OK;
}

gid_status gid_net_get_params(gid_net* net, float* host, int64_t count) {
    if (!net || !host || count != net->nparam) return nfail(net, GID_ERR_INVALID_ARG, "parameter count mismatch");
    NET_HIP(net, hipMemcpyAsync(host, net->P, 4 * (size_t)count, hipMemcpyDeviceToHost, net->stream));
    NET_HIP(net, hipStreamSynchronize(net->stream));
    return GID_OK;
}

gid_status gid_net_forward(gid_net* net, const float* frame_dev, const float* u_prev_dev, float* u_out_dev,
                           float* db_out_host) {
    if (!net || !frame_dev || !u_prev_dev || !u_out_dev) return nfail(net, GID_ERR_INVALID_ARG, "null pointer");
    NET_HIP(net, gidnet_forward_dev(net, net->stream, frame_dev, u_prev_dev, u_out_dev, nullptr));
    if (db_out_host) {
        NET_HIP(net, hipMemcpyAsync(net->h_db, net->db, 4 * 3 * net->K, hipMemcpyDeviceToHost, net->stream));
        NET_HIP(net, hipStreamSynchronize(net->stream));
        std::memcpy(db_out_host, net->h_db, 4 * 3 * net->K);
    }
    return GID_OK;
}

gid_status gid_net_gradients(gid_net* net, const float* frame_dev, const float* u_prev_dev, const float* du_tgt_dev,
                             const float* db_tgt_host, float w_b, float* grad_host, double* loss_out) {
    if (!net || !frame_dev || !u_prev_dev || !du_tgt_dev || !db_tgt_host || !grad_host)
        return nfail(net, GID_ERR_INVALID_ARG, "null pointer");
    NET_HIP(net, hipMemcpyAsync(net->tdb, db_tgt_host, 4 * 3 * net->K, hipMemcpyHostToDevice, net->stream));
    NET_HIP(net, train_pass(net, frame_dev, u_prev_dev, du_tgt_dev, w_b));
    NET_HIP(net, hipMemcpyAsync(grad_host, net->G, 4 * (size_t)net->nparam, hipMemcpyDeviceToHost, net->stream));
    NET_HIP(net, hipMemcpyAsync(net->h_loss, net->loss_tot, 8, hipMemcpyDeviceToHost, net->stream));
    NET_HIP(net, hipStreamSynchronize(net->stream));
    if (loss_out) *loss_out = net->h_loss[0];
    return GID_OK;
}

gid_status gid_net_train_step(gid_net* net, const float* frame_dev, const float* u_prev_dev, const float* du_tgt_dev,
                              const float* db_tgt_host, float w_b, float lr, double* loss_out) {
    if (!net || !frame_dev || !u_prev_dev || !du_tgt_dev || !db_tgt_host || !(lr >= 0.0f))
        return nfail(net, GID_ERR_INVALID_ARG, "bad argument");
    NET_HIP(net, hipMemcpyAsync(net->tdb, db_tgt_host, 4 * 3 * net->K, hipMemcpyHostToDevice, net->stream));
    NET_HIP(net, train_pass(net, frame_dev, u_prev_dev, du_tgt_dev, w_b));
    net->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, net->adam_t)), c2 = (float)(1.0 - std::pow(b2, net->adam_t));
    NET_HIP(net, launch_adam(net->P, net->Mo, net->Ve, net->G, net->nparam, lr, (float)b1, (float)b2, c1, c2, 1e-8f,
                             net->stream));
    NET_HIP(net, pack_all(net));
    if (loss_out) {
        NET_HIP(net, hipMemcpyAsync(net->h_loss, net->loss_tot, 8, hipMemcpyDeviceToHost, net->stream));
        NET_HIP(net, hipStreamSynchronize(net->stream));
        *loss_out = net->h_loss[0];
    }
    return GID_OK;
}

gid_status gid_net_layer_forward(gid_net* net, int32_t layer, const void* in_dev, float* out_dev) {
    if (!net || !in_dev || !out_dev || layer < 0 || layer >= NCONV)
        return nfail(net, GID_ERR_INVALID_ARG, "bad argument");
    ConvArgs a = conv_args(net, layer, static_cast<const __bf16*>(in_dev), M_RAW);
    a.out_f = out_dev;
    NET_HIP(net, launch_conv(a, 2, net->stream));
    NET_HIP(net, hipStreamSynchronize(net->stream));
    return GID_OK;
}

gid_status gid_net_layer_wgrad(gid_net* net, int32_t layer, const void* x_dev, const void* gy_dev, float* gw_host,
                               float* gb_host) {
    if (!net || !x_dev || !gy_dev || !gw_host || !gb_host || layer < 0 || layer >= NCONV)
        return nfail(net, GID_ERR_INVALID_ARG, "bad argument");
    WgradArgs w{};
    w.x = static_cast<const __bf16*>(x_dev);
    w.gy = static_cast<const __bf16*>(gy_dev);
    w.W = net->W;
    w.H = net->H;
    w.gw_part = net->gw_part;
    w.gb_part = net->gb_part;
    NET_HIP(net, launch_wgrad(w, net->nparts, net->lcin[layer], net->lcout[layer], net->G + net->woff[layer],
                              net->G + net->boff[layer], net->stream));
    const size_t nw = (size_t)net->lcout[layer] * net->lcin[layer] * 9;
    NET_HIP(net, hipMemcpyAsync(gw_host, net->G + net->woff[layer], 4 * nw, hipMemcpyDeviceToHost, net->stream));
    NET_HIP(net, hipMemcpyAsync(gb_host, net->G + net->boff[layer], 4 * (size_t)net->lcout[layer],
                                hipMemcpyDeviceToHost, net->stream));
    NET_HIP(net, hipStreamSynchronize(net->stream));
    return GID_OK;
}

gid_status gid_net_set_conv_workgroups(gid_net* net, int32_t workgroups) {
    if (!net || workgroups < 0) return nfail(net, GID_ERR_INVALID_ARG, "workgroups must be >= 0");
    net->conv_wg = workgroups;
    return GID_OK;
}

const char* gid_net_last_error(const gid_net* net) { return net ? net->err.c_str() : "null network"; }

}  // extern "C"

// Inference on a caller's stream (the solver's, for the warm start): u_out =
// u + du over the network's n planes, db (3K FP32) to db_dev or the network's
// own buffer.
hipError_t gidnet_forward_dev(gid_net* net, hipStream_t s, const float* frame, const float* u, float* u_out,
                              float* db_dev) {
    hipError_t e = forward_trunk(net, s, frame, u, 0);
    if (e != hipSuccess) return e;
    ConvArgs a = conv_args(net, NCONV - 1, net->act[NCONV - 1], M_ADD);
    a.out_f = u_out;
    a.uprev = u;
    if ((e = launch_conv(a, net->n <= 16 ? 1 : 2, s)) != hipSuccess) return e;
    if (db_dev) e = hipMemcpyAsync(db_dev, net->db, 4 * 3 * net->K, hipMemcpyDeviceToDevice, s);
    return e;
}

bool gidnet_matches(const gid_net* net, int K, int W, int H) {
    return net && net->K == K && net->W == W && net->H == H;
}
