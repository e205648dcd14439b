// libgid host runtime: context and workspace, the per-frame schedule of the
// alternating solve (Sec. 7.1), hipGraph replay of that schedule, single-step
// access, checkpoint/resume, and the C ABI declared in gid.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "gid_internal.h"
#include "gid_net_internal.h"

using namespace gid;

namespace {

constexpr int FINAL_SLOT = ELOG_FINAL_SLOT;
constexpr int PROBE_SLOT = ELOG_SLOTS - 1;   // single-step energy evaluation
constexpr int NSTATS = NSCAL + ELOG_SLOTS * ELOG_STRIDE + 3 * KMAX;   // doubles of the statistics block
constexpr int NB_MAX = 2048;                 // default cap on workgroups of a per-pixel launch (one tile each up to here)
static_assert(NB_MAX <= NB_TUNE_MAX, "site totals unroll their loads up to NB_TUNE_MAX workgroups");
constexpr uint32_t STATE_MAGIC = 0x67696431u; // "gid1"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct gid_ctx {
    gid_params prm{};
    int W = 0, H = 0, K = 0, n = 0;
    long long ps = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    void* arena = nullptr;
    // device workspace
    float *u = nullptr, *delta = nullptr, *zA = nullptr, *zB = nullptr, *pA = nullptr, *pB = nullptr, *qA = nullptr, *qB = nullptr,
          *minv = nullptr, *I = nullptr, *wsr = nullptr, *tg = nullptr, *Iprev = nullptr,
          *rprev = nullptr, *bf = nullptr, *lnb = nullptr, *bcf = nullptr;
    uint8_t* ids = nullptr;
    double *b64 = nullptr, *lnb64 = nullptr, *binit64 = nullptr, *scal = nullptr, *partials = nullptr,
           *elog = nullptr, *bsum = nullptr;
    unsigned* tickets = nullptr;
    long long part_stride = 0;
    // pinned host mirrors
    double* h_scal = nullptr;
    double* h_elog = nullptr;
    double* h_b64 = nullptr;
    double* h_small = nullptr;     // staging for host -> device colour uploads
    // tiling
    int ppt = 1, ntx = 0, nty = 0, ntiles = 0, nblocks = 0, nb_bs = 0;
    // clip state
    bool colors_set = false, have_prev = false;
    bool frame_ready = false;      // a frame's per-pixel data is loaded (the tuner times on it)
    int frame_index = 0;
    double binit_host[3 * KMAX] = {};
    // pending host outputs of the last frame
    bool pending = false;
    double* pend_b = nullptr;
    gid_frame_stats* pend_stats = nullptr;
    int pend_nhalf = 0, pend_final_slot = FINAL_SLOT, pend_frame = 0, pend_gn = 0;
    bool pend_had_prev = false;
    bool pend_target = false;
    // energy-target continuation: target > 0 runs up to target_gn outer
    // iterations and stops the frame on the device once E <= target
    double target = 0.0;
    int target_gn = 0;
    int target_first = 1;          // first outer iteration whose energy is checked (1-based)
    int pend_first = 1;
    double* h_target = nullptr;    // pinned slot the target is uploaded from
    // energy-target mode: the outer iterations after the first check are
    // enqueued by gid_synchronize, only when the frame has not met its target
    bool pend_rest = false;
    bool pend_refine = false;
    Args pend_args{};
    float* pend_layers = nullptr;
    // replayable schedules keyed by (refine, temporal, record, energy target,
    // iterations after the first check)
    hipGraphExec_t graphs[32] = {};
    hipStream_t cap_stream = nullptr;
    // kernel timing
    bool profiling = false;
    static constexpr int NEV = 8192;
    hipEvent_t ev[NEV] = {};
    int ev_kind[NEV / 2] = {};
    int ev_used = 0;
    double kind_ms[GID_NUM_KERNEL_KINDS] = {};
    int64_t kind_n[GID_NUM_KERNEL_KINDS] = {};
    // learned warm start
    gid_net* wnet = nullptr;
    void* warena = nullptr;
    float *ucand = nullptr, *dbc = nullptr, *bfc = nullptr, *lnbc = nullptr, *bcfc = nullptr;
    double *b64c = nullptr, *lnb64c = nullptr;
    bool pend_judged = false;
    std::string err;
};

namespace {

gid_status fail(gid_ctx* c, gid_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define GID_HIP(c, call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((c), GID_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Launch through fn; with profiling on, bracket the launch with an event pair.
template <typename Fn>
hipError_t timed(gid_ctx* c, int kind, Fn&& fn) {
    if (!c->profiling || c->ev_used + 2 > gid_ctx::NEV) return fn();
    hipEvent_t& e0 = c->ev[c->ev_used];
    hipEvent_t& e1 = c->ev[c->ev_used + 1];
    hipError_t e;
    if (!e0 && (e = hipEventCreate(&e0)) != hipSuccess) return e;
    if (!e1 && (e = hipEventCreate(&e1)) != hipSuccess) return e;
    if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) return e;
    if ((e = fn()) != hipSuccess) return e;
    if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) return e;
    c->ev_kind[c->ev_used / 2] = kind;
    c->ev_used += 2;
    return hipSuccess;
}

// Accumulate the recorded event pairs (the stream must be idle).
hipError_t collect_times(gid_ctx* c) {
    for (int i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]);
        if (e != hipSuccess) return e;
        c->kind_ms[c->ev_kind[i / 2]] += ms;
        c->kind_n[c->ev_kind[i / 2]] += 1;
    }
    c->ev_used = 0;
    return hipSuccess;
}

// Profiling kind of a kernel (-1: not timed).
int kind_of(Kern k) {
    switch (k) {
        case KN_SCAN: return GID_KERNEL_SCAN;
        case KN_PRECOMPUTE: return GID_KERNEL_PRECOMPUTE;
        case KN_GN_BUILD: return GID_KERNEL_GN_BUILD;
        case KN_PCG: return GID_KERNEL_PCG;
        case KN_APPLY_BSUM: return GID_KERNEL_APPLY_BSUM;
        case KN_BSOLVE: return GID_KERNEL_BSOLVE;
        case KN_ENERGY: return GID_KERNEL_ENERGY;
        case KN_OUTPUT: return GID_KERNEL_OUTPUT;
        default: return -1;
    }
}

// Launch kernel k of one clip on stream st (timed when profiling is on).
hipError_t L1(gid_ctx* c, hipStream_t st, Kern k, const Args& a, const Step& s) {
    const int kind = kind_of(k);
    if (kind < 0) return launch_kernel(k, a, s, st);
    return timed(c, kind, [&]() { return launch_kernel(k, a, s, st); });
}

Lam make_lam(const gid_params& p) {
    Lam L;
    L.data = p.lambda.data;
    L.cl = p.lambda.cluster;
    L.rs = p.lambda.r_sparsity;
    L.p = p.lambda.p;
    L.rc = p.lambda.r_consistency;
    L.mo = p.lambda.monochrome;
    L.is = p.lambda.i_sparsity;
    L.sm = p.lambda.smoothness;
    L.nn = p.lambda.non_neg;
    L.ir = p.lambda.ir;
    L.cr = p.lambda.cr;
    L.eps_nn = p.eps_nonneg;
    L.eps_irls = p.eps_irls;
    L.rk = p.retinex_k;
    L.gate = p.chroma_gate;
    L.cfloor = p.chroma_floor;
    return L;
}

Args base_args(const gid_ctx* c) {
    Args a;
    std::memset(&a, 0, sizeof(a));
    a.W = c->W;
    a.H = c->H;
    a.K = c->K;
    a.ppt = c->ppt;
    a.ntx = c->ntx;
    a.nty = c->nty;
    a.ntiles = c->ntiles;
    a.nblocks = c->nblocks;
    a.nb_bs = c->nb_bs;
    a.ps = c->ps;
    a.lam = make_lam(c->prm);
    a.cr_literal = c->prm.cr_mode == GID_CR_LITERAL;
    a.bstep_sum = c->prm.bstep_scale == GID_BSTEP_SUM;
    a.spatial = c->prm.spatial_pairs != 0;
    a.spatial_seed = c->prm.spatial_seed;
    a.u = c->u;
    a.delta = c->delta;
    a.zA = c->zA;
    a.zB = c->zB;
    a.pA = c->pA;
    a.pB = c->pB;
    a.qA = c->qA;
    a.qB = c->qB;
    a.minv = c->minv;
    a.I = c->I;
    a.ids = c->ids;
    a.wsr = c->wsr;
    a.tg = c->tg;
    a.Iprev = c->Iprev;
    a.rprev = c->rprev;
    a.bf = c->bf;
    a.lnb = c->lnb;
    a.bcf = c->bcf;
    a.b64 = c->b64;
    a.lnb64 = c->lnb64;
    a.binit64 = c->binit64;
    a.scal = c->scal;
    a.partials = c->partials;
    a.tickets = c->tickets;
    a.elog = c->elog;
    a.bsum = c->bsum;
    a.part_stride = c->part_stride;
    a.ucand = c->ucand;
    a.dbc = c->dbc;
    a.b64c = c->b64c;
    a.lnb64c = c->lnb64c;
    a.bfc = c->bfc;
    a.lnbc = c->lnbc;
    a.bcfc = c->bcfc;
    return a;
}

// Pixel rows per thread in a tile.
int choose_ppt(int, int) {
    return 1;   // the halo-staged stencil kernels work on 64 x 4 tiles
}

// Each workgroup of a per-pixel launch owns a contiguous chunk of tiles; the
// chunks are balanced (every workgroup gets the same number of tiles up to one)
// and the workgroup count is a multiple of 8 for the XCD-aware order.
void set_tiling(gid_ctx* c, int ppt) {
    c->ppt = ppt;
    c->ntx = (c->W + TX - 1) / TX;
    c->nty = (c->H + TYW * ppt - 1) / (TYW * ppt);
    c->ntiles = c->ntx * c->nty;
    const int per = (c->ntiles + NB_MAX - 1) / NB_MAX;
    const int nb = (c->ntiles + per - 1) / per;
    c->nblocks = (int)align_up((size_t)nb, 8);
    c->nb_bs = std::min(c->nblocks, NB_BS_MAX);
}

// Use nb workgroups for the per-pixel launches (rounded to a multiple of 8, at
// most one per tile); cached graphs are rebuilt on their next use.
void set_nblocks(gid_ctx* c, int nb) {
    nb = std::max(8, std::min(nb, (int)align_up((size_t)c->ntiles, 8)));
    c->nblocks = (int)align_up((size_t)nb, 8);
    c->nb_bs = std::min(c->nblocks, NB_BS_MAX);
    for (auto& g : c->graphs)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// Upload colours b (K x 3 doubles, and the initial estimate when init is true)
// through the pinned staging buffer; the derived tables are computed on the
// device by the same routine the base-colour solve uses.
gid_status upload_colours(gid_ctx* c, const double* b, bool init) {
    const int nk = 3 * c->K;
    GID_HIP(c, hipStreamSynchronize(c->stream));
    double* st = c->h_small;
    for (int i = 0; i < nk; ++i) {
        st[i] = b[i];
        st[3 * KMAX + i] = b[i];
    }
    GID_HIP(c, hipMemcpyAsync(c->b64, st, nk * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (init)
        GID_HIP(c, hipMemcpyAsync(c->binit64, st + 3 * KMAX, nk * sizeof(double), hipMemcpyHostToDevice, c->stream));
    GID_HIP(c, launch_kernel(KN_TABLES, base_args(c), Step{}, c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    return GID_OK;
}

bool colours_valid(const double* b, int nk) {
    for (int i = 0; i < nk; ++i)
        if (!std::isfinite(b[i]) || !(b[i] > 0.0)) return false;
    return true;
}

// Enqueue the G outer iterations of one frame (everything between the per-frame
// precompute and the output pass) through launch(kern, step); used for one clip
// and for batches.  Returns the number of energy slots used.
// With check (energy-target mode) the energy is evaluated after every outer
// iteration into slot g and compared with the frame's target on the device.
// Checks start after outer iteration first (1-based; the last iteration is
// always checked).  Outer iterations g0 .. g1 - 1 of the G are enqueued.
template <typename LaunchFn>
hipError_t enqueue_schedule(int G, int P, bool refine, bool record, LaunchFn&& launch, int* nslots,
                            bool check = false, int first = 1, int g0 = 0, int g1 = -1) {
    int slot = 0;
    hipError_t e = hipSuccess;
    if (check) record = false;
    if (g1 < 0) g1 = G;
    for (int g = g0; g < g1; ++g) {
        Step s{};
        s.gn = g;
        if ((e = launch(KN_GN_BUILD, s)) != hipSuccess) return e;
        for (int i = 0; i < P; ++i) {
            s.iter = i;
            if ((e = launch(KN_PCG, s)) != hipSuccess) return e;
        }
        s.refine = refine ? 1 : 0;
        s.add_delta = 1;
        s.log_rz = 1;
        s.iter = P - 1;
        if ((e = launch(KN_APPLY_BSUM, s)) != hipSuccess) return e;
        if (record) {
            s.slot = slot++;
            if ((e = launch(KN_ENERGY, s)) != hipSuccess) return e;
            if ((e = launch(KN_ENERGY_FINISH, s)) != hipSuccess) return e;
        }
        if (refine) {
            if ((e = launch(KN_BSOLVE, s)) != hipSuccess) return e;
            if (record) {
                s.slot = slot++;
                if ((e = launch(KN_ENERGY, s)) != hipSuccess) return e;
                if ((e = launch(KN_ENERGY_FINISH, s)) != hipSuccess) return e;
            }
        }
        if (check && (g + 1 >= first || g == G - 1)) {
            s.slot = g;
            s.check = 1;
            if ((e = launch(KN_ENERGY, s)) != hipSuccess) return e;
            if ((e = launch(KN_ENERGY_FINISH, s)) != hipSuccess) return e;
        }
    }
    if (check) {
        *nslots = 0;
        return hipSuccess;
    }
    if (!record) {
        Step s{};
        s.slot = FINAL_SLOT;
        if ((e = launch(KN_ENERGY, s)) != hipSuccess) return e;
        if ((e = launch(KN_ENERGY_FINISH, s)) != hipSuccess) return e;
    }
    *nslots = slot;
    return hipSuccess;
}

// Outer iterations of the frame's schedule: all of them (part 0), or in energy-
// target mode those through the first check (part 1) and those after it (part 2).
int target_split(const gid_ctx* c) { return std::min(std::max(c->target_first, 1), c->target_gn); }

hipError_t enqueue_outer(gid_ctx* c, hipStream_t st, const Args& base, bool refine, bool record, int* nslots,
                         int part = 0) {
    const bool check = c->target > 0.0;
    const int G = check ? c->target_gn : c->prm.gn_iters;
    const int g0 = part == 2 ? target_split(c) : 0, g1 = part == 1 ? target_split(c) : G;
    return enqueue_schedule(G, c->prm.pcg_iters, refine, record,
                            [&](Kern k, const Step& s) { return L1(c, st, k, base, s); }, nslots, check,
                            c->target_first, g0, g1);
}

// Capture a schedule into a graph on a private stream (the caller's may be the
// legacy null stream, which cannot be captured); the graph runs on any stream.
template <typename EnqueueFn>
hipError_t capture_graph(hipStream_t* cap, EnqueueFn&& enqueue, hipGraphExec_t* out) {
    hipError_t e;
    if (!*cap && (e = hipStreamCreateWithFlags(cap, hipStreamNonBlocking)) != hipSuccess) return e;
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(*cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    hipError_t e1 = enqueue(*cap);
    hipError_t e2 = hipStreamEndCapture(*cap, &g);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e1 != hipSuccess ? e1 : e2;
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

gid_status run_outer(gid_ctx* c, const Args& base, bool refine, bool record, int* nslots, int part = 0) {
    if (!c->prm.use_graph || c->profiling) {
        GID_HIP(c, enqueue_outer(c, c->stream, base, refine, record, nslots, part));
        return GID_OK;
    }
    const int key = (refine ? 1 : 0) | (base.temporal ? 2 : 0) | (record ? 4 : 0) | (c->target > 0.0 ? 8 : 0) |
                    (part == 2 ? 16 : 0);
    if (!c->graphs[key]) {
        hipGraphExec_t ex = nullptr;
        hipError_t e = capture_graph(&c->cap_stream, [&](hipStream_t cs) {
            return enqueue_outer(c, cs, base, refine, record, nslots, part);
        }, &ex);
        if (e != hipSuccess) return fail(c, GID_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        c->graphs[key] = ex;
    } else {
        *nslots = (record && !(c->target > 0.0)) ? (c->prm.gn_iters * (refine ? 2 : 1)) : 0;
    }
    GID_HIP(c, hipGraphLaunch(c->graphs[key], c->stream));
    return GID_OK;
}

gid_status check_params(const gid_params* p) {
    if (!p || p->struct_size != sizeof(gid_params)) return GID_ERR_INVALID_ARG;
    if (p->K < 1 || p->K > KMAX) return GID_ERR_INVALID_ARG;
    if (p->gn_iters < 1 || p->gn_iters > 64) return GID_ERR_INVALID_ARG;
    if (p->pcg_iters < 0 || p->pcg_iters > 4096) return GID_ERR_INVALID_ARG;
    if (p->refine_mode < 0 || p->refine_mode > 2) return GID_ERR_INVALID_ARG;
    if (p->cr_mode < 0 || p->cr_mode > 1) return GID_ERR_INVALID_ARG;
    if (p->bstep_scale < 0 || p->bstep_scale > 1) return GID_ERR_INVALID_ARG;
    if (p->spatial_pairs < 0 || p->spatial_pairs > 1) return GID_ERR_INVALID_ARG;
    if (p->record_energy && 2 * p->gn_iters > GID_MAX_HALF_STEPS) return GID_ERR_INVALID_ARG;
    if (!(p->eps_nonneg > 0.0f) || !(p->eps_irls > 0.0f)) return GID_ERR_INVALID_ARG;
    if (!(p->lambda.p > 0.0f) || !(p->lambda.p <= 2.0f)) return GID_ERR_INVALID_ARG;
    return GID_OK;
}

void release(gid_ctx* c) {
    for (auto& e : c->ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    for (auto& g : c->graphs)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    if (c->arena) (void)hipFree(c->arena);
    if (c->h_scal) (void)hipHostFree(c->h_scal);   // h_elog and h_b64 point into the same block
    if (c->h_small) (void)hipHostFree(c->h_small);   // h_target points into the same block
    if (c->warena) (void)hipFree(c->warena);
    c->warena = nullptr;
    c->arena = nullptr;
}

gid_status check_frame_ready(gid_ctx* c) {
    if (!c->colors_set) return fail(c, GID_ERR_STATE, "base colours not set");
    return GID_OK;
}

}  // namespace

extern "C" {

gid_status gid_default_params(int32_t K, gid_params* out) {
    if (!out || K < 1 || K > KMAX) return GID_ERR_INVALID_ARG;
    gid_params p;
    std::memset(&p, 0, sizeof(p));
    p.struct_size = sizeof(gid_params);
    p.K = K;
    p.lambda.data = 5000.0f;
    p.lambda.cluster = 200.0f;
    p.lambda.r_sparsity = 20.0f;
    p.lambda.p = 1.0f;
    p.lambda.r_consistency = 10.0f;
    p.lambda.monochrome = 10.0f;
    p.lambda.i_sparsity = 3.0f;
    p.lambda.smoothness = 3.0f;
    p.lambda.non_neg = 1000.0f;
    p.lambda.ir = 10.0f;
    p.lambda.cr = 100.0f;
    p.eps_nonneg = 0.002f;
    p.eps_irls = 0.002f;
    p.retinex_k = 50.0f;
    p.chroma_gate = 0.1;
    p.chroma_floor = 1e-6;
    p.gn_iters = 3;
    p.pcg_iters = 8;
    p.refine_mode = GID_REFINE_EVERY_STEP;
    p.temporal = 1;
    p.cr_mode = GID_CR_CHROMA;
    p.record_energy = 0;
    p.use_graph = 1;
    p.bstep_scale = GID_BSTEP_PER_PIXEL;
    p.spatial_pairs = 0;
    p.spatial_seed = 2019;
    *out = p;
    return GID_OK;
}

gid_status gid_create(const gid_params* params, int32_t width, int32_t height, void* hip_stream,
                      gid_ctx** out) {
    if (!out) return GID_ERR_INVALID_ARG;
    *out = nullptr;
    if (check_params(params) != GID_OK) return GID_ERR_INVALID_ARG;
    if (width < 2 || height < 2 || (long long)width * height > (1LL << 28)) return GID_ERR_INVALID_ARG;
    gid_ctx* c = new (std::nothrow) gid_ctx();
    if (!c) return GID_ERR_OUT_OF_MEMORY;
    c->prm = *params;
    c->W = width;
    c->H = height;
    c->K = params->K;
    c->n = params->K + 4;
    c->ps = (long long)width * height;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return GID_ERR_HIP;
    }
    set_tiling(c, choose_ppt(width, height));
    const int nsum = bstep_nsums(c->K);
    c->part_stride = (long long)align_up((size_t)std::max<long long>((long long)NTERMS * NB_TUNE_MAX,
                                                                      (long long)nsum * NB_BS_MAX), 32);
    // one arena: planes (exact stride width*height, each buffer 256-byte aligned),
    // ids, small tables, reductions
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t fplane = sizeof(float) * (size_t)c->ps;
    const size_t o_u = take(fplane * c->n), o_delta = take(fplane * c->n), o_zA = take(fplane * c->n),
                 o_zB = take(fplane * c->n), o_pA = take(fplane * c->n), o_pB = take(fplane * c->n),
                 o_qA = take(fplane * c->n), o_qB = take(fplane * c->n), o_minv = take(fplane * c->n), o_I = take(fplane * 3), o_wsr = take(fplane),
                 o_tg = take(fplane * 6), o_Iprev = take(fplane * 3), o_rprev = take(fplane * 3);
    const size_t o_ids = take((size_t)c->ps);
    const size_t o_bf = take(sizeof(float) * 3 * KMAX);
    const size_t o_lnb = take(sizeof(float) * 3 * KMAX);
    const size_t o_bcf = take(sizeof(float) * 3 * KMAX);
    // scalars, energy log and FP64 colours back to back: one copy returns a frame's statistics
    const size_t o_stats = take(sizeof(double) * NSTATS);
    const size_t o_lnb64 = take(sizeof(double) * 3 * KMAX);
    const size_t o_binit = take(sizeof(double) * 3 * KMAX);
    const size_t o_tick = take(sizeof(unsigned) * NRED);
    const size_t o_bsum = take(sizeof(double) * bstep_nsums(KMAX));
    const size_t o_part = take(sizeof(double) * (size_t)c->part_stride * NRED);
    if (hipMalloc(&c->arena, off) != hipSuccess) {
        delete c;
        return GID_ERR_OUT_OF_MEMORY;
    }
    char* base = static_cast<char*>(c->arena);
    auto fp = [&](size_t o) { return reinterpret_cast<float*>(base + o); };
    c->u = fp(o_u);
    c->delta = fp(o_delta);
    c->zA = fp(o_zA);
    c->zB = fp(o_zB);
    c->pA = fp(o_pA);
    c->pB = fp(o_pB);
    c->qA = fp(o_qA);
    c->qB = fp(o_qB);
    c->minv = fp(o_minv);
    c->I = fp(o_I);
    c->wsr = fp(o_wsr);
    c->tg = fp(o_tg);
    c->Iprev = fp(o_Iprev);
    c->rprev = fp(o_rprev);
    c->ids = reinterpret_cast<uint8_t*>(base + o_ids);
    c->bf = reinterpret_cast<float*>(base + o_bf);
    c->lnb = reinterpret_cast<float*>(base + o_lnb);
    c->bcf = reinterpret_cast<float*>(base + o_bcf);
    c->scal = reinterpret_cast<double*>(base + o_stats);
    c->elog = c->scal + NSCAL;
    c->b64 = c->elog + ELOG_SLOTS * ELOG_STRIDE;
    c->lnb64 = reinterpret_cast<double*>(base + o_lnb64);
    c->binit64 = reinterpret_cast<double*>(base + o_binit);
    c->tickets = reinterpret_cast<unsigned*>(base + o_tick);
    c->bsum = reinterpret_cast<double*>(base + o_bsum);
    c->partials = reinterpret_cast<double*>(base + o_part);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_scal), sizeof(double) * NSTATS) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_small), sizeof(double) * (8 * 3 * KMAX + 1)) != hipSuccess) {
        release(c);
        delete c;
        return GID_ERR_OUT_OF_MEMORY;
    }
    c->h_elog = c->h_scal + NSCAL;
    c->h_b64 = c->h_elog + ELOG_SLOTS * ELOG_STRIDE;
    c->h_target = c->h_small + 8 * 3 * KMAX;
    // zero the whole workspace once (tickets must start at zero)
    if (hipMemsetAsync(c->arena, 0, off, c->stream) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        release(c);
        delete c;
        return GID_ERR_HIP;
    }
    *out = c;
    return GID_OK;
}

gid_status gid_destroy(gid_ctx* c) {
    if (!c) return GID_OK;
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
    return GID_OK;
}

gid_status gid_set_base_colors(gid_ctx* c, const double* rgb) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!rgb || !colours_valid(rgb, 3 * c->K)) return fail(c, GID_ERR_INVALID_ARG, "base colours must be finite and > 0");
    for (int i = 0; i < 3 * c->K; ++i) c->binit_host[i] = rgb[i];
    gid_status s = upload_colours(c, rgb, true);
    if (s != GID_OK) return s;
    c->colors_set = true;
    c->have_prev = false;
    c->frame_index = 0;
    return GID_OK;
}

gid_status gid_reset_clip(gid_ctx* c) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!c->colors_set) return fail(c, GID_ERR_STATE, "base colours not set");
    return gid_set_base_colors(c, c->binit_host);
}

static gid_status load_frame_impl(gid_ctx* c, const float* frame, const uint8_t* ids, Args& a) {
    a = base_args(c);
    a.in_frame = frame;
    a.in_ids = ids;
    a.first = c->frame_index == 0;
    a.temporal = (c->prm.temporal && c->have_prev) ? 1 : 0;
    const Step s{};
    GID_HIP(c, L1(c, c->stream, KN_SCAN, a, s));
    GID_HIP(c, L1(c, c->stream, KN_PRECOMPUTE, a, s));
    c->frame_ready = true;
    return GID_OK;
}

// The learned warm start's judge, between the frame's precompute and its
// schedule: energy at the previous frame's result, the network's prediction
// from it, energy at the prediction, then the device-side choice of the start.
static gid_status enqueue_judge(gid_ctx* c, const Args& a) {
    Step sp{};
    sp.slot = JUDGE_PREV_SLOT;
    GID_HIP(c, L1(c, c->stream, KN_ENERGY, a, sp));
    GID_HIP(c, L1(c, c->stream, KN_ENERGY_FINISH, a, sp));
    GID_HIP(c, gidnet_forward_dev(c->wnet, c->stream, c->I, c->u, c->ucand, c->dbc));
    GID_HIP(c, L1(c, c->stream, KN_CAND_TABLES, a, Step{}));
    Args ac = a;
    ac.u = c->ucand;
    ac.b64 = c->b64c;
    ac.lnb64 = c->lnb64c;
    ac.bf = c->bfc;
    ac.lnb = c->lnbc;
    ac.bcf = c->bcfc;
    Step sn{};
    sn.slot = JUDGE_NET_SLOT;
    GID_HIP(c, L1(c, c->stream, KN_ENERGY, ac, sn));
    GID_HIP(c, L1(c, c->stream, KN_ENERGY_FINISH, ac, sn));
    GID_HIP(c, L1(c, c->stream, KN_JUDGE, a, Step{}));
    return GID_OK;
}

gid_status gid_set_warmstart(gid_ctx* c, gid_net* net) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!net) {
        c->wnet = nullptr;
        return GID_OK;
    }
    if (!gidnet_matches(net, c->K, c->W, c->H))
        return fail(c, GID_ERR_INVALID_ARG, "the network's width, height and K must match the context's");
    if (!c->warena) {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off += (bytes + 255) & ~(size_t)255;
            return o;
        };
        const size_t o_u = take(sizeof(float) * (size_t)c->n * c->ps), o_db = take(sizeof(float) * 3 * KMAX);
        const size_t o_b = take(sizeof(double) * 3 * KMAX), o_lb = take(sizeof(double) * 3 * KMAX);
        const size_t o_bf = take(sizeof(float) * 3 * KMAX), o_lnb = take(sizeof(float) * 3 * KMAX),
                     o_bc = take(sizeof(float) * 3 * KMAX);
        char* base = nullptr;
        if (hipMalloc(reinterpret_cast<void**>(&base), off) != hipSuccess)
            return fail(c, GID_ERR_OUT_OF_MEMORY, "warm-start workspace");
        c->warena = base;
        c->ucand = reinterpret_cast<float*>(base + o_u);
        c->dbc = reinterpret_cast<float*>(base + o_db);
        c->b64c = reinterpret_cast<double*>(base + o_b);
        c->lnb64c = reinterpret_cast<double*>(base + o_lb);
        c->bfc = reinterpret_cast<float*>(base + o_bf);
        c->lnbc = reinterpret_cast<float*>(base + o_lnb);
        c->bcfc = reinterpret_cast<float*>(base + o_bc);
    }
    c->wnet = net;
    return GID_OK;
}

gid_status gid_decompose_frame(gid_ctx* c, const float* frame, const uint8_t* ids, float* layers,
                               double* b_out, gid_frame_stats* stats) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!frame) return fail(c, GID_ERR_INVALID_ARG, "a frame is required");
    if (c->pending) return fail(c, GID_ERR_STATE, "the previous frame is pending: call gid_synchronize first");
    gid_status s = check_frame_ready(c);
    if (s != GID_OK) return s;
    if (c->target > 0.0) {
        // the pinned slot is not touched again before gid_synchronize
        *c->h_target = c->target;
        GID_HIP(c, hipMemcpyAsync(c->scal + S_TARGET, c->h_target, sizeof(double), hipMemcpyHostToDevice, c->stream));
    }
    Args a;
    if ((s = load_frame_impl(c, frame, ids, a)) != GID_OK) return s;
    const bool judged = c->wnet != nullptr && c->have_prev;
    if (judged && (s = enqueue_judge(c, a)) != GID_OK) return s;
    const int mode = c->prm.refine_mode;
    const bool refine = mode == GID_REFINE_EVERY_STEP || (mode == GID_REFINE_FIRST_FRAME && c->frame_index == 0);
    const bool record = c->prm.record_energy != 0;
    int nslots = 0;
    // energy-target mode: the iterations through the first check now; the rest,
    // and the output pass, from gid_synchronize once the device flags are back
    // (a frame that met its target skips them instead of replaying them as
    // launches that return at once)
    const bool split = c->target > 0.0 && target_split(c) < c->target_gn;
    if ((s = run_outer(c, a, refine, record, &nslots, split ? 1 : 0)) != GID_OK) return s;
    if (!split) {
        Args o = a;
        o.out = layers;
        GID_HIP(c, L1(c, c->stream, KN_OUTPUT, o, Step{}));
    }
    GID_HIP(c, hipMemcpyAsync(c->h_scal, c->scal, sizeof(double) * NSTATS, hipMemcpyDeviceToHost, c->stream));
    c->pend_rest = split;
    c->pend_refine = refine;
    c->pend_args = a;
    c->pend_layers = layers;
    c->pending = true;
    c->pend_b = b_out;
    c->pend_stats = stats;
    c->pend_nhalf = nslots;
    c->pend_target = c->target > 0.0;
    c->pend_first = c->target_first;
    c->pend_final_slot = (record && !c->pend_target) ? nslots - 1 : FINAL_SLOT;
    c->pend_frame = c->frame_index;
    c->pend_gn = c->prm.gn_iters;
    c->pend_had_prev = c->have_prev;
    c->pend_judged = judged;
    c->frame_index += 1;
    c->have_prev = true;
    return GID_OK;
}

gid_status gid_set_energy_target(gid_ctx* c, double target, int32_t max_gn) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (std::isnan(target) || (target > 0.0 && (max_gn < 1 || max_gn > 64)))
        return fail(c, GID_ERR_INVALID_ARG, "energy target must not be NaN and max_gn must be in 1..64");
    if (c->pending) return fail(c, GID_ERR_STATE, "the previous frame is pending: call gid_synchronize first");
    const int gn = target > 0.0 ? max_gn : 0;
    if (gn != c->target_gn) {   // the target-mode schedule is captured for one iteration count
        for (int k = 8; k < 32; ++k)
            if ((k & 8) && c->graphs[k]) {
                (void)hipGraphExecDestroy(c->graphs[k]);
                c->graphs[k] = nullptr;
            }
    }
    c->target = target > 0.0 ? target : 0.0;
    c->target_gn = gn;
    return GID_OK;
}

gid_status gid_set_energy_check_from(gid_ctx* c, int32_t first_gn) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (first_gn < 1 || first_gn > 64) return fail(c, GID_ERR_INVALID_ARG, "first_gn must be in 1..64");
    if (c->pending) return fail(c, GID_ERR_STATE, "the previous frame is pending: call gid_synchronize first");
    if (first_gn != c->target_first) {   // the target-mode schedule is captured for one first check
        for (int k = 8; k < 32; ++k)
            if ((k & 8) && c->graphs[k]) {
                (void)hipGraphExecDestroy(c->graphs[k]);
                c->graphs[k] = nullptr;
            }
    }
    c->target_first = first_gn;
    return GID_OK;
}

gid_status gid_synchronize(gid_ctx* c) {
    if (!c) return GID_ERR_INVALID_ARG;
    GID_HIP(c, hipStreamSynchronize(c->stream));
    if (c->pending && c->pend_rest) {
        // the flags after the first energy check: the frame's remaining outer
        // iterations only while it has not met its target (nor was rejected)
        c->pend_rest = false;
        if (c->h_scal[S_BADIN] == 0.0 && c->h_scal[S_DONE] == 0.0) {
            int ns = 0;
            const gid_status s = run_outer(c, c->pend_args, c->pend_refine, false, &ns, 2);
            if (s != GID_OK) {
                c->pending = false;
                return s;
            }
        }
        Args o = c->pend_args;
        o.out = c->pend_layers;
        GID_HIP(c, L1(c, c->stream, KN_OUTPUT, o, Step{}));
        GID_HIP(c, hipMemcpyAsync(c->h_scal, c->scal, sizeof(double) * NSTATS, hipMemcpyDeviceToHost, c->stream));
        GID_HIP(c, hipStreamSynchronize(c->stream));
    }
    if (c->ev_used) GID_HIP(c, collect_times(c));
    if (!c->pending) return GID_OK;
    c->pending = false;
    if (c->h_scal[S_BADIN] != 0.0) {
        // the frame was rejected on the device before any state changed
        c->frame_index = c->pend_frame;
        c->have_prev = c->pend_had_prev;
        return fail(c, GID_ERR_NUMERIC, "frame has non-finite values or cluster ids outside [0, K); state unchanged");
    }
    const double* fin = c->h_elog + (long long)c->pend_final_slot * ELOG_STRIDE;
    if (c->pend_b)
        for (int i = 0; i < 3 * c->K; ++i) c->pend_b[i] = c->h_b64[i];
    if (c->pend_stats) {
        gid_frame_stats* st = c->pend_stats;
        std::memset(st, 0, sizeof(*st));
        st->energy_final = fin[0];
        for (int v = 0; v < NTERMS; ++v) st->energy_terms[v] = fin[1 + v];
        const int gn_done = c->pend_target ? (int)c->h_scal[S_GN_DONE] : c->pend_gn;
        st->n_half = c->pend_target ? gn_done : c->pend_nhalf;
        for (int h = 0; h < st->n_half && h < GID_MAX_HALF_STEPS; ++h)   // unchecked iterations: NaN
            st->energy_half[h] = (c->pend_target && h + 1 < c->pend_first && h + 1 < gn_done)
                                     ? std::nan("")
                                     : c->h_elog[(long long)h * ELOG_STRIDE];
        for (int g = 0; g < 64; ++g) st->pcg_rz_last[g] = c->h_scal[S_RZ_LOG + g];
        st->gn_done = gn_done;
        st->pcg_breakdowns = (int32_t)c->h_scal[S_BREAKDOWNS];
        st->bstep_rejected = (int32_t)c->h_scal[S_BREJECT];
        st->frame_index = c->pend_frame;
        st->warm_start_learned = c->pend_judged ? (c->h_scal[S_LEARNED] != 0.0 ? 1 : 0) : -1;
        st->energy_start_previous =
            c->pend_judged ? c->h_elog[(long long)JUDGE_PREV_SLOT * ELOG_STRIDE] : std::nan("");
        st->energy_start_learned = c->pend_judged ? c->h_elog[(long long)JUDGE_NET_SLOT * ELOG_STRIDE] : std::nan("");
    }
    if (!std::isfinite(fin[0])) return fail(c, GID_ERR_NUMERIC, "final energy is not finite");
    return GID_OK;
}

// ------------------------------------------------------------ single steps

gid_status gid_load_frame(gid_ctx* c, const float* frame, const uint8_t* ids) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!frame) return fail(c, GID_ERR_INVALID_ARG, "a frame is required");
    if (c->pending) return fail(c, GID_ERR_STATE, "the previous frame is pending: call gid_synchronize first");
    gid_status s = check_frame_ready(c);
    if (s != GID_OK) return s;
    Args a;
    if ((s = load_frame_impl(c, frame, ids, a)) != GID_OK) return s;
    GID_HIP(c, hipStreamSynchronize(c->stream));
    return GID_OK;
}

static Args step_args(gid_ctx* c) {
    Args a = base_args(c);
    a.temporal = (c->prm.temporal && c->have_prev) ? 1 : 0;
    return a;
}

gid_status gid_set_state(gid_ctx* c, const float* u, const double* b) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!u) return fail(c, GID_ERR_INVALID_ARG, "u is required");
    if (b && !colours_valid(b, 3 * c->K)) return fail(c, GID_ERR_INVALID_ARG, "colours must be finite and > 0");
    GID_HIP(c, hipMemcpyAsync(c->u, u, sizeof(float) * c->ps * c->n, hipMemcpyDeviceToDevice, c->stream));
    if (b) {
        gid_status s = upload_colours(c, b, false);
        if (s != GID_OK) return s;
    }
    GID_HIP(c, hipStreamSynchronize(c->stream));
    return GID_OK;
}

gid_status gid_set_prev_frame(gid_ctx* c, const float* frame_prev, const float* r_prev) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!frame_prev || !r_prev) return fail(c, GID_ERR_INVALID_ARG, "previous frame and reflectance are required");
    gid_status s = check_frame_ready(c);
    if (s != GID_OK) return s;
    GID_HIP(c, hipMemcpyAsync(c->Iprev, frame_prev, sizeof(float) * 3 * c->ps, hipMemcpyDeviceToDevice, c->stream));
    GID_HIP(c, hipMemcpyAsync(c->rprev, r_prev, sizeof(float) * 3 * c->ps, hipMemcpyDeviceToDevice, c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    c->have_prev = true;
    c->frame_index = std::max(c->frame_index, 1);
    return GID_OK;
}

gid_status gid_get_state(gid_ctx* c, float* u, double* b) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (u) GID_HIP(c, hipMemcpyAsync(u, c->u, sizeof(float) * c->ps * c->n, hipMemcpyDeviceToDevice, c->stream));
    if (b) GID_HIP(c, hipMemcpyAsync(c->h_b64, c->b64, sizeof(double) * 3 * c->K, hipMemcpyDeviceToHost, c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    if (b)
        for (int i = 0; i < 3 * c->K; ++i) b[i] = c->h_b64[i];
    return GID_OK;
}

gid_status gid_eval_energy(gid_ctx* c, double* e, double* terms) {
    if (!c) return GID_ERR_INVALID_ARG;
    Args a = step_args(c);
    Step s{};
    s.slot = PROBE_SLOT;
    GID_HIP(c, launch_kernel(KN_ENERGY, a, s, c->stream));
    GID_HIP(c, launch_kernel(KN_ENERGY_FINISH, a, s, c->stream));
    GID_HIP(c, hipMemcpyAsync(c->h_elog, c->elog, sizeof(double) * ELOG_SLOTS * ELOG_STRIDE, hipMemcpyDeviceToHost,
                              c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    const double* pr = c->h_elog + (long long)PROBE_SLOT * ELOG_STRIDE;
    if (e) *e = pr[0];
    if (terms)
        for (int v = 0; v < NTERMS; ++v) terms[v] = pr[1 + v];
    return GID_OK;
}

gid_status gid_eval_rhs(gid_ctx* c, float* g, float* diag) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!g || !diag) return fail(c, GID_ERR_INVALID_ARG, "g and diag are required");
    Args a = step_args(c);
    Step s{};
    s.debug = 1;
    a.out = g;
    a.out2 = diag;
    GID_HIP(c, launch_kernel(KN_GN_BUILD, a, s, c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    return GID_OK;
}

gid_status gid_apply_normal(gid_ctx* c, const float* p, float* q) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!p || !q) return fail(c, GID_ERR_INVALID_ARG, "p and q are required");
    Args a = step_args(c);
    Step s{};
    s.debug = 1;
    a.pdebug = p;
    a.out = q;
    GID_HIP(c, launch_kernel(KN_PCG, a, s, c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    return GID_OK;
}

gid_status gid_layer_step(gid_ctx* c, double* rz) {
    if (!c) return GID_ERR_INVALID_ARG;
    Args a = step_args(c);
    Step s{};
    GID_HIP(c, launch_kernel(KN_GN_BUILD, a, s, c->stream));
    for (int i = 0; i < c->prm.pcg_iters; ++i) {
        s.iter = i;
        GID_HIP(c, launch_kernel(KN_PCG, a, s, c->stream));
    }
    s.refine = 0;
    s.add_delta = 1;
    s.log_rz = 1;
    s.iter = c->prm.pcg_iters - 1;
    s.gn = 0;
    GID_HIP(c, launch_kernel(KN_APPLY_BSUM, a, s, c->stream));
    GID_HIP(c, hipMemcpyAsync(c->h_scal, c->scal, sizeof(double) * NSCAL, hipMemcpyDeviceToHost, c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    if (rz) *rz = c->h_scal[S_RZ_LOG];
    return GID_OK;
}

gid_status gid_bstep_sums(gid_ctx* c, double* A, double* h) {
    if (!c) return GID_ERR_INVALID_ARG;
    if (!A || !h) return fail(c, GID_ERR_INVALID_ARG, "A and h are required");
    Args a = step_args(c);
    Step s{};
    s.refine = 1;
    GID_HIP(c, launch_kernel(KN_APPLY_BSUM, a, s, c->stream));
    s.debug = 1;
    GID_HIP(c, launch_kernel(KN_BSOLVE, a, s, c->stream));
    const int ns = bstep_nsums(c->K);
    double* tmp = c->h_elog;   // large enough pinned buffer (ELOG_SLOTS * ELOG_STRIDE >= ns)
    GID_HIP(c, hipMemcpyAsync(tmp, c->bsum, sizeof(double) * ns, hipMemcpyDeviceToHost, c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    const int K = c->K;
    for (int ch = 0; ch < 3; ++ch)
        for (int k = 0; k < K; ++k) {
            for (int l = 0; l < K; ++l) {
                const int kk = std::min(k, l), ll = std::max(k, l);
                A[(ch * K + k) * K + l] = tmp[ch * (K * (K + 1) / 2) + (kk * K - kk * (kk - 1) / 2) + (ll - kk)];
            }
            h[ch * K + k] = tmp[3 * K * (K + 1) / 2 + ch * K + k];
        }
    return GID_OK;
}

gid_status gid_base_step(gid_ctx* c, int32_t* accepted) {
    if (!c) return GID_ERR_INVALID_ARG;
    Args a = step_args(c);
    Step s{};
    s.refine = 1;
    GID_HIP(c, launch_kernel(KN_APPLY_BSUM, a, s, c->stream));
    GID_HIP(c, launch_kernel(KN_BSOLVE, a, s, c->stream));
    GID_HIP(c, hipMemcpyAsync(c->h_scal, c->scal, sizeof(double) * NSCAL, hipMemcpyDeviceToHost, c->stream));
    GID_HIP(c, hipStreamSynchronize(c->stream));
    if (accepted) *accepted = c->h_scal[S_BACCEPT] != 0.0;
    return GID_OK;
}

// --------------------------------------------------------- checkpoint

namespace {
struct StateHeader {
    uint32_t magic, version;
    int32_t W, H, K, frame_index, have_prev, colors_set;
};
size_t state_bytes(const gid_ctx* c) {
    return sizeof(StateHeader) + sizeof(double) * 2 * 3 * c->K + sizeof(float) * c->ps * (c->n + 6);
}
}  // namespace

gid_status gid_save_state(gid_ctx* c, void* buf, size_t* inout) {
    if (!c || !inout) return GID_ERR_INVALID_ARG;
    const size_t need = state_bytes(c);
    if (!buf) {
        *inout = need;
        return GID_OK;
    }
    if (*inout < need) return fail(c, GID_ERR_INVALID_ARG, "state buffer too small");
    char* p = static_cast<char*>(buf);
    StateHeader hd{STATE_MAGIC, 1, c->W, c->H, c->K, c->frame_index, c->have_prev, c->colors_set};
    std::memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    GID_HIP(c, hipStreamSynchronize(c->stream));
    GID_HIP(c, hipMemcpy(p, c->b64, sizeof(double) * 3 * c->K, hipMemcpyDeviceToHost));
    p += sizeof(double) * 3 * c->K;
    GID_HIP(c, hipMemcpy(p, c->binit64, sizeof(double) * 3 * c->K, hipMemcpyDeviceToHost));
    p += sizeof(double) * 3 * c->K;
    GID_HIP(c, hipMemcpy(p, c->u, sizeof(float) * c->ps * c->n, hipMemcpyDeviceToHost));
    p += sizeof(float) * c->ps * c->n;
    GID_HIP(c, hipMemcpy(p, c->Iprev, sizeof(float) * c->ps * 3, hipMemcpyDeviceToHost));
    p += sizeof(float) * c->ps * 3;
    GID_HIP(c, hipMemcpy(p, c->rprev, sizeof(float) * c->ps * 3, hipMemcpyDeviceToHost));
    *inout = need;
    return GID_OK;
}

gid_status gid_load_state(gid_ctx* c, const void* buf, size_t bytes) {
    if (!c || !buf) return GID_ERR_INVALID_ARG;
    if (bytes < state_bytes(c)) return fail(c, GID_ERR_INVALID_ARG, "state buffer too small");
    const char* p = static_cast<const char*>(buf);
    StateHeader hd;
    std::memcpy(&hd, p, sizeof(hd));
    if (hd.magic != STATE_MAGIC || hd.version != 1 || hd.W != c->W || hd.H != c->H || hd.K != c->K)
        return fail(c, GID_ERR_INVALID_ARG, "state does not match this context");
    p += sizeof(hd);
    double b[3 * KMAX], b0[3 * KMAX];
    std::memcpy(b, p, sizeof(double) * 3 * c->K);
    p += sizeof(double) * 3 * c->K;
    std::memcpy(b0, p, sizeof(double) * 3 * c->K);
    p += sizeof(double) * 3 * c->K;
    if (!colours_valid(b, 3 * c->K) || !colours_valid(b0, 3 * c->K))
        return fail(c, GID_ERR_INVALID_ARG, "state holds invalid colours");
    GID_HIP(c, hipStreamSynchronize(c->stream));
    gid_status s = upload_colours(c, b0, true);
    if (s != GID_OK) return s;
    if ((s = upload_colours(c, b, false)) != GID_OK) return s;
    for (int i = 0; i < 3 * c->K; ++i) c->binit_host[i] = b0[i];
    GID_HIP(c, hipMemcpy(c->u, p, sizeof(float) * c->ps * c->n, hipMemcpyHostToDevice));
    p += sizeof(float) * c->ps * c->n;
    GID_HIP(c, hipMemcpy(c->Iprev, p, sizeof(float) * c->ps * 3, hipMemcpyHostToDevice));
    p += sizeof(float) * c->ps * 3;
    GID_HIP(c, hipMemcpy(c->rprev, p, sizeof(float) * c->ps * 3, hipMemcpyHostToDevice));
    c->frame_index = hd.frame_index;
    c->have_prev = hd.have_prev != 0;
    c->colors_set = hd.colors_set != 0;
    return GID_OK;
}

gid_status gid_set_profiling(gid_ctx* c, int32_t enable) {
    if (!c) return GID_ERR_INVALID_ARG;
    GID_HIP(c, hipStreamSynchronize(c->stream));
    if (c->ev_used) GID_HIP(c, collect_times(c));
    c->profiling = enable != 0;
    if (c->profiling)
        for (int k = 0; k < GID_NUM_KERNEL_KINDS; ++k) {
            c->kind_ms[k] = 0.0;
            c->kind_n[k] = 0;
        }
    return GID_OK;
}

gid_status gid_get_kernel_times(gid_ctx* c, double* ms, int64_t* n) {
    if (!c || !ms || !n) return GID_ERR_INVALID_ARG;
    GID_HIP(c, hipStreamSynchronize(c->stream));
    if (c->ev_used) GID_HIP(c, collect_times(c));
    for (int k = 0; k < GID_NUM_KERNEL_KINDS; ++k) {
        ms[k] = c->kind_ms[k];
        n[k] = c->kind_n[k];
    }
    return GID_OK;
}

// ---------------------------------------------------------------- batches

struct gid_batch {
    std::vector<gid_ctx*> clips;
    std::vector<int> nb_snapshot;      // per-clip workgroup counts the batch was built with
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    double* h_out = nullptr;           // pinned: per clip final energy and input-check flag
    // cached schedule graphs by (active clips, refine, clips with the temporal prior on):
    // the descriptors are baked into the graph's kernel arguments
    std::map<std::tuple<unsigned long long, int, unsigned long long>, hipGraphExec_t> graphs;
    std::vector<int> active;           // clips of the pending step
    int launch = GID_BATCH_ONE_LAUNCH; // launch layout of a step
    ClipTable* d_table = nullptr;      // clip descriptors of the one-launch layout (device)
    ClipTable* h_table = nullptr;      // their pinned staging copy
    bool pending = false;
    std::string err;
};

namespace {
gid_status bfail(gid_batch* b, gid_status s, const std::string& m) {
    if (b) b->err = m;
    return s;
}
#define GID_BHIP(b, call)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return bfail((b), GID_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void batch_release(gid_batch* b) {
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->h_out) (void)hipHostFree(b->h_out);
    if (b->h_table) (void)hipHostFree(b->h_table);
    if (b->d_table) (void)hipFree(b->d_table);
}

// The launch layouts of one step over the active clips act (sorted by K) with
// their descriptors: per-K groups of at most BATCH_LAUNCH_MAX clips, and the clip
// table of the one-launch layout (filled in b->h_table; the caller uploads it).
struct BatchPlan {
    std::vector<BatchGrid> groups;
    TableGrid table{};
};

// A buffer as the table stores it: its byte offset from the table's device
// address, carried in the pointer field (0 for a null buffer).
extern "C++" {
template <typename T>
T* table_offset(T* p, const void* table) {
    if (!p) return nullptr;
    const std::ptrdiff_t off = reinterpret_cast<const char*>(p) - static_cast<const char*>(table);
    return reinterpret_cast<T*>(static_cast<std::uintptr_t>(off));
}
}

void plan_batch(gid_batch* b, const std::vector<int>& act, const std::vector<Args>& args, BatchPlan& p) {
    const int na = (int)act.size();
    p.groups.clear();
    for (int j = 0; j < na;) {
        const int K = b->clips[act[j]]->K;
        int m = 0;
        while (j + m < na && m < BATCH_LAUNCH_MAX && b->clips[act[j + m]]->K == K) ++m;
        BatchGrid g{};
        g.ba.n = m;
        g.ba.wg_pix[0] = g.ba.wg_bs[0] = 0;
        for (int q = 0; q < m; ++q) {
            const gid_ctx* c = b->clips[act[j + q]];
            g.ba.a[q] = args[j + q];
            g.ba.wg_pix[q + 1] = g.ba.wg_pix[q] + c->nblocks;
            g.ba.wg_bs[q + 1] = g.ba.wg_bs[q] + c->nb_bs;
        }
        g.total_pix = g.ba.wg_pix[m];
        g.total_bs = g.ba.wg_bs[m];
        g.k = K;
        p.groups.push_back(g);
        j += m;
    }
    ClipTable* t = b->h_table;
    t->n = na;
    t->wg_pix[0] = t->wg_bs[0] = 0;
    TableGrid& tg = p.table;
    tg = TableGrid{};
    tg.t = b->d_table;
    tg.n = na;
    for (int j = 0; j < na; ++j) {
        const gid_ctx* c = b->clips[act[j]];
        // the kernels decode every buffer as the table's device address plus a
        // byte offset (0 for a null buffer)
        Args e = args[j];
#define GID_ENC(f) e.f = table_offset(e.f, b->d_table);
        GID_TABLE_POINTERS(GID_ENC)
#undef GID_ENC
        t->a[j] = e;
        t->wg_pix[j + 1] = t->wg_pix[j] + c->nblocks;
        t->wg_bs[j + 1] = t->wg_bs[j] + c->nb_bs;
        tg.kmax = std::max(tg.kmax, c->K);
        tg.kmask |= 1u << c->K;
    }
    tg.total_pix = t->wg_pix[na];
    tg.total_bs = t->wg_bs[na];
}

// Every launch of kernel k for one step under the batch's layout.
hipError_t launch_plan(const gid_batch* b, const BatchPlan& p, Kern k, const Step& s, hipStream_t cs) {
    if (b->launch == GID_BATCH_ONE_LAUNCH) return launch_table(k, p.table, s, cs);
    for (const BatchGrid& g : p.groups) {
        const hipError_t e = launch_batch(k, g, s, cs);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

gid_status gid_batch_create(gid_ctx* const* ctxs, int32_t n, gid_batch** out) {
    if (!out || !ctxs || n < 1 || n > 64) return GID_ERR_INVALID_ARG;
    *out = nullptr;
    const gid_ctx* c0 = ctxs[0];
    if (!c0) return GID_ERR_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        const gid_ctx* c = ctxs[i];
        if (!c || c->stream != c0->stream || c->device != c0->device) return GID_ERR_INVALID_ARG;
        if (c->prm.gn_iters != c0->prm.gn_iters || c->prm.pcg_iters != c0->prm.pcg_iters ||
            c->prm.refine_mode != c0->prm.refine_mode || c->prm.record_energy != 0)
            return GID_ERR_INVALID_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return GID_ERR_INVALID_ARG;
    }
    gid_batch* b = new (std::nothrow) gid_batch();
    if (!b) return GID_ERR_OUT_OF_MEMORY;
    b->stream = c0->stream;
    for (int i = 0; i < n; ++i) {
        b->clips.push_back(ctxs[i]);
        b->nb_snapshot.push_back(ctxs[i]->nblocks);
    }
    int dev = 0;
    bool ok = hipGetDevice(&dev) == hipSuccess && hipSetDevice(c0->device) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_out), sizeof(double) * 2 * n) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_table), sizeof(ClipTable)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&b->d_table), sizeof(ClipTable)) == hipSuccess;
    (void)hipSetDevice(dev);
    if (!ok) {
        batch_release(b);
        delete b;
        return GID_ERR_OUT_OF_MEMORY;
    }
    std::memset(b->h_table, 0, sizeof(ClipTable));
    *out = b;
    return GID_OK;
}

gid_status gid_batch_destroy(gid_batch* b) {
    if (!b) return GID_OK;
    (void)hipStreamSynchronize(b->stream);
    batch_release(b);
    delete b;
    return GID_OK;
}

gid_status gid_batch_decompose(gid_batch* b, const float* const* frames, const uint8_t* const* ids,
                               float* const* layers) {
    if (!b || !frames || !ids) return bfail(b, GID_ERR_INVALID_ARG, "frames and ids are required");
    if (b->pending) return bfail(b, GID_ERR_STATE, "synchronize the previous batch step first");
    for (gid_ctx* c : b->clips) {
        if (c->wnet) return bfail(b, GID_ERR_UNSUPPORTED, "batched clips run without a learned warm start");
        if (c->target > 0.0) return bfail(b, GID_ERR_UNSUPPORTED, "batched clips run the fixed schedule (no energy target)");
        if (c->pending) return bfail(b, GID_ERR_STATE, "a clip has a pending single frame: synchronize it first");
    }
    const int n = (int)b->clips.size();
    std::vector<int> act;
    unsigned long long mask = 0;
    int first_count = 0;
    for (int i = 0; i < n; ++i) {
        if (!frames[i]) continue;
        gid_ctx* c = b->clips[i];
        if (!ids[i]) return bfail(b, GID_ERR_INVALID_ARG, "ids missing for an active clip");
        if (!c->colors_set) return bfail(b, GID_ERR_STATE, "base colours not set for a clip");
        if (c->nblocks != b->nb_snapshot[i]) return bfail(b, GID_ERR_STATE, "a clip was retuned after gid_batch_create");
        act.push_back(i);
        mask |= 1ull << i;
        first_count += c->frame_index == 0;
    }
    if (act.empty()) return GID_OK;
    const int mode = b->clips[0]->prm.refine_mode;
    if (mode == GID_REFINE_FIRST_FRAME && first_count != 0 && first_count != (int)act.size())
        return bfail(b, GID_ERR_UNSUPPORTED, "refine-first-frame needs the active clips at the same frame");
    const bool refine = mode == GID_REFINE_EVERY_STEP || (mode == GID_REFINE_FIRST_FRAME && first_count > 0);
    // active clips sorted by K (stable), their descriptors, and the step's launch
    // layout: one launch per kernel over all of them (the clip table, uploaded
    // ahead of the step's kernels in stream order), or one per K group
    std::stable_sort(act.begin(), act.end(), [&](int x, int y) { return b->clips[x]->K < b->clips[y]->K; });
    const int na = (int)act.size();
    std::vector<Args> args(na);
    unsigned long long tmask = 0;
    for (int j = 0; j < na; ++j) {
        const int i = act[j];
        gid_ctx* c = b->clips[i];
        Args a = base_args(c);
        a.in_frame = frames[i];
        a.in_ids = ids[i];
        a.out = layers ? layers[i] : nullptr;
        a.first = c->frame_index == 0;
        a.temporal = (c->prm.temporal && c->have_prev) ? 1 : 0;
        if (a.temporal) tmask |= 1ull << i;
        args[j] = a;
    }
    BatchPlan plan;
    plan_batch(b, act, args, plan);
    hipStream_t st = b->stream;
    if (b->launch == GID_BATCH_ONE_LAUNCH)
        GID_BHIP(b, hipMemcpyAsync(b->d_table, b->h_table, sizeof(ClipTable), hipMemcpyHostToDevice, st));
    auto each = [&](Kern k, const Step& s, hipStream_t cs) { return launch_plan(b, plan, k, s, cs); };
    const Step s0{};
    GID_BHIP(b, each(KN_SCAN, s0, st));
    GID_BHIP(b, each(KN_PRECOMPUTE, s0, st));
    const gid_params& prm = b->clips[0]->prm;
    auto enqueue = [&](hipStream_t cs) {
        int ns = 0;
        return enqueue_schedule(prm.gn_iters, prm.pcg_iters, refine, false,
                                [&](Kern k, const Step& s) { return each(k, s, cs); }, &ns);
    };
    if (prm.use_graph) {
        const auto key = std::make_tuple(mask, (refine ? 1 : 0) | (b->launch << 1), tmask);
        auto it = b->graphs.find(key);
        if (it == b->graphs.end()) {
            hipGraphExec_t ex = nullptr;
            hipError_t e = capture_graph(&b->cap_stream, enqueue, &ex);
            if (e != hipSuccess) return bfail(b, GID_ERR_HIP, std::string("batch graph capture: ") + hipGetErrorString(e));
            it = b->graphs.emplace(key, ex).first;
        }
        GID_BHIP(b, hipGraphLaunch(it->second, st));
    } else {
        GID_BHIP(b, enqueue(st));
    }
    GID_BHIP(b, each(KN_OUTPUT, s0, st));
    for (int j = 0; j < na; ++j) {
        gid_ctx* c = b->clips[act[j]];
        GID_BHIP(b, hipMemcpyAsync(b->h_out + 2 * act[j], c->elog + (long long)FINAL_SLOT * ELOG_STRIDE,
                                   sizeof(double), hipMemcpyDeviceToHost, st));
        GID_BHIP(b, hipMemcpyAsync(b->h_out + 2 * act[j] + 1, c->scal + S_BADIN, sizeof(double),
                                   hipMemcpyDeviceToHost, st));
        c->frame_index += 1;
        c->have_prev = true;
        c->frame_ready = true;
    }
    b->active = act;
    b->pending = true;
    return GID_OK;
}

gid_status gid_batch_synchronize(gid_batch* b, double* energies) {
    if (!b) return GID_ERR_INVALID_ARG;
    GID_BHIP(b, hipStreamSynchronize(b->stream));
    if (!b->pending) return GID_OK;
    b->pending = false;
    const int n = (int)b->clips.size();
    if (energies)
        for (int i = 0; i < n; ++i) energies[i] = std::nan("");
    gid_status st = GID_OK;
    for (int i : b->active) {
        if (b->h_out[2 * i + 1] != 0.0) {
            gid_ctx* c = b->clips[i];      // frame rejected on the device: no state changed
            c->frame_index -= 1;
            c->have_prev = c->frame_index > 0;
            st = GID_ERR_NUMERIC;
            continue;
        }
        if (energies) energies[i] = b->h_out[2 * i];
        if (!std::isfinite(b->h_out[2 * i])) st = GID_ERR_NUMERIC;
    }
    if (st != GID_OK) b->err = "a clip's frame was rejected or its energy is not finite";
    return st;
}

const char* gid_batch_last_error(const gid_batch* b) { return b ? b->err.c_str() : "no batch"; }

gid_status gid_batch_set_launch(gid_batch* b, int32_t mode) {
    if (!b) return GID_ERR_INVALID_ARG;
    if (mode != GID_BATCH_ONE_LAUNCH && mode != GID_BATCH_PER_K) return bfail(b, GID_ERR_INVALID_ARG, "unknown launch layout");
    if (b->pending) return bfail(b, GID_ERR_STATE, "synchronize the pending batch step first");
    b->launch = mode;
    return GID_OK;
}

gid_status gid_batch_get_launch(const gid_batch* b, int32_t* mode) {
    if (!b || !mode) return GID_ERR_INVALID_ARG;
    *mode = b->launch;
    return GID_OK;
}

gid_status gid_batch_autotune(gid_batch* b, int32_t* chosen) {
    if (!b) return GID_ERR_INVALID_ARG;
    if (b->pending) return bfail(b, GID_ERR_STATE, "synchronize the pending batch step first");
    for (const gid_ctx* c : b->clips)
        if (!c->frame_ready) return bfail(b, GID_ERR_STATE, "every clip needs a loaded frame: the tuner times the real layer step");
    GID_BHIP(b, hipStreamSynchronize(b->stream));
    const int n = (int)b->clips.size();
    std::vector<int> act(n);
    for (int i = 0; i < n; ++i) act[i] = i;
    std::stable_sort(act.begin(), act.end(), [&](int x, int y) { return b->clips[x]->K < b->clips[y]->K; });
    std::vector<Args> args(n);
    for (int j = 0; j < n; ++j) args[j] = step_args(b->clips[act[j]]);
    BatchPlan plan;
    plan_batch(b, act, args, plan);
    GID_BHIP(b, hipMemcpyAsync(b->d_table, b->h_table, sizeof(ClipTable), hipMemcpyHostToDevice, b->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GID_BHIP(b, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(b, GID_ERR_HIP, "hipEventCreate failed");
    }
    // one outer iteration of every clip without its updates (the build, the
    // pcg_iters PCG iterations and the base-colour sums; u and the colours are not
    // changed) under each layout, the best of five repetitions after one that warms
    // the caches.  The per-K layout is kept only when it is 5% faster: the
    // kernels the timing leaves out (scan, solve, energy, output) favour the
    // one-launch layout, which issues one launch where the other issues one per K.
    const int saved = b->launch;
    const int P = b->clips[0]->prm.pcg_iters;
    const int modes[2] = {GID_BATCH_ONE_LAUNCH, GID_BATCH_PER_K};
    double ms_of[2] = {1e30, 1e30};
    gid_status status = GID_OK;
    for (int mi = 0; mi < 2 && status == GID_OK; ++mi) {
        b->launch = modes[mi];
        for (int rep = 0; rep < 6; ++rep) {
            bool ok = hipEventRecord(e0, b->stream) == hipSuccess &&
                      launch_plan(b, plan, KN_GN_BUILD, Step{}, b->stream) == hipSuccess;
            for (int i = 0; ok && i < P; ++i) {
                Step s{};
                s.iter = i;
                ok = launch_plan(b, plan, KN_PCG, s, b->stream) == hipSuccess;
            }
            Step sb{};
            sb.iter = P - 1;
            sb.refine = 1;
            sb.add_delta = 0;     // sums only: the layer step is not applied
            ok = ok && launch_plan(b, plan, KN_APPLY_BSUM, sb, b->stream) == hipSuccess;
            if (!ok || hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                status = bfail(b, GID_ERR_HIP, "batch autotune launch failed");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) ms_of[mi] = std::min(ms_of[mi], (double)ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != GID_OK) {
        b->launch = saved;
        return status;
    }
    b->launch = ms_of[1] < 0.95 * ms_of[0] ? GID_BATCH_PER_K : GID_BATCH_ONE_LAUNCH;
    if (chosen) *chosen = b->launch;
    return GID_OK;
}

// ------------------------------------------------------------- autotuner

namespace {
bool cache_lookup(const char* path, int W, int H, int K, int* nb) {
    FILE* f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return false;
    int w, h, k, v;
    bool found = false;
    while (std::fscanf(f, "%d %d %d %d", &w, &h, &k, &v) == 4)
        if (w == W && h == H && k == K) {
            *nb = v;
            found = true;
        }
    std::fclose(f);
    return found;
}
}  // namespace

gid_status gid_autotune(gid_ctx* c, const char* cache_path, int32_t* chosen) {
    if (!c) return GID_ERR_INVALID_ARG;
    int nb = 0;
    if (cache_lookup(cache_path, c->W, c->H, c->K, &nb)) {
        set_nblocks(c, nb);
        if (chosen) *chosen = c->nblocks;
        return GID_OK;
    }
    // time the real layer-step kernels (the build and the P PCG iterations) on the
    // loaded frame for each candidate grid; u and the colours are not changed
    if (!c->frame_ready)
        return fail(c, GID_ERR_STATE, "load or decompose a frame first: the tuner times the real layer step on it");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GID_HIP(c, hipEventCreate(&e0));
    GID_HIP(c, hipEventCreate(&e1));
    // candidates: the default shape (one tile per workgroup up to NB_MAX) first,
    // then fixed counts; another shape replaces the default only when it is 3%
    // faster (differences below that are within the run-to-run spread)
    // (every multiple of 64 up to NB_MAX: the best count sits near the number of
    // workgroups the CUs hold at once, which depends on K, and a count that deals
    // the tiles evenly avoids a partly filled last round)
    const int def_nb = std::min((int)align_up((size_t)c->ntiles, 8), NB_MAX);
    std::vector<int> cand{def_nb};
    for (int v = 64; v <= NB_MAX; v += 64) cand.push_back(v);
    double best_ms = 1e30;
    int best = c->nblocks;
    gid_status status = GID_OK;
    for (int ci = 0; ci < (int)cand.size(); ++ci) {
        const int nbc = cand[ci];
        if (ci > 0 && (nbc == def_nb || nbc > (int)align_up((size_t)c->ntiles, 8))) continue;
        set_nblocks(c, nbc);
        const Args a = step_args(c);
        float ms_total = 0.0f;
        for (int rep = 0; rep < 4; ++rep) {
            bool ok = hipEventRecord(e0, c->stream) == hipSuccess &&
                      launch_kernel(KN_GN_BUILD, a, Step{}, c->stream) == hipSuccess;
            for (int i = 0; ok && i < c->prm.pcg_iters; ++i) {
                Step s{};
                s.iter = i;
                ok = launch_kernel(KN_PCG, a, s, c->stream) == hipSuccess;
            }
            if (!ok || hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                status = fail(c, GID_ERR_HIP, "autotune launch failed");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) ms_total += ms;      // the first repetition warms caches
        }
        if (status != GID_OK) break;
        const double need = (ci == 0) ? 1.0 : (best == def_nb ? 0.97 : 1.0);
        if (ms_total < best_ms * need) {
            best_ms = ms_total;
            best = c->nblocks;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_nblocks(c, best);
    if (status != GID_OK) return status;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%d %d %d %d\n", c->W, c->H, c->K, c->nblocks);
            std::fclose(f);
        }
    }
    if (chosen) *chosen = c->nblocks;
    return GID_OK;
}

gid_status gid_set_workgroups(gid_ctx* c, int32_t nb) {
    if (!c || nb < 8 || nb > NB_TUNE_MAX) return GID_ERR_INVALID_ARG;
    GID_HIP(c, hipStreamSynchronize(c->stream));
    set_nblocks(c, nb);
    return GID_OK;
}

int32_t gid_get_workgroups(const gid_ctx* c) { return c ? c->nblocks : 0; }

const char* gid_status_string(gid_status s) {
    switch (s) {
        case GID_OK: return "ok";
        case GID_ERR_INVALID_ARG: return "invalid argument";
        case GID_ERR_OUT_OF_MEMORY: return "out of memory";
        case GID_ERR_HIP: return "HIP runtime error";
        case GID_ERR_NUMERIC: return "non-finite value";
        case GID_ERR_STATE: return "call out of order";
        case GID_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* gid_last_error(const gid_ctx* c) { return c ? c->err.c_str() : "no context"; }

}  // extern "C"
