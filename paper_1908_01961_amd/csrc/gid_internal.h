// Internal declarations of libgid: device workspace, kernel arguments and the
// launchers of the solver kernels (gid_kernels.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "gid.h"

namespace gid {

constexpr int TX = 64;            // tile width = one wavefront row
constexpr int TYW = 4;            // thread rows per workgroup (256 threads)
constexpr int NTHREADS = TX * TYW;
constexpr int KMAX = 16;
constexpr int NTERMS = GID_NUM_TERMS;
constexpr int ELOG_STRIDE = 1 + NTERMS;   // total + terms per energy slot
constexpr int ELOG_SLOTS = GID_MAX_HALF_STEPS + 4;
constexpr int JUDGE_PREV_SLOT = ELOG_SLOTS - 4;    // warm-start judge: energy at the previous frame's result
constexpr int JUDGE_NET_SLOT = ELOG_SLOTS - 3;     // warm-start judge: energy at the network's prediction
constexpr int ELOG_FINAL_SLOT = ELOG_SLOTS - 2;    // the frame's final energy when half-steps are not recorded
constexpr int NB_TUNE_MAX = 2048;   // workgroups of a per-pixel launch (at most)
constexpr int NB_BS_MAX = 1024;  // workgroups of the apply + base-colour-sum pass (at most)

// Slots of the device scalar array (doubles).
enum Scal : int {
    S_STOP = 0,         // nonzero: PCG stopped by a guard (rest of the layer step is a no-op);
                        // 1 + the iteration whose launch refused the update before it (apply = P)
    S_BREAKDOWNS,   // count of PCG breakdowns this frame
    S_BREJECT,      // count of rejected base-colour steps this frame
    S_BACCEPT,      // 1 if the last base-colour step was accepted
    S_BADIN,        // non-finite frame values or out-of-range ids in this frame's input
    S_CAND_OK,      // 1 if the network's colour prediction is admissible (every component in (1e-4, inf))
    S_LEARNED,      // 1 if the judge kept the network's prediction as this frame's start
    S_DONE,         // 1 once the frame reached its energy target (its remaining iterations are no-ops)
    S_GN_DONE,      // outer iterations completed in this frame (energy-target mode)
    S_TARGET,       // the frame's energy target (set by the host before the frame; not reset)
    S_RZ_LOG,       // first of 64 slots: final <r, z> of each layer step
    NSCAL = S_RZ_LOG + 64
};

// Reduction buffers (one partial array and ticket per reduction site).
// R_RZ0: <r0, z0> of the Gauss-Newton build; PCG iteration i publishes its sums
// (PcgVal) to R_PCGA / R_PCGB by the parity of i.
enum RedSite : int { R_RZ0 = 0, R_PCGA, R_PCGB, R_EN, R_BS, R_SCAN, NRED };

// Per-workgroup sums of one PCG iteration: <p, q>, <q, z>, <q, M^-1 q>, <r, z>
// with q = A p and z = M^-1 r.
enum PcgVal : int { PV_PQ = 0, PV_QZ, PV_QMQ, PV_RZ, PV_N };
static_assert(PV_N <= NTERMS, "a reduction site holds NTERMS values per workgroup");

struct Lam {
    float data, cl, rs, p, rc, mo, is, sm, nn, ir, cr;
    float eps_nn, eps_irls, rk;
    double gate, cfloor;     // compared in FP64 against FP64 chromaticity distances
};

// Fields that change from launch to launch of one schedule.
struct Step {
    int iter;       // PCG iteration (matvec, update); apply pass: index of the last one
    int slot;       // energy log slot
    int gn;         // Gauss-Newton iteration (log of <r, z>)
    int refine;     // apply pass: accumulate the base-colour sums
    int add_delta;  // apply pass: u += delta (0: sums only)
    int log_rz;     // apply pass: record the final <r, z> of the layer step
    int debug;      // single-step access: skip scalar bookkeeping / use caller buffers
    int check;      // energy total: compare with the frame's target after an outer iteration
};

// One clip: its geometry, parameters and every buffer a kernel may touch (every
// pointer field is listed in GID_TABLE_POINTERS below, which the clip table
// encodes and decodes).
// Passed by value to single-clip launches and, up to BATCH_LAUNCH_MAX of them,
// inside a BatchArgs to batched launches.
struct Args {
    int W, H, K;
    int ppt;                 // pixel rows per thread (tile height = TYW * ppt)
    int ntx, nty, ntiles;    // tile grid
    int nblocks;             // workgroups of a per-pixel launch (multiple of 8)
    int nb_bs;               // workgroups of the apply + base-colour-sum launch (multiple of 8)
    long long ps;            // plane stride in elements
    Lam lam;
    int temporal;            // consistency prior active for this frame
    int first;               // initialise the unknowns (first frame of a clip)
    int cr_literal;
    int bstep_sum;           // base-colour data sum not divided by the pixel count
    int spatial;             // spatial pairs of the consistency prior (Sec. 6.1)
    unsigned spatial_seed;   // their sampler's seed
    float* u;                // n planes
    float* delta;            // x: the layer step accumulated by PCG
    float* zA;               // preconditioned residual z = M^-1 r, even PCG iterations from 2
    float* zB;               // z, odd iterations (z0 = p0 lives in pA)
    float* pA;               // search direction, even iterations (and p0)
    float* pB;               // search direction, odd iterations
    float* qA;               // M^-1 q with q = A p, even iterations
    float* qB;               // M^-1 q, odd iterations
    float* minv;             // n planes of debug output (the Jacobi diagonal is rebuilt from u where needed)
    float* I;                // 3 planes (frame copy)
    uint8_t* ids;
    float* wsr;              // 1 plane
    float* tg;               // 6 planes: number of temporal pairs, sum of paired r_prev per channel,
                             // bit mask of the paired 3 x 3 window positions, bit mask of the
                             // active spatial pairs (neighbours right, down-right, down, down-left,
                             // left, up-left, up, up-right)
    float* Iprev;            // 3 planes, previous frame
    float* rprev;            // 3 planes, previous frame's final r
    float* bf;               // K x 3 base colours, float
    float* lnb;              // K x 3 ln b, float
    float* bcf;              // K x 3 base colours minus their channel mean, float
    double* b64;             // K x 3 base colours, double (master)
    double* lnb64;           // K x 3 ln b, double
    double* binit64;         // K x 3 initial estimate
    double* scal;
    double* partials;        // NRED sites x max partial count x max values
    unsigned* tickets;       // NRED
    double* elog;            // ELOG_SLOTS x ELOG_STRIDE
    double* bsum;            // reduced base-colour sums
    const float* in_frame;   // caller frame (precompute)
    const uint8_t* in_ids;   // caller ids (precompute)
    float* out;              // caller output planes (output / debug)
    float* out2;             // second caller output (debug diag)
    const float* pdebug;     // caller p (debug apply)
    long long part_stride;   // doubles per reduction site
    // learned warm start (null unless a network is attached)
    float* ucand;            // n planes: the network's prediction
    float* dbc;              // 3K predicted colour change (FP32)
    double* b64c;            // K x 3 candidate colours and their tables
    double* lnb64c;
    float* bfc;
    float* lnbc;
    float* bcfc;
};

// Number of base-colour step sums: 3 K(K+1)/2 Gram entries + 3K right-hand side entries.
__host__ __device__ inline int bstep_nsums(int K) { return 3 * K * (K + 1) / 2 + 3 * K; }

enum Kern : int {
    KN_SCAN = 0, KN_PRECOMPUTE, KN_GN_BUILD, KN_PCG, KN_APPLY_BSUM, KN_BSOLVE,
    KN_ENERGY, KN_ENERGY_FINISH, KN_OUTPUT, KN_TABLES, KN_CAND_TABLES, KN_JUDGE
};

// A batched launch over several clips of one K.  The descriptors travel as a
// kernel argument (kernel arguments are read with scalar loads and pointers read
// from them are known to be global, so the kernels keep the single-clip code);
// wg_pix / wg_bs are prefix sums of the per-clip workgroup counts (each a
// multiple of 8) of the per-pixel and of the apply + base-colour-sum launches.
constexpr int BATCH_LAUNCH_MAX = 8;
struct BatchArgs {
    Args a[BATCH_LAUNCH_MAX];
    int wg_pix[BATCH_LAUNCH_MAX + 1];
    int wg_bs[BATCH_LAUNCH_MAX + 1];
    int n;
};
static_assert(sizeof(BatchArgs) + sizeof(Step) <= 4096, "kernel arguments are limited to 4 KB");

struct BatchGrid {
    BatchArgs ba;
    int total_pix, total_bs;
    int k;                  // the K every clip of this launch has
};

// Every active clip of a batch in one launch per kernel, whatever its K.  The
// descriptors do not fit the kernel arguments, so they live in a device table
// uploaded before the step; each workgroup finds its clip by a binary search over
// the workgroup prefix sums and runs the body compiled for that clip's K.  A
// kernel of this family holds the bodies of every K up to its bound (4, 8, 12 or
// 16, the smallest at or above the largest K of the batch), so its registers and
// dynamic LDS are those of the largest body.
constexpr int TABLE_CLIPS_MAX = 64;
// The pointer fields of Args; in a ClipTable each holds the byte offset of its
// buffer from the table's device address (0 for a null buffer).
#define GID_TABLE_POINTERS(X)                                                                         \
    X(u) X(delta) X(zA) X(zB) X(pA) X(pB) X(qA) X(qB) X(minv) X(I) X(ids) X(wsr) X(tg) X(Iprev)        \
    X(rprev) X(bf) X(lnb) X(bcf) X(b64) X(lnb64) X(binit64) X(scal) X(partials) X(tickets) X(elog)     \
    X(bsum) X(in_frame) X(in_ids) X(out) X(out2) X(pdebug) X(ucand) X(dbc) X(b64c) X(lnb64c) X(bfc)    \
    X(lnbc) X(bcfc)
struct ClipTable {
    int n;
    int wg_pix[TABLE_CLIPS_MAX + 1];
    int wg_bs[TABLE_CLIPS_MAX + 1];
    Args a[TABLE_CLIPS_MAX];
};

struct TableGrid {
    const ClipTable* t;     // device copy
    int n, total_pix, total_bs;
    int kmax;               // largest K of the clips
    unsigned kmask;         // bit K set when a clip has that K
};

// Launch one kernel for one clip / for a batch of one K / for a whole batch
// (returns the launch error).
hipError_t launch_kernel(Kern k, const Args& a, const Step& st, hipStream_t s);
hipError_t launch_batch(Kern k, const BatchGrid& g, const Step& st, hipStream_t s);
hipError_t launch_table(Kern k, const TableGrid& g, const Step& st, hipStream_t s);
// the four clip-table families (gid_table4.hip ... gid_table16.hip)
hipError_t launch_table4(Kern k, const TableGrid& g, const Step& st, hipStream_t s);
hipError_t launch_table8(Kern k, const TableGrid& g, const Step& st, hipStream_t s);
hipError_t launch_table12(Kern k, const TableGrid& g, const Step& st, hipStream_t s);
hipError_t launch_table16(Kern k, const TableGrid& g, const Step& st, hipStream_t s);

}  // namespace gid
