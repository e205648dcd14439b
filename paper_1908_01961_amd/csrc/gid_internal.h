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
constexpr int ELOG_SLOTS = GID_MAX_HALF_STEPS + 2;

// Slots of the device scalar array (doubles).
enum Scal : int {
    S_STOP = 0,         // 1: PCG stopped by a guard (rest of the layer step is a no-op)
    S_BREAKDOWNS,   // count of PCG breakdowns this frame
    S_BREJECT,      // count of rejected base-colour steps this frame
    S_BACCEPT,      // 1 if the last base-colour step was accepted
    S_BADIN,        // non-finite frame values or out-of-range ids in this frame's input
    S_RZ_LOG,       // first of 64 slots: final <r, z> of each layer step
    NSCAL = S_RZ_LOG + 64
};

// Reduction buffers (one partial array and ticket per reduction site).
// <r, z> alternates between R_RZA and R_RZB by PCG iteration parity.
enum RedSite : int { R_RZA = 0, R_RZB, R_PQ, R_EN, R_BS, R_SCAN, NRED };

struct Lam {
    float data, cl, rs, p, rc, mo, is, sm, nn, ir, cr;
    float eps_nn, eps_irls, rk;
    double gate, cfloor;     // compared in FP64 against FP64 chromaticity distances
};

// Everything a kernel may touch; passed by value.
struct Args {
    int W, H, K;
    int ppt;                 // pixel rows per thread (tile height = TYW * ppt)
    int ntx, nty, ntiles;    // tile grid
    int nblocks;             // launched workgroups (multiple of 8)
    long long ps;            // plane stride in elements
    Lam lam;
    int temporal;            // consistency prior active for this frame
    int first;               // initialise the unknowns (first frame of a clip)
    int refine;              // base-colour step active in this GN iteration
    int cr_literal;
    int iter;                // PCG iteration index (matvec / update)
    int slot;                // energy log slot
    int debug;               // single-step access: skip scalar bookkeeping
    int gn;                  // GN iteration index (rz log)
    int add_delta;           // apply pass: u += delta (0: sums only)
    int log_rz;              // apply pass: record the final <r, z> of the layer step
    float* u;                // n planes
    float* delta;
    float* res;
    float* pold;             // p of the previous PCG iteration
    float* pnew;             // p of this iteration
    float* q;
    float* minv;
    float* I;                // 3 planes (frame copy)
    uint8_t* ids;
    float* wsr;              // 1 plane
    float* tg;               // 4 planes: number of temporal pairs, sum of paired r_prev per channel
    float* Iprev;            // 3 planes, previous frame
    float* rprev;            // 3 planes, previous frame's final r
    float* bf;               // K x 3 base colours, float
    float* lnb;              // K x 3 ln b, float
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
};

// Number of base-colour step sums: 3 K(K+1)/2 Gram entries + 3K right-hand side entries.
__host__ __device__ inline int bstep_nsums(int K) { return 3 * K * (K + 1) / 2 + 3 * K; }

// Launchers (return hipError_t of the launch).
hipError_t launch_precompute(const Args& a, hipStream_t s);
hipError_t launch_gn_build(const Args& a, hipStream_t s);
hipError_t launch_matvec(const Args& a, hipStream_t s);
hipError_t launch_update(const Args& a, hipStream_t s);
hipError_t launch_apply_bsum(const Args& a, int nblocks_bs, hipStream_t s);
hipError_t launch_bsolve(const Args& a, int nblocks_bs, hipStream_t s);
hipError_t launch_energy(const Args& a, hipStream_t s);
hipError_t launch_energy_finish(const Args& a, hipStream_t s);
hipError_t launch_output(const Args& a, hipStream_t s);
hipError_t launch_reset_frame(const Args& a, hipStream_t s);
hipError_t launch_scan(const Args& a, hipStream_t s);

}  // namespace gid
