// Batched 2D solves (one persistent launch for many problems): device
// structures shared by k_batch.hip and vfs_batch.hip.
#pragma once

#include "vfs_internal.h"

namespace vfs {

constexpr int kBatchVariants = 6;   // tile shapes (BX x BY): 64x4, 64x8, 32x8, 128x2, 64x12, 64x16

// One problem as seen by the batched kernels (pointers into its context).
struct BProb {
    Geo g;
    int item0, nt;                // first work item and item count of this step (active tiles)
    int ntx, nty, full0;          // tile grid and first tile in the list of all tiles
    float *x32, *r32, *p0, *p1, *q32;
    float *r32b, *q32b;           // second r and q buffers (iteration parity)
    const float *a, *c, *K, *dinv;
    const float* ead;             // e = a D^-1, the weight of the residual and A p
    double *x64, *r64;
    const double *a64, *c64, *K64, *b64;
};

// Per-problem mode inside the persistent solve.  The owner item writes the
// mode of the next phase into slot (phase+1)&1 while every item reads slot
// phase&1, so a mode change never races with the problem's other items.
enum BMode : int { BM_CG = 0, BM_AXPY = 1, BM_RESID = 2, BM_DECIDE = 3, BM_DONE = 4 };
struct BPhase {
    int mode;
    int kloc;   // CG iteration within the current inner solve
};

// Per-problem solver state (written by the owner item / finalize workgroup;
// a field is never written in the phase in which the problem's other items
// read it).
struct BState {
    BPhase ph[2];
    double bb;        // |r32|^2 at the start of the pass (1 up to rounding)
    double rho2;      // |r64|^2 of the current iterate
    double bb64;      // |b|^2
    double rel;       // FP64 true relative residual
    double tol_in2;   // inner (FP32) relative tolerance squared for the next pass
    int needs;        // 1: the problem needs a solve (set before the persistent launch)
    int retired;      // 1 once the problem is DONE (read when gathering a phase's items)
    int last_iter;    // iterations of the last inner solve
    int iters_total;  // iterations over all passes
    int passes;
    unsigned long long t_start, t_done;   // device wall clock
};

// Grid barrier: workgroup b arrives at group counter b % kBarGroups, the last
// arrival of each group at the top counter, the last of those advances the
// generation.  Group counters sit kBarStride words apart (own cache lines).
constexpr int kBarGroups = 16, kBarStride = 32;
struct BatchCtl {
    unsigned bar_count;   // top-level arrivals
    unsigned bar_gen;
    int abort;
    int n_done;
    int n_need;
    int pad;
    unsigned long long spin_ticks;   // barrier wait deadline (wall-clock ticks)
    unsigned bar_grp[kBarGroups * kBarStride];
};

// Work items are the active tiles of every problem, rebuilt after each
// assembly: item w is tile item_tile[w] of problem item_prob[w], a problem's
// items are contiguous and in tile order, and *nlive holds their number (read
// on the device, so a captured graph stays valid when the count changes).
struct BatchArgs {
    BProb* prob;
    BState* state;
    BatchCtl* ctl;
    const int* item_prob;
    const int* item_tile;
    const int* nlive;
    int nprob;
    double* partF[2];   // five CG partials per item, by iteration parity
    double* partR;      // FP64 |r64|^2 partial per item
    double tol;
    int max_iter, max_iter_pass, max_passes;
    int first_pass;
    int bx, by;
};

void batch_tile_shape(int variant, int* bx, int* by);
size_t batch_lds_bytes(int variant, int word);
int batch_pcg_occupancy(int variant, int* blocks_per_cu);
void launch_batch_pcg(int variant, const BatchArgs& A, int grid, hipStream_t s);
void launch_batch_resid(int variant, const BatchArgs& A, int grid, hipStream_t s);
void launch_batch_finalize(const BatchArgs& A, hipStream_t s);
void launch_batch_zero(const BatchArgs& A, hipStream_t s);
void launch_batch_tile_flags(const BProb* prob, const int* full_prob, int nfull, int bx, int by,
                             int* flags, hipStream_t s);
void launch_batch_reset_ctl(BatchCtl* ctl, hipStream_t s);

// single-problem pieces reused by the batch (vfs_api.hip)
int ctx_assemble(vfs_ctx* ctx, double dt);
int ctx_recover(vfs_ctx* ctx);

}  // namespace vfs
