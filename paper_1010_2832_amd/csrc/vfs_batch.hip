// C ABI of the batched 2D solver: many independent steps of different grid
// sizes whose CG solves run in one persistent launch per refinement pass.
// Each pass (reset, persistent FP32 PCG over all problems, x64 update, FP64
// residual, per-problem decision) is captured once in a hipGraph and
// replayed.  Assembly and velocity recovery reuse the single-problem
// kernels on each problem's own context.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "vfs_batch.h"

using namespace vfs;

struct vfs_batch {
    int n = 0;
    std::vector<vfs_ctx*> ctx;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;   // created here: graph capture needs a non-null stream
    std::string err;
    // solver settings
    double tol = 1e-6;
    int max_iter = 200000;
    int max_iter_pass = 50000;
    int max_passes = 8;
    // launch configuration (autotuned)
    int variant = 1;
    int blocks_per_cu = 2;   // requested
    int bpc_used = 0;        // after the occupancy limit
    int grid = 0;
    int ncu = 0;
    // device structures
    BProb* d_prob = nullptr;
    BState* d_state = nullptr;
    BatchCtl* d_ctl = nullptr;
    int* d_item_prob = nullptr;   // live items (capacity nfull): problem, tile
    int* d_item_tile = nullptr;
    int* d_nlive = nullptr;       // live item count, read by the kernels
    int* d_full_prob = nullptr;   // problem of each tile in the list of all tiles
    int* d_flags = nullptr;       // active flag of each tile in that list
    int* h_flags = nullptr;       // pinned staging: flags, then the live lists
    double* d_part = nullptr;
    int nfull = 0;                // tiles of all problems
    int nlive = 0;                // items of the current step
    long long part_cap = 0;
    std::vector<BProb> h_prob;
    BState* h_state = nullptr;   // pinned
    BatchCtl* h_ctl = nullptr;   // pinned
    // graph of one refinement pass
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_ok = false;
    double clock_khz = 100000.0;
    vfs_batch_stats stats{};
    hipEvent_t ev[4] = {};
};

namespace {

thread_local std::string g_batch_err;

int bfail(vfs_batch* b, int code, const std::string& m) {
    if (b)
        b->err = m;
    else
        g_batch_err = m;
    return code;
}

#define BCHK(call)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return bfail(b, VFS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

BatchArgs args(vfs_batch* b, int first_pass) {
    BatchArgs A{};
    A.prob = b->d_prob;
    A.state = b->d_state;
    A.ctl = b->d_ctl;
    A.item_prob = b->d_item_prob;
    A.item_tile = b->d_item_tile;
    A.nlive = b->d_nlive;
    A.nprob = b->n;
    A.partF[0] = b->d_part;
    A.partF[1] = b->d_part + 5 * b->part_cap;
    A.partR = b->d_part + 10 * b->part_cap;
    A.tol = b->tol;
    A.max_iter = b->max_iter;
    A.max_iter_pass = b->max_iter_pass;
    A.max_passes = b->max_passes;
    A.first_pass = first_pass;
    batch_tile_shape(b->variant, &A.bx, &A.by);
    return A;
}

// Upload the live item lists (problem, tile) held in h_flags[nfull...] and
// the per-problem item ranges; blocks until the copies are done.
int upload_items(vfs_batch* b) {
    hipStream_t s = b->stream;
    const int* hp = b->h_flags + b->nfull;
    const int* ht = hp + b->nfull;
    BCHK(hipMemcpyAsync(b->d_item_prob, hp, sizeof(int) * b->nlive, hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(b->d_item_tile, ht, sizeof(int) * b->nlive, hipMemcpyHostToDevice, s));
    b->h_flags[3 * b->nfull] = b->nlive;
    BCHK(hipMemcpyAsync(b->d_nlive, b->h_flags + 3 * b->nfull, sizeof(int), hipMemcpyHostToDevice,
                        s));
    BCHK(hipMemcpyAsync(b->d_prob, b->h_prob.data(), sizeof(BProb) * b->n, hipMemcpyHostToDevice,
                        s));
    BCHK(hipStreamSynchronize(s));
    return VFS_OK;
}

// Live items of the assembled step: the tiles of each problem holding an
// active sample, in problem and tile order.  A problem without one keeps its
// first tile, so that it still has an owner item (it retires at once).
int compact_items(vfs_batch* b) {
    hipStream_t s = b->stream;
    int bx, by;
    batch_tile_shape(b->variant, &bx, &by);
    launch_batch_tile_flags(b->d_prob, b->d_full_prob, b->nfull, bx, by, b->d_flags, s);
    BCHK(hipGetLastError());
    BCHK(hipMemcpyAsync(b->h_flags, b->d_flags, sizeof(int) * b->nfull, hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    int* hp = b->h_flags + b->nfull;
    int* ht = hp + b->nfull;
    int n = 0;
    for (int p = 0; p < b->n; ++p) {
        BProb& P = b->h_prob[p];
        P.item0 = n;
        for (int t = 0; t < P.ntx * P.nty; ++t)
            if (b->h_flags[P.full0 + t]) {
                hp[n] = p;
                ht[n] = t;
                ++n;
            }
        if (n == P.item0) {
            hp[n] = p;
            ht[n] = 0;
            ++n;
        }
        P.nt = n - P.item0;
    }
    b->nlive = n;
    return upload_items(b);
}

bool all_assembled(const vfs_batch* b) {
    for (auto* c : b->ctx)
        if (!c->assembled) return false;
    return true;
}

// (re)build the tile list of every problem for the current tile variant; the
// live items are all tiles until the next assembly compacts them
int build_items(vfs_batch* b) {
    int bx, by;
    batch_tile_shape(b->variant, &bx, &by);
    std::vector<int> full_prob;
    b->h_prob.assign(b->n, BProb{});
    for (int p = 0; p < b->n; ++p) {
        vfs_ctx* c = b->ctx[p];
        BProb& P = b->h_prob[p];
        P.g = c->g;
        P.ntx = (c->g.nx + 1 + bx - 1) / bx;
        P.nty = (c->g.ny + 1 + by - 1) / by;
        P.full0 = (int)full_prob.size();
        P.item0 = P.full0;
        P.nt = P.ntx * P.nty;
        for (int t = 0; t < P.nt; ++t) full_prob.push_back(p);
        P.x32 = c->x32;
        P.r32 = c->r32;
        P.p0 = c->p032;
        P.p1 = c->p132;
        P.q32 = c->q32;
        P.r32b = c->z32;
        P.q32b = c->f32b;
        P.a = c->a32;
        P.c = c->c32;
        P.K = c->K32;
        P.dinv = c->dinv32;
        P.ead = c->ead32;
        P.x64 = c->x;
        P.r64 = c->r;
        P.a64 = c->a;
        P.c64 = c->c;
        P.K64 = c->K;
        P.b64 = c->b;
    }
    b->nfull = (int)full_prob.size();
    int* dev[] = {b->d_item_prob, b->d_item_tile, b->d_nlive, b->d_full_prob, b->d_flags};
    for (int* q : dev)
        if (q) (void)hipFree(q);
    if (b->d_part) (void)hipFree(b->d_part);
    if (b->h_flags) (void)hipHostFree(b->h_flags);
    b->d_item_prob = b->d_item_tile = b->d_nlive = b->d_full_prob = b->d_flags = nullptr;
    b->d_part = nullptr;
    b->h_flags = nullptr;
    const size_t nf = sizeof(int) * b->nfull;
    BCHK(hipMalloc((void**)&b->d_item_prob, nf));
    BCHK(hipMalloc((void**)&b->d_item_tile, nf));
    BCHK(hipMalloc((void**)&b->d_full_prob, nf));
    BCHK(hipMalloc((void**)&b->d_flags, nf));
    BCHK(hipMalloc((void**)&b->d_nlive, sizeof(int)));
    BCHK(hipHostMalloc((void**)&b->h_flags, 3 * nf + sizeof(int), hipHostMallocDefault));
    b->part_cap = (long long)b->nfull + 64;
    BCHK(hipMalloc((void**)&b->d_part, sizeof(double) * 11 * b->part_cap));
    BCHK(hipMemcpy(b->d_full_prob, full_prob.data(), nf, hipMemcpyHostToDevice));
    int* hp = b->h_flags + b->nfull;
    int* ht = hp + b->nfull;
    for (int p = 0, n = 0; p < b->n; ++p)
        for (int t = 0; t < b->h_prob[p].nt; ++t, ++n) {
            hp[n] = p;
            ht[n] = t;
        }
    b->nlive = b->nfull;
    int rc = upload_items(b);
    if (rc) return rc;
    if (all_assembled(b) && (rc = compact_items(b))) return rc;
    int bpc = 0;
    if (batch_pcg_occupancy(b->variant, &bpc) != 0 || bpc < 1)
        return bfail(b, VFS_EHIP, "occupancy query failed");
    const int use = std::max(1, std::min(b->blocks_per_cu, bpc));
    b->bpc_used = use;
    b->grid = std::max(1, std::min(b->ncu * use, b->nfull));
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    b->graph_ok = false;
    return VFS_OK;
}

// the whole solve: x64 = 0, r64 = b, |b|, then the persistent kernel
// (inner FP32 CG, FP64 residual and refinement for every problem)
void enqueue_solve(vfs_batch* b, hipStream_t s) {
    const BatchArgs A0 = args(b, 1);
    launch_batch_zero(A0, s);
    launch_batch_resid(b->variant, A0, b->grid, s);
    launch_batch_finalize(A0, s);
    const BatchArgs A = args(b, 0);
    launch_batch_reset_ctl(b->d_ctl, s);
    launch_batch_pcg(b->variant, A, b->grid, s);
}

int ensure_graph(vfs_batch* b) {
    if (b->graph_ok) return VFS_OK;
    BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    enqueue_solve(b, b->stream);
    hipGraph_t g = nullptr;
    BCHK(hipStreamEndCapture(b->stream, &g));
    b->graph = g;
    BCHK(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    b->graph_ok = true;
    return VFS_OK;
}

int read_state(vfs_batch* b) {
    BCHK(hipMemcpyAsync(b->h_state, b->d_state, sizeof(BState) * b->n, hipMemcpyDeviceToHost,
                        b->stream));
    BCHK(hipMemcpyAsync(b->h_ctl, b->d_ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, b->stream));
    BCHK(hipStreamSynchronize(b->stream));
    if (b->h_ctl->abort) return bfail(b, VFS_EHIP, "batched grid barrier timed out (aborted)");
    return VFS_OK;
}

// solve phase of a step on assembled problems (one graph launch); returns status
int solve_all(vfs_batch* b, bool use_graph) {
    if (use_graph) {
        int rc = ensure_graph(b);
        if (rc) return rc;
        BCHK(hipGraphLaunch(b->gexec, b->stream));
    } else {
        enqueue_solve(b, b->stream);
    }
    BCHK(hipGetLastError());
    int rc = read_state(b);
    if (rc) return rc;
    int status = VFS_OK;
    for (int p = 0; p < b->n; ++p)
        if (b->h_state[p].rel > b->tol) status = VFS_ENOTCONV;
    return status;
}

float ev_ms(hipEvent_t a, hipEvent_t c) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, c) != hipSuccess) return 0.f;
    return ms;
}

}  // namespace

extern "C" {

const char* vfs_batch_last_error(const vfs_batch* b) {
    return b ? b->err.c_str() : g_batch_err.c_str();
}

int vfs_batch_num_variants(void) { return kBatchVariants; }

int vfs_batch_variant_shape(int variant, int* bx, int* by) {
    if (variant < 0 || variant >= kBatchVariants || !bx || !by) return VFS_EINVAL;
    batch_tile_shape(variant, bx, by);
    return VFS_OK;
}

int vfs_batch_destroy(vfs_batch* b) {
    if (!b) return VFS_OK;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto* c : b->ctx) vfs_destroy(c);
    void* bufs[] = {b->d_prob,      b->d_state,   b->d_ctl,   b->d_item_prob, b->d_item_tile,
                    b->d_full_prob, b->d_flags,   b->d_nlive, b->d_part};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    if (b->h_flags) (void)hipHostFree(b->h_flags);
    if (b->h_state) (void)hipHostFree(b->h_state);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
    for (auto& e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
    delete b;
    return VFS_OK;
}

int vfs_batch_create(vfs_batch** out, int n, const int* nx, const int* ny, const double* h) {
    if (!out || !nx || !ny || !h) return bfail(nullptr, VFS_EINVAL, "NULL argument");
    *out = nullptr;
    if (n < 1 || n > 4096) return bfail(nullptr, VFS_EINVAL, "problem count must be in [1, 4096]");
    vfs_batch* b = new vfs_batch();
    b->n = n;
    b->ctx.assign(n, nullptr);
    for (int p = 0; p < n; ++p) {
        const double org[3] = {0, 0, 0};
        int rc = vfs_create(&b->ctx[p], 2, nx[p], ny[p], 1, h[p], org);
        if (rc) {
            std::string m = std::string("problem ") + std::to_string(p) + ": " + vfs_last_error(nullptr);
            vfs_batch_destroy(b);
            return bfail(nullptr, rc, m);
        }
        b->ctx[p]->precision = VFS_MIXED;
    }
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        vfs_batch_destroy(b);
        return bfail(nullptr, VFS_EHIP, "device query failed");
    }
    b->ncu = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        b->clock_khz = khz;
    if (hipMalloc((void**)&b->d_prob, sizeof(BProb) * n) != hipSuccess ||
        hipMalloc((void**)&b->d_state, sizeof(BState) * n) != hipSuccess ||
        hipMalloc((void**)&b->d_ctl, sizeof(BatchCtl)) != hipSuccess ||
        hipHostMalloc((void**)&b->h_state, sizeof(BState) * n, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_ctl, sizeof(BatchCtl), hipHostMallocDefault) != hipSuccess) {
        vfs_batch_destroy(b);
        return bfail(nullptr, VFS_ENOMEM, "batch allocation failed");
    }
    (void)hipMemset(b->d_state, 0, sizeof(BState) * n);
    BatchCtl ctl{};
    ctl.spin_ticks = (unsigned long long)(b->clock_khz * 2000.0);   // 2 s per barrier wait
    (void)hipMemcpy(b->d_ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice);
    for (auto& e : b->ev) (void)hipEventCreate(&e);
    if (hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking) != hipSuccess) {
        vfs_batch_destroy(b);
        return bfail(nullptr, VFS_EHIP, "stream creation failed");
    }
    b->stream = b->own_stream;
    for (auto* c : b->ctx) c->stream = b->stream;
    int rc = build_items(b);
    if (rc) {
        std::string m = b->err;
        vfs_batch_destroy(b);
        return bfail(nullptr, rc, m);
    }
    *out = b;
    return VFS_OK;
}

int vfs_batch_set_stream(vfs_batch* b, void* stream) {
    if (!b) return VFS_EINVAL;
    b->stream = stream ? (hipStream_t)stream : b->own_stream;
    for (auto* c : b->ctx) c->stream = b->stream;
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    b->graph_ok = false;
    return VFS_OK;
}

int vfs_batch_set_problem(vfs_batch* b, int i, const double* phi_l, const double* phi_s,
                          const double* rho, const double* mu, const double* u, const double* v,
                          const double* ub, const double* vb, const double* g) {
    if (!b) return VFS_EINVAL;
    if (i < 0 || i >= b->n) return bfail(b, VFS_EINVAL, "problem index out of range");
    vfs_ctx* c = b->ctx[i];
    int rc;
    const std::string tag = "problem " + std::to_string(i) + ": ";
    if ((rc = vfs_set_level_sets(c, phi_l, phi_s)) || (rc = vfs_set_density(c, rho)) ||
        (rc = vfs_set_viscosity(c, mu)) || (rc = vfs_set_velocity(c, u, v, nullptr)) ||
        (rc = vfs_set_solid_velocity(c, ub, vb, nullptr)) || (rc = vfs_set_gravity(c, g)))
        return bfail(b, rc, tag + vfs_last_error(c));
    return VFS_OK;
}

int vfs_batch_set_solver(vfs_batch* b, double rel_tol, int max_iter, double w_min) {
    if (!b) return VFS_EINVAL;
    if (!(rel_tol > 0.0) || !(rel_tol < 1.0)) return bfail(b, VFS_EINVAL, "rel_tol must be in (0,1)");
    if (max_iter < 1) return bfail(b, VFS_EINVAL, "max_iter must be >= 1");
    for (auto* c : b->ctx) {
        int rc = vfs_set_solver(c, VFS_PRECOND_JACOBI, VFS_MIXED, rel_tol, max_iter, w_min);
        if (rc) return bfail(b, rc, vfs_last_error(c));
    }
    b->tol = rel_tol;
    b->max_iter = max_iter;
    b->max_iter_pass = std::min(max_iter, 50000);
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    b->graph_ok = false;
    return VFS_OK;
}

int vfs_batch_set_tiles(vfs_batch* b, int variant, int blocks_per_cu) {
    if (!b) return VFS_EINVAL;
    if (variant < 0 || variant >= kBatchVariants) return bfail(b, VFS_EINVAL, "bad tile variant");
    if (blocks_per_cu < 1 || blocks_per_cu > 16) return bfail(b, VFS_EINVAL, "bad blocks per CU");
    b->variant = variant;
    b->blocks_per_cu = blocks_per_cu;
    return build_items(b);
}

int vfs_batch_step(vfs_batch* b, double dt) {
    if (!b) return VFS_EINVAL;
    hipStream_t s = b->stream;
    BCHK(hipEventRecord(b->ev[0], s));
    for (int p = 0; p < b->n; ++p) {
        int rc = ctx_assemble(b->ctx[p], dt);
        if (rc) return bfail(b, rc, "problem " + std::to_string(p) + ": " + vfs_last_error(b->ctx[p]));
    }
    int rc = compact_items(b);
    if (rc) return rc;
    BCHK(hipEventRecord(b->ev[1], s));
    const int status = solve_all(b, true);
    if (status != VFS_OK && status != VFS_ENOTCONV) return status;
    BCHK(hipEventRecord(b->ev[2], s));
    for (int p = 0; p < b->n; ++p) {
        int rc = ctx_recover(b->ctx[p]);
        if (rc) return bfail(b, rc, vfs_last_error(b->ctx[p]));
    }
    BCHK(hipEventRecord(b->ev[3], s));
    BCHK(hipEventSynchronize(b->ev[3]));
    // stats
    vfs_batch_stats& S = b->stats;
    S = vfs_batch_stats{};
    S.n_problems = b->n;
    S.variant = b->variant;
    S.blocks_per_cu = b->bpc_used;
    S.grid = b->grid;
    S.graph_used = b->graph_ok ? 1 : 0;
    S.status = status;
    S.t_assemble_ms = ev_ms(b->ev[0], b->ev[1]);
    S.t_solve_ms = ev_ms(b->ev[1], b->ev[2]);
    S.t_step_ms = ev_ms(b->ev[0], b->ev[3]);
    {
        int bx, by;
        batch_tile_shape(b->variant, &bx, &by);
        S.n_items = b->nlive;
        S.n_tile_samples = (int64_t)b->nlive * bx * by * 3;
    }
    std::vector<double> lat;
    for (int p = 0; p < b->n; ++p) {
        const BState& st = b->h_state[p];
        // active count of each problem (from its assembly)
        Scalars sc{};
        BCHK(hipMemcpy(&sc, b->ctx[p]->sc, sizeof(Scalars), hipMemcpyDeviceToHost));
        b->ctx[p]->stats.n_active = sc.n_active;
        b->ctx[p]->stats.iterations = st.iters_total;
        b->ctx[p]->stats.outer_iterations = st.passes;
        b->ctx[p]->stats.rel_residual = st.rel;
        S.n_active_total += sc.n_active;
        S.dof_iters += (int64_t)sc.n_active * st.iters_total;
        S.max_iterations = std::max(S.max_iterations, st.iters_total);
        S.passes_max = std::max(S.passes_max, st.passes);
        const double ms = st.t_done > st.t_start ? (double)(st.t_done - st.t_start) / b->clock_khz : 0.0;
        lat.push_back(ms);
    }
    std::vector<double> l2 = lat;
    std::sort(l2.begin(), l2.end());
    auto pct = [&](double q) {
        const double pos = q * (l2.size() - 1);
        const size_t lo = (size_t)pos;
        const size_t hi = std::min(l2.size() - 1, lo + 1);
        return l2[lo] + (pos - lo) * (l2[hi] - l2[lo]);
    };
    S.latency_p50_ms = pct(0.50);
    S.latency_p90_ms = pct(0.90);
    S.latency_p99_ms = pct(0.99);
    S.latency_max_ms = l2.back();
    for (int p = 0; p < b->n; ++p) b->ctx[p]->stats.t_solve_ms = lat[p];
    return status;
}

int vfs_batch_get_velocity(vfs_batch* b, int i, double* u, double* v) {
    if (!b) return VFS_EINVAL;
    if (i < 0 || i >= b->n) return bfail(b, VFS_EINVAL, "problem index out of range");
    int rc = vfs_get_velocity(b->ctx[i], u, v, nullptr);
    if (rc) return bfail(b, rc, vfs_last_error(b->ctx[i]));
    return VFS_OK;
}

int vfs_batch_get_solution(vfs_batch* b, int i, double* x) {
    if (!b) return VFS_EINVAL;
    if (i < 0 || i >= b->n) return bfail(b, VFS_EINVAL, "problem index out of range");
    int rc = vfs_get_solution(b->ctx[i], x);
    if (rc) return bfail(b, rc, vfs_last_error(b->ctx[i]));
    return VFS_OK;
}

int vfs_batch_get_problem(vfs_batch* b, int i, int* iterations, int* passes,
                          double* rel_residual, double* latency_ms, int64_t* n_active) {
    if (!b) return VFS_EINVAL;
    if (i < 0 || i >= b->n) return bfail(b, VFS_EINVAL, "problem index out of range");
    const vfs_stats& st = b->ctx[i]->stats;
    if (iterations) *iterations = st.iterations;
    if (passes) *passes = st.outer_iterations;
    if (rel_residual) *rel_residual = st.rel_residual;
    if (latency_ms) *latency_ms = st.t_solve_ms;
    if (n_active) *n_active = st.n_active;
    return VFS_OK;
}

int vfs_batch_get_stats(vfs_batch* b, vfs_batch_stats* out) {
    if (!b || !out) return VFS_EINVAL;
    *out = b->stats;
    return VFS_OK;
}

int vfs_batch_max_blocks_per_cu(int variant) {
    if (variant < 0 || variant >= kBatchVariants) return VFS_EINVAL;
    int bpc = 0;
    if (batch_pcg_occupancy(variant, &bpc) != 0 || bpc < 1) return VFS_EHIP;
    return bpc;
}

int vfs_batch_time_variant(vfs_batch* b, int variant, int blocks_per_cu, int iterations,
                           double* ms_per_iteration) {
    if (!b || !ms_per_iteration) return VFS_EINVAL;
    if (iterations < 1) return bfail(b, VFS_EINVAL, "iterations must be >= 1");
    if (!all_assembled(b)) return bfail(b, VFS_ESTATE, "run vfs_batch_step once before timing");
    const int v0 = b->variant, c0 = b->blocks_per_cu;
    int rc = vfs_batch_set_tiles(b, variant, blocks_per_cu);
    if (rc) return rc;
    const int mip = b->max_iter_pass, mp = b->max_passes;
    b->max_iter_pass = iterations;
    b->max_passes = 1;
    hipStream_t s = b->stream;
    const BatchArgs A0 = args(b, 1);
    launch_batch_zero(A0, s);
    launch_batch_resid(b->variant, A0, b->grid, s);
    launch_batch_finalize(A0, s);
    const BatchArgs A = args(b, 0);
    launch_batch_reset_ctl(b->d_ctl, s);
    BCHK(hipEventRecord(b->ev[0], s));
    launch_batch_pcg(b->variant, A, b->grid, s);
    BCHK(hipEventRecord(b->ev[1], s));
    BCHK(hipGetLastError());
    BCHK(hipEventSynchronize(b->ev[1]));
    b->max_iter_pass = mip;
    b->max_passes = mp;
    rc = read_state(b);
    if (rc) return rc;
    *ms_per_iteration = ev_ms(b->ev[0], b->ev[1]) / iterations;
    return vfs_batch_set_tiles(b, v0, c0) == VFS_OK ? VFS_OK : VFS_EHIP;
}

}  // extern "C"
