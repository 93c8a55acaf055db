// C ABI of the variational Stokes step: context lifecycle, inputs, assembly,
// CG drivers (FP64 and mixed precision with iterative refinement), velocity
// recovery and result getters.  Every numerical step runs in the kernels of
// this library on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>

#include "vfs_internal.h"
#include "vfs_unet.h"

using namespace vfs;

namespace {

thread_local std::string g_create_err;

int fail(vfs_ctx* ctx, int code, const std::string& msg) {
    if (ctx)
        ctx->err = msg;
    else
        g_create_err = msg;
    return code;
}

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(ctx, VFS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
int dalloc(vfs_ctx* ctx, T** p, long long n) {
    *p = nullptr;
    if (n <= 0) n = 1;
    hipError_t e = hipMalloc((void**)p, (size_t)n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, VFS_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    e = hipMemset(*p, 0, (size_t)n * sizeof(T));
    if (e != hipSuccess) return fail(ctx, VFS_EHIP, "hipMemset failed");
    return VFS_OK;
}

long long node_count(const Geo& g) {
    return (long long)(g.nx + 1) * (g.ny + 1) * (g.dim == 3 ? g.nz + 1 : 1);
}
long long sub_count(const Geo& g) {
    return (long long)(2 * g.nx) * (2 * g.ny) * (g.dim == 3 ? 2 * g.nz : 1);
}
long long set_count(const Geo& g, int set) {
    int shp[3];
    set_shape(g, set, shp);
    return (long long)shp[0] * shp[1] * shp[2];
}

// stream-ordered check of a staged array: returns true if all values valid
int check_stage(vfs_ctx* ctx, const double* v, long long n, int positive, const char* what) {
    HIPCHK(hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream));
    launch_check(v, n, positive, ctx->flag, ctx->stream);
    HIPCHK(hipMemcpyAsync(ctx->flag_host, ctx->flag, sizeof(int), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (*ctx->flag_host)
        return fail(ctx, VFS_EINVAL,
                    std::string(what) + (positive ? ": non-finite or non-positive value"
                                                  : ": non-finite value"));
    return VFS_OK;
}

// user (host or device) compact array of a weight set -> padded device slice
int put_set(vfs_ctx* ctx, int set, const double* user, double* dst, int positive,
            const char* what) {
    int shp[3];
    set_shape(ctx->g, set, shp);
    const long long n = (long long)shp[0] * shp[1] * shp[2];
    HIPCHK(hipMemcpyAsync(ctx->stage, user, (size_t)n * sizeof(double), hipMemcpyDefault,
                          ctx->stream));
    int rc = check_stage(ctx, ctx->stage, n, positive, what);
    if (rc) return rc;
    launch_pack(ctx->g, shp, ctx->stage, dst, ctx->stream);
    HIPCHK(hipGetLastError());
    return VFS_OK;
}

// padded device slice of a weight set -> user (host or device) compact array
int get_set(vfs_ctx* ctx, int set, const double* src, double* user) {
    int shp[3];
    set_shape(ctx->g, set, shp);
    const long long n = (long long)shp[0] * shp[1] * shp[2];
    launch_unpack(ctx->g, shp, src, ctx->stage, ctx->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(user, ctx->stage, (size_t)n * sizeof(double), hipMemcpyDefault,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return VFS_OK;
}

int face_set(int a) { return 1 + a; }

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

int read_scalars(vfs_ctx* ctx, int which, Scalars* out) {
    HIPCHK(hipMemcpyAsync(ctx->sc_host + which, ctx->sc + which, sizeof(Scalars),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = ctx->sc_host[which];
    return VFS_OK;
}

// ---------------------------------------------------------------------------
// CG drivers.  Scalars slot 0: inner CG; slot 1: outer residual.
// ---------------------------------------------------------------------------
template <typename T>
struct Vecs {
    T *x, *r, *p0, *p1, *q, *z;
    const T *a, *c, *K, *dinv;
};

struct Parts {
    double *A, *B, *R;
};

Parts parts(vfs_ctx* ctx) {
    return Parts{ctx->partials, ctx->partials + ctx->capA, ctx->partials + ctx->capA + 2 * ctx->capB};
}

// Runs CG iterations in chunks until the device flag says done; returns the
// final scalars.  The r.z / r.r partials of the kernel before the first
// apply were written by the init or restart kernel (dense grid).
template <typename T>
int run_chunks(vfs_ctx* ctx, Vecs<T>& v, bool set_bb, Scalars* out) {
    const Geo& g = ctx->g;
    const Parts P = parts(ctx);
    const int nbA = dir_apply_blocks(g, ctx->tiles, (int)sizeof(T));
    const int nbU = update_blocks(g, ctx->tiles);
    const int nbV = vec_grid_blocks(g);
    int chunk = 8;
    int kidx = 0;
    for (;;) {
        for (int k = 0; k < chunk; ++k, ++kidx) {
            T* pin = (kidx & 1) ? v.p1 : v.p0;
            T* pout = (kidx & 1) ? v.p0 : v.p1;
            const bool timed = ctx->prof && k == 0;
            const RedArgs ra{ctx->sc, P.B, kidx == 0 ? nbV : nbU, P.A, kidx,
                             (set_bb && kidx == 0) ? 1 : 0};
            const RedArgs rb{ctx->sc, P.A, nbA, P.B, kidx, 0};
            if (timed) HIPCHK(hipEventRecord(ctx->pev[0], ctx->stream));
            launch_apply<T>(g, ctx->tiles, MODE_DIR, false, v.r, nullptr, v.dinv, pin, pout, v.q,
                            v.a, v.c, v.K, nullptr, ra, ctx->stream);
            if (timed) HIPCHK(hipEventRecord(ctx->pev[1], ctx->stream));
            launch_update<T>(g, ctx->tiles, v.x, pout, v.r, v.q, v.dinv, nullptr, rb, ctx->stream);
            if (timed) HIPCHK(hipEventRecord(ctx->pev[2], ctx->stream));
        }
        HIPCHK(hipGetLastError());
        int rc = read_scalars(ctx, 0, out);
        if (rc) return rc;
        // the flag read above synchronised the stream; the timed first
        // iteration of this chunk counts unless the solve stopped at it
        const int kidx0 = kidx - chunk;
        if (ctx->prof && (!out->done || out->iter > kidx0)) {
            ctx->prof_apply_ms += elapsed(ctx->pev[0], ctx->pev[1]);
            ctx->prof_update_ms += elapsed(ctx->pev[1], ctx->pev[2]);
            ++ctx->prof_apply_n;
            ++ctx->prof_update_n;
        }
        if (out->done) return VFS_OK;
        chunk = std::min(chunk * 2, 256);
    }
}

// 2D PCG with one fused launch per iteration (k_fused2d.hip) in FP32 over the
// tiles holding an active sample, on the residual that launch_cg_init placed
// in r32 (x32 = 0): an init launch
// (p = D^-1 r, q = A p, first partials), then launch k = 1, 2, ... carries
// out iteration k-1's update and forms direction k; partials alternate
// between two regions.
int run_chunks_fused(vfs_ctx* ctx, bool set_bb, Scalars* out) {
    const Geo& g = ctx->g;
    hipStream_t s = ctx->stream;
    const int nb = ctx->tiles2d;
    double* part[2] = {ctx->fpart, ctx->fpart + 5 * (long long)nb + 32};
    const FusedVecs fv{ctx->x32, {ctx->r32, ctx->z32}, {ctx->p032, ctx->p132}, {ctx->q32, ctx->f32b}};
    const RedArgs r0{ctx->sc, nullptr, 0, part[0], 0, 0};
    launch_fused2d<float>(g, true, fv, ctx->dinv32, ctx->a32, ctx->c32, ctx->K32, ctx->tile_list,
                          nb, r0, s);
    int chunk = 8;
    int kidx = 1;
    for (;;) {
        // live timing: the launches 2..chunk of a chunk back to back (the
        // first follows a host synchronisation and starts cold)
        for (int k = 0; k < chunk; ++k, ++kidx) {
            const RedArgs ra{ctx->sc, part[(kidx + 1) & 1], nb, part[kidx & 1], kidx,
                             (set_bb && kidx == 1) ? 1 : 0};
            if (ctx->prof && k == 1) HIPCHK(hipEventRecord(ctx->pev[0], s));
            launch_fused2d<float>(g, false, fv, ctx->dinv32, ctx->a32, ctx->c32, ctx->K32,
                                  ctx->tile_list, nb, ra, s);
        }
        if (ctx->prof) HIPCHK(hipEventRecord(ctx->pev[1], s));
        HIPCHK(hipGetLastError());
        int rc = read_scalars(ctx, 0, out);
        if (rc) return rc;
        // launch kidx performs iteration kidx - 1; a stop inside the chunk
        // leaves no-op launches in the bracket, so such chunks are not timed
        if (ctx->prof && !out->done) {
            ctx->prof_apply_ms += elapsed(ctx->pev[0], ctx->pev[1]) / (chunk - 1);
            ++ctx->prof_apply_n;
        }
        if (out->done) return VFS_OK;
        chunk = std::min(chunk * 2, 256);
    }
}

// 3D counterpart of run_chunks_fused (k_fused3d over the active tiles).
int run_chunks_fused3d(vfs_ctx* ctx, bool set_bb, Scalars* out) {
    const Geo& g = ctx->g;
    // the kernel addresses the six FP32 slices of a vector with 32-bit byte offsets
    if ((long long)g.nsamp() * g.NP * 4 >= (1LL << 32))
        return fail(ctx, VFS_EINVAL,
                    "grid too large for the mixed-precision 3D solve (a FP32 vector over 4 GiB)");
    hipStream_t s = ctx->stream;
    const int nb = fused3d_grid(ctx->ftiles.items());
    double* part[2] = {ctx->fpart, ctx->fpart + 5 * (long long)kMaxTileBlocks + 32};
    // the first launch reads the plain residual from r32 and writes e r to z32
    const FusedVecs fv{ctx->x32, {ctx->z32, ctx->r32}, {ctx->p032, ctx->p132}, {ctx->q32, ctx->f32b}};
    const RedArgs r0{ctx->sc, nullptr, 0, part[0], 0, 0};
    launch_fused3d(g, ctx->ftiles, true, fv, ctx->ead32, ctx->a32, ctx->c32, ctx->K32,
                   ctx->rowbits, ctx->counter, r0, s);
    int chunk = 8;
    int kidx = 1;
    for (;;) {
        for (int k = 0; k < chunk; ++k, ++kidx) {
            const RedArgs ra{ctx->sc, part[(kidx + 1) & 1], nb, part[kidx & 1], kidx,
                             (set_bb && kidx == 1) ? 1 : 0};
            if (ctx->prof && k == 1) HIPCHK(hipEventRecord(ctx->pev[0], s));
            launch_fused3d(g, ctx->ftiles, false, fv, ctx->ead32, ctx->a32, ctx->c32, ctx->K32,
                           ctx->rowbits, ctx->counter, ra, s);
        }
        if (ctx->prof) HIPCHK(hipEventRecord(ctx->pev[1], s));
        HIPCHK(hipGetLastError());
        int rc = read_scalars(ctx, 0, out);
        if (rc) return rc;
        if (ctx->prof && !out->done) {
            ctx->prof_apply_ms += elapsed(ctx->pev[0], ctx->pev[1]) / (chunk - 1);
            ++ctx->prof_apply_n;
        }
        if (out->done) return VFS_OK;
        chunk = std::min(chunk * 2, 256);
    }
}

// Truncated flexible CG (kFcgMax previous directions) with the learned
// two-level preconditioner (3D, FP32): z = a1 D^-1 r + w network(r1) from the
// (r.D^-1 r, r.r) partials of the previous kernel (net_precond), then the
// direction p = z - sum beta_i P_i (MODE_FDIR; Jacobi z when z is not a
// descent direction) + apply, then the update.  Directions and their images
// live in rings of kFcgMax + 1 slots.  Every launch after a stop sees
// sc->done and does nothing.
int run_chunks_fcg(vfs_ctx* ctx, Vecs<float>& v, bool set_bb, Scalars* out) {
    const Geo& g = ctx->g;
    const Parts P = parts(ctx);
    vfs_unet* u = ctx->net;
    hipStream_t s = ctx->stream;
    const int nbA = apply_blocks(g, ctx->tiles, 4), nbU = update_blocks(g, ctx->tiles);
    const int nbV = vec_grid_blocks(g), nbZ = coarse_blocks(g);
    const int* skip = &ctx->sc->done;
    constexpr int R = kFcgMax + 1;
    auto pring = [&](int k) { return net_vec(ctx, 5 + (k % R)); };
    auto qring = [&](int k) { return net_vec(ctx, 5 + R + (k % R)); };
    int chunk = 4;
    int kidx = 0;
    for (;;) {
        for (int k = 0; k < chunk; ++k, ++kidx) {
            FcgHist fh{};
            fh.mk = std::min(kidx, kFcgMax);
            for (int i = 0; i < fh.mk; ++i) {
                fh.P[i] = pring(kidx - 1 - i);
                fh.Q[i] = qring(kidx - 1 - i);
            }
            float* pout = pring(kidx);
            float* q = qring(kidx);
            const int nb2 = kidx == 0 ? nbV : nbU;
            const bool timed = ctx->prof && k == 0;
            if (timed) HIPCHK(hipEventRecord(ctx->pev[3], s));
            int rc = net_precond(u, ctx, v.r, v.dinv, v.a, v.c, v.K, P.B, nb2, fh, skip);
            if (rc) return fail(ctx, rc, u->err);
            RedArgs ra{ctx->sc, net_region(ctx, 4), nbZ, P.A, kidx, (set_bb && kidx == 0) ? 1 : 0,
                       P.B, nb2};
            ra.fh = fh;
            const RedArgs rb{ctx->sc, P.A, nbA, P.B, kidx, 0};
            if (timed) HIPCHK(hipEventRecord(ctx->pev[0], s));
            launch_apply<float>(g, ctx->tiles, MODE_FDIR, false, v.r, ctx->z32, v.dinv, nullptr,
                                pout, q, v.a, v.c, v.K, nullptr, ra, s);
            if (timed) HIPCHK(hipEventRecord(ctx->pev[1], s));
            launch_update<float>(g, ctx->tiles, v.x, pout, v.r, q, v.dinv, nullptr, rb, s);
            if (timed) HIPCHK(hipEventRecord(ctx->pev[2], s));
        }
        HIPCHK(hipGetLastError());
        int rc = read_scalars(ctx, 0, out);
        if (rc) return rc;
        const int kidx0 = kidx - chunk;
        if (ctx->prof && (!out->done || out->iter > kidx0)) {
            ctx->prof_apply_ms += elapsed(ctx->pev[0], ctx->pev[1]);
            ctx->prof_update_ms += elapsed(ctx->pev[1], ctx->pev[2]);
            ctx->prof_precond_ms += elapsed(ctx->pev[3], ctx->pev[0]);
            ++ctx->prof_apply_n;
            ++ctx->prof_update_n;
        }
        if (out->done) return VFS_OK;
        chunk = std::min(chunk * 2, 64);
    }
}

// r = b - A x in FP64 and ||r||^2 -> sc[1].aux0 (host copy in *so)
int true_residual(vfs_ctx* ctx, const double* b, const double* x, Scalars* so) {
    const Geo& g = ctx->g;
    const Parts P = parts(ctx);
    const RedArgs rr{ctx->sc + 1, nullptr, 0, P.R, 0, 0};
    launch_apply<double>(g, ctx->tiles, MODE_RESID, false, nullptr, nullptr, nullptr, x, nullptr,
                         ctx->r, ctx->a, ctx->c, ctx->K, b, rr, ctx->stream);
    launch_finalize(P.R, apply_blocks(g, ctx->tiles, 8), 1, ctx->sc + 1, 0, ctx->stream);
    HIPCHK(hipGetLastError());
    return read_scalars(ctx, 1, so);
}

// direction buffers and q start at zero (tiles that stay inactive are never
// written by the 3D kernels or the fused 2D kernel, and their halo values are
// read; the active tiles can change from one assembly to the next)
int zero_dirs(vfs_ctx* ctx, bool f32) {
    const size_t n = (size_t)ctx->g.nsamp() * ctx->g.NP;
    if (f32) {
        HIPCHK(hipMemsetAsync(ctx->p032, 0, n * sizeof(float), ctx->stream));
        HIPCHK(hipMemsetAsync(ctx->p132, 0, n * sizeof(float), ctx->stream));
        HIPCHK(hipMemsetAsync(ctx->q32, 0, n * sizeof(float), ctx->stream));
        // second r and q buffers of the fused iteration
        HIPCHK(hipMemsetAsync(ctx->z32, 0, n * sizeof(float), ctx->stream));
        HIPCHK(hipMemsetAsync(ctx->f32b, 0, n * sizeof(float), ctx->stream));
    } else {
        HIPCHK(hipMemsetAsync(ctx->p0, 0, n * sizeof(double), ctx->stream));
        HIPCHK(hipMemsetAsync(ctx->p1, 0, n * sizeof(double), ctx->stream));
        HIPCHK(hipMemsetAsync(ctx->q, 0, n * sizeof(double), ctx->stream));
    }
    return VFS_OK;
}

// FP64 solve of A x = b (padded device vectors); fills stats.
int solve_fp64(vfs_ctx* ctx, const double* b, double* x) {
    const Geo& g = ctx->g;
    if (int rc0 = zero_dirs(ctx, false)) return rc0;
    const Parts P = parts(ctx);
    Vecs<double> v{x, ctx->r, ctx->p0, ctx->p1, ctx->q, nullptr, ctx->a, ctx->c, ctx->K,
                   ctx->dinv};
    launch_cg_init<double>(g, b, x, ctx->r, ctx->dinv, nullptr, ctx->tol, ctx->max_iter, ctx->sc,
                           P.B, ctx->stream);
    HIPCHK(hipGetLastError());
    Scalars s{};
    int rc = run_chunks<double>(ctx, v, true, &s);
    if (rc) return rc;
    int total = s.iter, outer = 0, status = VFS_OK;
    const double bb = s.bb;
    ctx->stats.rel_residual_start = bb > 0.0 ? 1.0 : 0.0;
    const double bnorm = std::sqrt(bb);
    double rel = 0.0;
    while (bb > 0.0) {
        Scalars so{};
        rc = true_residual(ctx, b, x, &so);   // replaces r by the true residual
        if (rc) return rc;
        rel = std::sqrt(so.aux0 / bb);
        if (rel <= ctx->tol) break;
        if (s.done == 3 || !std::isfinite(rel)) {
            status = VFS_EBREAKDOWN;
            break;
        }
        if (s.done == 2 || total >= ctx->max_iter || ++outer > 20) {
            status = VFS_ENOTCONV;
            break;
        }
        launch_cg_restart<double>(g, ctx->r, ctx->dinv, nullptr, ctx->sc, P.B,
                                  ctx->max_iter - total, ctx->stream);
        HIPCHK(hipGetLastError());
        rc = run_chunks<double>(ctx, v, false, &s);
        if (rc) return rc;
        total += s.iter;
    }
    ctx->stats.iterations = total;
    ctx->stats.outer_iterations = outer;
    ctx->stats.rel_residual = rel;
    ctx->stats.b_norm = bnorm;
    ctx->stats.status = status;
    return status;
}

// Mixed precision: FP32 CG on the scaled residual, FP64 residual and
// iterative-refinement update x64 += |r64| d32.
int solve_mixed(vfs_ctx* ctx, const double* b, double* x) {
    const Geo& g = ctx->g;
    const long long n = (long long)g.nsamp() * g.NP;
    const Parts P = parts(ctx);
    Vecs<float> v{ctx->x32, ctx->r32, ctx->p032, ctx->p132, ctx->q32, nullptr, ctx->a32, ctx->c32,
                  ctx->K32, ctx->dinv32};
    if (int rc0 = zero_dirs(ctx, true)) return rc0;
    const bool learned = ctx->precond == VFS_PRECOND_LEARNED;
    if (learned) {
        if (!ctx->net) return fail(ctx, VFS_ESTATE, "no preconditioner network attached");
        if (!ctx->net->have_weights) return fail(ctx, VFS_ESTATE, "the network has no weights");
        if (ctx->net->stream != ctx->stream)
            return fail(ctx, VFS_EINVAL, "network and context must use the same stream");
        if (int rc0 = net_prepare_ctx(ctx->net, ctx)) return fail(ctx, rc0, ctx->net->err);
    }
    int fallbacks = 0;
    // warm start: keep the last solution on the samples that are still active
    const bool warm = ctx->warm_start && ctx->have_x && x == ctx->x;
    if (warm)
        HIPCHK(hipMemcpyAsync(ctx->z, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice,
                              ctx->stream));
    HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), ctx->stream));
    Scalars so{};
    int rc = true_residual(ctx, b, x, &so);
    if (rc) return rc;
    const double bnorm = std::sqrt(so.aux0);
    double rho = bnorm;
    if (warm && bnorm > 0.0) {
        launch_mask(x, ctx->z, ctx->a, n, ctx->stream);
        HIPCHK(hipGetLastError());
        rc = true_residual(ctx, b, x, &so);
        if (rc) return rc;
        rho = std::sqrt(so.aux0);
    }
    int total = 0, outer = 0, status = VFS_OK, stalls = 0;
    double rel = bnorm > 0 ? rho / bnorm : 0.0;
    ctx->stats.rel_residual_start = rel;
    while (bnorm > 0.0) {
        rel = rho / bnorm;
        if (rel <= ctx->tol) break;
        if (total >= ctx->max_iter || outer >= 40) {
            status = VFS_ENOTCONV;
            break;
        }
        // each FP32 pass reduces its residual at most 1e-4: beyond that, its
        // rounding slows the recurrence more than a fresh pass on the FP64
        // residual costs
        const double tol_in = std::min(0.5, std::max(0.5 * ctx->tol * bnorm / rho, 1e-4));
        launch_scale_to_f32(g, ctx->r, ctx->r32, ctx->sc + 1, ctx->stream);
        launch_cg_init<float>(g, ctx->r32, ctx->x32, ctx->r32, ctx->dinv32, nullptr, tol_in,
                              ctx->max_iter - total, ctx->sc, P.B, ctx->stream);
        HIPCHK(hipGetLastError());
        Scalars s{};
        if (learned)
            rc = run_chunks_fcg(ctx, v, true, &s);
        else if (g.dim == 2)
            rc = run_chunks_fused(ctx, true, &s);
        else
            rc = run_chunks_fused3d(ctx, true, &s);
        if (rc) return rc;
        total += s.iter;
        fallbacks += s.fallbacks;
        launch_axpy_f32_to_f64(g, x, ctx->x32, ctx->sc + 1, ctx->stream);
        rc = true_residual(ctx, b, x, &so);
        if (rc) return rc;
        const double rho_new = std::sqrt(so.aux0);
        ++outer;
        if (!(rho_new < 0.9 * rho)) {
            if (++stalls >= 3 || !std::isfinite(rho_new)) {
                rho = rho_new;
                rel = rho / bnorm;
                status = rel <= ctx->tol ? VFS_OK : VFS_EBREAKDOWN;
                break;
            }
        } else {
            stalls = 0;
        }
        rho = rho_new;
    }
    ctx->stats.precond_fallbacks = fallbacks;
    ctx->stats.iterations = total;
    ctx->stats.outer_iterations = outer;
    ctx->stats.rel_residual = rel;
    ctx->stats.b_norm = bnorm;
    ctx->stats.status = status;
    return status;
}

// FP64 PCG with the brick-local Schwarz (overlap 1) or block symmetric
// Gauss-Seidel (overlap 0) preconditioner; every scalar stays on the device
// (Scalars slot 3), the host polls the stop flag once per chunk.  A stop on
// the recursive residual is confirmed on the true FP64 residual; otherwise
// PCG restarts from it.
int solve_schwarz(vfs_ctx* ctx, const double* b, double* x) {
    const Geo& g = ctx->g;
    hipStream_t s = ctx->stream;
    const long long n = (long long)g.nsamp() * g.NP;
    const int overlap = ctx->precond == VFS_PRECOND_SCHWARZ ? 1 : 0;
    if (int rc0 = zero_dirs(ctx, false)) return rc0;
    const Parts P = parts(ctx);
    double* part = P.B;
    const int nb = pcg_blocks(g);
    Scalars* S = ctx->sc + 3;
    const int* done = &S->done;
    double* r = ctx->r;
    double* z = ctx->z;
    double* p = ctx->p0;
    double* q = ctx->q;
    const RedArgs none{ctx->sc + 2, nullptr, 0, nullptr, 0, 0};
    // 3D: the vector kernels sweep the rows holding an active sample
    RowList rl{nullptr, -1};
    if (g.dim == 3) {
        if (ctx->rowlist_n < 0) {
            if (!ctx->rowlist) {
                if (hipMalloc((void**)&ctx->rowlist, (size_t)row_items(g) * sizeof(int)) !=
                        hipSuccess ||
                    hipMalloc((void**)&ctx->rowlist_cnt,
                              (size_t)(row_list_chunks(g) + 1) * sizeof(int)) != hipSuccess)
                    return fail(ctx, VFS_ENOMEM, "hipMalloc failed (row list)");
            }
            launch_row_list(g, ctx->rowbits, ctx->rowlist, ctx->rowlist_cnt, s);
            HIPCHK(hipMemcpyAsync(ctx->tile_count_host + 2, ctx->rowlist_cnt + row_list_chunks(g),
                                  sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            ctx->rowlist_n = ctx->tile_count_host[2];
        }
        rl = RowList{ctx->rowlist, ctx->rowlist_n};
    }
    HIPCHK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s));
    HIPCHK(hipMemcpyAsync(r, b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_pcg_dot(g, rl, r, r, part, nullptr, s);
    launch_pcg_start(part, nb, S, ctx->tol, ctx->max_iter, false, s);
    HIPCHK(hipGetLastError());
    int total = 0, outer = 0, status = VFS_OK;
    double rel = 0.0, bb = 0.0;
    for (;;) {
        Scalars sc{};
        int chunk = 8;
        for (;;) {
            for (int k = 0; k < chunk; ++k) {
                const bool timed = ctx->prof && k == 0;
                if (timed) HIPCHK(hipEventRecord(ctx->pev[3], s));
                launch_schwarz(g, overlap, r, ctx->a, ctx->c, ctx->dinv, ctx->K, ctx->rowbits, z,
                               done, s);
                if (timed) HIPCHK(hipEventRecord(ctx->pev[0], s));
                launch_pcg_dot(g, rl, r, z, part, done, s);
                launch_pcg_rz(part, nb, S, s);
                launch_pcg_dir(g, rl, z, p, S, s);
                launch_apply<double>(g, ctx->tiles, MODE_APPLY, false, nullptr, nullptr, nullptr, p,
                                     nullptr, q, ctx->a, ctx->c, ctx->K, nullptr, none, s);
                launch_pcg_dot(g, rl, p, q, part, done, s);
                launch_pcg_pq(part, nb, S, s);
                if (timed) HIPCHK(hipEventRecord(ctx->pev[1], s));
                launch_pcg_update(g, rl, x, r, p, q, S, part, s);
                launch_pcg_check(part, nb, S, s);
                if (timed) HIPCHK(hipEventRecord(ctx->pev[2], s));
            }
            HIPCHK(hipGetLastError());
            int rc = read_scalars(ctx, 3, &sc);
            if (rc) return rc;
            if (ctx->prof && !sc.done) {
                ctx->prof_precond_ms += elapsed(ctx->pev[3], ctx->pev[0]);
                ctx->prof_apply_ms += elapsed(ctx->pev[0], ctx->pev[1]);
                ctx->prof_update_ms += elapsed(ctx->pev[1], ctx->pev[2]);
                ++ctx->prof_apply_n;
                ++ctx->prof_update_n;
            }
            if (sc.done) break;
            chunk = std::min(chunk * 2, 128);
        }
        total += sc.iter;
        bb = sc.bb;
        if (!(bb > 0.0)) {
            rel = 0.0;
            break;
        }
        Scalars so{};
        int rc = true_residual(ctx, b, x, &so);   // r = b - A x
        if (rc) return rc;
        rel = std::sqrt(so.aux0 / bb);
        if (rel <= ctx->tol) break;
        if (sc.done == 3 || !std::isfinite(rel)) {
            status = VFS_EBREAKDOWN;
            break;
        }
        if (sc.done == 2 || total >= ctx->max_iter || ++outer > 20) {
            status = VFS_ENOTCONV;
            break;
        }
        launch_pcg_dot(g, rl, r, r, part, nullptr, s);
        launch_pcg_start(part, nb, S, ctx->tol, ctx->max_iter - total, true, s);
        HIPCHK(hipGetLastError());
    }
    ctx->stats.iterations = total;
    ctx->stats.outer_iterations = outer;
    ctx->stats.rel_residual = rel;
    ctx->stats.rel_residual_start = bb > 0.0 ? 1.0 : 0.0;
    ctx->stats.b_norm = std::sqrt(bb);
    ctx->stats.status = status;
    return status;
}

int solve_internal(vfs_ctx* ctx, const double* b, double* x) {
    if (ctx->g.dim == 3 && ctx->tiles.count == 0) {   // nothing active: x = 0
        HIPCHK(hipMemsetAsync(x, 0, (size_t)ctx->g.nsamp() * ctx->g.NP * sizeof(double),
                              ctx->stream));
        ctx->stats.iterations = 0;
        ctx->stats.outer_iterations = 0;
        ctx->stats.rel_residual = 0.0;
        ctx->stats.b_norm = 0.0;
        ctx->stats.status = VFS_OK;
        return VFS_OK;
    }
    if (ctx->precond == VFS_PRECOND_IC || ctx->precond == VFS_PRECOND_SCHWARZ)
        return solve_schwarz(ctx, b, x);
    if (ctx->precision == VFS_MIXED) return solve_mixed(ctx, b, x);
    return solve_fp64(ctx, b, x);
}

int assemble_internal(vfs_ctx* ctx, double dt) {
    const Geo& g = ctx->g;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, VFS_EINVAL, "dt must be > 0 and finite");
    if (!ctx->have_phi || !ctx->have_rho || !ctx->have_mu || !ctx->have_u)
        return fail(ctx, VFS_ESTATE, "level sets, density, viscosity and velocity must be set");
    hipStream_t s = ctx->stream;
    launch_subcell_fractions(g, ctx->phi_l, ctx->thL, false, s);
    if (ctx->has_solid)
        launch_subcell_fractions(g, ctx->phi_s, ctx->thF, true, s);
    else
        launch_fill(ctx->thF, sub_count(g), 1.0, s);
    launch_weights(g, ctx->thL, ctx->thF, ctx->w_min, ctx->WL, ctx->WF, s);
    HIPCHK(hipMemsetAsync(&ctx->sc->n_active, 0, sizeof(long long), s));
    if (g.dim == 2) {
        launch_face_coef2d(g, dt, ctx->gravity, ctx->WL, ctx->WF, ctx->rho, ctx->u, ctx->ustar,
                           ctx->rhof, ctx->K, ctx->fflag, s);
        launch_sample_coef2d(g, ctx->WL, ctx->WF, ctx->mu, ctx->K, ctx->fflag, ctx->ustar,
                             ctx->ubc, ctx->a, ctx->c, ctx->dinv, ctx->b, ctx->sc, s);
    } else {
        launch_face_coef3d(g, dt, ctx->gravity, ctx->WL, ctx->WF, ctx->rho, ctx->u, ctx->ustar,
                           ctx->rhof, ctx->K, ctx->fflag, s);
        launch_sample_coef3d(g, ctx->WL, ctx->WF, ctx->mu, ctx->K, ctx->fflag, ctx->ustar,
                             ctx->ubc, ctx->a, ctx->c, ctx->dinv, ctx->b, ctx->sc, s);
    }
    if (ctx->have_traction) {
        // the traction terms change u* on faces with K > 0; the sample pass
        // then forms b from the new u* (a, c and D^-1 do not depend on it)
        if (g.dim == 2)
            launch_traction2d(g, dt, ctx->ybc, ctx->a, ctx->rhof, ctx->WL, ctx->fflag, ctx->ustar, s);
        else
            launch_traction3d(g, dt, ctx->ybc, ctx->a, ctx->rhof, ctx->WL, ctx->fflag, ctx->ustar, s);
        HIPCHK(hipMemsetAsync(&ctx->sc->n_active, 0, sizeof(long long), s));
        if (g.dim == 2) {
            launch_sample_coef2d(g, ctx->WL, ctx->WF, ctx->mu, ctx->K, ctx->fflag, ctx->ustar,
                                 ctx->ubc, ctx->a, ctx->c, ctx->dinv, ctx->b, ctx->sc, s);
        } else {
            launch_sample_coef3d(g, ctx->WL, ctx->WF, ctx->mu, ctx->K, ctx->fflag, ctx->ustar,
                                 ctx->ubc, ctx->a, ctx->c, ctx->dinv, ctx->b, ctx->sc, s);
            launch_traction_pair3d(g, ctx->ybc, ctx->a, ctx->c, ctx->b, s);
        }
    }
    if (g.dim == 2) {
        launch_tiles2d(g, ctx->a, ctx->tile_flags, ctx->tile_list, ctx->tile_count, s);
        HIPCHK(hipMemcpyAsync(ctx->tile_count_host, ctx->tile_count, sizeof(int),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ctx->tiles2d = *ctx->tile_count_host;
        ctx->stats.n_tile_samples = (int64_t)ctx->tiles2d * tile2d_anchors() * g.nsamp();
    }
    if (g.dim == 3) {
        launch_tiles(g, ctx->a, ctx->tile_flags, ctx->tile_list, ctx->tile_count, s);
        launch_fused_tiles(g, ctx->tile_flags, ctx->ftile_flags, ctx->ftile_list,
                           ctx->tile_count + 1, s);
        launch_row_bits(g, ctx->a, ctx->rowbits, s);
        ctx->rowlist_n = -1;   // the row list follows the new row bits
        HIPCHK(hipMemcpyAsync(ctx->tile_count_host, ctx->tile_count, 2 * sizeof(int),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ctx->tiles.list = ctx->tile_list;
        ctx->tiles.count = ctx->tile_count_host[0];
        ctx->ftiles.list = ctx->ftile_list;
        ctx->ftiles.count = ctx->tile_count_host[1];
        // main kernel of the solve: the fused FP32 iteration (mixed, over its
        // own work tiles) or the pipelined FP64 direction + apply
        const int cap = ctx->precision == VFS_MIXED ? fused3d_grid(1 << 30)
                                                    : dir3d_grid(1 << 30, (int)sizeof(double));
        ctx->tiles.split = tile_split(ctx->tiles.count, cap);
        ctx->ftiles.split = fused_split(ctx->ftiles.count, fused3d_grid(1 << 30));
        ctx->stats.n_tile_samples = (int64_t)ctx->tiles.count * tile3d_anchors() * g.nsamp();
    }
    if (ctx->precision == VFS_MIXED) {
        const long long ns = (long long)g.nsamp() * g.NP, nf = (long long)g.dim * g.NP;
        launch_to_f32(ctx->K, ctx->K32, nf, s);
        launch_to_f32(ctx->a, ctx->a32, ns, s);
        launch_to_f32(ctx->c, ctx->c32, ns, s);
        launch_to_f32(ctx->dinv, ctx->dinv32, ns, s);
        launch_mul_to_f32(ctx->a, ctx->dinv, ctx->ead32, ns, s);
    }
    HIPCHK(hipGetLastError());
    ctx->assembled = true;
    ctx->dt_assembled = dt;
    ctx->netvec_dirty = true;   // the active tiles may have changed
    return VFS_OK;
}

int recover_internal(vfs_ctx* ctx) {
    const Geo& g = ctx->g;
    if (g.dim == 2)
        launch_velocity2d(g, ctx->dt_assembled, ctx->x, ctx->a, ctx->ustar, ctx->ubc, ctx->rhof,
                          ctx->WL, ctx->WF, ctx->fflag, ctx->u, ctx->stream);
    else
        launch_velocity3d(g, ctx->dt_assembled, ctx->x, ctx->a, ctx->ustar, ctx->ubc, ctx->rhof,
                          ctx->WL, ctx->WF, ctx->fflag, ctx->u, ctx->stream);
    HIPCHK(hipGetLastError());
    return VFS_OK;
}

int pack_samples(vfs_ctx* ctx, const double* user, double* dst) {
    const Geo& g = ctx->g;
    long long off = 0;
    for (int s = 0; s < g.nsamp(); ++s) {
        const int set = sample_set(g.dim, s);
        int shp[3];
        set_shape(g, set, shp);
        const long long n = (long long)shp[0] * shp[1] * shp[2];
        HIPCHK(hipMemcpyAsync(ctx->stage, user + off, (size_t)n * sizeof(double),
                              hipMemcpyDefault, ctx->stream));
        int rc = check_stage(ctx, ctx->stage, n, 0, "vector");
        if (rc) return rc;
        launch_pack(g, shp, ctx->stage, dst + s * g.NP, ctx->stream);
        off += n;
    }
    HIPCHK(hipGetLastError());
    return VFS_OK;
}

int unpack_samples(vfs_ctx* ctx, const double* src, double* user) {
    const Geo& g = ctx->g;
    long long off = 0;
    for (int s = 0; s < g.nsamp(); ++s) {
        const int set = sample_set(g.dim, s);
        int rc = get_set(ctx, set, src + s * g.NP, user + off);
        if (rc) return rc;
        off += set_count(g, set);
    }
    return VFS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
namespace vfs {

int ctx_assemble(vfs_ctx* ctx, double dt) { return assemble_internal(ctx, dt); }
int ctx_recover(vfs_ctx* ctx) { return recover_internal(ctx); }
int ctx_put_samples(vfs_ctx* ctx, const double* user, double* dst) {
    return pack_samples(ctx, user, dst);
}
int ctx_get_samples(vfs_ctx* ctx, const double* src, double* user) {
    return unpack_samples(ctx, src, user);
}
int ctx_fail(vfs_ctx* ctx, int code, const std::string& msg) { return fail(ctx, code, msg); }
int fail_global(int code, const std::string& msg) { return fail(nullptr, code, msg); }

Geo make_geo(int dim, int nx, int ny, int nz, double h) {
    Geo g{};
    g.dim = dim;
    g.nx = nx;
    g.ny = ny;
    g.nz = dim == 3 ? nz : 1;
    // 3D: rows of 32-element multiples after a 32-element front, slices of
    // 32-element multiples, so every row starts on a 128-byte line in FP32 and
    // each half of a 64-anchor row (the unit of the row bits) is one line; 2D
    // rows stay 16-element multiples (64-byte aligned)
    const int ra = dim == 3 ? 32 : 16;
    g.PX = ((nx + 3) + ra - 1) / ra * ra;
    g.PY = ny + 3;
    g.PZ = dim == 3 ? nz + 3 : 1;
    const long long body = (long long)g.PX * g.PY * g.PZ;
    g.NP = (kFront + body + 32 + 31) / 32 * 32;
    g.h = h;
    return g;
}

void set_stagger(int dim, int set, int st[3]) {
    static const int s2[4][3] = {{1, 1, 1}, {0, 1, 1}, {1, 0, 1}, {0, 0, 1}};
    static const int s3[7][3] = {{1, 1, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0},
                                 {0, 0, 1}, {0, 1, 0}, {1, 0, 0}};
    for (int a = 0; a < 3; ++a) st[a] = dim == 2 ? s2[set][a] : s3[set][a];
}

int sample_set(int dim, int s) {
    if (dim == 2) return s < 2 ? 0 : 3;
    return s < 3 ? 0 : s + 1;
}

void set_shape(const Geo& g, int set, int shp[3]) {
    int st[3];
    set_stagger(g.dim, set, st);
    shp[0] = g.nx + 1 - st[0];
    shp[1] = g.ny + 1 - st[1];
    shp[2] = g.dim == 3 ? g.nz + 1 - st[2] : 1;
}

}  // namespace vfs

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* vfs_last_error(const vfs_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int vfs_destroy(vfs_ctx* ctx) {
    if (!ctx) return VFS_OK;
    void* bufs[] = {ctx->phi_l, ctx->phi_s, ctx->rho,  ctx->mu,     ctx->u,      ctx->ubc,
                    ctx->thL,   ctx->thF,   ctx->WL,   ctx->WF,     ctx->fflag,  ctx->ustar,
                    ctx->rhof,  ctx->K,     ctx->a,    ctx->c,      ctx->dinv,   ctx->b,
                    ctx->K32,   ctx->a32,   ctx->c32,  ctx->dinv32, ctx->x,      ctx->r,
                    ctx->p0,    ctx->p1,    ctx->q,    ctx->z,      ctx->x32,    ctx->r32,
                    ctx->p032,  ctx->p132,  ctx->q32,  ctx->z32,    ctx->partials, ctx->counter,
                    ctx->sc,    ctx->flag,  ctx->stage, ctx->netvec, ctx->netpart, ctx->netcoef,
                    ctx->f32b,  ctx->fpart, ctx->ybc, ctx->adv_a, ctx->adv_b, ctx->adv_ka,
                    ctx->adv_kb, ctx->phi_tmp, ctx->ead32};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    if (ctx->net_owned) (void)vfs_unet_destroy(ctx->net_owned);
    if (ctx->tile_flags) (void)hipFree(ctx->tile_flags);
    if (ctx->tile_list) (void)hipFree(ctx->tile_list);
    if (ctx->tile_count) (void)hipFree(ctx->tile_count);
    if (ctx->ftile_flags) (void)hipFree(ctx->ftile_flags);
    if (ctx->ftile_list) (void)hipFree(ctx->ftile_list);
    if (ctx->rowbits) (void)hipFree(ctx->rowbits);
    if (ctx->rowlist) (void)hipFree(ctx->rowlist);
    if (ctx->rowlist_cnt) (void)hipFree(ctx->rowlist_cnt);
    if (ctx->tile_count_host) (void)hipHostFree(ctx->tile_count_host);
    if (ctx->sc_host) (void)hipHostFree(ctx->sc_host);
    if (ctx->flag_host) (void)hipHostFree(ctx->flag_host);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->pev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
    return VFS_OK;
}

int vfs_create(vfs_ctx** out, int dim, int nx, int ny, int nz, double h, const double* origin) {
    if (!out) return fail(nullptr, VFS_EINVAL, "out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(nullptr, VFS_EINVAL, "dim must be 2 or 3");
    if (nx < 1 || ny < 1 || (dim == 3 && nz < 1)) return fail(nullptr, VFS_EINVAL, "grid size < 1");
    if (nx > 16384 || ny > 16384 || (dim == 3 && nz > 2048))
        return fail(nullptr, VFS_EINVAL, "grid size too large");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(nullptr, VFS_EINVAL, "h must be > 0");
    vfs_ctx* ctx = new vfs_ctx();
    ctx->g = make_geo(dim, nx, ny, nz, h);
    if (origin)
        for (int a = 0; a < dim; ++a) ctx->origin[a] = origin[a];
    const Geo& g = ctx->g;
    const long long NP = g.NP;
    const int ns = g.nsamp(), nf = g.dim, nsets = g.nsets();
    int rc = VFS_OK;
#define ALLOC(p, n)                                  \
    if ((rc = dalloc(ctx, &(p), (n))) != VFS_OK) {   \
        std::string m = ctx->err;                    \
        vfs_destroy(ctx);                            \
        return fail(nullptr, rc, m);                 \
    }
    ALLOC(ctx->phi_l, node_count(g));
    ALLOC(ctx->phi_s, node_count(g));
    ALLOC(ctx->rho, NP);
    ALLOC(ctx->mu, NP);
    ALLOC(ctx->u, nf * NP);
    ALLOC(ctx->ubc, nf * NP);
    ALLOC(ctx->thL, sub_count(g));
    ALLOC(ctx->thF, sub_count(g));
    ALLOC(ctx->WL, nsets * NP);
    ALLOC(ctx->WF, nsets * NP);
    ALLOC(ctx->fflag, nf * NP);
    ALLOC(ctx->ustar, nf * NP);
    ALLOC(ctx->rhof, nf * NP);
    ALLOC(ctx->K, nf * NP);
    ALLOC(ctx->a, ns * NP);
    ALLOC(ctx->c, ns * NP);
    ALLOC(ctx->dinv, ns * NP);
    ALLOC(ctx->b, ns * NP);
    ALLOC(ctx->K32, nf * NP);
    ALLOC(ctx->a32, ns * NP);
    ALLOC(ctx->c32, ns * NP);
    ALLOC(ctx->dinv32, ns * NP);
    ALLOC(ctx->ead32, ns * NP);
    ALLOC(ctx->x, ns * NP);
    ALLOC(ctx->r, ns * NP);
    ALLOC(ctx->p0, ns * NP);
    ALLOC(ctx->p1, ns * NP);
    ALLOC(ctx->q, ns * NP);
    ALLOC(ctx->z, ns * NP);
    ALLOC(ctx->x32, ns * NP);
    ALLOC(ctx->r32, ns * NP);
    ALLOC(ctx->p032, ns * NP);
    ALLOC(ctx->p132, ns * NP);
    ALLOC(ctx->q32, ns * NP);
    ALLOC(ctx->z32, ns * NP);
    int ntx2 = 0, nty2 = 0;
    if (dim == 2) fused2d_tile_dims(g, ntx2, nty2);
    const long long nt2 = (long long)ntx2 * nty2;
    // second r / q buffers and the two partial regions of the fused iteration
    ALLOC(ctx->f32b, ns * NP);
    ALLOC(ctx->fpart, 10 * (dim == 2 ? nt2 : (long long)kMaxTileBlocks) + 64);
    // 3D grids are capped at kMaxTileBlocks workgroups, not at the tile count
    const int maxA = std::max(apply_grid_blocks(g), dim == 3 ? kMaxTileBlocks : 0);
    ctx->capA = maxA + 16;
    ctx->capB = std::max(maxA, vec_grid_blocks(g)) + 16;
    ALLOC(ctx->partials, 2 * ctx->capA + 2 * ctx->capB + 64);
    ALLOC(ctx->counter, 16);
    ALLOC(ctx->sc, 4);
    ALLOC(ctx->flag, 4);
    ctx->stage_elems = (long long)(g.nx + 2) * (g.ny + 2) * (g.dim == 3 ? g.nz + 2 : 1);
    ALLOC(ctx->stage, ctx->stage_elems);
    if (dim == 3) {
        tile_dims(g, ctx->tiles.ntx, ctx->tiles.nty, ctx->tiles.ntz);
        const long long nt = (long long)ctx->tiles.ntx * ctx->tiles.nty * ctx->tiles.ntz;
        ALLOC(ctx->tile_flags, nt);
        ALLOC(ctx->tile_list, nt);
        ALLOC(ctx->tile_count, 4);
        fused_tile_dims(g, ctx->ftiles.ntx, ctx->ftiles.nty, ctx->ftiles.ntz);
        const long long nf = (long long)ctx->ftiles.ntx * ctx->ftiles.nty * ctx->ftiles.ntz;
        ALLOC(ctx->ftile_flags, nf);
        ALLOC(ctx->ftile_list, nf);
        ALLOC(ctx->rowbits, row_bytes(g));
    } else {
        ALLOC(ctx->tile_flags, nt2);
        ALLOC(ctx->tile_list, nt2);
        ALLOC(ctx->tile_count, 4);
    }
#undef ALLOC
    if (hipHostMalloc((void**)&ctx->sc_host, 4 * sizeof(Scalars), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&ctx->flag_host, 4 * sizeof(int), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&ctx->tile_count_host, 4 * sizeof(int), hipHostMallocDefault) !=
            hipSuccess) {
        vfs_destroy(ctx);
        return fail(nullptr, VFS_ENOMEM, "hipHostMalloc failed");
    }
    for (auto& e : ctx->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            vfs_destroy(ctx);
            return fail(nullptr, VFS_EHIP, "hipEventCreate failed");
        }
    }
    for (auto& e : ctx->pev) {
        if (hipEventCreate(&e) != hipSuccess) {
            vfs_destroy(ctx);
            return fail(nullptr, VFS_EHIP, "hipEventCreate failed");
        }
    }
    ctx->stats.n_samples = 0;
    for (int s = 0; s < ns; ++s) ctx->stats.n_samples += set_count(g, sample_set(g.dim, s));
    *out = ctx;
    return VFS_OK;
}

int vfs_set_stream(vfs_ctx* ctx, void* hip_stream) {
    if (!ctx) return VFS_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    if (ctx->net_owned) (void)vfs_unet_set_stream(ctx->net_owned, hip_stream);
    return VFS_OK;
}

int vfs_set_level_sets(vfs_ctx* ctx, const double* phi_liquid, const double* phi_solid) {
    if (!ctx) return VFS_EINVAL;
    if (!phi_liquid) return fail(ctx, VFS_EINVAL, "phi_liquid is NULL");
    const long long n = node_count(ctx->g);
    HIPCHK(hipMemcpyAsync(ctx->phi_l, phi_liquid, (size_t)n * sizeof(double), hipMemcpyDefault,
                          ctx->stream));
    int rc = check_stage(ctx, ctx->phi_l, n, 0, "phi_liquid");
    if (rc) return rc;
    if (phi_solid) {
        HIPCHK(hipMemcpyAsync(ctx->phi_s, phi_solid, (size_t)n * sizeof(double), hipMemcpyDefault,
                              ctx->stream));
        rc = check_stage(ctx, ctx->phi_s, n, 0, "phi_solid");
        if (rc) return rc;
    }
    ctx->has_solid = phi_solid != nullptr;
    ctx->have_phi = true;
    ctx->assembled = false;
    return VFS_OK;
}

int vfs_set_density(vfs_ctx* ctx, const double* rho) {
    if (!ctx) return VFS_EINVAL;
    if (!rho) return fail(ctx, VFS_EINVAL, "rho is NULL");
    int rc = put_set(ctx, 0, rho, ctx->rho, 1, "density");
    if (rc) return rc;
    ctx->have_rho = true;
    ctx->assembled = false;
    return VFS_OK;
}

int vfs_set_viscosity(vfs_ctx* ctx, const double* mu) {
    if (!ctx) return VFS_EINVAL;
    if (!mu) return fail(ctx, VFS_EINVAL, "mu is NULL");
    int rc = put_set(ctx, 0, mu, ctx->mu, 1, "viscosity");
    if (rc) return rc;
    ctx->have_mu = true;
    ctx->assembled = false;
    return VFS_OK;
}

int vfs_set_velocity(vfs_ctx* ctx, const double* u, const double* v, const double* w) {
    if (!ctx) return VFS_EINVAL;
    const double* comp[3] = {u, v, w};
    for (int a = 0; a < ctx->g.dim; ++a) {
        if (!comp[a]) return fail(ctx, VFS_EINVAL, "velocity component is NULL");
        int rc = put_set(ctx, face_set(a), comp[a], ctx->u + a * ctx->g.NP, 0, "velocity");
        if (rc) return rc;
    }
    ctx->have_u = true;
    ctx->u_from_step = false;
    ctx->assembled = false;
    return VFS_OK;
}

int vfs_set_solid_velocity(vfs_ctx* ctx, const double* ub, const double* vb, const double* wb) {
    if (!ctx) return VFS_EINVAL;
    const double* comp[3] = {ub, vb, wb};
    for (int a = 0; a < ctx->g.dim; ++a) {
        double* dst = ctx->ubc + a * ctx->g.NP;
        if (!comp[a]) {
            HIPCHK(hipMemsetAsync(dst, 0, (size_t)ctx->g.NP * sizeof(double), ctx->stream));
            continue;
        }
        int rc = put_set(ctx, face_set(a), comp[a], dst, 0, "solid velocity");
        if (rc) return rc;
    }
    launch_zero_box_faces(ctx->g, ctx->ubc, ctx->stream);
    HIPCHK(hipGetLastError());
    ctx->assembled = false;
    return VFS_OK;
}

int vfs_set_traction(vfs_ctx* ctx, const double* p_bc, const double* const* tau_bc) {
    if (!ctx) return VFS_EINVAL;
    const Geo& g = ctx->g;
    bool any = p_bc != nullptr;
    for (int s = 1; tau_bc && s < g.nsamp(); ++s) any = any || tau_bc[s - 1] != nullptr;
    ctx->assembled = false;
    if (!any) {
        ctx->have_traction = false;
        return VFS_OK;
    }
    if (!ctx->ybc) {
        int rc = dalloc(ctx, &ctx->ybc, (long long)g.nsamp() * g.NP);
        if (rc) return rc;
    }
    ctx->have_traction = false;
    for (int s = 0; s < g.nsamp(); ++s) {
        const double* src = s == 0 ? p_bc : (tau_bc ? tau_bc[s - 1] : nullptr);
        double* dst = ctx->ybc + s * g.NP;
        if (!src) {
            HIPCHK(hipMemsetAsync(dst, 0, (size_t)g.NP * sizeof(double), ctx->stream));
            continue;
        }
        int rc = put_set(ctx, sample_set(g.dim, s), src, dst, 0,
                         s == 0 ? "prescribed pressure" : "prescribed stress");
        if (rc) return rc;
    }
    HIPCHK(hipGetLastError());
    ctx->have_traction = true;
    return VFS_OK;
}

int vfs_advect(vfs_ctx* ctx, double dt) {
    if (!ctx) return VFS_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, VFS_EINVAL, "dt must be > 0 and finite");
    if (!ctx->have_u || !ctx->have_phi)
        return fail(ctx, VFS_ESTATE, "velocity and level sets must be set");
    const Geo& g = ctx->g;
    const long long nf = (long long)g.dim * g.NP;
    if (!ctx->adv_a) {
        int rc = dalloc(ctx, &ctx->adv_a, nf);
        if (!rc) rc = dalloc(ctx, &ctx->adv_b, nf);
        if (!rc) rc = dalloc(ctx, &ctx->adv_ka, nf);
        if (!rc) rc = dalloc(ctx, &ctx->adv_kb, nf);
        if (!rc) rc = dalloc(ctx, &ctx->phi_tmp, node_count(g));
        if (rc) return rc;
    }
    hipStream_t s = ctx->stream;
    // faces the last Stokes step defined; every face when the velocity came
    // from the caller (or from a previous advection)
    const bool all = !(ctx->u_from_step && ctx->assembled);
    launch_known_faces(g, ctx->fflag, ctx->WF, all, ctx->adv_kb, s);
    launch_extend(g, ctx->u, ctx->adv_kb, ctx->adv_a, ctx->adv_ka, s);
    launch_extend(g, ctx->adv_a, ctx->adv_ka, ctx->adv_b, ctx->adv_kb, s);
    launch_extend(g, ctx->adv_b, ctx->adv_kb, ctx->adv_a, ctx->adv_ka, s);
    launch_advect_u(g, dt, ctx->adv_a, ctx->u, s);
    launch_advect_phi(g, dt, ctx->adv_a, ctx->phi_l, ctx->phi_tmp, s);
    HIPCHK(hipGetLastError());
    std::swap(ctx->phi_l, ctx->phi_tmp);
    ctx->u_from_step = false;
    ctx->assembled = false;
    return VFS_OK;
}

int vfs_get_level_set(vfs_ctx* ctx, double* phi_liquid) {
    if (!ctx || !phi_liquid) return ctx ? fail(ctx, VFS_EINVAL, "NULL output") : VFS_EINVAL;
    HIPCHK(hipMemcpyAsync(phi_liquid, ctx->phi_l, (size_t)node_count(ctx->g) * sizeof(double),
                          hipMemcpyDefault, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return VFS_OK;
}

int vfs_set_warm_start(vfs_ctx* ctx, int on) {
    if (!ctx) return VFS_EINVAL;
    ctx->warm_start = on != 0;
    return VFS_OK;
}

int vfs_set_gravity(vfs_ctx* ctx, const double* g) {
    if (!ctx) return VFS_EINVAL;
    if (!g) return fail(ctx, VFS_EINVAL, "g is NULL");
    for (int a = 0; a < ctx->g.dim; ++a) {
        if (!std::isfinite(g[a])) return fail(ctx, VFS_EINVAL, "gravity must be finite");
        ctx->gravity[a] = g[a];
    }
    ctx->assembled = false;
    return VFS_OK;
}

int vfs_set_solver(vfs_ctx* ctx, int precond, int precision, double rel_tol, int max_iter,
                   double w_min) {
    if (!ctx) return VFS_EINVAL;
    if (precond != VFS_PRECOND_JACOBI && precond != VFS_PRECOND_LEARNED &&
        precond != VFS_PRECOND_IC && precond != VFS_PRECOND_SCHWARZ)
        return fail(ctx, VFS_EINVAL, "unsupported preconditioner");
    if ((precond == VFS_PRECOND_IC || precond == VFS_PRECOND_SCHWARZ) && precision != VFS_FP64)
        return fail(ctx, VFS_EINVAL, "the brick preconditioners run in VFS_FP64");
    if (precision != VFS_FP64 && precision != VFS_MIXED)
        return fail(ctx, VFS_EINVAL, "precision must be VFS_FP64 or VFS_MIXED");
    if (precond == VFS_PRECOND_LEARNED && (ctx->g.dim != 3 || precision != VFS_MIXED))
        return fail(ctx, VFS_EINVAL, "the learned preconditioner needs a 3D grid and VFS_MIXED");
    if (!(rel_tol > 0.0) || !(rel_tol < 1.0)) return fail(ctx, VFS_EINVAL, "rel_tol must be in (0,1)");
    if (max_iter < 1) return fail(ctx, VFS_EINVAL, "max_iter must be >= 1");
    if (!(w_min >= 0.0) || !(w_min < 0.5)) return fail(ctx, VFS_EINVAL, "w_min must be in [0,0.5)");
    ctx->precond = precond;
    ctx->precision = precision;
    ctx->tol = rel_tol;
    ctx->max_iter = max_iter;
    if (w_min != ctx->w_min) ctx->assembled = false;
    ctx->w_min = w_min;
    ctx->stats.precision = precision;
    return VFS_OK;
}

int vfs_assemble(vfs_ctx* ctx, double dt) {
    if (!ctx) return VFS_EINVAL;
    int rc = assemble_internal(ctx, dt);
    if (rc) return rc;
    Scalars s{};
    rc = read_scalars(ctx, 0, &s);
    if (rc) return rc;
    ctx->stats.n_active = s.n_active;
    return VFS_OK;
}

int vfs_step(vfs_ctx* ctx, double dt) {
    if (!ctx) return VFS_EINVAL;
    hipStream_t s = ctx->stream;
    HIPCHK(hipEventRecord(ctx->ev[0], s));
    int rc = assemble_internal(ctx, dt);
    if (rc) return rc;
    HIPCHK(hipEventRecord(ctx->ev[1], s));
    const int status = solve_internal(ctx, ctx->b, ctx->x);
    if (status != VFS_OK && status != VFS_ENOTCONV && status != VFS_EBREAKDOWN) return status;
    HIPCHK(hipEventRecord(ctx->ev[2], s));
    rc = recover_internal(ctx);
    if (rc) return rc;
    ctx->u_from_step = true;
    ctx->have_x = true;
    HIPCHK(hipEventRecord(ctx->ev[3], s));
    HIPCHK(hipEventSynchronize(ctx->ev[3]));
    ctx->stats.t_assemble_ms = elapsed(ctx->ev[0], ctx->ev[1]);
    ctx->stats.t_solve_ms = elapsed(ctx->ev[1], ctx->ev[2]);
    ctx->stats.t_recover_ms = elapsed(ctx->ev[2], ctx->ev[3]);
    ctx->stats.t_step_ms = elapsed(ctx->ev[0], ctx->ev[3]);
    Scalars sc{};
    rc = read_scalars(ctx, 0, &sc);
    if (rc) return rc;
    ctx->stats.n_active = sc.n_active;
    return status;
}

int vfs_apply(vfs_ctx* ctx, const double* x, double* y) {
    if (!ctx || !x || !y) return ctx ? fail(ctx, VFS_EINVAL, "NULL vector") : VFS_EINVAL;
    if (!ctx->assembled) return fail(ctx, VFS_ESTATE, "call vfs_assemble first");
    int rc = pack_samples(ctx, x, ctx->z);
    if (rc) return rc;
    const RedArgs none{ctx->sc + 2, nullptr, 0, nullptr, 0, 0};
    launch_apply<double>(ctx->g, ctx->tiles, MODE_APPLY, false, nullptr, nullptr, nullptr, ctx->z,
                         nullptr, ctx->q, ctx->a, ctx->c, ctx->K, nullptr, none, ctx->stream);
    HIPCHK(hipGetLastError());
    return unpack_samples(ctx, ctx->q, y);
}

int vfs_solve(vfs_ctx* ctx, const double* b, double* x) {
    if (!ctx || !x || !b) return ctx ? fail(ctx, VFS_EINVAL, "NULL vector") : VFS_EINVAL;
    if (!ctx->assembled) return fail(ctx, VFS_ESTATE, "call vfs_assemble first");
    int rc = pack_samples(ctx, b, ctx->z);
    if (rc) return rc;
    ctx->have_x = false;   // a raw solve starts from 0
    launch_mask(ctx->b, ctx->z, ctx->a, (long long)ctx->g.nsamp() * ctx->g.NP, ctx->stream);
    HIPCHK(hipEventRecord(ctx->ev[1], ctx->stream));
    const int status = solve_internal(ctx, ctx->b, ctx->x);
    if (status != VFS_OK && status != VFS_ENOTCONV && status != VFS_EBREAKDOWN) return status;
    HIPCHK(hipEventRecord(ctx->ev[2], ctx->stream));
    HIPCHK(hipEventSynchronize(ctx->ev[2]));
    ctx->stats.t_solve_ms = elapsed(ctx->ev[1], ctx->ev[2]);
    rc = unpack_samples(ctx, ctx->x, x);
    if (rc) return rc;
    return status;
}

int vfs_get_velocity(vfs_ctx* ctx, double* u, double* v, double* w) {
    if (!ctx) return VFS_EINVAL;
    double* comp[3] = {u, v, w};
    for (int a = 0; a < ctx->g.dim; ++a) {
        if (!comp[a]) continue;
        int rc = get_set(ctx, face_set(a), ctx->u + a * ctx->g.NP, comp[a]);
        if (rc) return rc;
    }
    return VFS_OK;
}

int vfs_get_pressure(vfs_ctx* ctx, double* p) {
    if (!ctx || !p) return VFS_EINVAL;
    return get_set(ctx, 0, ctx->x, p);
}

int vfs_get_stress(vfs_ctx* ctx, double* const* tau) {
    if (!ctx || !tau) return VFS_EINVAL;
    for (int s = 1; s < ctx->g.nsamp(); ++s) {
        if (!tau[s - 1]) continue;
        int rc = get_set(ctx, sample_set(ctx->g.dim, s), ctx->x + s * ctx->g.NP, tau[s - 1]);
        if (rc) return rc;
    }
    return VFS_OK;
}

int vfs_get_solution(vfs_ctx* ctx, double* x) {
    if (!ctx || !x) return VFS_EINVAL;
    return unpack_samples(ctx, ctx->x, x);
}

int vfs_get_rhs(vfs_ctx* ctx, double* b) {
    if (!ctx || !b) return VFS_EINVAL;
    if (!ctx->assembled) return fail(ctx, VFS_ESTATE, "nothing assembled");
    return unpack_samples(ctx, ctx->b, b);
}

int vfs_get_weights(vfs_ctx* ctx, int set, int which, double* out) {
    if (!ctx || !out) return VFS_EINVAL;
    if (!ctx->assembled) return fail(ctx, VFS_ESTATE, "nothing assembled");
    int internal;
    if (ctx->g.dim == 2) {
        if (set == VFS_SET_CELL || set == VFS_SET_FACE_X || set == VFS_SET_FACE_Y)
            internal = set;
        else if (set == VFS_SET_NODE)
            internal = 3;
        else
            return fail(ctx, VFS_EINVAL, "bad set for 2D");
    } else {
        if (set < 0 || set > 6) return fail(ctx, VFS_EINVAL, "bad set for 3D");
        internal = set;
    }
    if (which != VFS_WEIGHT_LIQUID && which != VFS_WEIGHT_FLUID)
        return fail(ctx, VFS_EINVAL, "bad weight kind");
    const double* src = (which == VFS_WEIGHT_LIQUID ? ctx->WL : ctx->WF) + internal * ctx->g.NP;
    return get_set(ctx, internal, src, out);
}

int vfs_get_active_mask(vfs_ctx* ctx, int sample, uint8_t* out) {
    if (!ctx || !out) return ctx ? fail(ctx, VFS_EINVAL, "NULL output") : VFS_EINVAL;
    if (!ctx->assembled) return fail(ctx, VFS_ESTATE, "nothing assembled");
    const Geo& g = ctx->g;
    if (sample < 0 || sample >= g.nsamp()) return fail(ctx, VFS_EINVAL, "bad sample type");
    int shp[3];
    set_shape(g, sample_set(g.dim, sample), shp);
    const long long n = (long long)shp[0] * shp[1] * shp[2];
    uint8_t* stage8 = (uint8_t*)ctx->stage;
    launch_unpack_active(g, shp, ctx->a + sample * g.NP, stage8, ctx->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, stage8, (size_t)n, hipMemcpyDefault, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return VFS_OK;
}

int vfs_training_pair(vfs_ctx* ctx, const double* x_star, const double* x_k, double* r,
                      double* e) {
    if (!ctx || !x_star || !x_k || !r || !e)
        return ctx ? fail(ctx, VFS_EINVAL, "NULL vector") : VFS_EINVAL;
    if (!ctx->assembled) return fail(ctx, VFS_ESTATE, "call vfs_assemble first");
    const Geo& g = ctx->g;
    // solver work vectors serve as staging: every solve re-initialises them
    int rc = pack_samples(ctx, x_k, ctx->z);
    if (rc) return rc;
    rc = pack_samples(ctx, x_star, ctx->p0);
    if (rc) return rc;
    Scalars so{};
    rc = true_residual(ctx, ctx->b, ctx->z, &so);   // ctx->r = b - A x_k
    if (rc) return rc;
    launch_sub_mask(ctx->q, ctx->p0, ctx->z, ctx->a, (long long)g.nsamp() * g.NP, ctx->stream);
    HIPCHK(hipGetLastError());
    rc = unpack_samples(ctx, ctx->r, r);
    if (rc) return rc;
    return unpack_samples(ctx, ctx->q, e);
}

int vfs_get_active(vfs_ctx* ctx, uint8_t* out) {
    if (!ctx || !out) return VFS_EINVAL;
    if (!ctx->assembled) return fail(ctx, VFS_ESTATE, "nothing assembled");
    const Geo& g = ctx->g;
    long long off = 0;
    uint8_t* stage8 = (uint8_t*)ctx->stage;
    for (int s = 0; s < g.nsamp(); ++s) {
        const int set = sample_set(g.dim, s);
        int shp[3];
        set_shape(g, set, shp);
        const long long n = (long long)shp[0] * shp[1] * shp[2];
        launch_unpack_active(g, shp, ctx->a + s * g.NP, stage8, ctx->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out + off, stage8, (size_t)n, hipMemcpyDefault, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        off += n;
    }
    return VFS_OK;
}

int vfs_get_stats(vfs_ctx* ctx, vfs_stats* out) {
    if (!ctx || !out) return VFS_EINVAL;
    ctx->stats.n_apply_timed = ctx->prof_apply_n;
    ctx->stats.n_update_timed = ctx->prof_update_n;
    ctx->stats.t_apply_avg_ms = ctx->prof_apply_n ? ctx->prof_apply_ms / ctx->prof_apply_n : 0.0;
    ctx->stats.t_update_avg_ms =
        ctx->prof_update_n ? ctx->prof_update_ms / ctx->prof_update_n : 0.0;
    ctx->stats.t_precond_avg_ms =
        ctx->prof_apply_n ? ctx->prof_precond_ms / ctx->prof_apply_n : 0.0;
    *out = ctx->stats;
    return VFS_OK;
}

int vfs_set_profiling(vfs_ctx* ctx, int on) {
    if (!ctx) return VFS_EINVAL;
    ctx->prof = on != 0;
    if (ctx->prof) {
        ctx->prof_apply_ms = ctx->prof_update_ms = ctx->prof_precond_ms = 0.0;
        ctx->prof_apply_n = ctx->prof_update_n = 0;
    }
    return VFS_OK;
}

int vfs_get_sizes(const vfs_ctx* ctx, int64_t* n_samples, int64_t* n_faces) {
    if (!ctx) return VFS_EINVAL;
    const Geo& g = ctx->g;
    if (n_samples) {
        int64_t s = 0;
        for (int q = 0; q < g.nsamp(); ++q) s += set_count(g, sample_set(g.dim, q));
        *n_samples = s;
    }
    if (n_faces) {
        int64_t f = 0;
        for (int a = 0; a < g.dim; ++a) f += set_count(g, face_set(a));
        *n_faces = f;
    }
    return VFS_OK;
}

}  // extern "C"
