// Host side of the learned preconditioner: the network object, its forward
// and backward passes as sequences of kernel launches, Adam, the C entry
// points, and the coupling to a 3D solver context (training step and the
// preconditioner application used by flexible CG).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "vfs_unet.h"

namespace vfs {
// sample-order user vectors <-> padded device vectors (vfs_api.hip)
int ctx_put_samples(vfs_ctx* ctx, const double* user, double* dst);
int ctx_get_samples(vfs_ctx* ctx, const double* src, double* user);
int ctx_fail(vfs_ctx* ctx, int code, const std::string& msg);
}  // namespace vfs

using namespace vfs;

namespace {

thread_local std::string g_unet_err;

int ufail(vfs_unet* u, int code, const std::string& m) {
    if (u)
        u->err = m;
    else
        g_unet_err = m;
    return code;
}

#define UCHK(call)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ufail(u, VFS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t tensor_bytes(const Level& L, int ch) { return align256((size_t)L.padded() * ch * 2); }

struct TSpec {
    uint16_t** ptr;
    int level, ch;
};

long long wf_elems(int l) { return (long long)pad16(kNet[l].cout) * conv_kp(kNet[l].cin); }
long long wd_elems(int l) { return (long long)kNet[l].cin * conv_kp(pad16(kNet[l].cout)); }

void prep_all(vfs_unet* u, hipStream_t s) {
    for (int l = 0; l < kNetLayers; ++l)
        launch_prep_weights(u->w + u->poff[l], u->wf[l], u->wd[l], kNet[l].cin, kNet[l].cout, s);
}

int conv(vfs_unet* u, int layer, bool grad, const uint16_t* in, uint16_t* out, float* out32,
         int epi, const uint16_t* mask, hipStream_t s, const int* skip) {
    const NetLayer& N = kNet[layer];
    ConvArgs a{in, grad ? u->wd[layer] : u->wf[layer], out, out32, mask, u->L[N.level], skip};
    const int ci = grad ? pad16(N.cout) : N.cin;
    const int co = grad ? N.cin : pad16(N.cout);
    if (!launch_conv3(ci, co, epi, a, s))
        return ufail(u, VFS_EINVAL, "unsupported convolution shape");
    return VFS_OK;
}

int wgrad(vfs_unet* u, int layer, const uint16_t* in, const uint16_t* g, float scale,
          hipStream_t s) {
    const NetLayer& N = kNet[layer];
    const Level& L = u->L[N.level];
    const int co = pad16(N.cout);
    if (!launch_wgrad(N.cin, co, in, g, L, u->wpart, nullptr, s))
        return ufail(u, VFS_EINVAL, "unsupported weight-gradient shape");
    launch_wgrad_reduce(N.cin, co, N.cout, u->wpart, wgrad_chunks(L), u->g + u->poff[layer], scale,
                        s);
    return VFS_OK;
}

// gradient of <gy, y> with respect to the weights, added to u->g (scaled)
int net_backward(vfs_unet* u, hipStream_t s, float scale) {
    const Level* L = u->L;
    int rc;
#define RUN(x)              \
    if ((rc = (x)) != VFS_OK) return rc
    RUN(wgrad(u, 7, u->s0, u->gy, scale, s));
    RUN(conv(u, 7, true, u->gy, u->gs0, nullptr, EPI_PLAIN, nullptr, s, nullptr));
    launch_summask(u->gs0, u->d1, u->gd1, L[1], 16, s);
    RUN(wgrad(u, 6, u->s1, u->gd1, scale, s));
    RUN(conv(u, 6, true, u->gd1, u->gs1, nullptr, EPI_PLAIN, nullptr, s, nullptr));
    launch_summask(u->gs1, u->d2, u->gd2, L[2], 32, s);
    RUN(wgrad(u, 5, u->s2, u->gd2, scale, s));
    RUN(conv(u, 5, true, u->gd2, u->gs2, nullptr, EPI_PLAIN, nullptr, s, nullptr));
    launch_summask(u->gs2, u->d3, u->gd3, L[3], 64, s);
    RUN(wgrad(u, 4, u->c3, u->gd3, scale, s));
    RUN(conv(u, 4, true, u->gd3, u->gc3, nullptr, EPI_MASK, u->c3, s, nullptr));
    RUN(wgrad(u, 3, u->p2, u->gc3, scale, s));
    RUN(conv(u, 3, true, u->gc3, u->gp2, nullptr, EPI_PLAIN, nullptr, s, nullptr));
    launch_upaddmask(u->gs2, u->gp2, u->c2, u->gc2, L[2], 64, s);
    RUN(wgrad(u, 2, u->p1, u->gc2, scale, s));
    RUN(conv(u, 2, true, u->gc2, u->gp1, nullptr, EPI_PLAIN, nullptr, s, nullptr));
    launch_upaddmask(u->gs1, u->gp1, u->c1, u->gc1, L[1], 32, s);
    RUN(wgrad(u, 1, u->p0, u->gc1, scale, s));
    RUN(conv(u, 1, true, u->gc1, u->gp0, nullptr, EPI_PLAIN, nullptr, s, nullptr));
    launch_upaddmask(u->gs0, u->gp0, u->c0, u->gc0, L[0], 16, s);
    RUN(wgrad(u, 0, u->x, u->gc0, scale, s));
#undef RUN
    UCHK(hipGetLastError());
    return VFS_OK;
}

int check_level0(vfs_unet* u, int X, int Y, int Z) {
    if (X < 8 || Y < 8 || Z < 8 || X % 8 || Y % 8 || Z % 8)
        return ufail(u, VFS_EINVAL, "tensor extents must be positive multiples of 8");
    if ((long long)X * Y * Z > (1LL << 31))
        return ufail(u, VFS_EINVAL, "tensor too large");
    return VFS_OK;
}

int stage_floats(vfs_unet* u, size_t n) {
    if (u->stage_cap >= n) return VFS_OK;
    if (u->stage) (void)hipFree(u->stage);
    u->stage = nullptr;
    u->stage_cap = 0;
    UCHK(hipMalloc(&u->stage, n * sizeof(float)));
    u->stage_cap = n;
    return VFS_OK;
}

int check_floats(vfs_unet* u, const float* d, long long n, const char* what) {
    UCHK(hipMemsetAsync(u->flag, 0, sizeof(int), u->stream));
    launch_check_f32(d, n, u->flag, u->stream);
    UCHK(hipMemcpyAsync(u->flag_host, u->flag, sizeof(int), hipMemcpyDeviceToHost, u->stream));
    UCHK(hipStreamSynchronize(u->stream));
    if (*u->flag_host) return ufail(u, VFS_EINVAL, std::string(what) + ": non-finite value");
    return VFS_OK;
}

}  // namespace

namespace vfs {

Level net_level0(const Geo& g) {
    auto r8 = [](int n) { return (n + 1 + 7) / 8 * 8; };
    return Level{r8(g.nx), r8(g.ny), r8(g.nz)};
}

int net_ensure(vfs_unet* u, const Level& L0, bool grads) {
    const bool same = u->L[0].X == L0.X && u->L[0].Y == L0.Y && u->L[0].Z == L0.Z;
    if (same && u->fwd_ready && (!grads || u->bwd_ready)) return VFS_OK;
    if (!same) {
        u->fwd_ready = u->bwd_ready = false;
        u->fwd_valid = false;
    }
    for (int l = 0; l < 4; ++l) u->L[l] = Level{L0.X >> l, L0.Y >> l, L0.Z >> l};
    hipStream_t s = u->stream;
    if (!u->fwd_ready) {
        const TSpec f[] = {{&u->x, 0, 16},  {&u->c0, 0, 16}, {&u->p0, 1, 16}, {&u->c1, 1, 32},
                           {&u->p1, 2, 32}, {&u->c2, 2, 64}, {&u->p2, 3, 64}, {&u->c3, 3, 128},
                           {&u->d3, 3, 64}, {&u->s2, 2, 64}, {&u->d2, 2, 32}, {&u->s1, 1, 32},
                           {&u->d1, 1, 16}, {&u->s0, 0, 16}};
        size_t bytes = align256((size_t)L0.voxels() * 8 * sizeof(float));
        for (const auto& t : f) bytes += tensor_bytes(u->L[t.level], t.ch);
        if (bytes > u->fwd_cap) {
            if (u->fwd) (void)hipFree(u->fwd);
            u->fwd = nullptr;
            u->fwd_cap = 0;
            UCHK(hipMalloc(&u->fwd, bytes));
            u->fwd_cap = bytes;
        }
        UCHK(hipMemsetAsync(u->fwd, 0, bytes, s));
        size_t o = 0;
        for (const auto& t : f) {
            *t.ptr = reinterpret_cast<uint16_t*>(u->fwd + o);
            o += tensor_bytes(u->L[t.level], t.ch);
        }
        u->y32 = reinterpret_cast<float*>(u->fwd + o);
        u->fwd_ready = true;
    }
    if (grads && !u->bwd_ready) {
        const TSpec b[] = {{&u->gy, 0, 16},  {&u->gs0, 0, 16}, {&u->gd1, 1, 16}, {&u->gs1, 1, 32},
                           {&u->gd2, 2, 32}, {&u->gs2, 2, 64}, {&u->gd3, 3, 64}, {&u->gc3, 3, 128},
                           {&u->gp2, 3, 64}, {&u->gc2, 2, 64}, {&u->gp1, 2, 32}, {&u->gc1, 1, 32},
                           {&u->gp0, 1, 16}, {&u->gc0, 0, 16}};
        size_t part = 0;
        for (int l = 0; l < kNetLayers; ++l)
            part = std::max(part, (size_t)wgrad_chunks(u->L[kNet[l].level]) * 27 *
                                      pad16(kNet[l].cout) * kNet[l].cin);
        size_t bytes = align256(part * sizeof(float));
        for (const auto& t : b) bytes += tensor_bytes(u->L[t.level], t.ch);
        if (bytes > u->bwd_cap) {
            if (u->bwd) (void)hipFree(u->bwd);
            u->bwd = nullptr;
            u->bwd_cap = 0;
            UCHK(hipMalloc(&u->bwd, bytes));
            u->bwd_cap = bytes;
        }
        UCHK(hipMemsetAsync(u->bwd, 0, bytes, s));
        size_t o = 0;
        for (const auto& t : b) {
            *t.ptr = reinterpret_cast<uint16_t*>(u->bwd + o);
            o += tensor_bytes(u->L[t.level], t.ch);
        }
        u->wpart = reinterpret_cast<float*>(u->bwd + o);
        u->bwd_ready = true;
    }
    return VFS_OK;
}

int net_forward(vfs_unet* u, hipStream_t s, const int* skip) {
    const Level* L = u->L;
    int rc;
#define RUN(x)              \
    if ((rc = (x)) != VFS_OK) return rc
    RUN(conv(u, 0, false, u->x, u->c0, nullptr, EPI_RELU, nullptr, s, skip));
    launch_pool(u->c0, u->p0, L[1], 16, skip, s);
    RUN(conv(u, 1, false, u->p0, u->c1, nullptr, EPI_RELU, nullptr, s, skip));
    launch_pool(u->c1, u->p1, L[2], 32, skip, s);
    RUN(conv(u, 2, false, u->p1, u->c2, nullptr, EPI_RELU, nullptr, s, skip));
    launch_pool(u->c2, u->p2, L[3], 64, skip, s);
    RUN(conv(u, 3, false, u->p2, u->c3, nullptr, EPI_RELU, nullptr, s, skip));
    RUN(conv(u, 4, false, u->c3, u->d3, nullptr, EPI_RELU, nullptr, s, skip));
    launch_upadd(u->d3, u->c2, u->s2, L[2], 64, skip, s);
    RUN(conv(u, 5, false, u->s2, u->d2, nullptr, EPI_RELU, nullptr, s, skip));
    launch_upadd(u->d2, u->c1, u->s1, L[1], 32, skip, s);
    RUN(conv(u, 6, false, u->s1, u->d1, nullptr, EPI_RELU, nullptr, s, skip));
    launch_upadd(u->d1, u->c0, u->s0, L[0], 16, skip, s);
    RUN(conv(u, 7, false, u->s0, nullptr, u->y32, EPI_F32, nullptr, s, skip));
#undef RUN
    UCHK(hipGetLastError());
    u->fwd_valid = true;
    return VFS_OK;
}

int net_bufs(vfs_ctx* ctx) {
    if (ctx->netvec) return VFS_OK;
    const size_t n = (size_t)ctx->g.nsamp() * ctx->g.NP;
    const size_t np = (size_t)kNetPartRegions * kNetPartVals * kNetPartCap;
    if (hipMalloc(&ctx->netvec, kNetVecs * n * sizeof(float)) != hipSuccess ||
        hipMalloc(&ctx->netpart, np * sizeof(double)) != hipSuccess ||
        hipMalloc(&ctx->netcoef, 4 * sizeof(double)) != hipSuccess) {
        if (ctx->netvec) (void)hipFree(ctx->netvec);
        if (ctx->netpart) (void)hipFree(ctx->netpart);
        if (ctx->netcoef) (void)hipFree(ctx->netcoef);
        ctx->netvec = nullptr;
        ctx->netpart = nullptr;
        ctx->netcoef = nullptr;
        return ctx_fail(ctx, VFS_ENOMEM, "device allocation failed: preconditioner work space");
    }
    // entries outside the active tiles are read as halo values and stay zero
    if (hipMemset(ctx->netvec, 0, kNetVecs * n * sizeof(float)) != hipSuccess ||
        hipMemset(ctx->netcoef, 0, 4 * sizeof(double)) != hipSuccess)
        return ctx_fail(ctx, VFS_EHIP, "hipMemset failed");
    return VFS_OK;
}

int net_precond(vfs_unet* u, vfs_ctx* ctx, const float* r, const float* dinv, const float* a,
                const float* c, const float* K, const double* part_rdr, int nb_rdr,
                const FcgHist& fh, const int* skip) {
    const Geo& g = ctx->g;
    hipStream_t s = ctx->stream;
    const long long n = (long long)g.nsamp() * g.NP;
    float* D = ctx->netvec;
    float* QD = D + n;
    float* R1 = D + 2 * n;
    float* NV = D + 3 * n;
    float* QN = D + 4 * n;
    const int nbA = apply_blocks(g, ctx->tiles, 4);
    // Jacobi step: d = D^-1 r, A d
    const RedArgs j1{ctx->sc, nullptr, 0, net_region(ctx, 0), 0, 0, nullptr, 0, skip};
    launch_apply<float>(g, ctx->tiles, MODE_JDIR, false, r, nullptr, dinv, nullptr, D, QD, a, c, K,
                        nullptr, j1, s);
    launch_coarse_prep(g, ctx->tiles, r, QD, dinv, part_rdr, nb_rdr, net_region(ctx, 0), nbA, R1,
                       net_region(ctx, 1), ctx->netcoef, nullptr, nullptr, nullptr, skip, s);
    // network on r1
    launch_net_scale(net_region(ctx, 1), coarse_blocks(g), ctx->sc, u->dscal, s);
    launch_net_pack<float>(g, u->L[0], R1, dinv, u->dscal, u->x, skip, s);
    int rc = net_forward(u, s, skip);
    if (rc) return rc;
    launch_net_unpack(g, ctx->tiles, u->L[0], u->y32, dinv, u->dscal, R1, R1, NV,
                      net_region(ctx, 2), skip, s);
    // A n and the combination z = a1 d + w n
    const RedArgs j2{ctx->sc, nullptr, 0, net_region(ctx, 3), 0, 0, nullptr, 0, skip};
    launch_apply<float>(g, ctx->tiles, MODE_JDIR, true, nullptr, NV, dinv, nullptr, nullptr, QN, a,
                        c, K, nullptr, j2, s);
    launch_coarse_finish(g, ctx->tiles, D, NV, r, dinv, ctx->netcoef, net_region(ctx, 2),
                         net_unpack_blocks(g),
                         net_region(ctx, 3), nbA, fh, ctx->z32, net_region(ctx, 4), skip, s);
    if (hipGetLastError() != hipSuccess) return ufail(u, VFS_EHIP, "launch failed");
    return VFS_OK;
}

int net_prepare_ctx(vfs_unet* u, vfs_ctx* ctx) {
    const Geo& g = ctx->g;
    int rc = net_bufs(ctx);
    if (rc) return ufail(u, rc, ctx->err);
    if (ctx->netvec_dirty) {
        // the work vectors are read as halo values next to the active tiles:
        // values a previous assembly left in now-inactive tiles must go
        UCHK(hipMemsetAsync(ctx->netvec, 0,
                            (size_t)kNetVecs * g.nsamp() * g.NP * sizeof(float), ctx->stream));
        ctx->netvec_dirty = false;
    }
    rc = net_ensure(u, net_level0(g), false);
    if (rc) return rc;
    launch_net_geometry(g, u->L[0], ctx->WL, ctx->WF, ctx->rho, ctx->mu, ctx->dt_assembled, u->x,
                        ctx->stream);
    UCHK(hipGetLastError());
    return VFS_OK;
}

}  // namespace vfs

namespace {

// FP32 copies of the assembled coefficients (the mixed path makes them at
// assembly; an FP64 context gets them here)
int ctx_f32(vfs_ctx* ctx) {
    if (ctx->precision == VFS_MIXED) return VFS_OK;
    const Geo& g = ctx->g;
    const long long ns = (long long)g.nsamp() * g.NP, nf = (long long)g.dim * g.NP;
    launch_to_f32(ctx->K, ctx->K32, nf, ctx->stream);
    launch_to_f32(ctx->a, ctx->a32, ns, ctx->stream);
    launch_to_f32(ctx->c, ctx->c32, ns, ctx->stream);
    launch_to_f32(ctx->dinv, ctx->dinv32, ns, ctx->stream);
    return VFS_OK;
}

int ctx_ready(vfs_unet* u, vfs_ctx* ctx) {
    if (!ctx) return ufail(u, VFS_EINVAL, "context is NULL");
    if (ctx->g.dim != 3) return ufail(u, VFS_EINVAL, "the learned preconditioner is 3D only");
    if (!ctx->assembled) return ufail(u, VFS_ESTATE, "assemble the context first");
    if (!u->have_weights) return ufail(u, VFS_ESTATE, "set the network weights first");
    if (ctx->stream != u->stream)
        return ufail(u, VFS_EINVAL, "network and context must use the same stream");
    return VFS_OK;
}

}  // namespace

extern "C" {

const char* vfs_unet_last_error(const vfs_unet* u) {
    return u ? u->err.c_str() : g_unet_err.c_str();
}

int64_t vfs_unet_param_count(void) {
    long long n = 0;
    for (int l = 0; l < kNetLayers; ++l) n += (long long)kNet[l].cout * kNet[l].cin * 27;
    return n;
}

int vfs_unet_destroy(vfs_unet* u) {
    if (!u) return VFS_OK;
    void* bufs[] = {u->w, u->m, u->v, u->g, u->wbuf, u->flag, u->dscal, u->dpart, u->fwd, u->bwd,
                    u->stage};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    if (u->flag_host) (void)hipHostFree(u->flag_host);
    if (u->hscal) (void)hipHostFree(u->hscal);
    delete u;
    return VFS_OK;
}

int vfs_unet_create(vfs_unet** out) {
    if (!out) return ufail(nullptr, VFS_EINVAL, "out is NULL");
    *out = nullptr;
    vfs_unet* u = new vfs_unet();
    u->nparam = vfs_unet_param_count();
    long long o = 0, wb = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        u->poff[l] = o;
        o += (long long)kNet[l].cout * kNet[l].cin * 27;
        wb += wf_elems(l) + wd_elems(l);
    }
    u->poff[kNetLayers] = o;
    auto fail_alloc = [&](const char* what) {
        const std::string m = std::string("device allocation failed: ") + what;
        vfs_unet_destroy(u);
        return ufail(nullptr, VFS_ENOMEM, m);
    };
    const size_t pb = (size_t)u->nparam * sizeof(float);
    if (hipMalloc(&u->w, pb) != hipSuccess) return fail_alloc("weights");
    if (hipMalloc(&u->m, pb) != hipSuccess) return fail_alloc("moments");
    if (hipMalloc(&u->v, pb) != hipSuccess) return fail_alloc("moments");
    if (hipMalloc(&u->g, pb) != hipSuccess) return fail_alloc("gradient");
    if (hipMalloc(&u->wbuf, (size_t)wb * 2) != hipSuccess) return fail_alloc("bf16 weights");
    if (hipMalloc(&u->flag, sizeof(int)) != hipSuccess) return fail_alloc("flag");
    if (hipMalloc(&u->dscal, 8 * sizeof(double)) != hipSuccess) return fail_alloc("scalars");
    if (hipMalloc(&u->dpart, (size_t)kMaxNetPartials * 3 * sizeof(double)) != hipSuccess)
        return fail_alloc("partials");
    if (hipHostMalloc(&u->flag_host, sizeof(int)) != hipSuccess) return fail_alloc("pinned flag");
    if (hipHostMalloc(&u->hscal, 8 * sizeof(double)) != hipSuccess)
        return fail_alloc("pinned scalars");
    long long ow = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        u->wf[l] = u->wbuf + ow;
        ow += wf_elems(l);
        u->wd[l] = u->wbuf + ow;
        ow += wd_elems(l);
    }
    if (hipMemset(u->w, 0, pb) != hipSuccess || hipMemset(u->m, 0, pb) != hipSuccess ||
        hipMemset(u->v, 0, pb) != hipSuccess || hipMemset(u->g, 0, pb) != hipSuccess ||
        hipMemset(u->wbuf, 0, (size_t)wb * 2) != hipSuccess ||
        hipMemset(u->dscal, 0, 8 * sizeof(double)) != hipSuccess)
        return fail_alloc("initialisation");
    *out = u;
    return VFS_OK;
}

int vfs_unet_set_stream(vfs_unet* u, void* hip_stream) {
    if (!u) return VFS_EINVAL;
    u->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return VFS_OK;
}

int vfs_unet_set_weights(vfs_unet* u, const float* w, int64_t count) {
    if (!u || !w) return u ? ufail(u, VFS_EINVAL, "weights pointer is NULL") : VFS_EINVAL;
    if (count != u->nparam) return ufail(u, VFS_EINVAL, "weight count does not match the network");
    UCHK(hipMemcpyAsync(u->g, w, (size_t)count * sizeof(float), hipMemcpyDefault, u->stream));
    int rc = check_floats(u, u->g, count, "weights");
    if (rc) return rc;
    UCHK(hipMemcpyAsync(u->w, u->g, (size_t)count * sizeof(float), hipMemcpyDeviceToDevice,
                        u->stream));
    UCHK(hipMemsetAsync(u->g, 0, (size_t)count * sizeof(float), u->stream));
    UCHK(hipMemsetAsync(u->m, 0, (size_t)count * sizeof(float), u->stream));
    UCHK(hipMemsetAsync(u->v, 0, (size_t)count * sizeof(float), u->stream));
    prep_all(u, u->stream);
    UCHK(hipGetLastError());
    UCHK(hipStreamSynchronize(u->stream));
    u->adam_t = 0;
    u->have_weights = true;
    u->fwd_valid = false;
    return VFS_OK;
}

int vfs_unet_get_weights(vfs_unet* u, float* w, int64_t count) {
    if (!u || !w) return VFS_EINVAL;
    if (count != u->nparam) return ufail(u, VFS_EINVAL, "weight count does not match the network");
    UCHK(hipMemcpyAsync(w, u->w, (size_t)count * sizeof(float), hipMemcpyDefault, u->stream));
    UCHK(hipStreamSynchronize(u->stream));
    return VFS_OK;
}

int vfs_unet_get_grad(vfs_unet* u, float* g, int64_t count) {
    if (!u || !g) return VFS_EINVAL;
    if (count != u->nparam) return ufail(u, VFS_EINVAL, "gradient count does not match the network");
    UCHK(hipMemcpyAsync(g, u->g, (size_t)count * sizeof(float), hipMemcpyDefault, u->stream));
    UCHK(hipStreamSynchronize(u->stream));
    return VFS_OK;
}

int vfs_unet_zero_grad(vfs_unet* u) {
    if (!u) return VFS_EINVAL;
    UCHK(hipMemsetAsync(u->g, 0, (size_t)u->nparam * sizeof(float), u->stream));
    return VFS_OK;
}

int vfs_unet_forward(vfs_unet* u, int X, int Y, int Z, const float* x, float* y) {
    if (!u || !x || !y) return u ? ufail(u, VFS_EINVAL, "NULL tensor") : VFS_EINVAL;
    if (!u->have_weights) return ufail(u, VFS_ESTATE, "set the network weights first");
    int rc = check_level0(u, X, Y, Z);
    if (rc) return rc;
    const Level L0{X, Y, Z};
    rc = net_ensure(u, L0, false);
    if (rc) return rc;
    const long long V = L0.voxels();
    rc = stage_floats(u, (size_t)V * kNetIn);
    if (rc) return rc;
    UCHK(hipMemcpyAsync(u->stage, x, (size_t)V * kNetIn * sizeof(float), hipMemcpyDefault,
                        u->stream));
    rc = check_floats(u, u->stage, V * kNetIn, "input tensor");
    if (rc) return rc;
    launch_import16(u->stage, kNetIn, L0, u->x, u->stream);
    rc = net_forward(u, u->stream, nullptr);
    if (rc) return rc;
    launch_export6(u->y32, V, u->stage, u->stream);
    UCHK(hipGetLastError());
    UCHK(hipMemcpyAsync(y, u->stage, (size_t)V * kNetOut * sizeof(float), hipMemcpyDefault,
                        u->stream));
    UCHK(hipStreamSynchronize(u->stream));
    return VFS_OK;
}

int vfs_unet_backward(vfs_unet* u, const float* gy) {
    if (!u || !gy) return u ? ufail(u, VFS_EINVAL, "NULL tensor") : VFS_EINVAL;
    if (!u->fwd_valid) return ufail(u, VFS_ESTATE, "run vfs_unet_forward first");
    int rc = net_ensure(u, u->L[0], true);
    if (rc) return rc;
    const long long V = u->L[0].voxels();
    rc = stage_floats(u, (size_t)V * kNetIn);
    if (rc) return rc;
    UCHK(hipMemcpyAsync(u->stage, gy, (size_t)V * kNetOut * sizeof(float), hipMemcpyDefault,
                        u->stream));
    rc = check_floats(u, u->stage, V * kNetOut, "output gradient");
    if (rc) return rc;
    launch_import16(u->stage, kNetOut, u->L[0], u->gy, u->stream);
    rc = net_backward(u, u->stream, 1.0f);
    if (rc) return rc;
    UCHK(hipStreamSynchronize(u->stream));
    return VFS_OK;
}

int vfs_unet_adam(vfs_unet* u, double lr, double beta1, double beta2, double eps,
                  double grad_scale) {
    if (!u) return VFS_EINVAL;
    if (!u->have_weights) return ufail(u, VFS_ESTATE, "set the network weights first");
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
        !(eps > 0.0) || !std::isfinite(grad_scale))
        return ufail(u, VFS_EINVAL, "bad Adam hyper-parameters");
    ++u->adam_t;
    const double c1 = 1.0 - std::pow(beta1, u->adam_t), c2 = 1.0 - std::pow(beta2, u->adam_t);
    launch_adam(u->w, u->m, u->v, u->g, u->nparam, (float)lr, (float)beta1, (float)beta2,
                (float)eps, (float)c1, (float)c2, (float)grad_scale, u->stream);
    UCHK(hipMemsetAsync(u->g, 0, (size_t)u->nparam * sizeof(float), u->stream));
    prep_all(u, u->stream);
    UCHK(hipGetLastError());
    u->fwd_valid = false;
    return VFS_OK;
}

int vfs_unet_train_step(vfs_unet* u, vfs_ctx* ctx, const double* r, const double* e,
                        double* loss) {
    if (!u) return VFS_EINVAL;
    int rc = ctx_ready(u, ctx);
    if (rc) return rc;
    if (!r || !e) return ufail(u, VFS_EINVAL, "NULL vector");
    const Geo& g = ctx->g;
    hipStream_t s = ctx->stream;
    const long long n = (long long)g.nsamp() * g.NP;
    if ((rc = ctx_f32(ctx))) return rc;
    if ((rc = net_prepare_ctx(u, ctx))) return rc;
    if ((rc = net_ensure(u, u->L[0], true))) return rc;
    if ((rc = ctx_put_samples(ctx, r, ctx->z))) return ufail(u, rc, vfs_last_error(ctx));
    launch_mask(ctx->r, ctx->z, ctx->a, n, s);
    if ((rc = ctx_put_samples(ctx, e, ctx->q))) return ufail(u, rc, vfs_last_error(ctx));
    launch_mask(ctx->z, ctx->q, ctx->a, n, s);
    launch_to_f32(ctx->r, ctx->r32, n, s);
    float* D = ctx->netvec;
    float* QD = D + n;
    float* R1 = D + 2 * n;
    float* NV = D + 3 * n;
    float* QN = D + 4 * n;
    const int nbA = apply_blocks(g, ctx->tiles, 4);
    // Jacobi step on (r, e): r1 = r - a1 A d, e1 = e - a1 d (FP64 copies in ctx->r, ctx->z)
    launch_net_rdr(g, ctx->r32, ctx->dinv32, u->dpart, s);
    const RedArgs j1{ctx->sc, nullptr, 0, net_region(ctx, 0), 0, 0, nullptr, 0, nullptr};
    launch_apply<float>(g, ctx->tiles, MODE_JDIR, false, ctx->r32, nullptr, ctx->dinv32, nullptr, D,
                        QD, ctx->a32, ctx->c32, ctx->K32, nullptr, j1, s);
    launch_coarse_prep(g, ctx->tiles, ctx->r32, QD, ctx->dinv32, u->dpart, net_rdr_blocks(g),
                       net_region(ctx, 0),
                       nbA, R1, net_region(ctx, 1), ctx->netcoef, D, ctx->r, ctx->z, nullptr, s);
    // network direction f of r1 and A f
    launch_net_scale(net_region(ctx, 1), coarse_blocks(g), ctx->sc, u->dscal, s);
    launch_net_pack<float>(g, u->L[0], R1, ctx->dinv32, u->dscal, u->x, nullptr, s);
    rc = net_forward(u, s, nullptr);
    if (rc) return rc;
    launch_net_unpack(g, ctx->tiles, u->L[0], u->y32, ctx->dinv32, u->dscal, nullptr, nullptr,
                      NV, nullptr, nullptr, s);
    const RedArgs j2{ctx->sc, nullptr, 0, net_region(ctx, 3), 0, 0, nullptr, 0, nullptr};
    launch_apply<float>(g, ctx->tiles, MODE_JDIR, true, nullptr, NV, ctx->dinv32, nullptr, nullptr,
                        QN, ctx->a32, ctx->c32, ctx->K32, nullptr, j2, s);
    // loss on (r1, e1) and its gradient back through the network
    const int nb = train_dot_blocks(g);
    launch_train_dots(g, NV, QN, ctx->r, ctx->z, u->dpart, nb, s);
    launch_train_grad(g, u->L[0], u->dpart, nb, QN, ctx->r, ctx->dinv32, u->dscal, u->gy,
                      u->dscal + 1, s);
    rc = net_backward(u, s, 1.0f);
    if (rc) return rc;
    UCHK(hipMemcpyAsync(u->hscal, u->dscal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    UCHK(hipStreamSynchronize(s));
    if (loss) *loss = u->hscal[1];
    return VFS_OK;
}

int vfs_set_preconditioner(vfs_ctx* ctx, vfs_unet* u) {
    if (!ctx) return VFS_EINVAL;
    if (u && ctx->g.dim != 3)
        return ctx_fail(ctx, VFS_EINVAL, "the learned preconditioner is 3D only");
    if (u) {
        int rc = net_bufs(ctx);
        if (rc) return rc;
    }
    ctx->net = u;
    return VFS_OK;
}

int vfs_load_preconditioner(vfs_ctx* ctx, const void* weights, size_t bytes) {
    if (!ctx) return VFS_EINVAL;
    if (!weights) return ctx_fail(ctx, VFS_EINVAL, "weights pointer is NULL");
    if (ctx->g.dim != 3) return ctx_fail(ctx, VFS_EINVAL, "the learned preconditioner is 3D only");
    if (bytes != (size_t)vfs_unet_param_count() * sizeof(float))
        return ctx_fail(ctx, VFS_EINVAL, "weight bytes do not match the network's FP32 weights");
    if (!ctx->net_owned) {
        vfs_unet* u = nullptr;
        int rc = vfs_unet_create(&u);
        if (rc) return ctx_fail(ctx, rc, std::string("network: ") + vfs_unet_last_error(nullptr));
        ctx->net_owned = u;
    }
    vfs_unet* u = ctx->net_owned;
    u->stream = ctx->stream;
    int rc = vfs_unet_set_weights(u, (const float*)weights, vfs_unet_param_count());
    if (rc) return ctx_fail(ctx, rc, std::string("network: ") + u->err);
    return vfs_set_preconditioner(ctx, u);
}

int vfs_precond_apply(vfs_ctx* ctx, const double* r, double* z) {
    if (!ctx) return VFS_EINVAL;
    if (!r || !z) return ctx_fail(ctx, VFS_EINVAL, "NULL vector");
    if (ctx->precond == VFS_PRECOND_IC || ctx->precond == VFS_PRECOND_SCHWARZ) {
        if (!ctx->assembled) return ctx_fail(ctx, VFS_ESTATE, "call vfs_assemble first");
        const Geo& g = ctx->g;
        const long long n = (long long)g.nsamp() * g.NP;
        int rc = ctx_put_samples(ctx, r, ctx->q);
        if (rc) return rc;
        launch_mask(ctx->r, ctx->q, ctx->a, n, ctx->stream);
        launch_schwarz(g, ctx->precond == VFS_PRECOND_SCHWARZ ? 1 : 0, ctx->r, ctx->a, ctx->c,
                       ctx->dinv, ctx->K, ctx->rowbits, ctx->z, nullptr, ctx->stream);
        if (hipGetLastError() != hipSuccess) return ctx_fail(ctx, VFS_EHIP, "launch failed");
        return ctx_get_samples(ctx, ctx->z, z);
    }
    vfs_unet* u = ctx->net;
    if (!u) return ctx_fail(ctx, VFS_ESTATE, "no preconditioner network attached");
    int rc = ctx_ready(u, ctx);
    if (rc) return ctx_fail(ctx, rc, u->err);
    const Geo& g = ctx->g;
    hipStream_t s = ctx->stream;
    const long long n = (long long)g.nsamp() * g.NP;
    if ((rc = ctx_f32(ctx))) return rc;
    if ((rc = net_prepare_ctx(u, ctx))) return ctx_fail(ctx, rc, u->err);
    if ((rc = ctx_put_samples(ctx, r, ctx->z))) return rc;
    launch_mask(ctx->r, ctx->z, ctx->a, n, s);
    launch_to_f32(ctx->r, ctx->r32, n, s);
    launch_net_rdr(g, ctx->r32, ctx->dinv32, u->dpart, s);
    FcgHist none{};
    rc = net_precond(u, ctx, ctx->r32, ctx->dinv32, ctx->a32, ctx->c32, ctx->K32, u->dpart,
                     net_rdr_blocks(g), none, nullptr);
    if (rc) return ctx_fail(ctx, rc, u->err);
    launch_f32_to_f64(ctx->z32, ctx->z, n, s);
    if (hipGetLastError() != hipSuccess) return ctx_fail(ctx, VFS_EHIP, "launch failed");
    return ctx_get_samples(ctx, ctx->z, z);
}

}  // extern "C"
