// Preconditioned conjugate gradients on A = dt B^T K B + Dg (paper eq.
// stokesmixedsystemspd; the factored form of Section 8 is what makes the
// matrix-free apply two sparse passes: faces g = K (B x), then samples
// y = B^T g + Dg x).
//
// One CG iteration k is two kernels:
//   apply  (MODE_DIR): sum the r.z and r.r partials of the previous kernel,
//          decide convergence (every workgroup decides identically), beta =
//          r_k.z_k / r_{k-1}.z_{k-1}; p = z + beta p_old (z = D^-1 r on the
//          fly for Jacobi, or read for a stored preconditioner output),
//          q = A p, partials of p.q.
//   update: sum the p.q partials, alpha = r.z / p.q; x += alpha p,
//          r -= alpha q, z = D^-1 r, partials of r.z and r.r.
// The 2D apply is one fused LDS-tiled stencil: a 64x4 tile stages the
// weighted samples of its (66x6) halo in LDS, forms the face values g on the
// (65x5) faces it needs, then the sample outputs.  All reductions are FP64
// and deterministic (see vfs_reduce.h).
#include "vfs_internal.h"
#include "vfs_reduce.h"

namespace vfs {
namespace {

constexpr int BX = 64;
constexpr int BY = 4;
constexpr int NT = 256;

// ---------------------------------------------------------------------------
// 2D fused apply.  Sample slices: 0 p (cell), 1 tau_xx (cell), 2 tau_xy (node);
// face slices: 0 u, 1 v.  K already carries dt/h^2.
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool ZIN>
__global__ __launch_bounds__(NT) void k_apply2d(Geo g, const T* __restrict__ r,
                                                const T* __restrict__ zs,
                                                const T* __restrict__ dinv,
                                                const T* __restrict__ pin, T* __restrict__ pout,
                                                T* __restrict__ q, const T* __restrict__ a,
                                                const T* __restrict__ c, const T* __restrict__ K,
                                                const T* __restrict__ bv, RedArgs ra) {
    const int bid = blockIdx.x + gridDim.x * blockIdx.y;
    T beta = T(0);
    bool first = true;
    if (MODE == MODE_DIR) {
        if (ra.sc->done) return;
        double bd;
        if (!cg_direction_preamble<NT>(ra, bid, bd)) return;
        first = ra.kidx == 0;
        beta = (T)bd;
    }
    __shared__ T sW[3][BY + 2][BX + 2];
    __shared__ T sV[3][BY + 2][BX + 2];
    __shared__ T sG[2][BY + 1][BX + 1];
    const long long NP = g.NP;
    const int i0 = blockIdx.x * BX, j0 = blockIdx.y * BY;
    const int tid = threadIdx.x;

    // stage 1: direction (or input) values and weighted values on the halo
    for (int e = tid; e < (BX + 2) * (BY + 2); e += NT) {
        const int li = e % (BX + 2), lj = e / (BX + 2);
        const int i = i0 - 1 + li, j = j0 - 1 + lj;
        T v[3] = {T(0), T(0), T(0)};
        T w[3] = {T(0), T(0), T(0)};
        if (i <= g.nx + 1 && j <= g.ny + 1) {
            const long long o = g.idx(i, j);
            const bool own = li >= 1 && li <= BX && lj >= 1 && lj <= BY && i <= g.nx && j <= g.ny;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const long long os = o + s * NP;
                T val;
                if (MODE == MODE_DIR) {
                    const T z = ZIN ? zs[os] : dinv[os] * r[os];
                    val = first ? z : z + beta * pin[os];
                    if (own) pout[os] = val;
                } else {
                    val = pin[os];
                }
                v[s] = val;
                w[s] = a[os] * val;
            }
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            sV[s][lj][li] = v[s];
            sW[s][lj][li] = w[s];
        }
    }
    __syncthreads();

    // stage 2: g = K (B x) on u faces (i0..i0+BX, j0-1..j0+BY-1) and
    //          v faces (i0-1..i0+BX-1, j0..j0+BY)
    for (int e = tid; e < (BX + 1) * (BY + 1); e += NT) {
        const int li = e % (BX + 1), lj = e / (BX + 1);
        {
            const int i = i0 + li, j = j0 - 1 + lj;
            T gv = T(0);
            if (i <= g.nx && j >= 0 && j < g.ny) {
                const T k = K[g.idx(i, j)];
                gv = k * ((sW[0][lj][li + 1] - sW[0][lj][li]) + (sW[1][lj][li] - sW[1][lj][li + 1]) +
                          (sW[2][lj][li + 1] - sW[2][lj + 1][li + 1]));
            }
            sG[0][lj][li] = gv;
        }
        {
            const int i = i0 - 1 + li, j = j0 + lj;
            T gv = T(0);
            if (i >= 0 && i < g.nx && j <= g.ny) {
                const T k = K[NP + g.idx(i, j)];
                gv = k * ((sW[0][lj + 1][li] - sW[0][lj][li]) + (sW[1][lj + 1][li] - sW[1][lj][li]) +
                          (sW[2][lj + 1][li] - sW[2][lj + 1][li + 1]));
            }
            sG[1][lj][li] = gv;
        }
    }
    __syncthreads();

    // stage 3: y = B^T g + Dg x at the tile's anchors
    const int tx = tid % BX, ty = tid / BX;
    const int i = i0 + tx, j = j0 + ty;
    double acc = 0.0;
    if (i <= g.nx && j <= g.ny) {
        const long long o = g.idx(i, j);
        const T gu0 = sG[0][ty + 1][tx], gu1 = sG[0][ty + 1][tx + 1], gum = sG[0][ty][tx];
        const T gv0 = sG[1][ty][tx + 1], gv1 = sG[1][ty + 1][tx + 1], gvm = sG[1][ty][tx];
        const T v0 = sV[0][ty + 1][tx + 1], v1 = sV[1][ty + 1][tx + 1], v2 = sV[2][ty + 1][tx + 1];
        const T y0 = a[o] * ((gu0 - gu1) + (gv0 - gv1));
        const T y1 = a[NP + o] * ((gu1 - gu0) + (gv0 - gv1)) + c[NP + o] * v1;
        const T y2 = a[2 * NP + o] * ((gu0 - gum) + (gv0 - gvm)) + c[2 * NP + o] * v2;
        if (MODE == MODE_RESID) {
            const T r0 = bv[o] - y0, r1 = bv[NP + o] - y1, r2 = bv[2 * NP + o] - y2;
            q[o] = r0;
            q[NP + o] = r1;
            q[2 * NP + o] = r2;
            acc = (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2;
        } else {
            q[o] = y0;
            q[NP + o] = y1;
            q[2 * NP + o] = y2;
            if (MODE == MODE_DIR) acc = (double)v0 * y0 + (double)v1 * y1 + (double)v2 * y2;
        }
    }
    if (MODE == MODE_APPLY) return;
    double vv[1] = {acc};
    block_partial<1, NT>(vv, ra.part_out, gridDim.x * gridDim.y, bid);
}

// ---------------------------------------------------------------------------
// pointwise kernels over whole padded vectors (n = nsamp * NP elements)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_update(long long n, T* __restrict__ x,
                                               const T* __restrict__ p, T* __restrict__ r,
                                               const T* __restrict__ q,
                                               const T* __restrict__ dinv, T* __restrict__ z,
                                               RedArgs ra) {
    Scalars* sc = ra.sc;
    if (sc->done) return;
    double tot[1];
    reduce_partials<1, NT>(ra.part_in, ra.nb_in, tot);
    const double pq = tot[0];
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->done = 3;
            sc->iter = ra.kidx;
        }
        return;
    }
    const double alpha_d = sc->rz[ra.kidx & 1] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = alpha_d;
    }
    const T alpha = (T)alpha_d;
    double rz = 0.0, rr = 0.0;
    const long long stride = (long long)gridDim.x * NT;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < n; t += stride) {
        const T ri = r[t] - alpha * q[t];
        const T zi = dinv[t] * ri;
        x[t] = x[t] + alpha * p[t];
        r[t] = ri;
        if (z) z[t] = zi;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    double vv[2] = {rz, rr};
    block_partial<2, NT>(vv, ra.part_out, gridDim.x, blockIdx.x);
}

// x = 0, r = b (b may alias r), z = D^-1 r; partials of r.z and r.r; resets
// the flags of a new solve.
template <typename T>
__global__ __launch_bounds__(NT) void k_cg_init(long long n, const T* bsrc, T* __restrict__ x,
                                                T* r, const T* __restrict__ dinv,
                                                T* __restrict__ z, double tol, int max_iter,
                                                Scalars* sc, double* part_out) {
    double rz = 0.0, rr = 0.0;
    const long long stride = (long long)gridDim.x * NT;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < n; t += stride) {
        const T bi = bsrc[t];
        const T zi = dinv[t] * bi;
        r[t] = bi;
        x[t] = T(0);
        if (z) z[t] = zi;
        rz += (double)bi * (double)zi;
        rr += (double)bi * (double)bi;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = 0;
        sc->iter = 0;
        sc->tol2 = tol * tol;
        sc->max_iter = max_iter;
        sc->alpha = sc->beta = sc->pq = 0.0;
    }
    double vv[2] = {rz, rr};
    block_partial<2, NT>(vv, part_out, gridDim.x, blockIdx.x);
}

// Restart on the current r (after residual replacement): partials of r.z
// and r.r; a new run of iterations follows (bb is kept).
template <typename T>
__global__ __launch_bounds__(NT) void k_cg_restart(long long n, const T* __restrict__ r,
                                                   const T* __restrict__ dinv,
                                                   T* __restrict__ z, Scalars* sc,
                                                   double* part_out, int max_iter) {
    double rz = 0.0, rr = 0.0;
    const long long stride = (long long)gridDim.x * NT;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < n; t += stride) {
        const T ri = r[t];
        const T zi = dinv[t] * ri;
        if (z) z[t] = zi;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = 0;
        sc->iter = 0;
        sc->max_iter = max_iter;
    }
    double vv[2] = {rz, rr};
    block_partial<2, NT>(vv, part_out, gridDim.x, blockIdx.x);
}

__global__ __launch_bounds__(NT) void k_norm2(long long n, const double* __restrict__ v,
                                              double* part_out) {
    double s = 0.0;
    const long long stride = (long long)gridDim.x * NT;
    for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < n; t += stride)
        s += v[t] * v[t];
    double vv[1] = {s};
    block_partial<1, NT>(vv, part_out, gridDim.x, blockIdx.x);
}

__global__ __launch_bounds__(NT) void k_finalize1(const double* __restrict__ part, int nb,
                                                  Scalars* sc, int slot) {
    double tot[1];
    reduce_partials<1, NT>(part, nb, tot);
    if (threadIdx.x == 0) {
        if (slot == 0)
            sc->aux0 = tot[0];
        else
            sc->aux1 = tot[0];
    }
}

// r32 = r64 / sqrt(aux0) (scaled residual for the FP32 inner solve)
__global__ void k_scale_to_f32(long long n, const double* __restrict__ r64,
                               float* __restrict__ r32, const Scalars* sc) {
    const double s = sc->aux0 > 0.0 ? 1.0 / sqrt(sc->aux0) : 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        r32[t] = (float)(r64[t] * s);
}

// x64 += sqrt(aux0) * d32
__global__ void k_axpy_f32_to_f64(long long n, double* __restrict__ x64,
                                  const float* __restrict__ d32, const Scalars* sc) {
    const double s = sqrt(sc->aux0);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        x64[t] += s * (double)d32[t];
}

}  // namespace

int apply_grid_blocks(const Geo& g) {
    if (g.dim == 2) return ((g.nx + 1 + BX - 1) / BX) * ((g.ny + 1 + BY - 1) / BY);
    int ntx, nty, ntz;
    tile_dims(g, ntx, nty, ntz);
    return ntx * nty * ntz;
}

int vec_grid_blocks(const Geo& g) {
    const long long n = (long long)g.nsamp() * g.NP;
    long long nb = (n + NT * 4 - 1) / (NT * 4);
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    return (int)nb;
}

int apply_blocks(const Geo& g, const Tiles& tl) {
    return g.dim == 2 ? apply_grid_blocks(g) : tl.count;
}

int update_blocks(const Geo& g, const Tiles& tl) {
    return g.dim == 2 ? vec_grid_blocks(g) : tl.count;
}

template <typename T>
void launch_apply(const Geo& g, const Tiles& tl, int mode, bool zin, const T* r, const T* zsrc,
                  const T* dinv, const T* pin, T* pout, T* q, const T* a, const T* c, const T* K,
                  const T* bvec, const RedArgs& ra, hipStream_t s) {
    if (g.dim == 3) {
        launch_apply3d<T>(g, tl, mode, zin, r, zsrc, dinv, pin, pout, q, a, c, K, bvec, ra, s);
        return;
    }
    dim3 gs((g.nx + 1 + BX - 1) / BX, (g.ny + 1 + BY - 1) / BY);
    if (mode == MODE_DIR) {
        if (zin)
            hipLaunchKernelGGL((k_apply2d<T, MODE_DIR, true>), gs, dim3(NT), 0, s, g, r, zsrc, dinv,
                               pin, pout, q, a, c, K, bvec, ra);
        else
            hipLaunchKernelGGL((k_apply2d<T, MODE_DIR, false>), gs, dim3(NT), 0, s, g, r, zsrc,
                               dinv, pin, pout, q, a, c, K, bvec, ra);
    } else if (mode == MODE_APPLY) {
        hipLaunchKernelGGL((k_apply2d<T, MODE_APPLY, false>), gs, dim3(NT), 0, s, g, r, zsrc, dinv,
                           pin, pout, q, a, c, K, bvec, ra);
    } else {
        hipLaunchKernelGGL((k_apply2d<T, MODE_RESID, false>), gs, dim3(NT), 0, s, g, r, zsrc, dinv,
                           pin, pout, q, a, c, K, bvec, ra);
    }
}

template <typename T>
void launch_update(const Geo& g, const Tiles& tl, T* x, const T* p, T* r, const T* q,
                   const T* dinv, T* z, const RedArgs& ra, hipStream_t s) {
    if (g.dim == 3) {
        launch_update3d<T>(g, tl, x, p, r, q, dinv, z, ra, s);
        return;
    }
    const long long n = (long long)g.nsamp() * g.NP;
    hipLaunchKernelGGL((k_update<T>), dim3(vec_grid_blocks(g)), dim3(NT), 0, s, n, x, p, r, q, dinv,
                       z, ra);
}

template <typename T>
void launch_cg_init(const Geo& g, const T* bsrc, T* x, T* r, const T* dinv, T* z, double tol,
                    int max_iter, Scalars* sc, double* part_out, hipStream_t s) {
    const long long n = (long long)g.nsamp() * g.NP;
    hipLaunchKernelGGL((k_cg_init<T>), dim3(vec_grid_blocks(g)), dim3(NT), 0, s, n, bsrc, x, r,
                       dinv, z, tol, max_iter, sc, part_out);
}

template <typename T>
void launch_cg_restart(const Geo& g, const T* r, const T* dinv, T* z, Scalars* sc,
                       double* part_out, int max_iter, hipStream_t s) {
    const long long n = (long long)g.nsamp() * g.NP;
    hipLaunchKernelGGL((k_cg_restart<T>), dim3(vec_grid_blocks(g)), dim3(NT), 0, s, n, r, dinv, z,
                       sc, part_out, max_iter);
}

void launch_finalize(const double* part, int nb, int nv, Scalars* sc, int slot, hipStream_t s) {
    (void)nv;
    hipLaunchKernelGGL(k_finalize1, dim3(1), dim3(NT), 0, s, part, nb, sc, slot);
}

void launch_norm2(const Geo& g, const double* v, double* part_out, hipStream_t s) {
    const long long n = (long long)g.nsamp() * g.NP;
    hipLaunchKernelGGL(k_norm2, dim3(vec_grid_blocks(g)), dim3(NT), 0, s, n, v, part_out);
}

void launch_scale_to_f32(const Geo& g, const double* r64, float* r32, const Scalars* sc,
                         hipStream_t s) {
    const long long n = (long long)g.nsamp() * g.NP;
    hipLaunchKernelGGL(k_scale_to_f32, dim3(vec_grid_blocks(g)), dim3(NT), 0, s, n, r64, r32, sc);
}

void launch_axpy_f32_to_f64(const Geo& g, double* x64, const float* d32, const Scalars* sc,
                            hipStream_t s) {
    const long long n = (long long)g.nsamp() * g.NP;
    hipLaunchKernelGGL(k_axpy_f32_to_f64, dim3(vec_grid_blocks(g)), dim3(NT), 0, s, n, x64, d32,
                       sc);
}

#define VFS_INST(T)                                                                              \
    template void launch_apply<T>(const Geo&, const Tiles&, int, bool, const T*, const T*,       \
                                  const T*, const T*, T*, T*, const T*, const T*, const T*,      \
                                  const T*, const RedArgs&, hipStream_t);                        \
    template void launch_update<T>(const Geo&, const Tiles&, T*, const T*, T*, const T*,         \
                                   const T*, T*, const RedArgs&, hipStream_t);                   \
    template void launch_cg_init<T>(const Geo&, const T*, T*, T*, const T*, T*, double, int,      \
                                    Scalars*, double*, hipStream_t);                             \
    template void launch_cg_restart<T>(const Geo&, const T*, const T*, T*, Scalars*, double*,     \
                                       int, hipStream_t);
VFS_INST(double)
VFS_INST(float)

}  // namespace vfs
