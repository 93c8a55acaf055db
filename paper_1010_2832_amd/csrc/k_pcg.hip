// Preconditioned conjugate gradients on A = dt B^T K B + Dg (paper eq.
// stokesmixedsystemspd; the factored form of Section 7 is what makes the
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
// The 2D apply is one fused LDS-tiled stencil: a 64x8 tile stages the
// weighted samples of its (66x10) halo in LDS, forms the face values g on the
// (65x9) faces it needs, then the sample outputs (two rows per thread).  All reductions are FP64
// and deterministic (see vfs_reduce.h).
#include "vfs_internal.h"
#include "vfs_reduce.h"

#include <algorithm>

namespace vfs {
namespace {

constexpr int BX = 64;
constexpr int BY = 8;
constexpr int NT = 256;
constexpr int RPT = BY * BX / NT;   // anchor rows per thread in the output stage

// ---------------------------------------------------------------------------
// 2D fused apply.  Sample slices: 0 p (cell), 1 tau_xx (cell), 2 tau_xy (node);
// face slices: 0 u, 1 v.  K already carries dt/h^2.
// ---------------------------------------------------------------------------
// Latency structure: every global load that does not depend on the r.z /
// r.r totals (partials, halo values, K, a, c) is issued before the totals
// are formed, so one memory round trip covers the whole kernel.
template <typename T, int MODE, bool ZIN>
__global__ __launch_bounds__(NT) void k_apply2d(Geo g, const T* __restrict__ r,
                                                const T* __restrict__ zs,
                                                const T* __restrict__ dinv,
                                                const T* __restrict__ pin, T* __restrict__ pout,
                                                T* __restrict__ q, const T* __restrict__ a,
                                                const T* __restrict__ c, const T* __restrict__ K,
                                                const T* __restrict__ bv, RedArgs ra) {
    constexpr int NE1 = ((BX + 2) * (BY + 2) + NT - 1) / NT;   // halo elements per thread
    constexpr int NE2 = ((BX + 1) * (BY + 1) + NT - 1) / NT;   // faces per thread
    const int bid = blockIdx.x + gridDim.x * blockIdx.y;
    if (MODE == MODE_DIR && ra.sc->done) return;
    __shared__ T sW[3][BY + 2][BX + 2];
    __shared__ T sV[3][BY + 2][BX + 2];
    __shared__ T sG[2][BY + 1][BX + 1];
    const long long NP = g.NP;
    const int i0 = blockIdx.x * BX, j0 = blockIdx.y * BY;
    const int tid = threadIdx.x;

    // (1) partial sums of the previous kernel
    PartialLoads<2, NT, 4> pl;
    if (MODE == MODE_DIR) pl.load(ra.part_in, ra.nb_in);

    // (2) independent loads: halo raw values, face K, output a and c
    T Rr[NE1][3], Dd[NE1][3], Pp[NE1][3], Aa[NE1][3];
    bool in1[NE1], own1[NE1];
#pragma unroll
    for (int m = 0; m < NE1; ++m) {
        const int e = tid + m * NT;
        const int li = e % (BX + 2), lj = e / (BX + 2);
        const int i = i0 - 1 + li, j = j0 - 1 + lj;
        in1[m] = e < (BX + 2) * (BY + 2) && i <= g.nx + 1 && j <= g.ny + 1;
        own1[m] = in1[m] && li >= 1 && li <= BX && lj >= 1 && lj <= BY && i <= g.nx && j <= g.ny;
        const long long o = in1[m] ? g.idx(i, j) : 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const long long os = o + s * NP;
            Rr[m][s] = Dd[m][s] = Pp[m][s] = Aa[m][s] = T(0);
            if (in1[m]) {
                if (MODE == MODE_DIR) {
                    Rr[m][s] = ZIN ? zs[os] : r[os];
                    if (!ZIN) Dd[m][s] = dinv[os];
                }
                Pp[m][s] = pin[os];
                Aa[m][s] = a[os];
            }
        }
    }
    T Ku[NE2], Kv[NE2];
#pragma unroll
    for (int m = 0; m < NE2; ++m) {
        const int e = tid + m * NT;
        const int li = e % (BX + 1), lj = e / (BX + 1);
        Ku[m] = Kv[m] = T(0);
        if (e < (BX + 1) * (BY + 1)) {
            const int iu = i0 + li, ju = j0 - 1 + lj;
            if (iu <= g.nx && ju >= 0 && ju < g.ny) Ku[m] = K[g.idx(iu, ju)];
            const int iv = i0 - 1 + li, jv = j0 + lj;
            if (iv >= 0 && iv < g.nx && jv <= g.ny) Kv[m] = K[NP + g.idx(iv, jv)];
        }
    }
    const int tx = tid % BX;
    T Ao[RPT][3], Co[RPT][2], Bo[RPT][3];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int ty = tid / BX + rr * (NT / BX);
        const int i = i0 + tx, j = j0 + ty;
        const bool ok = i <= g.nx && j <= g.ny;
        const long long o = ok ? g.idx(i, j) : 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            Ao[rr][s] = ok ? a[o + s * NP] : T(0);
            Bo[rr][s] = (MODE == MODE_RESID && ok) ? bv[o + s * NP] : T(0);
        }
        Co[rr][0] = ok ? c[NP + o] : T(0);
        Co[rr][1] = ok ? c[2 * NP + o] : T(0);
    }

    // (3) totals -> beta
    T beta = T(0);
    bool first = true;
    if (MODE == MODE_DIR) {
        double tot[2];
        pl.finish(tot);
        double bd;
        if (!cg_direction_decide(ra, bid, tot[0], tot[1], bd)) return;
        first = ra.kidx == 0;
        beta = (T)bd;
    }

    // (4) stage 1: direction values and weighted values on the halo
#pragma unroll
    for (int m = 0; m < NE1; ++m) {
        const int e = tid + m * NT;
        if (e >= (BX + 2) * (BY + 2)) continue;
        const int li = e % (BX + 2), lj = e / (BX + 2);
        const int i = i0 - 1 + li, j = j0 - 1 + lj;
        const long long o = in1[m] ? g.idx(i, j) : 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            T val;
            if (MODE == MODE_DIR) {
                const T z = ZIN ? Rr[m][s] : Dd[m][s] * Rr[m][s];
                val = first ? z : z + beta * Pp[m][s];
                if (own1[m]) pout[o + s * NP] = val;
            } else {
                val = Pp[m][s];
            }
            sV[s][lj][li] = val;
            sW[s][lj][li] = Aa[m][s] * val;
        }
    }
    __syncthreads();

    // (5) stage 2: g = K (B x) on u faces (i0..i0+BX, j0-1..j0+BY-1) and
    //     v faces (i0-1..i0+BX-1, j0..j0+BY)
#pragma unroll
    for (int m = 0; m < NE2; ++m) {
        const int e = tid + m * NT;
        if (e >= (BX + 1) * (BY + 1)) continue;
        const int li = e % (BX + 1), lj = e / (BX + 1);
        sG[0][lj][li] = Ku[m] * ((sW[0][lj][li + 1] - sW[0][lj][li]) +
                                 (sW[1][lj][li] - sW[1][lj][li + 1]) +
                                 (sW[2][lj][li + 1] - sW[2][lj + 1][li + 1]));
        sG[1][lj][li] = Kv[m] * ((sW[0][lj + 1][li] - sW[0][lj][li]) +
                                 (sW[1][lj + 1][li] - sW[1][lj][li]) +
                                 (sW[2][lj + 1][li] - sW[2][lj + 1][li + 1]));
    }
    __syncthreads();

    // (6) stage 3: y = B^T g + Dg x at the tile's anchors (RPT rows per thread)
    double acc = 0.0;
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int ty = tid / BX + rr * (NT / BX);
        const int i = i0 + tx, j = j0 + ty;
        if (i <= g.nx && j <= g.ny) {
            const long long o = g.idx(i, j);
            const T gu0 = sG[0][ty + 1][tx], gu1 = sG[0][ty + 1][tx + 1], gum = sG[0][ty][tx];
            const T gv0 = sG[1][ty][tx + 1], gv1 = sG[1][ty + 1][tx + 1], gvm = sG[1][ty][tx];
            const T v0 = sV[0][ty + 1][tx + 1], v1 = sV[1][ty + 1][tx + 1], v2 = sV[2][ty + 1][tx + 1];
            const T y0 = Ao[rr][0] * ((gu0 - gu1) + (gv0 - gv1));
            const T y1 = Ao[rr][1] * ((gu1 - gu0) + (gv0 - gv1)) + Co[rr][0] * v1;
            const T y2 = Ao[rr][2] * ((gu0 - gum) + (gv0 - gvm)) + Co[rr][1] * v2;
            if (MODE == MODE_RESID) {
                const T r0 = Bo[rr][0] - y0, r1 = Bo[rr][1] - y1, r2 = Bo[rr][2] - y2;
                q[o] = r0;
                q[NP + o] = r1;
                q[2 * NP + o] = r2;
                acc += (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2;
            } else {
                q[o] = y0;
                q[NP + o] = y1;
                q[2 * NP + o] = y2;
                if (MODE == MODE_DIR) acc += (double)v0 * y0 + (double)v1 * y1 + (double)v2 * y2;
            }
        }
    }
    if (MODE == MODE_APPLY) return;
    double vv[1] = {acc};
    block_partial<1, NT>(vv, ra.part_out, gridDim.x * gridDim.y, bid);
}

// ---------------------------------------------------------------------------
// pointwise kernels over whole padded vectors (n = nsamp * NP elements)
// ---------------------------------------------------------------------------
// The first EPT elements of every thread are loaded before the p.q total is
// formed (latency hiding); the rest, if any, follow in a grid-stride loop.
template <typename T>
__global__ __launch_bounds__(NT) void k_update(long long n, T* __restrict__ x,
                                               const T* __restrict__ p, T* __restrict__ r,
                                               const T* __restrict__ q,
                                               const T* __restrict__ dinv, T* __restrict__ z,
                                               RedArgs ra) {
    constexpr int EPT = 8;
    Scalars* sc = ra.sc;
    if (sc->done) return;
    PartialLoads<1, NT, 6> pl;
    pl.load(ra.part_in, ra.nb_in);
    const long long base = (long long)blockIdx.x * NT * EPT + threadIdx.x;
    T X[EPT], P[EPT], R[EPT], Q[EPT], D[EPT];
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
        const long long t = base + (long long)m * NT;
        const bool ok = t < n;
        X[m] = ok ? x[t] : T(0);
        P[m] = ok ? p[t] : T(0);
        R[m] = ok ? r[t] : T(0);
        Q[m] = ok ? q[t] : T(0);
        D[m] = ok ? dinv[t] : T(0);
    }
    double tot[1];
    pl.finish(tot);
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
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
        const long long t = base + (long long)m * NT;
        if (t < n) {
            const T ri = R[m] - alpha * Q[m];
            const T zi = D[m] * ri;
            x[t] = X[m] + alpha * P[m];
            r[t] = ri;
            if (z) z[t] = zi;
            rz += (double)ri * (double)zi;
            rr += (double)ri * (double)ri;
        }
    }
    const long long stride = (long long)gridDim.x * NT * EPT;
    for (long long t0 = base + stride; t0 < n; t0 += stride) {
        for (int m = 0; m < EPT; ++m) {
            const long long t = t0 + (long long)m * NT;
            if (t >= n) break;
            const T ri = r[t] - alpha * q[t];
            const T zi = dinv[t] * ri;
            x[t] = x[t] + alpha * p[t];
            r[t] = ri;
            if (z) z[t] = zi;
            rz += (double)ri * (double)zi;
            rr += (double)ri * (double)ri;
        }
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
        sc->fallbacks = 0;
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
    long long nb = (n + NT * 8 - 1) / (NT * 8);
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    return (int)nb;
}

int apply_blocks(const Geo& g, const Tiles& tl, int word) {
    return g.dim == 2 ? apply_grid_blocks(g) : apply3d_grid(tl.items(), word);
}

int dir_apply_blocks(const Geo& g, const Tiles& tl, int word) {
    return g.dim == 2 ? apply_grid_blocks(g) : dir3d_grid(tl.items(), word);
}

int update_blocks(const Geo& g, const Tiles& tl) {
    return g.dim == 2 ? vec_grid_blocks(g) : std::min(update3d_tiles(tl).items(), kMaxTileBlocks);
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
    } else if (mode == MODE_RESID) {
        hipLaunchKernelGGL((k_apply2d<T, MODE_RESID, false>), gs, dim3(NT), 0, s, g, r, zsrc, dinv,
                           pin, pout, q, a, c, K, bvec, ra);
    }
    // MODE_FDIR exists in 3D only (the learned preconditioner is 3D); the
    // host never requests it for a 2D grid
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
