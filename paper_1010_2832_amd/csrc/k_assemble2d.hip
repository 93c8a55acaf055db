// 2D assembly of the SPD stress/pressure system (paper eq.
// stokesmixedsystemspd in the factored form of Section 7), null-space
// elimination (Section 8), moving-solid right-hand side (Section 6.2) and
// velocity recovery from the velocity row of eq. stokesmixedsystem.
//
// Samples (Section 5, Fig. 1): p and tau_xx at cells, tau_xy at nodes; u, v
// on faces.  With reduced stresses (tau_yy = -tau_xx) the face operator is
//   (B x)_u(i,j) = [P(i,j)-P(i-1,j) + X(i-1,j)-X(i,j) + Y(i,j)-Y(i,j+1)] / h
//   (B x)_v(i,j) = [P(i,j)-P(i,j-1) + X(i,j)-X(i,j-1) + Y(i,j)-Y(i+1,j)] / h
// with P = W_Lp p, X = W_Lt tau_xx, Y = W_Lt tau_xy (the G and D^T of the
// paper), and A = dt B^T K B + Dg with K = W_F / (rho W_L) on faces and
// Dg = W_F W_L / mu on stresses.
#include "vfs_internal.h"

namespace vfs {
namespace {

enum : uint8_t { FK = 1, FBAD = 2, FINV = 4 };

__device__ __forceinline__ double rho_face(const double* rho, long long o_lo, long long o_hi,
                                           bool lo_in, bool hi_in) {
    if (lo_in && hi_in) return (rho[o_lo] + rho[o_hi]) * 0.5;
    return lo_in ? rho[o_lo] : rho[o_hi];
}

// One thread per anchor (i,j): u face (i,j) and v face (i,j).
__global__ void k_face2d(Geo g, double dt, double g0, double g1, const double* __restrict__ WL,
                         double* __restrict__ WF, const double* __restrict__ rho,
                         const double* __restrict__ u, double* __restrict__ ustar,
                         double* __restrict__ rhof, double* __restrict__ K,
                         uint8_t* __restrict__ fflag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nx || j > g.ny) return;
    const long long NP = g.NP;
    const long long o = g.idx(i, j);
    const double sK = dt / (g.h * g.h);
    const double* WFc = WF;            // cells (set 0)
    const double* WFn = WF + 3 * NP;   // nodes (set 3)
    if (j < g.ny) {  // u face: cells (i-1,j),(i,j); nodes (i,j),(i,j+1)
        const double wl = WL[NP + o];
        const double wf = WF[NP + o];
        bool inval = false;
        if (wf > 0.0)
            inval = WFc[g.idx(i - 1, j)] == 0.0 || WFc[o] == 0.0 || WFn[o] == 0.0 ||
                    WFn[g.idx(i, j + 1)] == 0.0;
        const double wfe = inval ? 0.0 : wf;
        const bool kp = wfe > 0.0 && wl > 0.0;
        const bool bad = wfe > 0.0 && wl == 0.0;
        const double r = rho_face(rho, g.idx(i - 1, j), o, i > 0, i < g.nx);
        WF[NP + o] = wfe;
        rhof[o] = r;
        K[o] = kp ? sK * (wfe / (r * wl)) : 0.0;
        fflag[o] = (uint8_t)((kp ? FK : 0) | (bad ? FBAD : 0) | (inval ? FINV : 0));
        ustar[o] = u[o] + dt * g0;
    }
    if (i < g.nx) {  // v face: cells (i,j-1),(i,j); nodes (i,j),(i+1,j)
        const double wl = WL[2 * NP + o];
        const double wf = WF[2 * NP + o];
        bool inval = false;
        if (wf > 0.0)
            inval = WFc[g.idx(i, j - 1)] == 0.0 || WFc[o] == 0.0 || WFn[o] == 0.0 ||
                    WFn[g.idx(i + 1, j)] == 0.0;
        const double wfe = inval ? 0.0 : wf;
        const bool kp = wfe > 0.0 && wl > 0.0;
        const bool bad = wfe > 0.0 && wl == 0.0;
        const double r = rho_face(rho, g.idx(i, j - 1), o, j > 0, j < g.ny);
        WF[2 * NP + o] = wfe;
        rhof[NP + o] = r;
        K[NP + o] = kp ? sK * (wfe / (r * wl)) : 0.0;
        fflag[NP + o] = (uint8_t)((kp ? FK : 0) | (bad ? FBAD : 0) | (inval ? FINV : 0));
        ustar[NP + o] = u[NP + o] + dt * g1;
    }
}

// One thread per anchor: cell (p, tau_xx) and node (tau_xy) coefficients,
// classification, Jacobi diagonal and right-hand side.
__global__ void k_sample2d(Geo g, const double* __restrict__ WL, const double* __restrict__ WF,
                           const double* __restrict__ mu, const double* __restrict__ K,
                           const uint8_t* __restrict__ fflag, const double* __restrict__ ustar,
                           const double* __restrict__ ubc, double* __restrict__ a,
                           double* __restrict__ c, double* __restrict__ dinv,
                           double* __restrict__ b, Scalars* sc) {
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    const int i = blockIdx.x * 64 + tx;
    const int j = blockIdx.y * 4 + ty;
    const long long NP = g.NP;
    const double ih = 1.0 / g.h;
    int nact = 0;
    if (i <= g.nx && j <= g.ny) {
        const long long o = g.idx(i, j);
        const double* Ku = K;
        const double* Kv = K + NP;
        const uint8_t* Fu = fflag;
        const uint8_t* Fv = fflag + NP;
        const double* Su = ustar;
        const double* Sv = ustar + NP;
        const double* Bu = ubc;
        const double* Bv = ubc + NP;
        const double* Wu = WF + NP;
        const double* Wv = WF + 2 * NP;
        // ---------------- cell: p and tau_xx share the stencil u(i),u(i+1),v(j),v(j+1)
        double ap = 0.0, cx = 0.0, dp = 0.0, dx = 0.0, bp = 0.0, bx = 0.0;
        if (i < g.nx && j < g.ny) {
            const long long ou1 = g.idx(i + 1, j), ov1 = g.idx(i, j + 1);
            const uint8_t f0 = Fu[o], f1 = Fu[ou1], f2 = Fv[o], f3 = Fv[ov1];
            const bool tb = ((f0 | f1 | f2 | f3) & FBAD) != 0;
            const bool tk = ((f0 | f1 | f2 | f3) & FK) != 0;
            const double wl = WL[o], wf = WF[o];
            const bool act = wl > 0.0 && !tb && tk;
            if (act) {
                ap = wl;
                cx = wf * wl / mu[o];
                const double sumK = (Ku[o] + Ku[ou1]) + (Kv[o] + Kv[ov1]);
                dp = 1.0 / (ap * ap * sumK);
                dx = 1.0 / (cx + ap * ap * sumK);
                // y = W_F u* + W_S u_BC on the four faces; W_S = 1 - W_F
                const double yu0 = Wu[o] * Su[o] + (1.0 - Wu[o]) * Bu[o];
                const double yu1 = Wu[ou1] * Su[ou1] + (1.0 - Wu[ou1]) * Bu[ou1];
                const double yv0 = Wv[o] * Sv[o] + (1.0 - Wv[o]) * Bv[o];
                const double yv1 = Wv[ov1] * Sv[ov1] + (1.0 - Wv[ov1]) * Bv[ov1];
                const double ws = 1.0 - wf;
                const double gt_y = (yu0 - yu1 + yv0 - yv1) * ih;          // G^T y
                const double gt_b = (Bu[o] - Bu[ou1] + Bv[o] - Bv[ov1]) * ih;
                const double dxx_y = (yu1 - yu0 - yv1 + yv0) * ih;         // D_xx y
                const double dxx_b = (Bu[ou1] - Bu[o] - Bv[ov1] + Bv[o]) * ih;
                bp = ap * (gt_y - ws * gt_b);
                bx = ap * (dxx_y - ws * dxx_b);
                nact += 2;
            }
        }
        a[o] = ap;
        a[NP + o] = ap;
        c[o] = 0.0;
        c[NP + o] = cx;
        dinv[o] = dp;
        dinv[NP + o] = dx;
        b[o] = bp;
        b[NP + o] = bx;
        // ---------------- node: tau_xy, stencil u(i,j-1), u(i,j), v(i-1,j), v(i,j)
        double ay = 0.0, cy = 0.0, dy = 0.0, by = 0.0;
        {
            const long long oum = g.idx(i, j - 1), ovm = g.idx(i - 1, j);
            const uint8_t f0 = Fu[oum], f1 = Fu[o], f2 = Fv[ovm], f3 = Fv[o];
            const bool tb = ((f0 | f1 | f2 | f3) & FBAD) != 0;
            const bool tk = ((f0 | f1 | f2 | f3) & FK) != 0;
            const double wl = WL[3 * NP + o], wf = WF[3 * NP + o];
            const bool act = wl > 0.0 && !tb && tk;
            if (act) {
                // viscosity: mean of the in-box cells sharing the node
                double ms = 0.0;
                int mc = 0;
                if (i > 0 && j > 0) { ms += mu[g.idx(i - 1, j - 1)]; ++mc; }
                if (i > 0 && j < g.ny) { ms += mu[g.idx(i - 1, j)]; ++mc; }
                if (i < g.nx && j > 0) { ms += mu[g.idx(i, j - 1)]; ++mc; }
                if (i < g.nx && j < g.ny) { ms += mu[o]; ++mc; }
                const double mun = ms / (double)mc;
                ay = wl;
                cy = wf * wl / mun;
                const double sumK = (Ku[oum] + Ku[o]) + (Kv[ovm] + Kv[o]);
                dy = 1.0 / (cy + ay * ay * sumK);
                const double yum = Wu[oum] * Su[oum] + (1.0 - Wu[oum]) * Bu[oum];
                const double yu0 = Wu[o] * Su[o] + (1.0 - Wu[o]) * Bu[o];
                const double yvm = Wv[ovm] * Sv[ovm] + (1.0 - Wv[ovm]) * Bv[ovm];
                const double yv0 = Wv[o] * Sv[o] + (1.0 - Wv[o]) * Bv[o];
                const double dxy_y = (yu0 - yum + yv0 - yvm) * ih;
                const double dxy_b = (Bu[o] - Bu[oum] + Bv[o] - Bv[ovm]) * ih;
                by = ay * (dxy_y - (1.0 - wf) * dxy_b);
                nact += 1;
            }
        }
        a[2 * NP + o] = ay;
        c[2 * NP + o] = cy;
        dinv[2 * NP + o] = dy;
        b[2 * NP + o] = by;
    }
    // count active samples (integer atomics: order independent)
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    if (nact) atomicAdd(&s_cnt, nact);
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt)
        atomicAdd((unsigned long long*)&sc->n_active, (unsigned long long)s_cnt);
}

// Velocity recovery: u = u* - dt (B x) / (rho W_L) where K > 0; u_BC where
// W_F = 0 (solid, box or invalid face); 0 elsewhere (air).
__global__ void k_velocity2d(Geo g, double dt, const double* __restrict__ x,
                             const double* __restrict__ a, const double* __restrict__ ustar,
                             const double* __restrict__ ubc, const double* __restrict__ rhof,
                             const double* __restrict__ WL, const double* __restrict__ WF,
                             const uint8_t* __restrict__ fflag, double* __restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nx || j > g.ny) return;
    const long long NP = g.NP;
    const long long o = g.idx(i, j);
    const double* P = x;
    const double* X = x + NP;
    const double* Y = x + 2 * NP;
    const double* aP = a;
    const double* aX = a + NP;
    const double* aY = a + 2 * NP;
    const double s = dt / g.h;
    if (j < g.ny) {
        const long long om = g.idx(i - 1, j), oy = g.idx(i, j + 1);
        double val;
        if (fflag[o] & FK) {
            const double d = (aP[o] * P[o] - aP[om] * P[om]) + (aX[om] * X[om] - aX[o] * X[o]) +
                             (aY[o] * Y[o] - aY[oy] * Y[oy]);
            val = ustar[o] - s * d / (rhof[o] * WL[NP + o]);
        } else {
            val = WF[NP + o] == 0.0 ? ubc[o] : 0.0;
        }
        u[o] = val;
    }
    if (i < g.nx) {
        const long long om = g.idx(i, j - 1), ox = g.idx(i + 1, j);
        double val;
        if (fflag[NP + o] & FK) {
            const double d = (aP[o] * P[o] - aP[om] * P[om]) + (aX[o] * X[o] - aX[om] * X[om]) +
                             (aY[o] * Y[o] - aY[ox] * Y[ox]);
            val = ustar[NP + o] - s * d / (rhof[NP + o] * WL[2 * NP + o]);
        } else {
            val = WF[2 * NP + o] == 0.0 ? ubc[NP + o] : 0.0;
        }
        u[NP + o] = val;
    }
}

// Prescribed traction (Section 6.1): with boundary values y = (p_BC, tau_BC)
// per sample, the air-region boundary work and the boundary values of the
// eliminated samples add f = B0 (a y) - W_L (B0 y) to the velocity rows; on a
// face with K > 0 eliminating the velocity folds it into the input velocity,
// u* += dt f / (rho W_L).  B0's stencils are those of k_velocity2d.
__global__ void k_traction2d(Geo g, double dt, const double* __restrict__ y,
                             const double* __restrict__ a, const double* __restrict__ rhof,
                             const double* __restrict__ WL, const uint8_t* __restrict__ fflag,
                             double* __restrict__ ustar) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nx || j > g.ny) return;
    const long long NP = g.NP;
    const long long o = g.idx(i, j);
    const double *P = y, *X = y + NP, *Y = y + 2 * NP;
    const double *aP = a, *aX = a + NP, *aY = a + 2 * NP;
    const double s = dt / g.h;
    if (j < g.ny && (fflag[o] & FK)) {
        const long long om = g.idx(i - 1, j), oy = g.idx(i, j + 1);
        const double day = (aP[o] * P[o] - aP[om] * P[om]) + (aX[om] * X[om] - aX[o] * X[o]) +
                           (aY[o] * Y[o] - aY[oy] * Y[oy]);
        const double dy = (P[o] - P[om]) + (X[om] - X[o]) + (Y[o] - Y[oy]);
        const double wl = WL[NP + o];
        ustar[o] += s * (day - wl * dy) / (rhof[o] * wl);
    }
    if (i < g.nx && (fflag[NP + o] & FK)) {
        const long long om = g.idx(i, j - 1), ox = g.idx(i + 1, j);
        const double day = (aP[o] * P[o] - aP[om] * P[om]) + (aX[o] * X[o] - aX[om] * X[om]) +
                           (aY[o] * Y[o] - aY[ox] * Y[ox]);
        const double dy = (P[o] - P[om]) + (X[o] - X[om]) + (Y[o] - Y[ox]);
        const double wl = WL[2 * NP + o];
        ustar[NP + o] += s * (day - wl * dy) / (rhof[NP + o] * wl);
    }
}

}  // namespace

void launch_traction2d(const Geo& g, double dt, const double* y, const double* a,
                       const double* rhof, const double* WL, const uint8_t* fflag, double* ustar,
                       hipStream_t s) {
    dim3 bs(64, 4);
    dim3 gs((g.nx + 1 + 63) / 64, (g.ny + 1 + 3) / 4);
    hipLaunchKernelGGL(k_traction2d, gs, bs, 0, s, g, dt, y, a, rhof, WL, fflag, ustar);
}

void launch_face_coef2d(const Geo& g, double dt, const double* g3, const double* WL, double* WF,
                        const double* rho, const double* u, double* ustar, double* rhof,
                        double* K, uint8_t* fflag, hipStream_t s) {
    dim3 bs(64, 4);
    dim3 gs((g.nx + 1 + 63) / 64, (g.ny + 1 + 3) / 4);
    hipLaunchKernelGGL(k_face2d, gs, bs, 0, s, g, dt, g3[0], g3[1], WL, WF, rho, u, ustar, rhof, K,
                       fflag);
}

void launch_sample_coef2d(const Geo& g, const double* WL, const double* WF, const double* mu,
                          const double* K, const uint8_t* fflag, const double* ustar,
                          const double* ubc, double* a, double* c, double* dinv, double* b,
                          Scalars* sc, hipStream_t s) {
    dim3 gs((g.nx + 1 + 63) / 64, (g.ny + 1 + 3) / 4);
    hipLaunchKernelGGL(k_sample2d, gs, dim3(256), 0, s, g, WL, WF, mu, K, fflag, ustar, ubc, a, c,
                       dinv, b, sc);
}

void launch_velocity2d(const Geo& g, double dt, const double* x, const double* a,
                       const double* ustar, const double* ubc, const double* rhof,
                       const double* WL, const double* WF, const uint8_t* fflag, double* u,
                       hipStream_t s) {
    dim3 bs(64, 4);
    dim3 gs((g.nx + 1 + 63) / 64, (g.ny + 1 + 3) / 4);
    hipLaunchKernelGGL(k_velocity2d, gs, bs, 0, s, g, dt, x, a, ustar, ubc, rhof, WL, WF, fflag, u);
}

}  // namespace vfs
