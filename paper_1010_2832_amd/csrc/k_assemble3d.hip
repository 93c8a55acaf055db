// 3D assembly of the SPD stress/pressure system (paper eq.
// stokesmixedsystemspd, factored form of Section 7), null-space elimination
// (Section 8), moving-solid right-hand side (Section 6.2) and velocity
// recovery from the velocity row of eq. stokesmixedsystem.
//
// Samples (Section 5, Fig. 2): p, tau_xx, tau_yy at cells (tau_zz =
// -tau_xx - tau_yy); tau_xy on z-edges, tau_xz on y-edges, tau_yz on
// x-edges; u, v, w on faces.  Reduced deformation rows:
//   D_xx = u_x - w_z, D_yy = v_y - w_z, D_xy = u_y + v_x, D_xz = u_z + w_x,
//   D_yz = v_z + w_y.
// Compliance: (1/mu)[[1, 1/2], [1/2, 1]] on each cell's (tau_xx, tau_yy) and
// 1/mu on the edges, times W_F W_L of the sample.
//
// Slices: samples 0 p, 1 txx, 2 tyy, 3 txy (z-edge), 4 txz (y-edge),
// 5 tyz (x-edge); faces 0 u, 1 v, 2 w; weight sets 0 cell, 1 u, 2 v, 3 w,
// 4 z-edge, 5 y-edge, 6 x-edge.
#include "vfs_internal.h"

namespace vfs {
namespace {

enum : uint8_t { FK = 1, FBAD = 2, FINV = 4 };

struct FaceIn {
    const double* WL;
    double* WF;
    const double* rho;
    const double* u;
    double* ustar;
    double* rhof;
    double* K;
    uint8_t* fflag;
};

// Classification and coefficients of face slice `a` at anchor o.
// s0, s1: the two cells sharing the face (in-box flags lo_in / hi_in),
// e0..e3: edge samples whose stencil holds the face (set index + offsets).
__device__ __forceinline__ void face_one(const Geo& g, const FaceIn& f, int a, long long o,
                                         long long oc_lo, bool lo_in, bool hi_in,
                                         int set_e0, long long oe0, long long oe1, int set_e1,
                                         long long oe2, long long oe3, double sK, double dt,
                                         double ga) {
    const long long NP = g.NP;
    const double wl = f.WL[(1 + a) * NP + o];
    const double wf = f.WF[(1 + a) * NP + o];
    bool inval = false;
    if (wf > 0.0) {
        const double* WFc = f.WF;
        inval = WFc[oc_lo] == 0.0 || WFc[o] == 0.0 || f.WF[set_e0 * NP + oe0] == 0.0 ||
                f.WF[set_e0 * NP + oe1] == 0.0 || f.WF[set_e1 * NP + oe2] == 0.0 ||
                f.WF[set_e1 * NP + oe3] == 0.0;
    }
    const double wfe = inval ? 0.0 : wf;
    const bool kp = wfe > 0.0 && wl > 0.0;
    const bool bad = wfe > 0.0 && wl == 0.0;
    double r;
    if (lo_in && hi_in)
        r = (f.rho[oc_lo] + f.rho[o]) * 0.5;
    else
        r = lo_in ? f.rho[oc_lo] : f.rho[o];
    f.WF[(1 + a) * NP + o] = wfe;
    f.rhof[a * NP + o] = r;
    f.K[a * NP + o] = kp ? sK * (wfe / (r * wl)) : 0.0;
    f.fflag[a * NP + o] = (uint8_t)((kp ? FK : 0) | (bad ? FBAD : 0) | (inval ? FINV : 0));
    f.ustar[a * NP + o] = f.u[a * NP + o] + dt * ga;
}

__global__ void k_face3d(Geo g, double dt, double g0, double g1, double g2, FaceIn f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i > g.nx || j > g.ny || k > g.nz) return;
    const long long o = g.idx(i, j, k);
    const double sK = dt / (g.h * g.h);
    // u face (i,j,k): i <= nx, j < ny, k < nz. cells (i-1,j,k),(i,j,k);
    // z-edges (i,j,k),(i,j+1,k) [set 4]; y-edges (i,j,k),(i,j,k+1) [set 5]
    if (j < g.ny && k < g.nz)
        face_one(g, f, 0, o, g.idx(i - 1, j, k), i > 0, i < g.nx, 4, o, g.idx(i, j + 1, k), 5, o,
                 g.idx(i, j, k + 1), sK, dt, g0);
    // v face: i < nx, j <= ny, k < nz. cells (i,j-1,k),(i,j,k);
    // z-edges (i,j,k),(i+1,j,k) [4]; x-edges (i,j,k),(i,j,k+1) [6]
    if (i < g.nx && k < g.nz)
        face_one(g, f, 1, o, g.idx(i, j - 1, k), j > 0, j < g.ny, 4, o, g.idx(i + 1, j, k), 6, o,
                 g.idx(i, j, k + 1), sK, dt, g1);
    // w face: i < nx, j < ny, k <= nz. cells (i,j,k-1),(i,j,k);
    // y-edges (i,j,k),(i+1,j,k) [5]; x-edges (i,j,k),(i,j+1,k) [6]
    if (i < g.nx && j < g.ny)
        face_one(g, f, 2, o, g.idx(i, j, k - 1), k > 0, k < g.nz, 5, o, g.idx(i + 1, j, k), 6, o,
                 g.idx(i, j + 1, k), sK, dt, g2);
}

struct SampleIn {
    const double* WL;
    const double* WF;
    const double* mu;
    const double* K;
    const uint8_t* fflag;
    const double* ustar;
    const double* ubc;
    double* a;
    double* c;
    double* dinv;
    double* b;
};

// y = W_F u* + W_S u_BC on face slice fa at offset o
__device__ __forceinline__ double yface(const Geo& g, const SampleIn& s, int fa, long long o) {
    const long long NP = g.NP;
    const double wf = s.WF[(1 + fa) * NP + o];
    return wf * s.ustar[fa * NP + o] + (1.0 - wf) * s.ubc[fa * NP + o];
}

// One sample with a 2- or 4-face stencil: faces (fa[q], off[q]) with signs sg[q]
// (the reduced-D row, or -div for pressure).
template <int NF>
__device__ __forceinline__ int sample_one(const Geo& g, const SampleIn& s, int slice, int set,
                                          long long o, const int (&fa)[NF],
                                          const long long (&of)[NF], const double (&sg)[NF],
                                          double mu_s, double& a_out, double& c_out,
                                          double& d_out, double& b_out) {
    const long long NP = g.NP;
    uint8_t fl = 0;
#pragma unroll
    for (int q = 0; q < NF; ++q) fl |= s.fflag[fa[q] * NP + of[q]];
    const double wl = s.WL[set * NP + o];
    const double wf = s.WF[set * NP + o];
    const bool act = wl > 0.0 && !(fl & FBAD) && (fl & FK);
    a_out = c_out = d_out = b_out = 0.0;
    if (!act) return 0;
    const double ih = 1.0 / g.h;
    double sumK = 0.0, ty = 0.0, tb = 0.0;
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        sumK += s.K[fa[q] * NP + of[q]];
        ty += sg[q] * yface(g, s, fa[q], of[q]);
        tb += sg[q] * s.ubc[fa[q] * NP + of[q]];
    }
    a_out = wl;
    c_out = slice == 0 ? 0.0 : wf * wl / mu_s;
    d_out = 1.0 / (c_out + wl * wl * sumK);
    b_out = wl * (ty * ih - (1.0 - wf) * (tb * ih));
    return 1;
}

__device__ __forceinline__ double mu_mean(const Geo& g, const double* mu, int i, int j, int k,
                                          int sx, int sy, int sz) {
    // mean of the in-box cells adjacent to a sample of stagger (sx,sy,sz)
    double s = 0.0;
    int n = 0;
    for (int di = (sx ? 0 : -1); di <= 0; ++di)
        for (int dj = (sy ? 0 : -1); dj <= 0; ++dj)
            for (int dk = (sz ? 0 : -1); dk <= 0; ++dk) {
                const int ci = i + di, cj = j + dj, ck = k + dk;
                if (ci < 0 || ci >= g.nx || cj < 0 || cj >= g.ny || ck < 0 || ck >= g.nz) continue;
                s += mu[g.idx(ci, cj, ck)];
                ++n;
            }
    return n ? s / (double)n : 1.0;
}

__global__ void k_sample3d(Geo g, SampleIn s, Scalars* sc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    int nact = 0;
    if (i <= g.nx && j <= g.ny && k <= g.nz) {
        const long long NP = g.NP;
        const long long o = g.idx(i, j, k);
        double av[6], cv[6], dv[6], bv[6];
        for (int q = 0; q < 6; ++q) av[q] = cv[q] = dv[q] = bv[q] = 0.0;
        if (i < g.nx && j < g.ny && k < g.nz) {
            const long long oi = g.idx(i + 1, j, k), oj = g.idx(i, j + 1, k), ok = g.idx(i, j, k + 1);
            const double muc = s.mu[o];
            {   // p: -div over the six faces
                const int fa[6] = {0, 0, 1, 1, 2, 2};
                const long long of[6] = {o, oi, o, oj, o, ok};
                const double sg[6] = {1, -1, 1, -1, 1, -1};
                nact += sample_one<6>(g, s, 0, 0, o, fa, of, sg, muc, av[0], cv[0], dv[0], bv[0]);
            }
            {   // txx: u_x - w_z
                const int fa[4] = {0, 0, 2, 2};
                const long long of[4] = {oi, o, ok, o};
                const double sg[4] = {1, -1, -1, 1};
                nact += sample_one<4>(g, s, 1, 0, o, fa, of, sg, muc, av[1], cv[1], dv[1], bv[1]);
            }
            {   // tyy: v_y - w_z
                const int fa[4] = {1, 1, 2, 2};
                const long long of[4] = {oj, o, ok, o};
                const double sg[4] = {1, -1, -1, 1};
                nact += sample_one<4>(g, s, 2, 0, o, fa, of, sg, muc, av[2], cv[2], dv[2], bv[2]);
            }
            // the (txx, tyy) compliance coupling: the diagonal of the 2x2
            // block is c; Jacobi uses the diagonal entries only
        }
        if (i <= g.nx && j <= g.ny && k < g.nz) {   // txy on z-edge: u_y + v_x
            const int fa[4] = {0, 0, 1, 1};
            const long long of[4] = {o, g.idx(i, j - 1, k), o, g.idx(i - 1, j, k)};
            const double sg[4] = {1, -1, 1, -1};
            nact += sample_one<4>(g, s, 3, 4, o, fa, of, sg, mu_mean(g, s.mu, i, j, k, 0, 0, 1),
                                  av[3], cv[3], dv[3], bv[3]);
        }
        if (i <= g.nx && j < g.ny && k <= g.nz) {   // txz on y-edge: u_z + w_x
            const int fa[4] = {0, 0, 2, 2};
            const long long of[4] = {o, g.idx(i, j, k - 1), o, g.idx(i - 1, j, k)};
            const double sg[4] = {1, -1, 1, -1};
            nact += sample_one<4>(g, s, 4, 5, o, fa, of, sg, mu_mean(g, s.mu, i, j, k, 0, 1, 0),
                                  av[4], cv[4], dv[4], bv[4]);
        }
        if (i < g.nx && j <= g.ny && k <= g.nz) {   // tyz on x-edge: v_z + w_y
            const int fa[4] = {1, 1, 2, 2};
            const long long of[4] = {o, g.idx(i, j, k - 1), o, g.idx(i, j - 1, k)};
            const double sg[4] = {1, -1, 1, -1};
            nact += sample_one<4>(g, s, 5, 6, o, fa, of, sg, mu_mean(g, s.mu, i, j, k, 1, 0, 0),
                                  av[5], cv[5], dv[5], bv[5]);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            s.a[q * NP + o] = av[q];
            s.c[q * NP + o] = cv[q];
            s.dinv[q * NP + o] = dv[q];
            s.b[q * NP + o] = bv[q];
        }
    }
    __shared__ int s_cnt;
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    if (nact) atomicAdd(&s_cnt, nact);
    __syncthreads();
    if (tid == 0 && s_cnt) atomicAdd((unsigned long long*)&sc->n_active, (unsigned long long)s_cnt);
}

// Velocity recovery (3D): u = u* - dt (B x) / (rho W_L) where K > 0; u_BC
// where W_F = 0; 0 elsewhere.
__global__ void k_velocity3d(Geo g, double dt, const double* __restrict__ x,
                             const double* __restrict__ a, const double* __restrict__ ustar,
                             const double* __restrict__ ubc, const double* __restrict__ rhof,
                             const double* __restrict__ WL, const double* __restrict__ WF,
                             const uint8_t* __restrict__ fflag, double* __restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i > g.nx || j > g.ny || k > g.nz) return;
    const long long NP = g.NP;
    const long long o = g.idx(i, j, k);
    auto W = [&](int s, long long off) { return a[s * NP + off] * x[s * NP + off]; };
    const double sc = dt / g.h;
    if (j < g.ny && k < g.nz) {
        double val;
        if (fflag[o] & FK) {
            const long long om = g.idx(i - 1, j, k);
            const double d = (W(0, o) - W(0, om)) + (W(1, om) - W(1, o)) +
                             (W(3, o) - W(3, g.idx(i, j + 1, k))) +
                             (W(4, o) - W(4, g.idx(i, j, k + 1)));
            val = ustar[o] - sc * d / (rhof[o] * WL[NP + o]);
        } else {
            val = WF[NP + o] == 0.0 ? ubc[o] : 0.0;
        }
        u[o] = val;
    }
    if (i < g.nx && k < g.nz) {
        double val;
        if (fflag[NP + o] & FK) {
            const long long om = g.idx(i, j - 1, k);
            const double d = (W(0, o) - W(0, om)) + (W(2, om) - W(2, o)) +
                             (W(3, o) - W(3, g.idx(i + 1, j, k))) +
                             (W(5, o) - W(5, g.idx(i, j, k + 1)));
            val = ustar[NP + o] - sc * d / (rhof[NP + o] * WL[2 * NP + o]);
        } else {
            val = WF[2 * NP + o] == 0.0 ? ubc[NP + o] : 0.0;
        }
        u[NP + o] = val;
    }
    if (i < g.nx && j < g.ny) {
        double val;
        if (fflag[2 * NP + o] & FK) {
            const long long om = g.idx(i, j, k - 1);
            const double d = (W(0, o) - W(0, om)) + (W(1, o) - W(1, om)) + (W(2, o) - W(2, om)) +
                             (W(4, o) - W(4, g.idx(i + 1, j, k))) +
                             (W(5, o) - W(5, g.idx(i, j + 1, k)));
            val = ustar[2 * NP + o] - sc * d / (rhof[2 * NP + o] * WL[3 * NP + o]);
        } else {
            val = WF[3 * NP + o] == 0.0 ? ubc[2 * NP + o] : 0.0;
        }
        u[2 * NP + o] = val;
    }
}

// Prescribed traction (Section 6.1), 3D counterpart of k_traction2d: on
// faces with K > 0, u* += dt f / (rho W_L), f = B0 (a y) - W_L (B0 y), with
// B0's stencils of k_velocity3d.
__global__ void k_traction3d(Geo g, double dt, const double* __restrict__ y,
                             const double* __restrict__ a, const double* __restrict__ rhof,
                             const double* __restrict__ WL, const uint8_t* __restrict__ fflag,
                             double* __restrict__ ustar) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i > g.nx || j > g.ny || k > g.nz) return;
    const long long NP = g.NP;
    const long long o = g.idx(i, j, k);
    auto AY = [&](int s, long long off) { return a[s * NP + off] * y[s * NP + off]; };
    auto Y = [&](int s, long long off) { return y[s * NP + off]; };
    const double sc = dt / g.h;
    if (j < g.ny && k < g.nz && (fflag[o] & FK)) {
        const long long om = g.idx(i - 1, j, k), oy = g.idx(i, j + 1, k), oz = g.idx(i, j, k + 1);
        const double day = (AY(0, o) - AY(0, om)) + (AY(1, om) - AY(1, o)) + (AY(3, o) - AY(3, oy)) +
                           (AY(4, o) - AY(4, oz));
        const double dy = (Y(0, o) - Y(0, om)) + (Y(1, om) - Y(1, o)) + (Y(3, o) - Y(3, oy)) +
                          (Y(4, o) - Y(4, oz));
        const double wl = WL[NP + o];
        ustar[o] += sc * (day - wl * dy) / (rhof[o] * wl);
    }
    if (i < g.nx && k < g.nz && (fflag[NP + o] & FK)) {
        const long long om = g.idx(i, j - 1, k), ox = g.idx(i + 1, j, k), oz = g.idx(i, j, k + 1);
        const double day = (AY(0, o) - AY(0, om)) + (AY(2, om) - AY(2, o)) + (AY(3, o) - AY(3, ox)) +
                           (AY(5, o) - AY(5, oz));
        const double dy = (Y(0, o) - Y(0, om)) + (Y(2, om) - Y(2, o)) + (Y(3, o) - Y(3, ox)) +
                          (Y(5, o) - Y(5, oz));
        const double wl = WL[2 * NP + o];
        ustar[NP + o] += sc * (day - wl * dy) / (rhof[NP + o] * wl);
    }
    if (i < g.nx && j < g.ny && (fflag[2 * NP + o] & FK)) {
        const long long om = g.idx(i, j, k - 1), ox = g.idx(i + 1, j, k), oy = g.idx(i, j + 1, k);
        const double day = (AY(0, o) - AY(0, om)) + (AY(1, o) - AY(1, om)) + (AY(2, o) - AY(2, om)) +
                           (AY(4, o) - AY(4, ox)) + (AY(5, o) - AY(5, oy));
        const double dy = (Y(0, o) - Y(0, om)) + (Y(1, o) - Y(1, om)) + (Y(2, o) - Y(2, om)) +
                          (Y(4, o) - Y(4, ox)) + (Y(5, o) - Y(5, oy));
        const double wl = WL[3 * NP + o];
        ustar[2 * NP + o] += sc * (day - wl * dy) / (rhof[2 * NP + o] * wl);
    }
}

// A cell whose tau_xx is active and tau_yy eliminated (or the reverse): the
// eliminated stress holds its boundary value, and the compliance coupling
// (1/2) W_F W_L / mu of the pair moves that value times the coupling to the
// right-hand side of the active one.  c holds W_F W_L / mu on active stresses.
__global__ void k_traction_pair3d(Geo g, const double* __restrict__ y,
                                  const double* __restrict__ a, const double* __restrict__ c,
                                  double* __restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    const long long NP = g.NP;
    const long long o = g.idx(i, j, k);
    const bool ax = a[NP + o] != 0.0, ay = a[2 * NP + o] != 0.0;
    if (ax && !ay) b[NP + o] -= 0.5 * c[NP + o] * y[2 * NP + o];
    if (ay && !ax) b[2 * NP + o] -= 0.5 * c[2 * NP + o] * y[NP + o];
}

dim3 grid3(const Geo& g, dim3 bs) {
    return dim3((g.nx + 1 + bs.x - 1) / bs.x, (g.ny + 1 + bs.y - 1) / bs.y,
                (g.nz + 1 + bs.z - 1) / bs.z);
}

}  // namespace

void launch_face_coef3d(const Geo& g, double dt, const double* g3, const double* WL, double* WF,
                        const double* rho, const double* u, double* ustar, double* rhof,
                        double* K, uint8_t* fflag, hipStream_t s) {
    FaceIn f{WL, WF, rho, u, ustar, rhof, K, fflag};
    dim3 bs(64, 2, 2);
    hipLaunchKernelGGL(k_face3d, grid3(g, bs), bs, 0, s, g, dt, g3[0], g3[1], g3[2], f);
}

void launch_traction3d(const Geo& g, double dt, const double* y, const double* a,
                       const double* rhof, const double* WL, const uint8_t* fflag, double* ustar,
                       hipStream_t s) {
    dim3 bs(64, 2, 2);
    hipLaunchKernelGGL(k_traction3d, grid3(g, bs), bs, 0, s, g, dt, y, a, rhof, WL, fflag, ustar);
}

void launch_traction_pair3d(const Geo& g, const double* y, const double* a, const double* c,
                            double* b, hipStream_t s) {
    dim3 bs(64, 2, 2);
    hipLaunchKernelGGL(k_traction_pair3d, grid3(g, bs), bs, 0, s, g, y, a, c, b);
}

void launch_sample_coef3d(const Geo& g, const double* WL, const double* WF, const double* mu,
                          const double* K, const uint8_t* fflag, const double* ustar,
                          const double* ubc, double* a, double* c, double* dinv, double* b,
                          Scalars* sc, hipStream_t s) {
    SampleIn si{WL, WF, mu, K, fflag, ustar, ubc, a, c, dinv, b};
    dim3 bs(64, 2, 2);
    hipLaunchKernelGGL(k_sample3d, grid3(g, bs), bs, 0, s, g, si, sc);
}

void launch_velocity3d(const Geo& g, double dt, const double* x, const double* a,
                       const double* ustar, const double* ubc, const double* rhof,
                       const double* WL, const double* WF, const uint8_t* fflag, double* u,
                       hipStream_t s) {
    dim3 bs(64, 2, 2);
    hipLaunchKernelGGL(k_velocity3d, grid3(g, bs), bs, 0, s, g, dt, x, a, ustar, ubc, rhof, WL, WF,
                       fflag, u);
}

}  // namespace vfs
