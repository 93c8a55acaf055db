// Advection half of the fractional step (Section 10): first-order
// semi-Lagrangian advection of the face velocities (bilinear in 2D,
// trilinear in 3D) and of the nodal liquid level set, FP64.
//
// * Velocity extension: faces the last Stokes step defined (K > 0, or
//   W_F = 0) are known; each of `layers` passes gives every unknown face with
//   a known neighbour of the same component (one index step along an axis)
//   the mean of those neighbours, summed along x (i-1, i+1), then y, then z.
// * Interpolation of a sample type of stagger s at a point given in index
//   units of h from the box corner: continuous index P - s/2, clamped to
//   [0, shape - 1] per axis, base min(floor, shape - 2), multilinear weights.
// * Departure point of a sample: its position minus dt v / h (index units),
//   v the interpolated extended velocity.
#include "vfs_internal.h"

namespace vfs {
namespace {

enum : uint8_t { FK = 1 };

struct Lattice {
    int n[3];   // samples per axis
    int s[3];   // stagger (1 = cell-centred along that axis)
};

__device__ __forceinline__ Lattice face_lattice(const Geo& g, int a) {
    Lattice L;
    const int nn[3] = {g.nx, g.ny, g.nz};
    for (int b = 0; b < 3; ++b) {
        L.s[b] = (b == a) ? 0 : 1;
        L.n[b] = (b < g.dim) ? nn[b] + 1 - L.s[b] : 1;
    }
    return L;
}

__device__ __forceinline__ void axis_weights(double P, int s, int n, int& i0, double& t) {
    double xi = P - 0.5 * s;
    xi = fmin(fmax(xi, 0.0), (double)(n - 1));
    int f = (int)floor(xi);
    i0 = min(f, max(n - 2, 0));
    t = xi - (double)i0;
}

// value of face component a (padded slice `u`) at the index-space point P
__device__ double interp_face(const Geo& g, const double* __restrict__ u, int a, const double P[3]) {
    const Lattice L = face_lattice(g, a);
    int i0[3];
    double t[3];
    for (int b = 0; b < 3; ++b) {
        if (b < g.dim) {
            axis_weights(P[b], L.s[b], L.n[b], i0[b], t[b]);
        } else {
            i0[b] = 0;
            t[b] = 0.0;
        }
    }
    const double* src = u + (long long)a * g.NP;
    double acc = 0.0;
    const int corners = 1 << g.dim;
    for (int c = 0; c < corners; ++c) {
        double w = 1.0;
        int ix[3] = {0, 0, 0};
        for (int b = 0; b < g.dim; ++b) {
            const int up = (c >> b) & 1;
            w *= up ? t[b] : 1.0 - t[b];
            ix[b] = min(i0[b] + up, L.n[b] - 1);
        }
        const long long o = g.dim == 2 ? g.idx(ix[0], ix[1]) : g.idx(ix[0], ix[1], ix[2]);
        acc += w * src[o];
    }
    return acc;
}

__device__ __forceinline__ bool face_valid(const Geo& g, int a, int i, int j, int k) {
    const int n[3] = {g.nx, g.ny, g.nz};
    const int id[3] = {i, j, k};
    for (int b = 0; b < g.dim; ++b) {
        const int lim = n[b] + (b == a ? 1 : 0);
        if (id[b] < 0 || id[b] >= lim) return false;
    }
    return true;
}

__device__ __forceinline__ long long anchor(const Geo& g, int i, int j, int k) {
    return g.dim == 2 ? g.idx(i, j) : g.idx(i, j, k);
}

// known flags of the velocity of the last Stokes step (all = 1: every face)
__global__ void k_known_faces(Geo g, const uint8_t* __restrict__ fflag,
                              const double* __restrict__ WF, int all, uint8_t* __restrict__ known) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i > g.nx || j > g.ny || k > (g.dim == 3 ? g.nz : 0)) return;
    const long long o = anchor(g, i, j, k);
    for (int a = 0; a < g.dim; ++a) {
        const long long q = (long long)a * g.NP + o;
        uint8_t kn = 0;
        if (face_valid(g, a, i, j, k))
            kn = (all || (fflag[q] & FK) || WF[(long long)(1 + a) * g.NP + o] == 0.0) ? 1 : 0;
        known[q] = kn;
    }
}

// one extension layer: vin/kin -> vout/kout
__global__ void k_extend(Geo g, const double* __restrict__ vin, const uint8_t* __restrict__ kin,
                         double* __restrict__ vout, uint8_t* __restrict__ kout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i > g.nx || j > g.ny || k > (g.dim == 3 ? g.nz : 0)) return;
    const long long o = anchor(g, i, j, k);
    const long long step[3] = {1, (long long)g.PX, (long long)g.PX * g.PY};
    const int id[3] = {i, j, k};
    for (int a = 0; a < g.dim; ++a) {
        const long long q = (long long)a * g.NP + o;
        if (!face_valid(g, a, i, j, k)) continue;
        if (kin[q]) {
            vout[q] = vin[q];
            kout[q] = 1;
            continue;
        }
        double acc = 0.0;
        int cnt = 0;
        for (int b = 0; b < g.dim; ++b) {
            int lo[3] = {id[0], id[1], id[2]};
            lo[b] -= 1;
            if (face_valid(g, a, lo[0], lo[1], lo[2]) && kin[q - step[b]]) {
                acc += vin[q - step[b]];
                ++cnt;
            }
            int hi[3] = {id[0], id[1], id[2]};
            hi[b] += 1;
            if (face_valid(g, a, hi[0], hi[1], hi[2]) && kin[q + step[b]]) {
                acc += vin[q + step[b]];
                ++cnt;
            }
        }
        if (cnt > 0) {
            vout[q] = acc / (double)cnt;
            kout[q] = 1;
        } else {
            vout[q] = vin[q];
            kout[q] = 0;
        }
    }
}

// semi-Lagrangian velocity: every valid face of every component
__global__ void k_advect_u(Geo g, double dt, const double* __restrict__ uext,
                           double* __restrict__ uout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i > g.nx || j > g.ny || k > (g.dim == 3 ? g.nz : 0)) return;
    const long long o = anchor(g, i, j, k);
    const double sc = dt / g.h;
    for (int a = 0; a < g.dim; ++a) {
        if (!face_valid(g, a, i, j, k)) continue;
        double P[3] = {(double)i, (double)j, (double)k};
        for (int b = 0; b < g.dim; ++b)
            if (b != a) P[b] += 0.5;
        double v[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < g.dim; ++b) v[b] = interp_face(g, uext, b, P);
        double D[3] = {P[0], P[1], P[2]};
        for (int b = 0; b < g.dim; ++b) D[b] -= sc * v[b];
        uout[(long long)a * g.NP + o] = interp_face(g, uext, a, D);
    }
}

// semi-Lagrangian level set at the nodes (compact arrays)
__global__ void k_advect_phi(Geo g, double dt, const double* __restrict__ uext,
                             const double* __restrict__ phi, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    const int n0 = g.nx + 1, n1 = g.ny + 1, n2 = g.dim == 3 ? g.nz + 1 : 1;
    if (i >= n0 || j >= n1 || k >= n2) return;
    const double sc = dt / g.h;
    const double P[3] = {(double)i, (double)j, (double)k};
    double D[3] = {P[0], P[1], P[2]};
    for (int b = 0; b < g.dim; ++b) D[b] -= sc * interp_face(g, uext, b, P);
    const int nn[3] = {n0, n1, n2};
    int i0[3] = {0, 0, 0};
    double t[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < g.dim; ++b) axis_weights(D[b], 0, nn[b], i0[b], t[b]);
    double acc = 0.0;
    const int corners = 1 << g.dim;
    for (int c = 0; c < corners; ++c) {
        double w = 1.0;
        int ix[3] = {0, 0, 0};
        for (int b = 0; b < g.dim; ++b) {
            const int up = (c >> b) & 1;
            w *= up ? t[b] : 1.0 - t[b];
            ix[b] = min(i0[b] + up, nn[b] - 1);
        }
        acc += w * phi[ix[0] + (long long)n0 * (ix[1] + (long long)n1 * ix[2])];
    }
    out[i + (long long)n0 * (j + (long long)n1 * k)] = acc;
}

dim3 grid_of(const Geo& g, dim3 bs, int extra) {
    return dim3((g.nx + extra + bs.x - 1) / bs.x, (g.ny + extra + bs.y - 1) / bs.y,
                g.dim == 3 ? (g.nz + extra + bs.z - 1) / bs.z : 1);
}

dim3 block_of(const Geo& g) { return g.dim == 2 ? dim3(64, 4, 1) : dim3(64, 2, 2); }

}  // namespace

void launch_known_faces(const Geo& g, const uint8_t* fflag, const double* WF, bool all,
                        uint8_t* known, hipStream_t s) {
    const dim3 bs = block_of(g);
    hipLaunchKernelGGL(k_known_faces, grid_of(g, bs, 1), bs, 0, s, g, fflag, WF, all ? 1 : 0, known);
}

void launch_extend(const Geo& g, const double* vin, const uint8_t* kin, double* vout,
                   uint8_t* kout, hipStream_t s) {
    const dim3 bs = block_of(g);
    hipLaunchKernelGGL(k_extend, grid_of(g, bs, 1), bs, 0, s, g, vin, kin, vout, kout);
}

void launch_advect_u(const Geo& g, double dt, const double* uext, double* uout, hipStream_t s) {
    const dim3 bs = block_of(g);
    hipLaunchKernelGGL(k_advect_u, grid_of(g, bs, 1), bs, 0, s, g, dt, uext, uout);
}

void launch_advect_phi(const Geo& g, double dt, const double* uext, const double* phi, double* out,
                       hipStream_t s) {
    const dim3 bs = block_of(g);
    hipLaunchKernelGGL(k_advect_phi, grid_of(g, bs, 1), bs, 0, s, g, dt, uext, phi, out);
}

}  // namespace vfs
