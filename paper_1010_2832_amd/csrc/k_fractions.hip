// Volume fractions of the sample control volumes (paper Section 5,
// Figs. 3-4: every term of the discrete functional is weighted by the
// fraction of material in an h-sized control volume around its sample).
//
// Estimator: nodal level set -> h/2 lattice by multilinear interpolation
// (midpoints averaged along x, then y, then z); each h/2 sub-cell split into
// Kuhn simplices sharing its min->max diagonal (2 triangles / 6 tetrahedra
// in axis-permutation order xyz, xzy, yxz, yzx, zxy, zyx); exact measure of
// {phi < 0} of each simplex under linear interpolation; control-volume
// weight = mean of its 2^d sub-cells, summed pairwise along x, then y, then
// z.  The operation order is part of the definition: together with
// -ffp-contract=off (set for this file by the build) it makes the weights,
// and therefore every classification decision taken on them, reproducible
// to the last bit.
//
// Box walls: sub-cells outside the box are solid (fluid fraction 0) and
// take the liquid fraction of the adjacent in-box sub-cell; faces on the
// box boundary have W_F = 0.  Weights below w_min are snapped to 0.
#include "vfs_internal.h"

namespace vfs {
namespace {

// Fraction of a triangle with phi < 0 for vertex values v0, v1, v2.
// Negative values are taken first in vertex order, then the others.
__device__ __forceinline__ double tri_frac(double v0, double v1, double v2) {
    double V[3] = {v0, v1, v2};
    double w[3];
    int m = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (V[q] < 0.0) w[m++] = V[q];
    const int k = m;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (!(V[q] < 0.0)) w[m++] = V[q];
    double f;
    if (k == 0) {
        f = 0.0;
    } else if (k == 3) {
        f = 1.0;
    } else if (k == 1) {
        const double a = w[0], b = w[1], c = w[2];
        f = (a * a) / ((a - b) * (a - c));
    } else {
        const double a = w[0], b = w[1], c = w[2];
        f = 1.0 - (c * c) / ((c - a) * (c - b));
    }
    return fmin(fmax(f, 0.0), 1.0);
}

// Fraction of a tetrahedron with phi < 0.
__device__ __forceinline__ double tet_frac(double v0, double v1, double v2, double v3) {
    double V[4] = {v0, v1, v2, v3};
    double w[4];
    int m = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (V[q] < 0.0) w[m++] = V[q];
    const int k = m;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (!(V[q] < 0.0)) w[m++] = V[q];
    const double a = w[0], b = w[1], c = w[2], d = w[3];
    double f;
    if (k == 0) {
        f = 0.0;
    } else if (k == 4) {
        f = 1.0;
    } else if (k == 1) {
        f = ((a * a) * a) / (((a - b) * (a - c)) * (a - d));
    } else if (k == 2) {
        const double num = ((a * a) * (b * b) - ((a * b) * (a + b)) * (c + d)) +
                           (c * d) * (((a * a) + (a * b)) + (b * b));
        const double den = ((a - c) * (a - d)) * ((b - c) * (b - d));
        f = num / den;
    } else {
        f = 1.0 - ((d * d) * d) / (((d - a) * (d - b)) * (d - c));
    }
    return fmin(fmax(f, 0.0), 1.0);
}

// h/2-lattice value at (A,B) from compact nodal values (x-fastest, NX1 per row).
__device__ __forceinline__ double half2(const double* __restrict__ phi, int NX1, int A, int B) {
    const int i = A >> 1, j = B >> 1;
    const bool ox = A & 1, oy = B & 1;
    const double* r0 = phi + (long long)j * NX1;
    const double x0 = ox ? (r0[i] + r0[i + 1]) * 0.5 : r0[i];
    if (!oy) return x0;
    const double* r1 = r0 + NX1;
    const double x1 = ox ? (r1[i] + r1[i + 1]) * 0.5 : r1[i];
    return (x0 + x1) * 0.5;
}

__device__ __forceinline__ double half3(const double* __restrict__ phi, int NX1, int NY1, int A,
                                        int B, int C) {
    const int k = C >> 1;
    const long long plane = (long long)NX1 * NY1;
    const double z0 = half2(phi + k * plane, NX1, A, B);
    if (!(C & 1)) return z0;
    const double z1 = half2(phi + (k + 1) * plane, NX1, A, B);
    return (z0 + z1) * 0.5;
}

__global__ void k_subcell2d(int nx, int ny, const double* __restrict__ phi,
                            double* __restrict__ th, int complement) {
    const long long n = 4LL * nx * ny;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int A = (int)(t % (2 * nx));
    const int B = (int)(t / (2 * nx));
    const int NX1 = nx + 1;
    const double c00 = half2(phi, NX1, A, B);
    const double c10 = half2(phi, NX1, A + 1, B);
    const double c01 = half2(phi, NX1, A, B + 1);
    const double c11 = half2(phi, NX1, A + 1, B + 1);
    const double t1 = tri_frac(c00, c10, c11);
    const double t2 = tri_frac(c00, c01, c11);
    const double f = (t1 + t2) * 0.5;
    th[t] = complement ? 1.0 - f : f;
}

__global__ void k_subcell3d(int nx, int ny, int nz, const double* __restrict__ phi,
                            double* __restrict__ th, int complement) {
    const long long sx = 2LL * nx, sy = 2LL * ny;
    const long long n = sx * sy * 2LL * nz;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int A = (int)(t % sx);
    const int B = (int)((t / sx) % sy);
    const int C = (int)(t / (sx * sy));
    const int NX1 = nx + 1, NY1 = ny + 1;
    double cv[2][2][2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx)
                cv[dx][dy][dz] = half3(phi, NX1, NY1, A + dx, B + dy, C + dz);
    const double c000 = cv[0][0][0], c111 = cv[1][1][1];
    // permutations xyz, xzy, yxz, yzx, zxy, zyx: v1 = +e_p0, v2 = v1 + e_p1
    double acc;
    acc = tet_frac(c000, cv[1][0][0], cv[1][1][0], c111);          // xyz
    acc = acc + tet_frac(c000, cv[1][0][0], cv[1][0][1], c111);    // xzy
    acc = acc + tet_frac(c000, cv[0][1][0], cv[1][1][0], c111);    // yxz
    acc = acc + tet_frac(c000, cv[0][1][0], cv[0][1][1], c111);    // yzx
    acc = acc + tet_frac(c000, cv[0][0][1], cv[1][0][1], c111);    // zxy
    acc = acc + tet_frac(c000, cv[0][0][1], cv[0][1][1], c111);    // zyx
    const double f = acc / 6.0;
    th[t] = complement ? 1.0 - f : f;
}

__global__ void k_fill(double* __restrict__ d, long long n, double v) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = v;
}

// Sub-cell value with the box rule: liquid mirrors (clamps) into the box,
// fluid is 0 outside.
__device__ __forceinline__ double sub2(const double* th, int SX, int SY, int A, int B,
                                       bool liquid) {
    if (A < 0 || A >= SX || B < 0 || B >= SY) {
        if (!liquid) return 0.0;
        A = A < 0 ? 0 : (A >= SX ? SX - 1 : A);
        B = B < 0 ? 0 : (B >= SY ? SY - 1 : B);
    }
    return th[(long long)B * SX + A];
}

__device__ __forceinline__ double sub3(const double* th, int SX, int SY, int SZ, int A, int B,
                                       int C, bool liquid) {
    if (A < 0 || A >= SX || B < 0 || B >= SY || C < 0 || C >= SZ) {
        if (!liquid) return 0.0;
        A = A < 0 ? 0 : (A >= SX ? SX - 1 : A);
        B = B < 0 ? 0 : (B >= SY ? SY - 1 : B);
        C = C < 0 ? 0 : (C >= SZ ? SZ - 1 : C);
    }
    return th[((long long)C * SY + B) * SX + A];
}

__device__ __forceinline__ double cvmean2(const double* th, int SX, int SY, int i, int j, int sx,
                                          int sy, bool liquid) {
    const int A = 2 * i + (sx ? 0 : -1);
    const int B = 2 * j + (sy ? 0 : -1);
    const double t00 = sub2(th, SX, SY, A, B, liquid);
    const double t10 = sub2(th, SX, SY, A + 1, B, liquid);
    const double t01 = sub2(th, SX, SY, A, B + 1, liquid);
    const double t11 = sub2(th, SX, SY, A + 1, B + 1, liquid);
    return ((t00 + t10) + (t01 + t11)) * 0.25;
}

__device__ __forceinline__ double cvmean3(const double* th, int SX, int SY, int SZ, int i, int j,
                                          int k, int sx, int sy, int sz, bool liquid) {
    const int A = 2 * i + (sx ? 0 : -1);
    const int B = 2 * j + (sy ? 0 : -1);
    const int C = 2 * k + (sz ? 0 : -1);
    const double t000 = sub3(th, SX, SY, SZ, A, B, C, liquid);
    const double t100 = sub3(th, SX, SY, SZ, A + 1, B, C, liquid);
    const double t010 = sub3(th, SX, SY, SZ, A, B + 1, C, liquid);
    const double t110 = sub3(th, SX, SY, SZ, A + 1, B + 1, C, liquid);
    const double t001 = sub3(th, SX, SY, SZ, A, B, C + 1, liquid);
    const double t101 = sub3(th, SX, SY, SZ, A + 1, B, C + 1, liquid);
    const double t011 = sub3(th, SX, SY, SZ, A, B + 1, C + 1, liquid);
    const double t111 = sub3(th, SX, SY, SZ, A + 1, B + 1, C + 1, liquid);
    return (((t000 + t100) + (t010 + t110)) + ((t001 + t101) + (t011 + t111))) * 0.125;
}

__device__ __forceinline__ double snap(double w, double w_min) { return w < w_min ? 0.0 : w; }

// 2D sets: 0 cell (1,1), 1 u (0,1), 2 v (1,0), 3 node (0,0)
__global__ void k_weights2d(Geo g, const double* __restrict__ thL,
                            const double* __restrict__ thF, double w_min,
                            double* __restrict__ WL, double* __restrict__ WF) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nx || j > g.ny) return;
    const int SX = 2 * g.nx, SY = 2 * g.ny;
    const long long o = g.idx(i, j);
    const int sxs[4] = {1, 0, 1, 0};
    const int sys[4] = {1, 1, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int sx = sxs[s], sy = sys[s];
        const bool valid = (i < g.nx + (sx ? 0 : 1)) && (j < g.ny + (sy ? 0 : 1));
        if (!valid) continue;
        double wl = snap(cvmean2(thL, SX, SY, i, j, sx, sy, true), w_min);
        double wf = snap(cvmean2(thF, SX, SY, i, j, sx, sy, false), w_min);
        if (s == 1 && (i == 0 || i == g.nx)) wf = 0.0;
        if (s == 2 && (j == 0 || j == g.ny)) wf = 0.0;
        WL[s * g.NP + o] = wl;
        WF[s * g.NP + o] = wf;
    }
}

// 3D sets: 0 cell (1,1,1), 1 u (0,1,1), 2 v (1,0,1), 3 w (1,1,0),
//          4 z-edge (0,0,1), 5 y-edge (0,1,0), 6 x-edge (1,0,0)
__global__ void k_weights3d(Geo g, const double* __restrict__ thL,
                            const double* __restrict__ thF, double w_min,
                            double* __restrict__ WL, double* __restrict__ WF) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i > g.nx || j > g.ny || k > g.nz) return;
    const int SX = 2 * g.nx, SY = 2 * g.ny, SZ = 2 * g.nz;
    const long long o = g.idx(i, j, k);
    const int sxs[7] = {1, 0, 1, 1, 0, 0, 1};
    const int sys[7] = {1, 1, 0, 1, 0, 1, 0};
    const int szs[7] = {1, 1, 1, 0, 1, 0, 0};
#pragma unroll
    for (int s = 0; s < 7; ++s) {
        const int sx = sxs[s], sy = sys[s], sz = szs[s];
        const bool valid = (i < g.nx + (sx ? 0 : 1)) && (j < g.ny + (sy ? 0 : 1)) &&
                           (k < g.nz + (sz ? 0 : 1));
        if (!valid) continue;
        double wl = snap(cvmean3(thL, SX, SY, SZ, i, j, k, sx, sy, sz, true), w_min);
        double wf = snap(cvmean3(thF, SX, SY, SZ, i, j, k, sx, sy, sz, false), w_min);
        if (s == 1 && (i == 0 || i == g.nx)) wf = 0.0;
        if (s == 2 && (j == 0 || j == g.ny)) wf = 0.0;
        if (s == 3 && (k == 0 || k == g.nz)) wf = 0.0;
        WL[s * g.NP + o] = wl;
        WF[s * g.NP + o] = wf;
    }
}

}  // namespace

void launch_subcell_fractions(const Geo& g, const double* phi, double* theta, bool complement,
                              hipStream_t s) {
    const int bs = 256;
    if (g.dim == 2) {
        const long long n = 4LL * g.nx * g.ny;
        hipLaunchKernelGGL(k_subcell2d, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, g.nx,
                           g.ny, phi, theta, complement ? 1 : 0);
    } else {
        const long long n = 8LL * g.nx * g.ny * g.nz;
        hipLaunchKernelGGL(k_subcell3d, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, g.nx,
                           g.ny, g.nz, phi, theta, complement ? 1 : 0);
    }
}

void launch_fill(double* dst, long long n, double v, hipStream_t s) {
    const int bs = 256;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, dst, n, v);
}

void launch_weights(const Geo& g, const double* thL, const double* thF, double w_min, double* WL,
                    double* WF, hipStream_t s) {
    if (g.dim == 2) {
        dim3 bs(64, 4);
        dim3 gs((g.nx + 1 + 63) / 64, (g.ny + 1 + 3) / 4);
        hipLaunchKernelGGL(k_weights2d, gs, bs, 0, s, g, thL, thF, w_min, WL, WF);
    } else {
        dim3 bs(64, 2, 2);
        dim3 gs((g.nx + 1 + 63) / 64, (g.ny + 1 + 1) / 2, (g.nz + 1 + 1) / 2);
        hipLaunchKernelGGL(k_weights3d, gs, bs, 0, s, g, thL, thF, w_min, WL, WF);
    }
}

}  // namespace vfs
