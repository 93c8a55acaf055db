// Layout conversion between the caller's compact x-fastest arrays and the
// padded device grid, input validation and precision conversion.
#include "vfs_internal.h"

namespace vfs {
namespace {

__global__ void k_pack(Geo g, int n0, int n1, int n2, const double* __restrict__ src,
                       double* __restrict__ dst) {
    const long long n = (long long)n0 * n1 * n2;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % n0);
    const int j = (int)((t / n0) % n1);
    const int k = (int)(t / ((long long)n0 * n1));
    const long long o = g.dim == 2 ? g.idx(i, j) : g.idx(i, j, k);
    dst[o] = src[t];
}

__global__ void k_unpack(Geo g, int n0, int n1, int n2, const double* __restrict__ src,
                         double* __restrict__ dst) {
    const long long n = (long long)n0 * n1 * n2;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % n0);
    const int j = (int)((t / n0) % n1);
    const int k = (int)(t / ((long long)n0 * n1));
    const long long o = g.dim == 2 ? g.idx(i, j) : g.idx(i, j, k);
    dst[t] = src[o];
}

__global__ void k_unpack_active(Geo g, int n0, int n1, int n2, const double* __restrict__ a,
                                uint8_t* __restrict__ dst) {
    const long long n = (long long)n0 * n1 * n2;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % n0);
    const int j = (int)((t / n0) % n1);
    const int k = (int)(t / ((long long)n0 * n1));
    const long long o = g.dim == 2 ? g.idx(i, j) : g.idx(i, j, k);
    dst[t] = a[o] != 0.0 ? 1 : 0;
}

__global__ void k_check(const double* __restrict__ v, long long n, int positive,
                        int* __restrict__ flag) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double x = v[t];
    const bool bad = !isfinite(x) || (positive && !(x > 0.0));
    if (bad) atomicOr(flag, 1);
}

__global__ void k_zero_box_faces(Geo g, double* __restrict__ f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i > g.nx || j > g.ny || (g.dim == 3 && k > g.nz)) return;
    const long long NP = g.NP;
    const long long o = g.dim == 2 ? g.idx(i, j) : g.idx(i, j, k);
    if (i == 0 || i == g.nx) f[o] = 0.0;
    if (j == 0 || j == g.ny) f[NP + o] = 0.0;
    if (g.dim == 3 && (k == 0 || k == g.nz)) f[2 * NP + o] = 0.0;
}

__global__ void k_to_f32(const double* __restrict__ s, float* __restrict__ d, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = (float)s[t];
}

// d = (float)(u v), the product rounded once
__global__ void k_mul_to_f32(const double* __restrict__ u, const double* __restrict__ v,
                             float* __restrict__ d, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = (float)(u[t] * v[t]);
}

__global__ void k_mask(double* __restrict__ d, const double* __restrict__ s,
                       const double* __restrict__ a, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = a[t] != 0.0 ? s[t] : 0.0;
}

// d = (x - y) on the samples with a != 0, 0 elsewhere
__global__ void k_sub_mask(double* __restrict__ d, const double* __restrict__ x,
                           const double* __restrict__ y, const double* __restrict__ a,
                           long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = a[t] != 0.0 ? x[t] - y[t] : 0.0;
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_pack(const Geo& g, const int shp[3], const double* src, double* dst, hipStream_t s) {
    const long long n = (long long)shp[0] * shp[1] * shp[2];
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pack, dim3(nblk(n, 256)), dim3(256), 0, s, g, shp[0], shp[1], shp[2], src,
                       dst);
}

void launch_unpack(const Geo& g, const int shp[3], const double* src, double* dst, hipStream_t s) {
    const long long n = (long long)shp[0] * shp[1] * shp[2];
    if (n <= 0) return;
    hipLaunchKernelGGL(k_unpack, dim3(nblk(n, 256)), dim3(256), 0, s, g, shp[0], shp[1], shp[2],
                       src, dst);
}

void launch_unpack_active(const Geo& g, const int shp[3], const double* a, uint8_t* dst,
                          hipStream_t s) {
    const long long n = (long long)shp[0] * shp[1] * shp[2];
    if (n <= 0) return;
    hipLaunchKernelGGL(k_unpack_active, dim3(nblk(n, 256)), dim3(256), 0, s, g, shp[0], shp[1],
                       shp[2], a, dst);
}

void launch_check(const double* v, long long n, int positive, int* flag, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_check, dim3(nblk(n, 256)), dim3(256), 0, s, v, n, positive, flag);
}

void launch_zero_box_faces(const Geo& g, double* faces, hipStream_t s) {
    dim3 bs(64, 4, 1);
    dim3 gs((g.nx + 1 + 63) / 64, (g.ny + 1 + 3) / 4, g.dim == 3 ? g.nz + 1 : 1);
    hipLaunchKernelGGL(k_zero_box_faces, gs, bs, 0, s, g, faces);
}

void launch_to_f32(const double* src, float* dst, long long n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_f32, dim3(nblk(n, 256)), dim3(256), 0, s, src, dst, n);
}

void launch_mul_to_f32(const double* u, const double* v, float* dst, long long n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mul_to_f32, dim3(nblk(n, 256)), dim3(256), 0, s, u, v, dst, n);
}

void launch_mask(double* dst, const double* src, const double* a, long long n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mask, dim3(nblk(n, 256)), dim3(256), 0, s, dst, src, a, n);
}

void launch_sub_mask(double* dst, const double* x, const double* y, const double* a, long long n,
                     hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sub_mask, dim3(nblk(n, 256)), dim3(256), 0, s, dst, x, y, a, n);
}

}  // namespace vfs
