// Kernels of the learned preconditioner network: 3x3x3 convolutions as
// implicit GEMMs on the gfx950 BF16 matrix cores (FP32 accumulation), the
// weight gradient, 2x2x2 level transfers, weight preparation, Adam, and the
// transfers between a 3D solver context's sample vectors and the network's
// cell-indexed tensors.
//
// Convolution as GEMM: out[co][v] = sum_K W[co][K] * B[K][v] with
// K = t * CIN + ci (tap t = 9 dz + 3 dy + dx) and B[K][v] = in[v + off_t][ci].
// v_mfma_f32_16x16x32_bf16 multiplies a 16x32 tile of W by a 32x16 tile of B.
// Lane l supplies W[m = l%16][k = 8(l/16) .. +7] and B[k = 8(l/16) .. +7][n =
// l%16] (8 contiguous channels of one voxel: one 16-byte load from the
// channels-last tensor) and receives D[m = 4(l/16) + i][n = l%16], i < 4
// (4 consecutive output channels of one voxel: one 8-byte store).
#include "vfs_unet.h"
#include "vfs_reduce.h"

#include <algorithm>

namespace vfs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CT = 256;

__device__ __forceinline__ float bf2f(uint32_t v) { return __uint_as_float(v << 16); }

// round to nearest, ties to even; NaN stays a quiet NaN
__device__ __forceinline__ uint32_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ bf16x8 ld16(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

// 8 bf16 values at stride `stride` (LDS) as one MFMA operand
__device__ __forceinline__ bf16x8 gather8(const uint16_t* p, int stride) {
    uint4 u;
    u.x = (uint32_t)p[0] | ((uint32_t)p[stride] << 16);
    u.y = (uint32_t)p[2 * stride] | ((uint32_t)p[3 * stride] << 16);
    u.z = (uint32_t)p[4 * stride] | ((uint32_t)p[5 * stride] << 16);
    u.w = (uint32_t)p[6 * stride] | ((uint32_t)p[7 * stride] << 16);
    return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ void unpack8(const uint4& u, float (&f)[8]) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = bf2f(w[i] & 0xffffu);
        f[2 * i + 1] = bf2f(w[i] >> 16);
    }
}

__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
    uint4 u;
    u.x = f2bf(f[0]) | (f2bf(f[1]) << 16);
    u.y = f2bf(f[2]) | (f2bf(f[3]) << 16);
    u.z = f2bf(f[4]) | (f2bf(f[5]) << 16);
    u.w = f2bf(f[6]) | (f2bf(f[7]) << 16);
    return u;
}

__device__ __forceinline__ long long voxel_off(const Level& L, long long v) {
    const int x = (int)(v % L.X);
    const long long t = v / L.X;
    const int y = (int)(t % L.Y);
    const int z = (int)(t / L.Y);
    return L.off(x, y, z);
}

__device__ __forceinline__ long long tap_off(const Level& L, int t) {
    const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
    return ((long long)(dz - 1) * (L.Y + 2) + (dy - 1)) * (L.X + 2) + (dx - 1);
}

// ---------------------------------------------------------------------------
// convolution (forward and input gradient)
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
struct ConvShape {
    static constexpr int KP = conv_kp(CIN);
    static constexpr int NKC = KP / 32;
    static constexpr int MT = COUT / 16;               // output-channel tiles
    static constexpr int NV = COUT >= 128 ? 2 : 4;      // 16-voxel tiles per wave
    static constexpr int VPB = 4 * 16 * NV;             // voxels per workgroup
};

template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(CT) void k_conv3(ConvArgs A) {
    if (A.skip && *A.skip) return;
    using S = ConvShape<CIN, COUT>;
    constexpr int KP = S::KP, NKC = S::NKC, MT = S::MT, NV = S::NV;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Level L = A.L;
    const long long V = L.voxels();
    const long long vbase = ((long long)blockIdx.x * 4 + wave) * (16 * NV);
    if (vbase >= V) return;   // the wave has no voxel; no workgroup barrier follows
    long long vof[NV];
    bool valid[NV];
#pragma unroll
    for (int nv = 0; nv < NV; ++nv) {
        const long long v = vbase + nv * 16 + (lane & 15);
        valid[nv] = v < V;
        vof[nv] = voxel_off(L, valid[nv] ? v : 0);
    }
    f32x4 acc[NV][MT];
#pragma unroll
    for (int nv = 0; nv < NV; ++nv)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[nv][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kq = lane >> 4;
    const uint16_t* wrow = A.w + (long long)(lane & 15) * KP + kq * 8;
    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, uint4{0u, 0u, 0u, 0u});
    for (int kc = 0; kc < NKC; ++kc) {
        const int K = kc * 32 + kq * 8;
        const int t = K / CIN, ci = K % CIN;
        bf16x8 b[NV];
        if (t < 27) {
            const long long to = tap_off(L, t);
#pragma unroll
            for (int nv = 0; nv < NV; ++nv) b[nv] = ld16(A.in + (vof[nv] + to) * CIN + ci);
        } else {
#pragma unroll
            for (int nv = 0; nv < NV; ++nv) b[nv] = zero8;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const bf16x8 a = ld16(wrow + (long long)mt * 16 * KP + kc * 32);
#pragma unroll
            for (int nv = 0; nv < NV; ++nv)
                acc[nv][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nv], acc[nv][mt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nv = 0; nv < NV; ++nv) {
        if (!valid[nv]) continue;
        const long long v = vbase + nv * 16 + (lane & 15);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int co0 = mt * 16 + kq * 4;
            float o[4] = {acc[nv][mt][0], acc[nv][mt][1], acc[nv][mt][2], acc[nv][mt][3]};
            if (EPI == EPI_F32) {
                if (co0 < 8)
                    *reinterpret_cast<float4*>(A.out32 + v * 8 + co0) = float4{o[0], o[1], o[2], o[3]};
                continue;
            }
            if (EPI == EPI_RELU) {
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = fmaxf(o[i], 0.f);
            } else if (EPI == EPI_MASK) {
                const uint2 mk = *reinterpret_cast<const uint2*>(A.mask + vof[nv] * COUT + co0);
                const uint32_t mw[4] = {mk.x & 0xffffu, mk.x >> 16, mk.y & 0xffffu, mk.y >> 16};
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = bf2f(mw[i]) > 0.f ? o[i] : 0.f;
            }
            uint2 st;
            st.x = f2bf(o[0]) | (f2bf(o[1]) << 16);
            st.y = f2bf(o[2]) | (f2bf(o[3]) << 16);
            *reinterpret_cast<uint2*>(A.out + vof[nv] * COUT + co0) = st;
        }
    }
}

// ---------------------------------------------------------------------------
// Convolutions with 16 or 32 channels on each side (the full-resolution and
// half-resolution layers): z-marching with the input planes staged in LDS.
// With few output channels a voxel operand feeds only COUT / 16 MFMAs, so
// operand bandwidth bounds these layers, not the matrix cores; here each
// input plane is read from global memory once per tile (plus its x,y halo)
// and the 27 taps read their operands from LDS, while the weight operands of
// a lane stay in registers for the whole launch.
//
// Workgroup: a 32 x ZY voxel tile in x,y marching kZZ planes in z.  LDS holds
// a ring of 4 input planes of 34 x (ZY + 2) voxels, each split into CIN / 8
// arrays of 8 channels (16 bytes per voxel, so the 16 lanes of one MFMA
// column group read 256 contiguous bytes).  Step z: issue the global loads of
// plane z+2, compute output plane z from the planes z-1, z, z+1, write the
// epilogue, store plane z+2 into its slot (which held plane z-2), one
// barrier.  K = 32 kc + 8 kq + j is tap t = K / CIN, channel K % CIN: with 16
// input channels lanes 0-31 of a wave read tap 2 kc and lanes 32-63 tap
// 2 kc + 1 (tap 27, for kc = 13 and kq >= 2, is the zero padding of K); with
// 32 they all read tap kc, 8 channels per lane group.
// ---------------------------------------------------------------------------
constexpr int kZX = 32, kZZ = 16;   // output tile in x and z (ZY in y)

template <int CIN, int ZY>
struct ZTile {
    static constexpr int HX = kZX + 2, HY = ZY + 2;
    static constexpr int PLANE = HX * HY;                 // voxels per input plane
    static constexpr int OCT = CIN / 8;                   // 16-byte channel octets per voxel
    static constexpr int CHUNKS = OCT * PLANE;            // 16-byte chunks per plane
    static constexpr int LOADS = (CHUNKS + CT - 1) / CT;  // chunks per thread
    static constexpr int NVW = ZY / 2;                    // 16-voxel column groups per wave
};

template <int CIN, int COUT, int ZY, int EPI>
__global__ __launch_bounds__(CT) void k_conv3_z(ConvArgs A, int ntx, int nty, int ntz) {
    if (A.skip && *A.skip) return;
    using Z = ZTile<CIN, ZY>;
    static_assert(CIN == 16 || CIN == 32, "input channels");
    static_assert(COUT % 16 == 0 && ZY % 4 == 0, "tile");
    constexpr int KP = conv_kp(CIN), NKC = KP / 32, MT = COUT / 16;
    constexpr int NVW = Z::NVW, HX = Z::HX;
    __shared__ __align__(16) uint4 sIn[4][Z::OCT][Z::PLANE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, n = lane & 15;
    const Level L = A.L;
    // XCD-contiguous tile order (workgroup b runs on XCD b % 8)
    const int G = gridDim.x, b = blockIdx.x;
    int tile = b;
    if (G >= 8) {
        const int x8 = b & 7, q = G >> 3, rem = G & 7;
        tile = x8 * q + min(x8, rem) + (b >> 3);
    }
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx * kZX, y0 = ty * ZY, z0 = tz * kZZ;
    const int zend = min(z0 + kZZ, L.Z);

    // weight operands: row co = 16 mt + n, K = 32 kc + 8 kq .. +7
    bf16x8 a[NKC][MT];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            a[kc][mt] = ld16(A.w + (long long)(16 * mt + n) * KP + kc * 32 + kq * 8);

    // plane loader: chunk e = OCT * voxel + octet of the input plane
    auto fetch = [&](int zz, uint4 (&r)[Z::LOADS]) {
#pragma unroll
        for (int m = 0; m < Z::LOADS; ++m) {
            const int e = threadIdx.x + m * CT;
            r[m] = uint4{0u, 0u, 0u, 0u};
            if (e < Z::CHUNKS) {
                const int v = e / Z::OCT, h = e % Z::OCT;
                const int x = x0 - 1 + v % HX, y = y0 - 1 + v / HX;
                if (x <= L.X && y <= L.Y && zz <= L.Z)
                    r[m] = *reinterpret_cast<const uint4*>(A.in + L.off(x, y, zz) * CIN + h * 8);
            }
        }
    };
    auto commit = [&](int zz, const uint4 (&r)[Z::LOADS]) {
        const int sl = (zz + 4) & 3;
#pragma unroll
        for (int m = 0; m < Z::LOADS; ++m) {
            const int e = threadIdx.x + m * CT;
            if (e < Z::CHUNKS) sIn[sl][e % Z::OCT][e / Z::OCT] = r[m];
        }
    };

    uint4 pre[Z::LOADS];
    fetch(z0 - 1, pre);
    commit(z0 - 1, pre);
    fetch(z0, pre);
    commit(z0, pre);
    fetch(z0 + 1, pre);
    commit(z0 + 1, pre);
    __syncthreads();

    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, uint4{0u, 0u, 0u, 0u});
    for (int z = z0; z < zend; ++z) {
        const bool more = z + 2 <= zend;
        if (more) fetch(z + 2, pre);
        f32x4 acc[NVW][MT];
#pragma unroll
        for (int nv = 0; nv < NVW; ++nv)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[nv][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
            const int K = 32 * kc + 8 * kq;
            const int t = K / CIN, oct = (K % CIN) / 8;
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
            const uint4* pl = sIn[(z + dz - 1 + 4) & 3][oct];
#pragma unroll
            for (int nv = 0; nv < NVW; ++nv) {
                const int yr = (ZY / 4) * wave + (nv >> 1), xo = 16 * (nv & 1);
                const bf16x8 bo = t < 27 ? __builtin_bit_cast(bf16x8, pl[(yr + dy) * HX + xo + n + dx])
                                         : zero8;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[nv][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kc][mt], bo, acc[nv][mt], 0, 0, 0);
            }
        }
        // epilogue: lane holds output channels 16 mt + 4 kq .. +3 of voxel n
#pragma unroll
        for (int nv = 0; nv < NVW; ++nv) {
            const int yr = (ZY / 4) * wave + (nv >> 1), xo = 16 * (nv & 1);
            const int x = x0 + xo + n, y = y0 + yr;
            if (x >= L.X || y >= L.Y) continue;
            const long long vo = L.off(x, y, z);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int co0 = 16 * mt + 4 * kq;
                float o[4] = {acc[nv][mt][0], acc[nv][mt][1], acc[nv][mt][2], acc[nv][mt][3]};
                if (EPI == EPI_F32) {
                    if (co0 < 8) {
                        const long long v = ((long long)z * L.Y + y) * L.X + x;
                        *reinterpret_cast<float4*>(A.out32 + v * 8 + co0) = float4{o[0], o[1], o[2], o[3]};
                    }
                    continue;
                }
                if (EPI == EPI_RELU) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) o[i] = fmaxf(o[i], 0.f);
                } else if (EPI == EPI_MASK) {
                    const uint2 mk = *reinterpret_cast<const uint2*>(A.mask + vo * COUT + co0);
                    const uint32_t mw[4] = {mk.x & 0xffffu, mk.x >> 16, mk.y & 0xffffu, mk.y >> 16};
#pragma unroll
                    for (int i = 0; i < 4; ++i) o[i] = bf2f(mw[i]) > 0.f ? o[i] : 0.f;
                }
                uint2 st;
                st.x = f2bf(o[0]) | (f2bf(o[1]) << 16);
                st.y = f2bf(o[2]) | (f2bf(o[3]) << 16);
                *reinterpret_cast<uint2*>(A.out + vo * COUT + co0) = st;
            }
        }
        // plane z + 2 replaces plane z - 2, which no wave reads any more
        if (more) commit(z + 2, pre);
        __syncthreads();
    }
}

template <int CIN, int COUT, int ZY, int EPI>
void conv_launch_z(const ConvArgs& a, hipStream_t s) {
    const int ntx = (a.L.X + kZX - 1) / kZX, nty = (a.L.Y + ZY - 1) / ZY;
    const int ntz = (a.L.Z + kZZ - 1) / kZZ;
    const long long nb = (long long)ntx * nty * ntz;
    if (nb == 0) return;
    hipLaunchKernelGGL((k_conv3_z<CIN, COUT, ZY, EPI>), dim3((unsigned)nb), dim3(CT), 0, s, a, ntx,
                       nty, ntz);
}

template <int CIN, int COUT, int EPI>
void conv_launch(const ConvArgs& a, hipStream_t s) {
    using S = ConvShape<CIN, COUT>;
    const long long V = a.L.voxels();
    const unsigned nb = (unsigned)((V + S::VPB - 1) / S::VPB);
    if (nb == 0) return;
    hipLaunchKernelGGL((k_conv3<CIN, COUT, EPI>), dim3(nb), dim3(CT), 0, s, a);
}

// ---------------------------------------------------------------------------
// weight gradient: per (voxel chunk, tap) workgroup, the COUT x CIN product
// of the output gradient and the tap-shifted input over the chunk.  Each
// wave stages 32 voxels of both operands in LDS per step and reads them
// transposed as MFMA operands (the reduction runs over voxels); the four
// waves' sums are added in wave order.
// ---------------------------------------------------------------------------
constexpr int kWgradStep = 32;
constexpr int kWgradTarget = 2048;   // voxels per chunk (before rounding)

template <int CIN, int COUT>
__global__ __launch_bounds__(CT) void k_wgrad(const uint16_t* __restrict__ in,
                                              const uint16_t* __restrict__ g, Level L,
                                              float* __restrict__ part, int chunk_vox,
                                              const int* skip) {
    if (skip && *skip) return;
    constexpr int MT = COUT / 16, NTc = CIN / 16;
    constexpr int STAGE = 4 * kWgradStep * (COUT + CIN) * 2;
    constexpr int RED = COUT * CIN * 4;
    constexpr int SMEM = STAGE > RED ? STAGE : RED;
    __shared__ __align__(16) unsigned char smem[SMEM];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = blockIdx.y;
    const long long V = L.voxels();
    const long long v0 = (long long)blockIdx.x * chunk_vox;
    const long long v1 = v0 + chunk_vox < V ? v0 + chunk_vox : V;
    const long long to = tap_off(L, t);
    uint16_t* sG = reinterpret_cast<uint16_t*>(smem) + wave * kWgradStep * (COUT + CIN);
    uint16_t* sX = sG + kWgradStep * COUT;
    f32x4 acc[MT][NTc];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTc; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nsteps = (chunk_vox + kWgradStep - 1) / kWgradStep;
    const int kq = lane >> 4, col = lane & 15;
    for (int s0 = 0; s0 < nsteps; s0 += 4) {
        const long long vs = v0 + (long long)(s0 + wave) * kWgradStep;
        for (int e = lane; e < kWgradStep * (COUT / 8); e += 64) {
            const int vi = e / (COUT / 8), cb = (e % (COUT / 8)) * 8;
            const long long v = vs + vi;
            uint4 val{0u, 0u, 0u, 0u};
            if (v < v1) val = *reinterpret_cast<const uint4*>(g + voxel_off(L, v) * COUT + cb);
            *reinterpret_cast<uint4*>(sG + vi * COUT + cb) = val;
        }
        for (int e = lane; e < kWgradStep * (CIN / 8); e += 64) {
            const int vi = e / (CIN / 8), cb = (e % (CIN / 8)) * 8;
            const long long v = vs + vi;
            uint4 val{0u, 0u, 0u, 0u};
            if (v < v1) val = *reinterpret_cast<const uint4*>(in + (voxel_off(L, v) + to) * CIN + cb);
            *reinterpret_cast<uint4*>(sX + vi * CIN + cb) = val;
        }
        __syncthreads();
        bf16x8 av[MT], bv[NTc];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            av[mt] = gather8(sG + kq * 8 * COUT + mt * 16 + col, COUT);
#pragma unroll
        for (int nt = 0; nt < NTc; ++nt)
            bv[nt] = gather8(sX + kq * 8 * CIN + nt * 16 + col, CIN);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NTc; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
        __syncthreads();
    }
    // D[co = mt*16 + 4 kq + i][ci = nt*16 + col]; waves add in order 0..3
    float* red = reinterpret_cast<float*>(smem);
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NTc; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int co = mt * 16 + kq * 4 + i, ci = nt * 16 + col;
                        float& r = red[co * CIN + ci];
                        r = (w == 0) ? acc[mt][nt][i] : r + acc[mt][nt][i];
                    }
        }
        __syncthreads();
    }
    float* dst = part + ((long long)blockIdx.x * 27 + t) * COUT * CIN;
    for (int e = threadIdx.x; e < COUT * CIN; e += CT) dst[e] = red[e];
}

__global__ void k_wgrad_reduce(int cin, int cout, int cout_real, const float* __restrict__ part,
                               int chunks, float* __restrict__ grad, float scale) {
    const long long n = (long long)cout_real * cin * 27;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e % 27);
        const long long oc = e / 27;
        const int ci = (int)(oc % cin), co = (int)(oc / cin);
        float s = 0.f;
        for (int c = 0; c < chunks; ++c) s += part[(((long long)c * 27 + t) * cout + co) * cin + ci];
        grad[e] += scale * s;
    }
}

// ---------------------------------------------------------------------------
// level transfers (one thread per voxel and 8 channels)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool vox8(const Level& L, int C, long long e, int& x, int& y, int& z,
                                     int& cb) {
    const int nc = C / 8;
    if (e >= L.voxels() * nc) return false;
    cb = (int)(e % nc) * 8;
    long long v = e / nc;
    x = (int)(v % L.X);
    v /= L.X;
    y = (int)(v % L.Y);
    z = (int)(v / L.Y);
    return true;
}

__global__ void k_pool(const uint16_t* __restrict__ fine, uint16_t* __restrict__ coarse, Level Lc,
                       int C, const int* skip) {
    if (skip && *skip) return;
    int x, y, z, cb;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (!vox8(Lc, C, e, x, y, z, cb)) return;
    const Level Lf{2 * Lc.X, 2 * Lc.Y, 2 * Lc.Z};
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < 8; ++c) {
        float f[8];
        unpack8(*reinterpret_cast<const uint4*>(
                    fine + Lf.off(2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + (c >> 2)) * C + cb),
                f);
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] += f[i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] *= 0.125f;
    *reinterpret_cast<uint4*>(coarse + Lc.off(x, y, z) * C + cb) = pack8(s);
}

__global__ void k_upadd(const uint16_t* __restrict__ coarse, const uint16_t* __restrict__ skipt,
                        uint16_t* __restrict__ fine, Level Lf, int C, const int* skip) {
    if (skip && *skip) return;
    int x, y, z, cb;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (!vox8(Lf, C, e, x, y, z, cb)) return;
    const Level Lc{Lf.X / 2, Lf.Y / 2, Lf.Z / 2};
    float a[8], b[8];
    unpack8(*reinterpret_cast<const uint4*>(coarse + Lc.off(x / 2, y / 2, z / 2) * C + cb), a);
    const long long o = Lf.off(x, y, z) * C + cb;
    unpack8(*reinterpret_cast<const uint4*>(skipt + o), b);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] += b[i];
    *reinterpret_cast<uint4*>(fine + o) = pack8(a);
}

__global__ void k_summask(const uint16_t* __restrict__ fine, const uint16_t* __restrict__ mask,
                          uint16_t* __restrict__ coarse, Level Lc, int C) {
    int x, y, z, cb;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (!vox8(Lc, C, e, x, y, z, cb)) return;
    const Level Lf{2 * Lc.X, 2 * Lc.Y, 2 * Lc.Z};
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < 8; ++c) {
        float f[8];
        unpack8(*reinterpret_cast<const uint4*>(
                    fine + Lf.off(2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + (c >> 2)) * C + cb),
                f);
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] += f[i];
    }
    const long long o = Lc.off(x, y, z) * C + cb;
    float m[8];
    unpack8(*reinterpret_cast<const uint4*>(mask + o), m);
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = m[i] > 0.f ? s[i] : 0.f;
    *reinterpret_cast<uint4*>(coarse + o) = pack8(s);
}

__global__ void k_upaddmask(const uint16_t* __restrict__ gskip, const uint16_t* __restrict__ gcoarse,
                            const uint16_t* __restrict__ mask, uint16_t* __restrict__ fine, Level Lf,
                            int C) {
    int x, y, z, cb;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (!vox8(Lf, C, e, x, y, z, cb)) return;
    const Level Lc{Lf.X / 2, Lf.Y / 2, Lf.Z / 2};
    float a[8], b[8], m[8];
    const long long o = Lf.off(x, y, z) * C + cb;
    unpack8(*reinterpret_cast<const uint4*>(gskip + o), a);
    unpack8(*reinterpret_cast<const uint4*>(gcoarse + Lc.off(x / 2, y / 2, z / 2) * C + cb), b);
    unpack8(*reinterpret_cast<const uint4*>(mask + o), m);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = m[i] > 0.f ? a[i] + b[i] * 0.125f : 0.f;
    *reinterpret_cast<uint4*>(fine + o) = pack8(a);
}

// ---------------------------------------------------------------------------
// weights and Adam
// ---------------------------------------------------------------------------
__global__ void k_prep_weights(const float* __restrict__ w, uint16_t* __restrict__ wf,
                               uint16_t* __restrict__ wd, int cin, int cout) {
    const int coutp = pad16(cout);
    const int kpf = conv_kp(cin), kpd = conv_kp(coutp);
    const long long nf = (long long)coutp * kpf, nd = (long long)cin * kpd;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nf + nd;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < nf) {
            const int co = (int)(e / kpf), K = (int)(e % kpf);
            const int t = K / cin, ci = K % cin;
            float v = 0.f;
            if (co < cout && t < 27) v = w[((long long)co * cin + ci) * 27 + t];
            wf[e] = (uint16_t)f2bf(v);
        } else {
            const long long d = e - nf;
            const int ci = (int)(d / kpd), K = (int)(d % kpd);
            const int t = K / coutp, co = K % coutp;
            float v = 0.f;
            if (co < cout && t < 27) v = w[((long long)co * cin + ci) * 27 + (26 - t)];
            wd[d] = (uint16_t)f2bf(v);
        }
    }
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2, float gscale) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const float gi = g[e] * gscale;
        const float mi = b1 * m[e] + (1.f - b1) * gi;
        const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
        m[e] = mi;
        v[e] = vi;
        w[e] = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// ---------------------------------------------------------------------------
// solver context <-> network tensors
// ---------------------------------------------------------------------------
__global__ void k_net_scale(const double* __restrict__ part, int nb, const Scalars* sc,
                            double* scale) {
    double tot[2];
    reduce_partials<2, CT>(part, nb, tot);
    if (threadIdx.x == 0) {
        const double n = (double)sc->n_active;
        *scale = (tot[0] > 0.0 && isfinite(tot[0])) ? sqrt(n / tot[0]) : 0.0;
    }
}

// sample set q of 3D: p, txx, tyy at cells; txy z-edges; txz y-edges; tyz x-edges
__device__ __forceinline__ bool sample_exists(const Geo& g, int q, int x, int y, int z) {
    const int sx = (q < 3 || q == 5) ? 1 : 0;
    const int sy = (q < 3 || q == 4) ? 1 : 0;
    const int sz = (q < 3 || q == 3) ? 1 : 0;
    return x <= g.nx - sx && y <= g.ny - sy && z <= g.nz - sz;
}

__global__ void k_net_geometry(Geo g, Level L0, const double* __restrict__ WL,
                               const double* __restrict__ WF, const double* __restrict__ rho,
                               const double* __restrict__ mu, double dt, uint16_t* __restrict__ x) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long long)g.nx * g.ny));
    const long long o = g.idx(i, j, k);
    const double lam = log10(1.0 + dt * mu[o] / (rho[o] * g.h * g.h)) / 6.0;
    float f[8] = {(float)WL[o], (float)WF[o], (float)lam, 0.f, 0.f, 0.f, 0.f, 0.f};
    *reinterpret_cast<uint4*>(x + L0.off(i, j, k) * kNetIn + kGeoChannel) = pack8(f);
}

template <typename T>
__global__ void k_net_pack(Geo g, Level L0, const T* __restrict__ r, const T* __restrict__ dinv,
                           const double* __restrict__ scale, uint16_t* __restrict__ x,
                           const int* skip) {
    if (skip && *skip) return;
    const long long n = (long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int i = (int)(e % (g.nx + 1)), j = (int)((e / (g.nx + 1)) % (g.ny + 1));
    const int k = (int)(e / ((long long)(g.nx + 1) * (g.ny + 1)));
    const long long o = g.idx(i, j, k);
    const float s = (float)*scale;
    float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!sample_exists(g, q, i, j, k)) continue;
        const long long os = o + q * g.NP;
        const float d = (float)dinv[os];
        f[q] = d > 0.f ? s * sqrtf(d) * (float)r[os] : 0.f;
    }
    *reinterpret_cast<uint4*>(x + L0.off(i, j, k) * kNetIn) = pack8(f);
}

constexpr int kVecBlocks = 1024;

int grid_for(long long n) {
    return (int)std::max<long long>(1, std::min<long long>(kVecBlocks, (n + CT - 1) / CT));
}

// Only the anchors of the active tiles are visited (one 64-wide row of anchors
// per wave, all six sample sets of each anchor): every sample outside them has
// D^-1 = 0, and z there keeps the zero the work space was cleared to.
__global__ __launch_bounds__(CT) void k_net_unpack(Geo g, Tiles tl, Level L0,
                                                   const float* __restrict__ y32,
                                                   const float* __restrict__ dinv,
                                                   const double* __restrict__ scale,
                                                   const float* __restrict__ r,
                                                   const float* __restrict__ q,
                                                   float* __restrict__ z,
                                                   double* __restrict__ part, const int* skip) {
    if (skip && *skip) return;
    const double sd = *scale;
    const float inv = sd > 0.0 ? (float)(1.0 / sd) : 0.f;
    double zr = 0.0, zq = 0.0, rdq = 0.0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long long rows = (long long)tl.count * kTile3Y * kTile3Z;
    for (long long u = (long long)blockIdx.x * (CT / 64) + wv; u < rows;
         u += (long long)gridDim.x * (CT / 64)) {
        bool ok;
        const long long o = tile_row_offset(g, tl, u, lane, 1, ok);
        if (!ok) continue;
        const int id = tl.list[u / (kTile3Y * kTile3Z)];
        const int rem = (int)(u % (kTile3Y * kTile3Z));
        const int i = (id % tl.ntx) * kTile3X + lane;
        const int j = ((id / tl.ntx) % tl.nty) * kTile3Y + rem / kTile3Z;
        const int k = (id / (tl.ntx * tl.nty)) * kTile3Z + rem % kTile3Z;
        const long long v = ((long long)k * L0.Y + j) * L0.X + i;
        const float4 ya = *reinterpret_cast<const float4*>(y32 + v * 8);
        const float4 yb = *reinterpret_cast<const float4*>(y32 + v * 8 + 4);
        const float yv[6] = {ya.x, ya.y, ya.z, ya.w, yb.x, yb.y};
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            if (!sample_exists(g, s, i, j, k)) continue;
            const long long os = o + s * g.NP;
            const float d = dinv[os];
            const float zi = d > 0.f ? sqrtf(d) * yv[s] * inv : 0.f;
            z[os] = zi;
            if (part) {
                const float ri = r[os], qi = q[os];
                zr += (double)zi * (double)ri;
                zq += (double)zi * (double)qi;
                rdq += (double)ri * (double)d * (double)qi;
            }
        }
    }
    if (part) {
        double vv[3] = {zr, zq, rdq};
        block_partial<3, CT>(vv, part, gridDim.x, blockIdx.x);
    }
}

__global__ __launch_bounds__(CT) void k_train_dots(long long n, const float* __restrict__ f,
                                                   const float* __restrict__ q,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ e,
                                                   double* __restrict__ part) {
    double a = 0.0, b = 0.0, E = 0.0;
    for (long long t = blockIdx.x * (long long)CT + threadIdx.x; t < n;
         t += (long long)gridDim.x * CT) {
        const double fi = f[t], ri = r[t];
        a += fi * ri;
        b += fi * (double)q[t];
        E += e[t] * ri;
    }
    double vv[3] = {a, b, E};
    block_partial<3, CT>(vv, part, gridDim.x, blockIdx.x);
}

__global__ __launch_bounds__(CT) void k_train_grad(Geo g, Level L0, const double* __restrict__ part,
                                                   int nb, const float* __restrict__ q,
                                                   const double* __restrict__ r,
                                                   const float* __restrict__ dinv,
                                                   const double* __restrict__ scale,
                                                   uint16_t* __restrict__ gy, double* loss) {
    double tot[3];
    reduce_partials<3, CT>(part, nb, tot);
    const double a = tot[0], b = tot[1], E = tot[2];
    const bool ok = b > 0.0 && E > 0.0 && isfinite(a) && isfinite(b) && isfinite(E);
    const double L = ok ? 1.0 - a * a / (b * E) : 1.0;
    const double c1 = ok ? 2.0 * a / (b * E) : 0.0, c2 = ok ? a / b : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        loss[0] = L;
        loss[1] = a;
        loss[2] = b;
        loss[3] = E;
    }
    const double sd = *scale;
    const double inv = sd > 0.0 ? 1.0 / sd : 0.0;
    const long long n = (long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    for (long long e = blockIdx.x * (long long)CT + threadIdx.x; e < n;
         e += (long long)gridDim.x * CT) {
        const int i = (int)(e % (g.nx + 1)), j = (int)((e / (g.nx + 1)) % (g.ny + 1));
        const int k = (int)(e / ((long long)(g.nx + 1) * (g.ny + 1)));
        const long long o = g.idx(i, j, k);
        float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            if (!sample_exists(g, s, i, j, k)) continue;
            const long long os = o + s * g.NP;
            const double d = dinv[os];
            if (d > 0.0) f[s] = (float)(sqrt(d) * inv * c1 * (c2 * (double)q[os] - r[os]));
        }
        uint16_t* dst = gy + L0.off(i, j, k) * 16;
        *reinterpret_cast<uint4*>(dst) = pack8(f);
    }
}

// ---------------------------------------------------------------------------
// dense FP32 tensors at the boundary <-> halo BF16 tensors
// ---------------------------------------------------------------------------
__global__ void k_check_f32(const float* __restrict__ v, long long n, int* flag) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        if (!isfinite(v[e])) *flag = 1;
}

// dense [V][cd] FP32 -> halo [..][16] BF16 (channels >= cd are zero)
__global__ void k_import16(const float* __restrict__ src, int cd, Level L, uint16_t* __restrict__ dst) {
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= L.voxels()) return;
    float a[8], b[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        a[c] = c < cd ? src[v * cd + c] : 0.f;
        b[c] = c + 8 < cd ? src[v * cd + c + 8] : 0.f;
    }
    uint16_t* d = dst + voxel_off(L, v) * 16;
    *reinterpret_cast<uint4*>(d) = pack8(a);
    *reinterpret_cast<uint4*>(d + 8) = pack8(b);
}

// dense [V][8] FP32 -> dense [V][6]
__global__ void k_export6(const float* __restrict__ y32, long long V, float* __restrict__ dst) {
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= V) return;
#pragma unroll
    for (int c = 0; c < 6; ++c) dst[v * 6 + c] = y32[v * 8 + c];
}

__global__ void k_f32_to_f64(const float* __restrict__ src, double* __restrict__ dst, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        dst[e] = (double)src[e];
}

// partials of (r.D^-1 r, r.r) over n padded samples
__global__ __launch_bounds__(CT) void k_net_rdr(long long n, const float* __restrict__ r,
                                                const float* __restrict__ dinv,
                                                double* __restrict__ part) {
    double a = 0.0, b = 0.0;
    for (long long t = blockIdx.x * (long long)CT + threadIdx.x; t < n;
         t += (long long)gridDim.x * CT) {
        const double ri = r[t];
        a += ri * (double)dinv[t] * ri;
        b += ri * ri;
    }
    double vv[2] = {a, b};
    block_partial<2, CT>(vv, part, gridDim.x, blockIdx.x);
}

// ---------------------------------------------------------------------------
// two-level preconditioner step (FP32 vectors over the padded samples):
//   d = D^-1 r and A d come from a MODE_JDIR apply; a1 = r.d / d.A d;
//   r1 = r - a1 A d (input of the network); n = network(r1); A n from a
//   second MODE_JDIR apply; w = n.r1 / n.A n; z = a1 d + w n.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double safe_ratio(double num, double den) {
    const double v = (den > 0.0 && isfinite(den) && isfinite(num)) ? num / den : 0.0;
    return isfinite(v) ? v : 0.0;
}

// a1 from (r.D^-1 r, .) partials and (d.Ad) partials; r1 = r - a1 qd;
// partials (r1.D^-1 r1, 0); coef[0] = a1.  Optionally also the FP64 pair
// r64 -= a1 qd, e64 -= a1 d (training).
__global__ __launch_bounds__(CT) void k_coarse_prep(Geo g, Tiles tl, const float* __restrict__ r,
                                                    const float* __restrict__ qd,
                                                    const float* __restrict__ dinv,
                                                    const double* __restrict__ part_rdr, int nb_rdr,
                                                    const double* __restrict__ part_dq, int nb_dq,
                                                    float* __restrict__ r1, double* __restrict__ part,
                                                    double* coef, const float* __restrict__ d,
                                                    double* __restrict__ r64,
                                                    double* __restrict__ e64, const int* skip) {
    if (skip && *skip) return;
    double t2[2], t1[1];
    reduce_partials<2, CT>(part_rdr, nb_rdr, t2);
    reduce_partials<1, CT>(part_dq, nb_dq, t1);
    const double a1d = safe_ratio(t2[0], t1[0]);
    const float a1 = (float)a1d;
    if (blockIdx.x == 0 && threadIdx.x == 0) coef[0] = a1d;
    double acc = 0.0;
    // only the positions of the active tiles: elsewhere every input is zero
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long long rows = (long long)tl.count * g.nsamp() * kTile3Y * kTile3Z;
    for (long long u = (long long)blockIdx.x * (CT / 64) + wv; u < rows;
         u += (long long)gridDim.x * (CT / 64)) {
        bool ok;
        const long long t = tile_row_offset(g, tl, u, lane, g.nsamp(), ok);
        if (!ok) continue;
        const float v = r[t] - a1 * qd[t];
        r1[t] = v;
        acc += (double)v * (double)dinv[t] * (double)v;
        if (r64) {
            r64[t] -= a1d * (double)qd[t];
            e64[t] -= a1d * (double)d[t];
        }
    }
    double vv[2] = {acc, 0.0};
    block_partial<2, CT>(vv, part, gridDim.x, blockIdx.x);
}

// w from (n.r1, ., .) and (n.An) partials; z = a1 d + w n; partials of
// (z.r, then z.Q_i and r.D^-1 Q_i for the previous directions of truncated
// flexible CG, zero past fh.mk); coef[1] = w.
__global__ __launch_bounds__(CT) void k_coarse_finish(Geo g, Tiles tl, const float* __restrict__ d,
                                                      const float* __restrict__ nv,
                                                      const float* __restrict__ r,
                                                      const float* __restrict__ dinv,
                                                      double* coef,
                                                      const double* __restrict__ part_nr, int nb_nr,
                                                      const double* __restrict__ part_nq, int nb_nq,
                                                      FcgHist fh, float* __restrict__ z,
                                                      double* __restrict__ part, const int* skip) {
    if (skip && *skip) return;
    double t3[3], t1[1];
    reduce_partials<3, CT>(part_nr, nb_nr, t3);
    reduce_partials<1, CT>(part_nq, nb_nq, t1);
    const double wd = safe_ratio(t3[0], t1[0]);
    const float w = (float)wd, a1 = (float)coef[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) coef[1] = wd;
    constexpr int NV = 1 + 2 * kFcgMax;
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    const int mk = fh.mk;
    // only the positions of the active tiles: elsewhere every input is zero
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long long rows = (long long)tl.count * g.nsamp() * kTile3Y * kTile3Z;
    for (long long u = (long long)blockIdx.x * (CT / 64) + wv; u < rows;
         u += (long long)gridDim.x * (CT / 64)) {
        bool ok;
        const long long t = tile_row_offset(g, tl, u, lane, g.nsamp(), ok);
        if (!ok) continue;
        const float zi = a1 * d[t] + w * nv[t];
        z[t] = zi;
        const double ri = r[t], rd = ri * (double)dinv[t];
        acc[0] += (double)zi * ri;
#pragma unroll
        for (int i = 0; i < kFcgMax; ++i) {
            if (i < mk) {
                const double qi = static_cast<const float*>(fh.Q[i])[t];
                acc[1 + 2 * i] += (double)zi * qi;
                acc[2 + 2 * i] += rd * qi;
            }
        }
    }
    block_partial<NV, CT>(acc, part, gridDim.x, blockIdx.x);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
bool launch_conv3(int cin, int cout, int epi, const ConvArgs& a, hipStream_t s) {
#define VFS_CONV(CI, CO)                                                          \
    if (cin == CI && cout == CO) {                                                \
        switch (epi) {                                                            \
            case EPI_RELU: conv_launch<CI, CO, EPI_RELU>(a, s); return true;      \
            case EPI_PLAIN: conv_launch<CI, CO, EPI_PLAIN>(a, s); return true;    \
            case EPI_MASK: conv_launch<CI, CO, EPI_MASK>(a, s); return true;      \
            case EPI_F32: conv_launch<CI, CO, EPI_F32>(a, s); return true;        \
        }                                                                         \
        return false;                                                             \
    }
#define VFS_CONVZ(CI, CO, ZY)                                                         \
    if (cin == CI && cout == CO) {                                                     \
        switch (epi) {                                                                 \
            case EPI_RELU: conv_launch_z<CI, CO, ZY, EPI_RELU>(a, s); return true;     \
            case EPI_PLAIN: conv_launch_z<CI, CO, ZY, EPI_PLAIN>(a, s); return true;   \
            case EPI_MASK: conv_launch_z<CI, CO, ZY, EPI_MASK>(a, s); return true;     \
            case EPI_F32: conv_launch_z<CI, CO, ZY, EPI_F32>(a, s); return true;       \
        }                                                                              \
        return false;                                                                  \
    }
    VFS_CONVZ(16, 16, 8)
    VFS_CONVZ(16, 32, 8)
    VFS_CONVZ(32, 16, 4)
#undef VFS_CONVZ
    VFS_CONV(32, 64)
    VFS_CONV(64, 128)
    VFS_CONV(128, 64)
    VFS_CONV(64, 32)
#undef VFS_CONV
    return false;
}

int wgrad_chunks(const Level& L) {
    const long long V = L.voxels();
    return (int)std::max<long long>(1, std::min<long long>(512, (V + kWgradTarget - 1) / kWgradTarget));
}

static int wgrad_chunk_vox(const Level& L) {
    const long long V = L.voxels();
    const int c = wgrad_chunks(L);
    const long long per = (V + c - 1) / c;
    const long long q = 4 * kWgradStep;
    return (int)((per + q - 1) / q * q);
}

bool launch_wgrad(int cin, int cout, const uint16_t* in, const uint16_t* g, const Level& L,
                  float* part, const int* skip, hipStream_t s) {
    const dim3 grid(wgrad_chunks(L), 27);
    const int cv = wgrad_chunk_vox(L);
#define VFS_WG(CI, CO)                                                                       \
    if (cin == CI && cout == CO) {                                                           \
        hipLaunchKernelGGL((k_wgrad<CI, CO>), grid, dim3(CT), 0, s, in, g, L, part, cv, skip); \
        return true;                                                                         \
    }
    VFS_WG(16, 16)
    VFS_WG(32, 16)
    VFS_WG(64, 32)
    VFS_WG(128, 64)
    VFS_WG(64, 128)
    VFS_WG(32, 64)
    VFS_WG(16, 32)
#undef VFS_WG
    return false;
}

void launch_wgrad_reduce(int cin, int cout, int cout_real, const float* part, int chunks,
                         float* grad, float scale, hipStream_t s) {
    const long long n = (long long)cout_real * cin * 27;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid_for(n)), dim3(CT), 0, s, cin, cout, cout_real, part,
                       chunks, grad, scale);
}

static unsigned blocks8(const Level& L, int C) {
    return (unsigned)((L.voxels() * (C / 8) + CT - 1) / CT);
}

void launch_pool(const uint16_t* fine, uint16_t* coarse, const Level& Lc, int C, const int* skip,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_pool, dim3(blocks8(Lc, C)), dim3(CT), 0, s, fine, coarse, Lc, C, skip);
}

void launch_upadd(const uint16_t* coarse, const uint16_t* skipt, uint16_t* fine, const Level& Lf,
                  int C, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_upadd, dim3(blocks8(Lf, C)), dim3(CT), 0, s, coarse, skipt, fine, Lf, C,
                       skip);
}

void launch_summask(const uint16_t* fine, const uint16_t* mask, uint16_t* coarse, const Level& Lc,
                    int C, hipStream_t s) {
    hipLaunchKernelGGL(k_summask, dim3(blocks8(Lc, C)), dim3(CT), 0, s, fine, mask, coarse, Lc, C);
}

void launch_upaddmask(const uint16_t* gskip, const uint16_t* gcoarse, const uint16_t* mask,
                      uint16_t* fine, const Level& Lf, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_upaddmask, dim3(blocks8(Lf, C)), dim3(CT), 0, s, gskip, gcoarse, mask, fine,
                       Lf, C);
}

void launch_prep_weights(const float* canon, uint16_t* wf, uint16_t* wd, int cin, int cout,
                         hipStream_t s) {
    const long long n = (long long)pad16(cout) * conv_kp(cin) + (long long)cin * conv_kp(pad16(cout));
    hipLaunchKernelGGL(k_prep_weights, dim3(grid_for(n)), dim3(CT), 0, s, canon, wf, wd, cin, cout);
}

void launch_adam(float* w, float* m, float* v, const float* g, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, float gscale, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(CT), 0, s, w, m, v, g, n, lr, b1, b2, eps, c1,
                       c2, gscale);
}

void launch_net_scale(const double* part, int nb, const Scalars* sc, double* scale,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_net_scale, dim3(1), dim3(CT), 0, s, part, nb, sc, scale);
}

void launch_net_geometry(const Geo& g, const Level& L0, const double* WL, const double* WF,
                         const double* rho, const double* mu, double dt, uint16_t* x,
                         hipStream_t s) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_net_geometry, dim3((unsigned)((n + CT - 1) / CT)), dim3(CT), 0, s, g, L0, WL,
                       WF, rho, mu, dt, x);
}

template <typename T>
void launch_net_pack(const Geo& g, const Level& L0, const T* r, const T* dinv, const double* scale,
                     uint16_t* x, const int* skip, hipStream_t s) {
    const long long n = (long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    hipLaunchKernelGGL((k_net_pack<T>), dim3((unsigned)((n + CT - 1) / CT)), dim3(CT), 0, s, g, L0, r,
                       dinv, scale, x, skip);
}
template void launch_net_pack<float>(const Geo&, const Level&, const float*, const float*,
                                     const double*, uint16_t*, const int*, hipStream_t);

int net_unpack_blocks(const Geo& g) {
    return grid_for((long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1));
}

void launch_net_unpack(const Geo& g, const Tiles& tl, const Level& L0, const float* y32,
                       const float* dinv, const double* scale, const float* r, const float* q,
                       float* z, double* part, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_net_unpack, dim3(net_unpack_blocks(g)), dim3(CT), 0, s, g, tl, L0, y32,
                       dinv, scale, r, q, z, part, skip);
}

int train_dot_blocks(const Geo& g) { return grid_for((long long)g.nsamp() * g.NP); }

void launch_train_dots(const Geo& g, const float* f, const float* q, const double* r,
                       const double* e, double* part, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_train_dots, dim3(nb), dim3(CT), 0, s, (long long)g.nsamp() * g.NP, f, q, r, e,
                       part);
}

void launch_train_grad(const Geo& g, const Level& L0, const double* part, int nb,
                       const float* q, const double* r, const float* dinv, const double* scale,
                       uint16_t* gy, double* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_train_grad, dim3(net_unpack_blocks(g)), dim3(CT), 0, s, g, L0, part, nb, q, r,
                       dinv, scale, gy, loss);
}

void launch_check_f32(const float* v, long long n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_f32, dim3(grid_for(n)), dim3(CT), 0, s, v, n, flag);
}

void launch_import16(const float* src, int cd, const Level& L, uint16_t* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_import16, dim3((unsigned)((L.voxels() + CT - 1) / CT)), dim3(CT), 0, s, src,
                       cd, L, dst);
}

void launch_export6(const float* y32, long long V, float* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_export6, dim3((unsigned)((V + CT - 1) / CT)), dim3(CT), 0, s, y32, V, dst);
}

void launch_f32_to_f64(const float* src, double* dst, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(CT), 0, s, src, dst, n);
}

int net_rdr_blocks(const Geo& g) { return grid_for((long long)g.nsamp() * g.NP); }

void launch_net_rdr(const Geo& g, const float* r, const float* dinv, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_net_rdr, dim3(net_rdr_blocks(g)), dim3(CT), 0, s,
                       (long long)g.nsamp() * g.NP, r, dinv, part);
}

int coarse_blocks(const Geo& g) { return grid_for((long long)g.nsamp() * g.NP); }

void launch_coarse_prep(const Geo& g, const Tiles& tl, const float* r, const float* qd,
                        const float* dinv, const double* part_rdr, int nb_rdr,
                        const double* part_dq, int nb_dq, float* r1, double* part, double* coef,
                        const float* d, double* r64, double* e64, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_prep, dim3(coarse_blocks(g)), dim3(CT), 0, s, g, tl, r, qd, dinv,
                       part_rdr, nb_rdr, part_dq, nb_dq, r1, part, coef, d, r64, e64, skip);
}

void launch_coarse_finish(const Geo& g, const Tiles& tl, const float* d, const float* nv,
                          const float* r, const float* dinv, double* coef, const double* part_nr,
                          int nb_nr, const double* part_nq, int nb_nq, const FcgHist& fh,
                          float* z, double* part, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_finish, dim3(coarse_blocks(g)), dim3(CT), 0, s, g, tl, d, nv, r,
                       dinv, coef, part_nr, nb_nr, part_nq, nb_nq, fh, z, part, skip);
}

}  // namespace vfs
