// Learned preconditioner network (U-Net style, 3D, BF16 on MFMA): layer
// table, tensor geometry and launchers shared by k_unet.hip and
// vfs_unet.hip.
//
// Tensors are channels-last BF16 with a one-voxel zero halo:
//   element (z, y, x, c) of a level with interior extents (Z, Y, X) and C
//   channels lives at ((z+1)*(Y+2) + (y+1))*(X+2) + (x+1)) * C + c.
// The halo is zeroed once at allocation and never written, so 3x3x3 taps
// need no bounds tests.  Level l has extents (Z0, Y0, X0) >> l; level 0 has
// extents roundup(n + 1, 8) per axis so that every sample of every set of
// a grid of n cells has a voxel and three 2x2x2 poolings divide evenly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "vfs_internal.h"

namespace vfs {

struct NetLayer {
    int cin, cout, level, relu;
};
// enc0..enc3, bottleneck, dec2..dec0 (additive skips, one conv per stage)
constexpr int kNetLayers = 8;
constexpr NetLayer kNet[kNetLayers] = {{16, 16, 0, 1},  {16, 32, 1, 1}, {32, 64, 2, 1},
                                       {64, 128, 3, 1}, {128, 64, 3, 1}, {64, 32, 2, 1},
                                       {32, 16, 1, 1},  {16, 6, 0, 0}};
constexpr int kNetIn = 16;    // input channels: 6 residual sets, 2 zero, 3 geometry, 5 zero
constexpr int kNetOut = 6;    // output channels (one per 3D sample set)
constexpr int kGeoChannel = 8;

__host__ __device__ constexpr int pad16(int c) { return c < 16 ? 16 : (c + 15) / 16 * 16; }
__host__ __device__ constexpr int conv_kp(int cin) { return (27 * cin + 31) / 32 * 32; }

struct Level {
    int X, Y, Z;   // interior extents
    __host__ __device__ long long voxels() const { return (long long)X * Y * Z; }
    __host__ __device__ long long padded() const {
        return (long long)(X + 2) * (Y + 2) * (Z + 2);
    }
    __host__ __device__ long long off(int x, int y, int z) const {
        return ((long long)(z + 1) * (Y + 2) + (y + 1)) * (X + 2) + (x + 1);
    }
};

enum ConvEpi : int {
    EPI_RELU = 0,    // out = bf16(max(acc, 0))
    EPI_PLAIN = 1,   // out = bf16(acc)
    EPI_MASK = 2,    // out = bf16(acc * [mask > 0])
    EPI_F32 = 3,     // out32[v * 8 + c] = acc for c < 8 (dense, no halo)
};

struct ConvArgs {
    const uint16_t* in;      // halo tensor, CIN channels
    const uint16_t* w;       // [COUTp][KP(CIN)] bf16
    uint16_t* out;           // halo tensor, COUT channels (bf16 epilogues)
    float* out32;            // dense [voxels][8] (EPI_F32)
    const uint16_t* mask;    // halo tensor, COUT channels (EPI_MASK)
    Level L;
    const int* skip;         // if set and *skip != 0 the launch does nothing
};

// out = conv3(in) with the given epilogue; (cin, cout) must be a pair the
// network uses (forward or input-gradient), else returns false.
bool launch_conv3(int cin, int cout, int epi, const ConvArgs& a, hipStream_t s);

// Weight gradient partials: part[chunk][t][cout][cin] = sum over the chunk's
// voxels of g[v][co] * in[v + off_t][ci]; then reduced in chunk order into
// grad (canonical [co][ci][t] layout, first cout_real rows) scaled by scale.
int wgrad_chunks(const Level& L);
bool launch_wgrad(int cin, int cout, const uint16_t* in, const uint16_t* g, const Level& L,
                  float* part, const int* skip, hipStream_t s);
void launch_wgrad_reduce(int cin, int cout, int cout_real, const float* part, int chunks,
                         float* grad, float scale, hipStream_t s);

// elementwise level transfers (C channels, C % 8 == 0)
void launch_pool(const uint16_t* fine, uint16_t* coarse, const Level& Lc, int C, const int* skip,
                 hipStream_t s);
void launch_upadd(const uint16_t* coarse, const uint16_t* skipt, uint16_t* fine, const Level& Lf,
                  int C, const int* skip, hipStream_t s);
void launch_summask(const uint16_t* fine, const uint16_t* mask, uint16_t* coarse,
                    const Level& Lc, int C, hipStream_t s);
void launch_upaddmask(const uint16_t* gskip, const uint16_t* gcoarse, const uint16_t* mask,
                      uint16_t* fine, const Level& Lf, int C, hipStream_t s);

// weights: canonical FP32 [co][ci][27] per layer -> BF16 forward [COUTp][KP(cin)] and
// input-gradient [cin][KP(COUTp)] (taps reversed, co/ci swapped)
void launch_prep_weights(const float* canon, uint16_t* wf, uint16_t* wd, int cin, int cout,
                         hipStream_t s);
// Adam on n FP32 parameters; c1 = 1 - b1^t, c2 = 1 - b2^t
void launch_adam(float* w, float* m, float* v, const float* g, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, float gscale, hipStream_t s);

// ---- coupling to a 3D solver context (padded sample layout, FP32) ----
// scale s = sqrt(n_active / sum(partials[0])) from nb two-value partials
// (r.D^-1 r, r.r) -> *scale (0 if the sum is not positive).
void launch_net_scale(const double* part, int nb, const Scalars* sc, double* scale,
                      hipStream_t s);
// channels 8..10 of the input tensor: W_L, W_F and log10(1 + dt mu / (rho h^2)) / 6 at cells
void launch_net_geometry(const Geo& g, const Level& L0, const double* WL, const double* WF,
                         const double* rho, const double* mu, double dt, uint16_t* x,
                         hipStream_t s);
// channels 0..5: s * sqrt(D^-1) r of each sample set; 6, 7 zero
template <typename T>
void launch_net_pack(const Geo& g, const Level& L0, const T* r, const T* dinv, const double* scale,
                     uint16_t* x, const int* skip, hipStream_t s);
// z = sqrt(D^-1) y / s on the samples of the active tiles (0 where D^-1 = 0 or
// s = 0; z elsewhere is left as it is, zero in the cleared work space); with
// partials: (z.r, z.q, r.D^-1 q) per workgroup -> part (nb = returned count)
int net_unpack_blocks(const Geo& g);
void launch_net_unpack(const Geo& g, const Tiles& tl, const Level& L0, const float* y32,
                       const float* dinv, const double* scale, const float* r, const float* q,
                       float* z, double* part, const int* skip, hipStream_t s);
// training: partials of (f.r, f.q, e.r) then the loss gradient pushed back to the
// network output: gy = P^T sqrt(D^-1) dL/df / s (bf16, 16 channels)
void launch_train_dots(const Geo& g, const float* f, const float* q, const double* r,
                       const double* e, double* part, int nb, hipStream_t s);
void launch_train_grad(const Geo& g, const Level& L0, const double* part, int nb,
                       const float* q, const double* r, const float* dinv, const double* scale,
                       uint16_t* gy, double* loss, hipStream_t s);
int train_dot_blocks(const Geo& g);

void launch_check_f32(const float* v, long long n, int* flag, hipStream_t s);
void launch_import16(const float* src, int cd, const Level& L, uint16_t* dst, hipStream_t s);
void launch_export6(const float* y32, long long V, float* dst, hipStream_t s);
// partials of (r.D^-1 r, r.r) over the padded samples (nb = net_rdr_blocks)
int net_rdr_blocks(const Geo& g);
void launch_net_rdr(const Geo& g, const float* r, const float* dinv, double* part, hipStream_t s);
void launch_f32_to_f64(const float* src, double* dst, long long n, hipStream_t s);

// Two-level preconditioner step (see k_unet.hip), over the positions of the
// active tiles tl (the other positions of every vector involved are zero).
// Partial counts of both kernels: coarse_blocks(g).
int coarse_blocks(const Geo& g);
void launch_coarse_prep(const Geo& g, const Tiles& tl, const float* r, const float* qd,
                        const float* dinv, const double* part_rdr, int nb_rdr,
                        const double* part_dq, int nb_dq, float* r1, double* part, double* coef,
                        const float* d, double* r64, double* e64, const int* skip, hipStream_t s);
void launch_coarse_finish(const Geo& g, const Tiles& tl, const float* d, const float* nv,
                          const float* r, const float* dinv, double* coef, const double* part_nr,
                          int nb_nr, const double* part_nq, int nb_nq, const FcgHist& fh,
                          float* z, double* part, const int* skip, hipStream_t s);

}  // namespace vfs

// The network object: FP32 master weights, Adam moments and gradient
// accumulator (canonical layout), their BF16 MFMA layouts, and activation /
// gradient tensors for one level-0 extent at a time.
struct vfs_unet {
    hipStream_t stream = nullptr;
    std::string err;
    long long nparam = 0;
    long long poff[vfs::kNetLayers + 1] = {};
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    uint16_t* wbuf = nullptr;
    uint16_t* wf[vfs::kNetLayers] = {};
    uint16_t* wd[vfs::kNetLayers] = {};
    int adam_t = 0;
    bool have_weights = false;
    int* flag = nullptr;         // device check flag
    int* flag_host = nullptr;    // pinned
    double* dscal = nullptr;     // device: [0] input scale, [1..4] loss, f.r, f.Af, e.r
    double* hscal = nullptr;     // pinned mirror
    double* dpart = nullptr;     // reduction partials (vfs::kMaxNetPartials x 3)
    // tensors of the current extent
    vfs::Level L[4] = {};
    unsigned char* fwd = nullptr;
    size_t fwd_cap = 0;
    bool fwd_ready = false;
    unsigned char* bwd = nullptr;
    size_t bwd_cap = 0;
    bool bwd_ready = false;
    uint16_t *x = nullptr, *c0 = nullptr, *p0 = nullptr, *c1 = nullptr, *p1 = nullptr,
             *c2 = nullptr, *p2 = nullptr, *c3 = nullptr, *d3 = nullptr, *s2 = nullptr,
             *d2 = nullptr, *s1 = nullptr, *d1 = nullptr, *s0 = nullptr;
    float* y32 = nullptr;
    uint16_t *gy = nullptr, *gs0 = nullptr, *gd1 = nullptr, *gs1 = nullptr, *gd2 = nullptr,
             *gs2 = nullptr, *gd3 = nullptr, *gc3 = nullptr, *gp2 = nullptr, *gc2 = nullptr,
             *gp1 = nullptr, *gc1 = nullptr, *gp0 = nullptr, *gc0 = nullptr;
    float* wpart = nullptr;
    bool fwd_valid = false;      // activations of the last forward are kept
    float* stage = nullptr;      // boundary staging (dense FP32 tensors)
    size_t stage_cap = 0;
};

namespace vfs {
constexpr int kMaxNetPartials = 1024;
// partial regions of a context's preconditioner work space, each room for
// kNetPartVals values x kNetPartCap workgroups
constexpr int kNetPartRegions = 5;
constexpr int kNetPartVals = 1 + 2 * kFcgMax;
constexpr int kNetPartCap = 1536;
// work-space vectors: d, A d, r1, n, A n, then the direction and image rings
// of truncated flexible CG (kFcgMax + 1 slots each)
constexpr int kNetVecs = 5 + 2 * (kFcgMax + 1);
// allocate the context's preconditioner work space (once)
int net_bufs(vfs_ctx* ctx);
// z (ctx->z32) = two-level preconditioner of the FP32 residual r; part_rdr:
// (r.D^-1 r, .) partials of r; fh: previous directions whose (z.Q_i,
// r.D^-1 Q_i) partials go with z.r to region 4 for flexible CG; skip:
// optional device flag.
int net_precond(vfs_unet* u, vfs_ctx* ctx, const float* r, const float* dinv, const float* a,
                const float* c, const float* K, const double* part_rdr, int nb_rdr,
                const FcgHist& fh, const int* skip);
inline double* net_region(vfs_ctx* ctx, int k) {
    return ctx->netpart + (long long)k * kNetPartVals * kNetPartCap;
}
inline float* net_vec(vfs_ctx* ctx, int k) {
    return ctx->netvec + (long long)k * ctx->g.nsamp() * ctx->g.NP;
}
// level-0 extents of the network tensor of a 3D grid
Level net_level0(const Geo& g);
// allocate / re-carve tensors for level-0 extents L0 (zeroing their halos)
int net_ensure(vfs_unet* u, const Level& L0, bool grads);
// forward pass x -> y32 (activations kept); skip: optional device flag
int net_forward(vfs_unet* u, hipStream_t s, const int* skip);
// solver coupling: tensors sized for ctx, geometry channels written
int net_prepare_ctx(vfs_unet* u, vfs_ctx* ctx);
}  // namespace vfs
