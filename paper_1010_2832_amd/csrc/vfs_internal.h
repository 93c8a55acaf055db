// Internal declarations of the vfstokes HIP library (gfx950).
//
// Device data layout ("padded grid"): every per-sample array of every type
// (cells, faces, nodes/edges) lives on the same padded 2D/3D array so that a
// thread anchored at logical index (i,j[,k]) finds every sample type anchored
// there at the same offset:
//   offset(i,j)   = FRONT + (j+1)*PX + i                   (2D)
//   offset(i,j,k) = FRONT + ((k+1)*PY + (j+1))*PX + i      (3D)
// PX >= nx+3 is rounded up to a multiple of 16 elements, PY = ny+3, PZ = nz+3.
// The ghost index -1 along x is the last (always zero) padding element of the
// previous row; along y/z it is a zero row/plane; FRONT (16 elements) holds
// the ghost of the very first row.  Elements outside a sample type's valid
// range stay zero for the lifetime of the array, so stencils never need a
// bounds test for reads at distance one.
//
// A multi-component quantity (all stress/pressure samples, all faces) is one
// allocation of S slices of NP elements; slice s starts at s*NP.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/vfstokes.h"

namespace vfs {

constexpr int kFront = 32;   // elements before the body (128-byte rows, see make_geo)
// 3D kernels run at most this many workgroups, each looping over tiles, so
// that the partial sums a consumer must read stay few.
constexpr int kMaxTileBlocks = 1536;
// 3D tile: 64 x 4 anchors in x, y, marching 8 planes in z
constexpr int kTile3X = 64, kTile3Y = 4, kTile3Z = 8;
// Work tile of the fused 3D CG iteration: kFused3X x kFused3Y anchors
// marching kFused3Z planes, one thread per anchor of a plane; in y and z a
// whole number of the tiles above, in x a part of one.  The row bits of the
// 3D solve (one byte per kFused3X-anchor row) share its x width.
#ifndef VFS_FUSED3_X
#define VFS_FUSED3_X 64
#endif
#ifndef VFS_FUSED3_Y
#define VFS_FUSED3_Y 4
#endif
#ifndef VFS_FUSED3_Z
#define VFS_FUSED3_Z 8
#endif
constexpr int kFused3X = VFS_FUSED3_X, kFused3Y = VFS_FUSED3_Y, kFused3Z = VFS_FUSED3_Z;
constexpr int kRow3X = kFused3X;
// Row bits of the 3D solve: one word per kRow3X-anchor row (x part, y, z);
// bit s (s < 6) is set if sample slice s has an active sample among the first
// kRow3X / 2 anchors of the row, bit 6 + s among the second half.  With rows
// that start on 128-byte lines, a half row of FP32 values is one line.
using RowBits = uint16_t;
static_assert(kTile3X % kFused3X == 0 && kFused3X >= 16 && kFused3Y % kTile3Y == 0 &&
                  kFused3Z % kTile3Z == 0 && kFused3X * kFused3Y <= 1024 &&
                  (kFused3X * kFused3Y) % 64 == 0,
              "a fused tile holds whole tiles in y, z and whole waves");

struct Geo {
    int dim;
    int nx, ny, nz;          // cells (nz = 1 in 2D)
    int PX, PY, PZ;          // padded extents (PZ = 1 in 2D)
    long long NP;            // elements of one padded array (incl. front/tail pads)
    double h;

    __host__ __device__ inline long long idx(int i, int j) const {
        return (long long)kFront + (long long)(j + 1) * PX + i;
    }
    __host__ __device__ inline long long idx(int i, int j, int k) const {
        return (long long)kFront + ((long long)(k + 1) * PY + (j + 1)) * PX + i;
    }
    // number of stress+pressure sample types and face types
    __host__ __device__ inline int nsamp() const { return dim == 2 ? 3 : 6; }
    __host__ __device__ inline int nface() const { return dim; }
    // number of weight sets: 2D cell,u,v,node; 3D cell,u,v,w,ez,ey,ex
    __host__ __device__ inline int nsets() const { return dim == 2 ? 4 : 7; }
};

Geo make_geo(int dim, int nx, int ny, int nz, double h);

// stagger of weight set s (1 = cell-centred along that axis): used for
// shapes of user-facing arrays.
void set_stagger(int dim, int set, int st[3]);
// weight set of sample slice s (p, txx, [tyy], txy, [txz, tyz])
int sample_set(int dim, int s);
// compact shape of a set
void set_shape(const Geo& g, int set, int shp[3]);

// Device scalars of one CG solve.  Written only by workgroup 0 of a kernel
// and read only by later kernels (r.z is double-buffered by iteration
// parity so that the kernel writing iteration k's value never overwrites the
// value of iteration k-1 that its other workgroups still read).
struct Scalars {
    double rz[2];       // r.z of iteration k in slot k&1
    double rr;          // r.r of the last checked iterate
    double bb;          // b.b of the system being solved
    double tol2;        // stop when rr <= tol2 * bb
    double pq;          // p.Ap of the last iteration
    double alpha, beta;
    double aux0, aux1;  // finalized norms (residual checks)
    double rz_prev_z;   // flexible CG: r_{k}.z_{k-1}
    int iter;           // iterations completed when done was set
    int max_iter;
    int done;           // 0 running, 1 converged, 2 max_iter, 3 breakdown
    int flexible;
    long long n_active;
    int fallbacks;      // flexible CG: iterations that used the Jacobi direction
    int pad[3];
    double pqh[8];      // p.Ap of iteration k in slot k & 7 (truncated flexible CG)
};

// Vectors of the fused CG iteration (one launch per iteration, 2D and 3D):
// x in place; r, p and q = A p double-buffered by launch parity.
struct FusedVecs {
    void* x;
    void* r[2];
    void* p[2];
    void* q[2];
};

// Truncated flexible CG: the m previous directions P_i and their images
// Q_i = A P_i (i = 1 most recent), mk of them valid.
constexpr int kFcgMax = 4;
struct FcgHist {
    const void* P[kFcgMax];
    const void* Q[kFcgMax];
    int mk;
};

// Partial-sum plumbing of one reduction-carrying launch.
struct RedArgs {
    Scalars* sc;
    const double* part_in;   // partials of the previous kernel
    int nb_in;               // how many workgroups wrote them
    double* part_out;        // this kernel's partials (one per workgroup)
    int kidx;                // CG iteration index within the current run
    int set_bb;              // first iteration of a fresh solve: bb := r.r
    const double* part_in2;  // flexible CG: (r.D^-1 r, r.r) partials of the update
    int nb_in2;
    const int* skip;         // MODE_JDIR: the launch does nothing if *skip != 0
    FcgHist fh;              // MODE_FDIR: previous directions
};

// Compacted list of active 3D tiles (64 x 4 anchors in x,y times 8 planes
// in z); unused in 2D.  When the list is short the planes of each tile are
// shared by `split` work items (1, 2, 4 or 8; item u covers tile u / split,
// planes part (u % split) of it), so a small active set still spreads over
// the whole chip and each workgroup marches fewer planes.
struct Tiles {
    const int* list;
    int count;
    int ntx, nty, ntz;
    int split = 1;
    __host__ __device__ int items() const { return count * split; }
};

// Offset (slice s included) of lane `lane` in row u of the active 3D tiles:
// row u is one 64-wide x run (fixed y, z and sample slice) of a tile, so an
// elementwise kernel that gives each wave one row at a time touches only the
// positions of active tiles.  ok is false past the grid's last anchor.
__device__ __forceinline__ long long tile_row_offset(const Geo& g, const Tiles& tl, long long u,
                                                     int lane, int ns, bool& ok) {
    constexpr int R = kTile3Y * kTile3Z;
    const int id = tl.list[u / (ns * R)];
    const int rem = (int)(u % (ns * R));
    const int s = rem / R, jj = (rem / kTile3Z) % kTile3Y, kk = rem % kTile3Z;
    const int tx = id % tl.ntx, ty = (id / tl.ntx) % tl.nty, tz = id / (tl.ntx * tl.nty);
    const int i = tx * kTile3X + lane, j = ty * kTile3Y + jj, k = tz * kTile3Z + kk;
    ok = i <= g.nx && j <= g.ny && k <= g.nz;
    return s * g.NP + (ok ? g.idx(i, j, k) : 0);
}

}  // namespace vfs

struct vfs_ctx {
    vfs::Geo g;
    hipStream_t stream = nullptr;
    std::string err;
    double origin[3] = {0, 0, 0};

    // settings
    int precond = VFS_PRECOND_JACOBI;
    int precision = VFS_FP64;
    double tol = 1e-6;
    int max_iter = 100000;
    double w_min = 1e-3;
    double gravity[3] = {0, 0, 0};

    // inputs (device)
    double* phi_l = nullptr;     // compact nodal
    double* phi_s = nullptr;     // compact nodal (valid if has_solid)
    bool has_solid = false;
    bool have_phi = false, have_rho = false, have_mu = false, have_u = false;
    double* rho = nullptr;       // padded cells
    double* mu = nullptr;        // padded cells
    double* u = nullptr;         // padded faces, dim slices (u^n, then u^{n+1})
    double* ubc = nullptr;       // padded faces, dim slices
    double* ybc = nullptr;       // padded samples: prescribed (p, tau) on the free surface
    bool have_traction = false;

    // fractional step (vfs_advect): extension buffers, known-face flags and
    // the advected level set; u_from_step: ctx->u is the last step's velocity
    double* adv_a = nullptr;
    double* adv_b = nullptr;
    uint8_t* adv_ka = nullptr;
    uint8_t* adv_kb = nullptr;
    double* phi_tmp = nullptr;
    bool u_from_step = false;
    bool warm_start = false;     // mixed solves start from the last solution
    bool have_x = false;         // ctx->x holds a solution of the last step

    // assembly (device)
    double* thL = nullptr;       // compact sub-cell liquid fractions (2n)^d
    double* thF = nullptr;       // compact sub-cell fluid fractions
    double* WL = nullptr;        // padded, nsets slices
    double* WF = nullptr;        // padded, nsets slices (faces: after invalidation)
    uint8_t* fflag = nullptr;    // padded faces, dim slices: bit0 K>0, bit1 bad, bit2 invalid
    double* ustar = nullptr;     // padded faces
    double* rhof = nullptr;      // padded faces
    double* K = nullptr;         // padded faces: dt/h^2 * W_F / (rho W_L)
    double* a = nullptr;         // padded samples: W_L * active
    double* c = nullptr;         // padded samples: W_F W_L / mu * active (stresses)
    double* dinv = nullptr;      // padded samples: 1 / diag(A) (0 inactive)
    double* b = nullptr;         // padded samples
    float* K32 = nullptr;
    float* a32 = nullptr;
    float* c32 = nullptr;
    float* dinv32 = nullptr;
    float* ead32 = nullptr;   // 3D: a D^-1, the weighted preconditioner of the fused iteration

    // solver vectors (padded samples)
    double* x = nullptr;
    double* r = nullptr;
    double* p0 = nullptr;
    double* p1 = nullptr;
    double* q = nullptr;
    double* z = nullptr;
    float* x32 = nullptr;
    float* r32 = nullptr;
    float* p032 = nullptr;
    float* p132 = nullptr;
    float* q32 = nullptr;
    float* z32 = nullptr;
    float* f32b = nullptr;       // 2D: second q buffer of the fused CG
    double* fpart = nullptr;     // 2D: its two 5-value partial regions

    // reductions
    double* partials = nullptr;  // per-workgroup partial sums: regions A, B, R
    long long capA = 0, capB = 0;
    unsigned* counter = nullptr;     // 3D: work-queue counters of the fused iteration
    vfs::Scalars* sc = nullptr;      // device
    vfs::Scalars* sc_host = nullptr; // pinned mirror
    int* flag = nullptr;             // device: input validation flag
    int* flag_host = nullptr;        // pinned

    // staging for user copies (device, compact)
    double* stage = nullptr;
    long long stage_elems = 0;

    // active tiles (3D)
    int* tile_flags = nullptr;
    int* tile_list = nullptr;
    int* tile_count = nullptr;
    int* tile_count_host = nullptr;  // pinned
    vfs::Tiles tiles{nullptr, 0, 0, 0, 0};
    int tiles2d = 0;                 // 2D: active tiles of the fused CG (in tile_list)
    // 3D: work tiles of the fused iteration holding an active tile, and one
    // byte per kRow3X-anchor row (x part, y, z) with bit s set if sample slice
    // s has an active sample in the row
    int* ftile_flags = nullptr;
    int* ftile_list = nullptr;
    vfs::Tiles ftiles{nullptr, 0, 0, 0, 0};
    vfs::RowBits* rowbits = nullptr;
    // the (slice, row) items of the set row bits, built on the first FP64
    // brick-preconditioned solve after an assembly (launch_row_list)
    int* rowlist = nullptr;
    int* rowlist_cnt = nullptr;
    int rowlist_n = -1;            // -1: to be built

    bool assembled = false;
    double dt_assembled = 0.0;

    // learned preconditioner (not owned) and its work space: 5 FP32 sample
    // vectors (d, A d, r1, n, A n), partial regions, line-search coefficients
    struct vfs_unet* net = nullptr;
    struct vfs_unet* net_owned = nullptr;  // created by vfs_load_preconditioner
    float* netvec = nullptr;
    double* netpart = nullptr;
    double* netcoef = nullptr;
    bool netvec_dirty = true;    // the work space must be zeroed (new assembly)
    vfs_stats stats{};
    hipEvent_t ev[6] = {};
    bool prof = false;
    hipEvent_t pev[4] = {};
    double prof_apply_ms = 0.0, prof_update_ms = 0.0, prof_precond_ms = 0.0;
    long long prof_apply_n = 0, prof_update_n = 0;
};

namespace vfs {

// error message of a call without a context (read by vfs_last_error(NULL))
int fail_global(int code, const std::string& msg);

// ---- launchers (defined in the .hip files) ----
// fractions / weights (k_fractions.hip)
void launch_subcell_fractions(const Geo& g, const double* phi, double* theta, bool complement,
                              hipStream_t s);
void launch_fill(double* dst, long long n, double v, hipStream_t s);
void launch_weights(const Geo& g, const double* thL, const double* thF, double w_min,
                    double* WL, double* WF, hipStream_t s);
// 2D assembly (k_assemble2d.hip)
void launch_face_coef2d(const Geo& g, double dt, const double* g3, const double* WL, double* WF,
                        const double* rho, const double* u, double* ustar, double* rhof,
                        double* K, uint8_t* fflag, hipStream_t s);
void launch_sample_coef2d(const Geo& g, const double* WL, const double* WF, const double* mu,
                          const double* K, const uint8_t* fflag, const double* ustar,
                          const double* ubc, double* a, double* c, double* dinv, double* b,
                          Scalars* sc, hipStream_t s);
void launch_velocity2d(const Geo& g, double dt, const double* x, const double* a,
                       const double* ustar, const double* ubc, const double* rhof,
                       const double* WL, const double* WF, const uint8_t* fflag, double* u,
                       hipStream_t s);
// 3D assembly (k_assemble3d.hip)
void launch_face_coef3d(const Geo& g, double dt, const double* g3, const double* WL, double* WF,
                        const double* rho, const double* u, double* ustar, double* rhof,
                        double* K, uint8_t* fflag, hipStream_t s);
void launch_sample_coef3d(const Geo& g, const double* WL, const double* WF, const double* mu,
                          const double* K, const uint8_t* fflag, const double* ustar,
                          const double* ubc, double* a, double* c, double* dinv, double* b,
                          Scalars* sc, hipStream_t s);
void launch_velocity3d(const Geo& g, double dt, const double* x, const double* a,
                       const double* ustar, const double* ubc, const double* rhof,
                       const double* WL, const double* WF, const uint8_t* fflag, double* u,
                       hipStream_t s);

// prescribed traction (Section 6.1): u* on faces with K > 0 and, in 3D, the
// coupling of an eliminated tau_xx / tau_yy on the right-hand side
void launch_traction2d(const Geo& g, double dt, const double* y, const double* a,
                       const double* rhof, const double* WL, const uint8_t* fflag, double* ustar,
                       hipStream_t s);
void launch_traction3d(const Geo& g, double dt, const double* y, const double* a,
                       const double* rhof, const double* WL, const uint8_t* fflag, double* ustar,
                       hipStream_t s);
void launch_traction_pair3d(const Geo& g, const double* y, const double* a, const double* c,
                            double* b, hipStream_t s);

// fractional step (k_advect.hip)
void launch_known_faces(const Geo& g, const uint8_t* fflag, const double* WF, bool all,
                        uint8_t* known, hipStream_t s);
void launch_extend(const Geo& g, const double* vin, const uint8_t* kin, double* vout,
                   uint8_t* kout, hipStream_t s);
void launch_advect_u(const Geo& g, double dt, const double* uext, double* uout, hipStream_t s);
void launch_advect_phi(const Geo& g, double dt, const double* uext, const double* phi, double* out,
                       hipStream_t s);

// brick-local Schwarz / block symmetric Gauss-Seidel preconditioner and the
// FP64 PCG around it (k_schwarz.hip); rows: the 3D row bits (bricks whose rows
// hold no active sample are skipped), ignored in 2D.  The PCG vector kernels
// sweep, in 3D, the compacted list of (slice, row) items whose row bit is set
// (RowList, built by launch_row_list: item u = slice * row_bytes + row, the
// count of cnt[row_list_chunks] after the build) and, in 2D (count < 0), the
// whole arrays.
struct RowList {
    const int* list;
    int count;
};
long long row_items(const Geo& g);
int row_list_chunks(const Geo& g);
void launch_row_list(const Geo& g, const RowBits* rows, int* list, int* cnt, hipStream_t st);
int schwarz_brick(int dim, int overlap);
void launch_schwarz(const Geo& g, int overlap, const double* r, const double* a, const double* c,
                    const double* dinv, const double* K, const RowBits* rows, double* z,
                    const int* done, hipStream_t st);
int pcg_blocks(const Geo& g);
void launch_pcg_dot(const Geo& g, const RowList& rl, const double* u, const double* v,
                    double* part, const int* done, hipStream_t st);
void launch_pcg_start(const double* part, int nb, Scalars* S, double tol, int max_iter,
                      bool keep_bb, hipStream_t st);
void launch_pcg_rz(const double* part, int nb, Scalars* S, hipStream_t st);
void launch_pcg_dir(const Geo& g, const RowList& rl, const double* z, double* p,
                    const Scalars* S, hipStream_t st);
void launch_pcg_pq(const double* part, int nb, Scalars* S, hipStream_t st);
void launch_pcg_update(const Geo& g, const RowList& rl, double* x, double* r, const double* p,
                       const double* q, const Scalars* S, double* part, hipStream_t st);
void launch_pcg_check(const double* part, int nb, Scalars* S, hipStream_t st);

// packing and checks (k_util.hip)
void launch_pack(const Geo& g, const int shp[3], const double* src, double* dst, hipStream_t s);
void launch_unpack(const Geo& g, const int shp[3], const double* src, double* dst, hipStream_t s);
void launch_unpack_active(const Geo& g, const int shp[3], const double* a, uint8_t* dst,
                          hipStream_t s);
void launch_check(const double* v, long long n, int positive, int* flag, hipStream_t s);
void launch_zero_box_faces(const Geo& g, double* faces, hipStream_t s);
void launch_to_f32(const double* src, float* dst, long long n, hipStream_t s);
void launch_mul_to_f32(const double* u, const double* v, float* dst, long long n, hipStream_t s);
void launch_mask(double* dst, const double* src, const double* a, long long n, hipStream_t s);
void launch_sub_mask(double* dst, const double* x, const double* y, const double* a, long long n,
                     hipStream_t s);

// CG building blocks (k_pcg.hip); T = double or float
// MODE_FDIR: flexible-CG direction from a given z (or the Jacobi z when the
// given one is not a descent direction) with the Polak-Ribiere beta.
// MODE_JDIR: v = D^-1 r (or a given vector), stored to pout if set, q = A v,
// partials of v.q; no CG scalars are touched.
enum ApplyMode { MODE_DIR = 0, MODE_APPLY = 1, MODE_RESID = 2, MODE_FDIR = 3, MODE_JDIR = 4 };
int apply_grid_blocks(const Geo& g);   // 2D apply grid / all 3D tiles (capacity)
int vec_grid_blocks(const Geo& g);     // dense pointwise kernels
// workgroups of one apply / update launch (the partial count they write)
// workgroups (= partials) of an apply launch on T = float (word 4) or double (8)
int apply_blocks(const Geo& g, const Tiles& tl, int word);
// workgroups of the Jacobi-PCG direction + apply launch (MODE_DIR without a
// given z), which in 3D runs the pipelined kernel
int dir_apply_blocks(const Geo& g, const Tiles& tl, int word);
int apply3d_grid(int count, int word);
int dir3d_grid(int count, int word);
// one launch per Jacobi-PCG iteration in 3D (FP32), k_apply3d.hip
// over the work tiles of fused_tile_dims (the list launch_fused_tiles builds
// from the tile flags), skipping the rows of rowbits without an active sample;
// wq: 16 work-queue counters (two slots of one per XCD), zero before the first
// solve, kept by the launches themselves afterwards
int fused3d_grid(int count);
void launch_fused3d(const Geo& g, const Tiles& ft, bool init, const FusedVecs& v,
                    const float* ead, const float* a, const float* c, const float* K,
                    const RowBits* rows, unsigned* wq, const RedArgs& ra, hipStream_t s);
void fused_tile_dims(const Geo& g, int& ntx, int& nty, int& ntz);
void launch_fused_tiles(const Geo& g, const int* tile_flags, int* flags, int* list, int* count,
                        hipStream_t s);
// plane split of the fused work tiles (their Tiles::split)
int fused_split(int count, int capacity);
long long row_bytes(const Geo& g);
void launch_row_bits(const Geo& g, const double* a, RowBits* rows, hipStream_t s);
// anchor positions of one tile of the 3D kernels and of the fused 2D kernel
int tile3d_anchors();
// plane split of a 3D tile list (Tiles::split)
int tile_split(int count, int capacity);
// the tile list as the 3D update kernel walks it (its own, finer split)
Tiles update3d_tiles(const Tiles& tl);
int tile2d_anchors();
// fused 2D CG over the compacted list of tiles holding an active sample
void fused2d_tile_dims(const Geo& g, int& ntx, int& nty);
void launch_tiles2d(const Geo& g, const double* a, int* flags, int* list, int* count,
                    hipStream_t s);
template <typename T>
void launch_fused2d(const Geo& g, bool init, const FusedVecs& v, const T* dinv, const T* a,
                    const T* c, const T* K, const int* tiles, int count, const RedArgs& ra,
                    hipStream_t s);
int update_blocks(const Geo& g, const Tiles& tl);
template <typename T>
void launch_apply(const Geo& g, const Tiles& tl, int mode, bool zin, const T* r, const T* zsrc,
                  const T* dinv, const T* pin, T* pout, T* q, const T* a, const T* c, const T* K,
                  const T* bvec, const RedArgs& ra, hipStream_t s);
template <typename T>
void launch_update(const Geo& g, const Tiles& tl, T* x, const T* p, T* r, const T* q,
                   const T* dinv, T* z, const RedArgs& ra, hipStream_t s);
template <typename T>
void launch_cg_restart(const Geo& g, const T* r, const T* dinv, T* z, Scalars* sc,
                       double* part_out, int max_iter, hipStream_t s);
template <typename T>
void launch_cg_init(const Geo& g, const T* bsrc, T* x, T* r, const T* dinv, T* z, double tol,
                    int max_iter, Scalars* sc, double* part_out, hipStream_t s);
// one workgroup sums nb partials (nv values each) into sc->aux0 (slot 0) / aux1
void launch_finalize(const double* part, int nb, int nv, Scalars* sc, int slot, hipStream_t s);
// mixed precision glue
void launch_scale_to_f32(const Geo& g, const double* r64, float* r32, const Scalars* sc,
                         hipStream_t s);
void launch_axpy_f32_to_f64(const Geo& g, double* x64, const float* d32, const Scalars* sc,
                            hipStream_t s);
void launch_norm2(const Geo& g, const double* v, double* part_out, hipStream_t s);
// 3D tiles (k_apply3d.hip)
void tile_dims(const Geo& g, int& ntx, int& nty, int& ntz);
void launch_tiles(const Geo& g, const double* a, int* flags, int* list, int* count,
                  hipStream_t s);
template <typename T>
void launch_apply3d(const Geo& g, const Tiles& tl, int mode, bool zin, const T* r, const T* zsrc,
                    const T* dinv, const T* pin, T* pout, T* q, const T* a, const T* c,
                    const T* K, const T* bvec, const RedArgs& ra, hipStream_t s);
template <typename T>
void launch_update3d(const Geo& g, const Tiles& tl, T* x, const T* p, T* r, const T* q,
                     const T* dinv, T* z, const RedArgs& ra, hipStream_t s);

}  // namespace vfs
