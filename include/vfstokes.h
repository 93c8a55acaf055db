/*
 * vfstokes.h -- C ABI of the MI355X (gfx950) variational Stokes step.
 *
 * The library performs one backward-Euler step of time-dependent,
 * variable-coefficient Stokes flow with free surfaces and (moving) solids,
 * following "A Simple Finite Difference Method for Time-Dependent, Variable
 * Coefficient Stokes Flow on Irregular Domains":
 *   u* = u^n + dt g                         (body force, Section 10)
 *   volume fractions W_L, W_F               (Section 5, Figs. 3-4)
 *   null-space elimination                  (Section 8)
 *   SPD stress/pressure system A x = b      (eq. stokesmixedsystemspd,
 *                                            factored form of Section 7,
 *                                            moving-solid RHS of Section 6.2)
 *   preconditioned CG on A                  (Section 7 end, Section 9)
 *   velocity recovery from the KKT velocity row (eq. stokesmixedsystem)
 *
 * Conventions for every entry point
 *   - Return value: VFS_OK (0) or a negative VFS_E* code; vfs_last_error()
 *     gives a message for the last failing call on that context.
 *   - Pointers passed in may be host or device memory (the library copies
 *     with hipMemcpyDefault); the caller owns them and may free them after
 *     the call returns.  The library owns all device memory it allocates.
 *   - All arrays are FP64, x-fastest (index i + nx_a*(j + ny_a*k)).
 *       nodes  (level sets):        (nx+1) x (ny+1) [x (nz+1)]
 *       cells  (rho, mu, p):        nx x ny [x nz]
 *       u faces: (nx+1) x ny [x nz]; v faces: nx x (ny+1) [x nz];
 *       w faces: nx x ny x (nz+1)
 *       2D tau_xy (nodes): (nx+1) x (ny+1)
 *       3D tau_xy (z-edges): (nx+1)x(ny+1)x nz; tau_xz (y-edges):
 *          (nx+1) x ny x (nz+1); tau_yz (x-edges): nx x (ny+1) x (nz+1)
 *   - "Sample order" vectors (vfs_apply, vfs_solve, vfs_get_solution,
 *     vfs_get_rhs) concatenate, in this order, p, tau_xx, [tau_yy,] tau_xy,
 *     [tau_xz, tau_yz], each block in its native shape above.  Entries of
 *     eliminated (inactive) samples are ignored on input and 0 on output.
 *   - Work is queued on the context's stream; calls that return data to the
 *     caller synchronise that stream.  A context must not be used from two
 *     threads at once.
 */
#ifndef VFSTOKES_H
#define VFSTOKES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define VFS_OK           0
#define VFS_EINVAL      -1   /* bad argument: NaN/Inf input, rho<=0, mu<=0, dt<=0, sizes */
#define VFS_ENOMEM      -2   /* device allocation failed */
#define VFS_EHIP        -3   /* a HIP runtime call failed */
#define VFS_ENOTCONV    -4   /* max_iter reached; best iterate and velocity still written */
#define VFS_EBREAKDOWN  -5   /* CG breakdown (p.Ap <= 0 or non-finite); best iterate kept */
#define VFS_ESTATE      -6   /* call out of order (e.g. solve before assemble) */

/* preconditioners */
#define VFS_PRECOND_NONE     0
#define VFS_PRECOND_JACOBI   1   /* diagonal of A */
#define VFS_PRECOND_IC       2   /* block symmetric Gauss-Seidel (the IC-style
                                    factorization (D+L) D^-1 (D+U) of A restricted to
                                    disjoint bricks of 16^2 / 4^3 anchors, multicolour
                                    order), VFS_FP64 only */
#define VFS_PRECOND_LEARNED  3   /* U-Net correction inside flexible CG (3D, VFS_MIXED;
                                    attach a network with vfs_set_preconditioner) */
#define VFS_PRECOND_SCHWARZ  4   /* overlapping additive Schwarz: the same brick solver on
                                    bricks extended by one anchor, corrections summed (a
                                    GPU analogue of the overlapping Schwarz decomposition
                                    the paper pairs with CG, Sections 7 and 9), VFS_FP64 only */

/* arithmetic of the solve */
#define VFS_FP64   0   /* FP64 vectors, coefficients, apply and reductions */
#define VFS_MIXED  1   /* FP32 apply/vectors, FP64 reductions, FP64 residual
                          and iterative-refinement outer steps; in 3D the six
                          FP32 sample slices of one vector must stay under
                          4 GiB (grids up to about 550^3), else the solve
                          returns VFS_EINVAL */

/* sample types, in sample order (index of a block of a sample-order vector);
 * the 3D-only types shift the 2D tau_xy to slot 3 */
#define VFS_SAMPLE_P      0
#define VFS_SAMPLE_TXX    1
#define VFS_SAMPLE_TXY_2D 2
#define VFS_SAMPLE_TYY    2   /* 3D */
#define VFS_SAMPLE_TXY    3   /* 3D */
#define VFS_SAMPLE_TXZ    4   /* 3D */
#define VFS_SAMPLE_TYZ    5   /* 3D */

/* sample sets for vfs_get_weights */
#define VFS_SET_CELL    0   /* p, tau_xx, tau_yy */
#define VFS_SET_FACE_X  1
#define VFS_SET_FACE_Y  2
#define VFS_SET_FACE_Z  3
#define VFS_SET_NODE    4   /* 2D tau_xy */
#define VFS_SET_EDGE_Z  4   /* 3D tau_xy (same slot as the 2D node set) */
#define VFS_SET_EDGE_Y  5   /* 3D tau_xz */
#define VFS_SET_EDGE_X  6   /* 3D tau_yz */

#define VFS_WEIGHT_LIQUID  0  /* W_L */
#define VFS_WEIGHT_FLUID   1  /* W_F as used by the system (0 on invalid faces) */

typedef struct vfs_ctx vfs_ctx;

typedef struct vfs_stats {
    int64_t n_samples;        /* candidate unknowns (all tau + p samples) */
    int64_t n_active;         /* unknowns after null-space elimination */
    int32_t iterations;       /* total inner CG iterations of the last solve */
    int32_t outer_iterations; /* refinement steps (mixed) or residual replacements */
    int32_t status;           /* status of the last solve */
    int32_t precision;        /* VFS_FP64 / VFS_MIXED */
    double  rel_residual;     /* FP64 true ||b - A x||_2 / ||b||_2 over active samples */
    double  b_norm;           /* ||b||_2 */
    double  t_assemble_ms;    /* (a1)-(a4) of the last step, device time */
    double  t_solve_ms;       /* first apply to convergence, device time */
    double  t_recover_ms;     /* velocity recovery, device time */
    double  t_step_ms;        /* whole step, device time */
    /* live kernel timing (vfs_set_profiling): average device duration of one
       launch of the CG apply kernel and of the CG update kernel, from HIP
       events on the context stream around one launch of each per chunk of
       iterations.  The VFS_MIXED Jacobi solve (2D and 3D) runs one fused
       launch per iteration: t_apply_avg_ms is then its average over the
       back-to-back launches of each chunk after the first, t_update_avg_ms
       is 0 and n_apply_timed counts the timed chunks. */
    double  t_apply_avg_ms;
    double  t_update_avg_ms;
    int64_t n_apply_timed;
    int64_t n_update_timed;
    /* preconditioned solves (VFS_PRECOND_LEARNED, _IC, _SCHWARZ): average
       device time of one preconditioner application under profiling (for
       the network: scale, pack, forward, unpack); for the learned solve also
       the number of iterations whose network direction was not a descent
       direction and was replaced by the Jacobi one */
    double  t_precond_avg_ms;
    int32_t precond_fallbacks;
    int32_t pad0;
    /* sample positions the solver kernels sweep: active tiles (tiles holding
       an active sample) x anchors per tile x sample types, counting positions
       past the grid edge; the solver vectors are zero outside these tiles.
       Set by assembly.  In 2D it describes the VFS_MIXED (fused) solve; the
       2D VFS_FP64 kernels sweep the whole grid. */
    int64_t n_tile_samples;
    /* ||b - A x0|| / ||b|| of the last solve's starting iterate x0: 1 from
       zero; when warm-started (vfs_set_warm_start) that of the previous
       solution masked to the new active set, which may well exceed 1 */
    double  rel_residual_start;
} vfs_stats;

/* Last error message of a context (or of the failed create when ctx is NULL). */
const char* vfs_last_error(const vfs_ctx* ctx);

/* Create a context for a dim-D grid (dim 2 or 3) of nx*ny[*nz] cells of size
 * h whose lower corner is origin[0..dim-1].  nz is ignored in 2D.  The box
 * walls act as static no-slip solids.  Allocates all device memory for the
 * grid; *out is NULL on failure. */
int vfs_create(vfs_ctx** out, int dim, int nx, int ny, int nz, double h, const double* origin);
int vfs_destroy(vfs_ctx* ctx);

/* Queue all work on this hipStream_t (NULL = the null stream). */
int vfs_set_stream(vfs_ctx* ctx, void* hip_stream);

/* Level sets at grid nodes (phi < 0 inside; phi == 0 counts as outside).
 * phi_liquid marks the liquid (non-air) region and must be given
 * everywhere, including inside solids (Fig. 4 caption: the interface is
 * extrapolated into the solid).  phi_solid may be NULL (no solid besides
 * the box walls).  Section 5 weights every term by the volume fraction of
 * its sample's h-sized control volume; the fractions are recomputed from
 * these level sets by the next assemble/step.  EINVAL on NaN/Inf. */
int vfs_set_level_sets(vfs_ctx* ctx, const double* phi_liquid, const double* phi_solid);

/* Cell-centred density (> 0) and viscosity (> 0).  Density at a face is
 * the mean of its in-box cells, viscosity at a node/edge the mean of the
 * in-box cells sharing it (the diagonal P and M of Section 5). */
int vfs_set_density(vfs_ctx* ctx, const double* rho_cells);
int vfs_set_viscosity(vfs_ctx* ctx, const double* mu_cells);

/* Face velocities u^n (w ignored in 2D). */
int vfs_set_velocity(vfs_ctx* ctx, const double* u, const double* v, const double* w);

/* Prescribed solid velocity u_BC per face (Section 6.2); NULL pointers mean
 * a static solid.  Values on box faces are ignored (box walls are static). */
int vfs_set_solid_velocity(vfs_ctx* ctx, const double* ub, const double* vb, const double* wb);

/* Prescribed traction on the free surface (Section 6.1), e.g. a surface-
 * tension pressure: boundary values of the pressure and of the deviatoric
 * stress, given as fields at their samples (p_bc: cells; tau_bc[0..1] in 2D:
 * tau_xx cells, tau_xy nodes; tau_bc[0..4] in 3D: xx, yy cells, xy, xz, yz
 * edges, the shapes of the conventions above).  Only their values in the air
 * part of the control volumes near the surface and at eliminated samples
 * matter: the air-region boundary work enters the right-hand side, and a
 * sample removed by the null-space elimination takes its boundary value
 * instead of 0 (Section 8).  The sign is such that a uniform p_bc = p0
 * raises the liquid pressure by p0 and leaves the flow unchanged.  NULL
 * pointers mean 0; p_bc and tau_bc both NULL (or every entry NULL) switch
 * the terms off.  Applied from the next assemble/step.  EINVAL on NaN/Inf. */
int vfs_set_traction(vfs_ctx* ctx, const double* p_bc, const double* const* tau_bc);

/* Advection half of the fractional step of Section 10, to call before
 * vfs_step: first-order semi-Lagrangian advection (bilinear in 2D, trilinear
 * in 3D) of the context's velocity and of its liquid level set, FP64.  The
 * velocity the last vfs_step defined (faces with K > 0, and solid or box
 * faces, W_F = 0) is first extended three face layers into the air, each
 * unknown face taking the mean of its known same-component neighbours; a
 * velocity given by vfs_set_velocity counts as known everywhere.  Each face
 * value (and each level-set node) becomes the interpolant of the extended
 * field at its departure point x - dt v(x), clamped to the box.  The solid
 * level set and solid velocity are unchanged.  Allocates its work buffers on
 * the first call.  ESTATE before velocity and level sets are set. */
int vfs_advect(vfs_ctx* ctx, double dt);
/* The current liquid level set (after vfs_advect), nodal shape. */
int vfs_get_level_set(vfs_ctx* ctx, double* phi_liquid);
/* Warm start (1) or not (0, default): the VFS_MIXED solve of vfs_step starts
 * from the previous step's solution on the samples that are still active,
 * instead of 0; the tolerance stays relative to |b|.  FP64 solves and
 * vfs_solve always start from 0. */
int vfs_set_warm_start(vfs_ctx* ctx, int on);

/* Body force per unit mass, g[0..dim-1]. */
int vfs_set_gravity(vfs_ctx* ctx, const double* g);

/* Solver settings: preconditioner (VFS_PRECOND_*), precision (VFS_FP64 or
 * VFS_MIXED), relative tolerance on the FP64 true residual ||b-Ax||/||b||
 * over active samples, iteration cap, and w_min: volume fractions strictly
 * below w_min are snapped to 0. Defaults: JACOBI, FP64, 1e-6, 100000, 1e-3. */
int vfs_set_solver(vfs_ctx* ctx, int precond, int precision, double rel_tol,
                   int max_iter, double w_min);

/* One full step: u* = u + dt g, fractions, coefficients, null-space
 * elimination, right-hand side, CG solve, velocity recovery.  The new
 * velocity replaces the context's velocity.  Returns VFS_ENOTCONV /
 * VFS_EBREAKDOWN with the best iterate applied when the solve fails. */
int vfs_step(vfs_ctx* ctx, double dt);

/* Steps (a1)-(a4) only: body force, fractions, coefficients, elimination
 * and right-hand side for this dt (for tests and vfs_apply/vfs_solve). */
int vfs_assemble(vfs_ctx* ctx, double dt);

/* y = A x on the assembled system (sample order, FP64 path). */
int vfs_apply(vfs_ctx* ctx, const double* x, double* y);

/* Solve A x = b on the assembled system with the configured solver
 * (sample order); x is the result, the iterate starts from 0. */
int vfs_solve(vfs_ctx* ctx, const double* b, double* x);

/* Results of the last step / assemble. */
int vfs_get_velocity(vfs_ctx* ctx, double* u, double* v, double* w);
int vfs_get_pressure(vfs_ctx* ctx, double* p);
/* tau[0..1] (2D: tau_xx, tau_xy) or tau[0..4] (3D: xx, yy, xy, xz, yz) */
int vfs_get_stress(vfs_ctx* ctx, double* const* tau);
int vfs_get_solution(vfs_ctx* ctx, double* x);   /* sample order */
int vfs_get_rhs(vfs_ctx* ctx, double* b);        /* sample order */
/* W_L or W_F of a sample set (VFS_SET_*), native shape of that set. */
int vfs_get_weights(vfs_ctx* ctx, int set, int which, double* out);
/* 1 for active (not eliminated) samples, sample order.  A sample is active
 * when its liquid weight is positive, no face of its stencil has positive
 * fluid weight and zero liquid weight, and some face of its stencil carries
 * K > 0 (the null-space elimination of Section 8); inactive samples hold
 * their boundary value 0.  ESTATE before the first assembly. */
int vfs_get_active(vfs_ctx* ctx, uint8_t* out);
/* The same mask for one sample type (VFS_SAMPLE_*) in that type's native
 * shape (cells for p, tau_xx, tau_yy; nodes or edges for the off-diagonal
 * stresses).  EINVAL for a type the grid's dimension does not have. */
int vfs_get_active_mask(vfs_ctx* ctx, int sample, uint8_t* out);
int vfs_get_stats(vfs_ctx* ctx, vfs_stats* out);
/* Turn live per-kernel timing on (1) or off (0); turning it on resets the
 * accumulated averages reported in vfs_stats.  Timing adds one event pair
 * per kernel per chunk of CG iterations. */
int vfs_set_profiling(vfs_ctx* ctx, int on);

/* Number of entries of a sample-order vector and of the face vector. */
int vfs_get_sizes(const vfs_ctx* ctx, int64_t* n_samples, int64_t* n_faces);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the liquid
 * volume fractions W_L of one sample set (VFS_SET_*) computed straight from a
 * nodal liquid level set, without a context, allocating nothing.  The result
 * is bit-identical to vfs_get_weights(ctx, set, VFS_WEIGHT_LIQUID, out) on a
 * context assembled from the same level set and w_min (W_L ignores solids).
 *   phi_liquid: DEVICE memory, (nx+1) x (ny+1) [x (nz+1)] FP64, x-fastest.
 *   out:        DEVICE memory, the set's native shape (see the conventions).
 * Work is queued on hip_stream (NULL = the null stream) and the call returns
 * without synchronising; NaN/Inf in phi_liquid are not checked.  The work
 * space is one fixed 96 MiB device array per GPU, held until the process
 * ends: it takes (16 (nx ny [nz]) + 2 nsets NP) doubles, NP the padded grid
 * size of the conventions above, which admits square 2D grids up to 882^2
 * and cubic 3D grids up to 69^3; larger grids return VFS_EINVAL.  Every call on a
 * GPU shares that GPU's array, so calls that overlap in time on one GPU
 * (different streams or threads) race and must be serialised by the caller.
 * Errors: VFS_EINVAL (sizes, set, w_min, NULL pointers), VFS_EHIP; the
 * message is vfs_last_error(NULL). */
int vfs_liquid_weights_noalloc(int dim, int nx, int ny, int nz, double w_min,
                               const double* phi_liquid, int set, double* out, void* hip_stream);

/* ------------------------------------------------------------------------
 * Batched 2D steps: many independent problems of different sizes.  All
 * their solves run in one persistent launch (FP32 Jacobi PCG with FP64
 * reductions, FP64 residual and iterative refinement per problem, each
 * problem retiring on its own), captured once in a hipGraph and replayed.
 * Every problem is a full step of the method above (same equations, inputs
 * and outputs as a single context), always in VFS_MIXED arithmetic.
 * ------------------------------------------------------------------------ */
typedef struct vfs_batch vfs_batch;

typedef struct vfs_batch_stats {
    int32_t n_problems;
    int32_t variant;          /* tile shape index (vfs_batch_variant_shape) */
    int32_t blocks_per_cu;    /* persistent workgroups per compute unit (the requested
                                 number, capped at what can be resident) */
    int32_t grid;             /* persistent workgroups launched */
    int32_t graph_used;       /* 1 if the pass ran from a hipGraph */
    int32_t status;           /* VFS_OK or VFS_ENOTCONV */
    int64_t n_active_total;   /* sum of active unknowns */
    int64_t dof_iters;        /* sum over problems of active unknowns x CG iterations */
    int32_t max_iterations;   /* largest per-problem CG iteration count */
    int32_t passes_max;       /* largest per-problem refinement pass count */
    double  t_assemble_ms, t_solve_ms, t_step_ms;   /* device time of the last step */
    double  latency_p50_ms, latency_p90_ms, latency_p99_ms, latency_max_ms;
                              /* per-problem solve latency: device wall clock from
                                 the start of the solve to the pass that met tol */
    int64_t n_items;          /* work items of the last step: the tiles holding an
                                 active sample (at least one per problem) */
    int64_t n_tile_samples;   /* sample positions those items sweep per CG iteration */
} vfs_batch_stats;

const char* vfs_batch_last_error(const vfs_batch* b);
/* n problems; problem i has nx[i] x ny[i] cells of size h[i], origin 0. */
int vfs_batch_create(vfs_batch** out, int n, const int* nx, const int* ny, const double* h);
int vfs_batch_destroy(vfs_batch* b);
/* NULL selects the batch's own (non-blocking, default priority) stream. */
int vfs_batch_set_stream(vfs_batch* b, void* hip_stream);
/* Inputs of problem i, same meaning and layout as vfs_set_level_sets,
 * vfs_set_density, vfs_set_viscosity, vfs_set_velocity,
 * vfs_set_solid_velocity (ub/vb may be NULL) and vfs_set_gravity. */
int vfs_batch_set_problem(vfs_batch* b, int i, const double* phi_liquid, const double* phi_solid,
                          const double* rho, const double* mu, const double* u, const double* v,
                          const double* ub, const double* vb, const double* g);
int vfs_batch_set_solver(vfs_batch* b, double rel_tol, int max_iter, double w_min);
/* Launch configuration: tile shape variant and persistent workgroups per
 * compute unit (clamped to the occupancy limit); chosen by the autotuner. */
int vfs_batch_num_variants(void);
int vfs_batch_variant_shape(int variant, int* bx, int* by);
int vfs_batch_set_tiles(vfs_batch* b, int variant, int blocks_per_cu);
/* Most persistent workgroups per compute unit that can be resident at once
 * with the given tile shape on the current device (vfs_batch_set_tiles caps
 * its request at this); < 0 for a bad variant or a failed query. */
int vfs_batch_max_blocks_per_cu(int variant);
/* Autotuner probe: device time per CG iteration of the persistent kernel
 * for a configuration, measured over `iterations` iterations on the
 * currently assembled problems (requires one vfs_batch_step before). */
int vfs_batch_time_variant(vfs_batch* b, int variant, int blocks_per_cu, int iterations,
                           double* ms_per_iteration);
/* One step of every problem: assemble all, solve all, recover all velocities.
 * VFS_ENOTCONV if some problem missed the tolerance (its best iterate is used). */
int vfs_batch_step(vfs_batch* b, double dt);
int vfs_batch_get_velocity(vfs_batch* b, int i, double* u, double* v);
int vfs_batch_get_solution(vfs_batch* b, int i, double* x);   /* sample order */
int vfs_batch_get_problem(vfs_batch* b, int i, int* iterations, int* passes,
                          double* rel_residual, double* latency_ms, int64_t* n_active);
int vfs_batch_get_stats(vfs_batch* b, vfs_batch_stats* out);

/* ------------------------------------------------------------------------
 * Learned preconditioner (3D).  Not part of the paper, whose CG uses an
 * algebraic Schwarz preconditioner (Section 7 end, Section 9): a U-Net
 * style network (Ronneberger et al. 2015) maps a residual r to a correction
 * z inside flexible CG (Golub and Ye 1999, Notay 2000; Polak-Ribiere beta),
 * with the Jacobi direction D^-1 r whenever z is not a descent direction.
 *
 * Network: 3x3x3 convolutions, no biases, ReLU, 2x2x2 mean pooling,
 * nearest upsampling, additive skips.  Layers (Cin -> Cout, level):
 *   enc0 16->16 L0, enc1 16->32 L1, enc2 32->64 L2, enc3 64->128 L3,
 *   bott 128->64 L3, dec2 64->32 L2, dec1 32->16 L1, dec0 16->6 L0
 *   c0 = relu(enc0(x)); c1 = relu(enc1(pool c0)); c2 = relu(enc2(pool c1));
 *   c3 = relu(enc3(pool c2)); d3 = relu(bott(c3));
 *   d2 = relu(dec2(up d3 + c2)); d1 = relu(dec1(up d2 + c1));
 *   y = dec0(up d1 + c0)
 * BF16 storage and MFMA operands, FP32 accumulation, FP32 master weights.
 * Weights: FP32, layers in the order above, each [Cout][Cin][dz][dy][dx]
 * (C order), out[z,y,x,co] = sum W[co,ci,dz,dy,dx] in[z+dz-1, y+dy-1, x+dx-1, ci]
 * with zero padding; vfs_unet_param_count() values in total.
 * Tensors at this boundary: FP32, dense, [Z][Y][X][C] (C fastest); X, Y, Z
 * positive multiples of 8.  Input C = 16, output C = 6.
 * Solver coupling: a grid of n cells uses extents roundup(n_a + 1, 8); input
 * channel q < 6 at voxel (i, j, k) is s sqrt(D^-1) r of sample set q
 * (p, txx, tyy, txy, txz, tyz) at index (i, j, k), s = sqrt(n_active) /
 * ||sqrt(D^-1) r||; channels 8, 9, 10 hold the cell's W_L, W_F and
 * log10(1 + dt mu / (rho h^2)) / 6; the others are 0.  The correction is
 * z = sqrt(D^-1) y / s on active samples.
 * ------------------------------------------------------------------------ */
typedef struct vfs_unet vfs_unet;
const char* vfs_unet_last_error(const vfs_unet* u);
int64_t vfs_unet_param_count(void);
/* New network with zero weights (set them before use). */
int vfs_unet_create(vfs_unet** out);
int vfs_unet_destroy(vfs_unet* u);
/* Stream for the network's work (must equal the stream of any context it
 * is used with). */
int vfs_unet_set_stream(vfs_unet* u, void* hip_stream);
/* Replace the FP32 master weights (count = vfs_unet_param_count(), host or
 * device); resets the Adam state and the gradient.  EINVAL on NaN/Inf. */
int vfs_unet_set_weights(vfs_unet* u, const float* w, int64_t count);
int vfs_unet_get_weights(vfs_unet* u, float* w, int64_t count);
/* Accumulated weight gradient (same layout as the weights). */
int vfs_unet_get_grad(vfs_unet* u, float* g, int64_t count);
int vfs_unet_zero_grad(vfs_unet* u);
/* y = network(x); keeps the activations for vfs_unet_backward. */
int vfs_unet_forward(vfs_unet* u, int X, int Y, int Z, const float* x, float* y);
/* Adds the gradient of <gy, y> with respect to the weights (chain rule
 * through the last forward) to the accumulated gradient.  ESTATE without a
 * preceding forward. */
int vfs_unet_backward(vfs_unet* u, const float* gy);
/* Adam (Kingma and Ba 2015, bias-corrected) on the weights with gradient
 * grad_scale * (accumulated gradient); clears the accumulated gradient. */
int vfs_unet_adam(vfs_unet* u, double lr, double beta1, double beta2, double eps,
                  double grad_scale);
/* One training sample on an assembled 3D context: network correction f of
 * the residual r (sample order; A e = r, e the exact correction), loss
 * L = 1 - (f.r)^2 / ((f.A f)(e.r)) (the A-norm error left after an exact
 * line search along f, relative to that of e), and its gradient added to
 * the accumulated weight gradient.  *loss receives L. */
int vfs_unet_train_step(vfs_unet* u, vfs_ctx* ctx, const double* r, const double* e,
                        double* loss);
/* Attach a network (not owned; NULL detaches) for VFS_PRECOND_LEARNED. */
int vfs_set_preconditioner(vfs_ctx* ctx, vfs_unet* u);
/* Load FP32 weights (the vfs_unet_set_weights layout, exactly
 * vfs_unet_param_count() * 4 bytes; host or device memory, copied) into a
 * network owned by the context (created on the first call, freed by
 * vfs_destroy, run on the context's stream) and attach it as by
 * vfs_set_preconditioner.  EINVAL for a 2D context, a size mismatch or
 * NaN/Inf weights. */
int vfs_load_preconditioner(vfs_ctx* ctx, const void* weights, size_t bytes);
/* One training pair from two iterates of a solve on the assembled context
 * (sample order, FP64): r = b - A x_k and e = x_star - x_k on the active
 * samples (0 on the others).  With x_star the solution of A x = b, A e = r:
 * e is the exact correction of the residual r. */
int vfs_training_pair(vfs_ctx* ctx, const double* x_star, const double* x_k, double* r,
                      double* e);
/* z = M^-1 r of the configured preconditioner on the assembled context
 * (sample order): the brick preconditioners (VFS_PRECOND_IC, _SCHWARZ) in
 * FP64, otherwise the attached network's two-level correction. */
int vfs_precond_apply(vfs_ctx* ctx, const double* r, double* z);

#ifdef __cplusplus
}
#endif
#endif /* VFSTOKES_H */
