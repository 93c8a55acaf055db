// Brick-local Schwarz preconditioners and the FP64 PCG that uses them.
//
// Preconditioner (the GPU analogue of the overlapping Schwarz domain
// decomposition the paper pairs with CG, Section 7's closing paragraph and
// Section 9): the anchor lattice (every sample of every type anchored at its
// array index, 0..n per axis) is cut into bricks of B anchors per axis; a
// brick's subdomain is the active samples anchored in the brick extended by OV
// anchors on each side.  Each subdomain is solved approximately by one
// symmetric multicolour Gauss-Seidel sweep on its principal submatrix of A,
// from zero: colours (sample type q, parity of the anchor index sum) in the
// order q = 0, 1, ..., parity 0 before 1, forward, then in reverse.  Samples
// of one colour share no face, so A couples none of them and a colour is
// relaxed at once.  z = sum over subdomains I of W_I G_I W_I r, W_I =
// diag(m^-1/2), m the number of extended bricks holding the sample's anchor
// (a symmetric partition of unity on the overlap): with OV = 0 the bricks are
// disjoint (m = 1, block symmetric Gauss-Seidel); with OV > 0 the launches
// take the bricks in 2^d colour classes whose extended bricks do not overlap,
// so each class adds its corrections without write conflicts.
//
// One workgroup per brick, one thread per anchor of the extended brick: the
// thread keeps r, a = W_L active, c = W_F W_L / mu (stresses), D^-1 and the
// local iterate x of its anchor's samples in registers, and the workgroup
// keeps the face coefficients K (one anchor beyond the extended brick) and the
// face values g in LDS.  (A_loc x)_s is evaluated matrix-free from the same
// stencils as the apply kernels:
//   (A x)_s = a_s sum_f sigma_fs K_f g_f + c_s x_s [+ (1/2) min(c_xx, c_yy) x
//   of the other diagonal stress in 3D],  g_f = sum_t sigma_ft a_t x_t,
// with x = 0 outside the subdomain.
#include <algorithm>

#include "vfs_internal.h"
#include "vfs_reduce.h"

namespace vfs {
namespace {

constexpr int NT = 256;

// Stencil terms of a sample's row: per sample type, the faces (axis, offset
// of the face anchor from the sample anchor, sign) of its (B0^T) column, so
// that (A x)_s = a_s sum_t sign_t K_t g_t over these faces.  Compile-time
// tables: the kernel's loops over types and terms are unrolled, so every
// entry folds into an immediate.
struct Term {
    int8_t q, dx, dy, dz, s;
};

// 2D: types p, txx, txy; faces u, v
constexpr Term kSamp2[3][4] = {
    {{0, 0, 0, 0, 1}, {0, 1, 0, 0, -1}, {1, 0, 0, 0, 1}, {1, 0, 1, 0, -1}},
    {{0, 0, 0, 0, -1}, {0, 1, 0, 0, 1}, {1, 0, 0, 0, 1}, {1, 0, 1, 0, -1}},
    {{0, 0, 0, 0, 1}, {0, 0, -1, 0, -1}, {1, 0, 0, 0, 1}, {1, -1, 0, 0, -1}},
};
// 3D: types p, txx, tyy, txy, txz, tyz; faces u, v, w
constexpr Term kSamp3[6][6] = {
    {{0, 0, 0, 0, 1}, {0, 1, 0, 0, -1}, {1, 0, 0, 0, 1}, {1, 0, 1, 0, -1}, {2, 0, 0, 0, 1}, {2, 0, 0, 1, -1}},
    {{0, 1, 0, 0, 1}, {0, 0, 0, 0, -1}, {2, 0, 0, 0, 1}, {2, 0, 0, 1, -1}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
    {{1, 0, 1, 0, 1}, {1, 0, 0, 0, -1}, {2, 0, 0, 0, 1}, {2, 0, 0, 1, -1}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
    {{0, 0, 0, 0, 1}, {0, 0, -1, 0, -1}, {1, 0, 0, 0, 1}, {1, -1, 0, 0, -1}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
    {{0, 0, 0, 0, 1}, {0, 0, 0, -1, -1}, {2, 0, 0, 0, 1}, {2, -1, 0, 0, -1}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
    {{1, 0, 0, 0, 1}, {1, 0, 0, -1, -1}, {2, 0, 0, 0, 1}, {2, 0, -1, 0, -1}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
};

template <int DIM>
__device__ __forceinline__ Term samp_term(int q, int t) {
    return DIM == 2 ? kSamp2[q][t] : kSamp3[q][t];
}

template <int DIM>
struct Shape;
template <>
struct Shape<2> {
    static constexpr int NS = 3, NF = 2, ST = 4;
};
template <>
struct Shape<3> {
    static constexpr int NS = 6, NF = 3, ST = 6;
};

struct SgsArgs {
    const double* r;
    const double* a;
    const double* c;
    const double* dinv;
    const double* K;
    double* z;
    int nb[3];        // bricks per axis
    int cls[3];       // brick class of this launch (parity per axis), -1: every brick
    int accumulate;   // z += correction (overlapping bricks) or z = correction
    const int* done;  // skip when set (a converged solve)
    const RowBits* rows;   // 3D row bits (active sample slices per row half) or null
    int rntx;              // x tiles of the row bits
};

// threads of a brick workgroup: one per anchor of the extended brick
template <int DIM, int B, int OV>
struct BrickShape {
    static constexpr int E = B + 2 * OV;                        // extended brick
    static constexpr int NE = DIM == 2 ? E * E : E * E * E;     // its anchors
    static constexpr int EK = E + 2;                            // with a face ring
    static constexpr int NK = DIM == 2 ? EK * EK : EK * EK * EK;
    static constexpr int T = (NE + 63) / 64 * 64;
};

template <int DIM, int B, int OV>
__global__ __launch_bounds__((BrickShape<DIM, B, OV>::T)) void k_sgs_bricks(Geo g, SgsArgs s) {
    static_assert(OV == 0 || OV == 1, "the overlap weights assume an overlap of 0 or 1");
    static_assert(B >= 2, "same-class extended bricks must not overlap");
    using S = Shape<DIM>;
    using BS = BrickShape<DIM, B, OV>;
    constexpr int E = BS::E, NE = BS::NE, EK = BS::EK, NK = BS::NK, T = BS::T;
    // per face: K and the face value g = sum_t sigma a_t x_t of the current
    // local iterate (read and updated by the neighbouring anchors); a thread's
    // own samples (local iterate, a, weighted r, D^-1, c) stay in registers
    __shared__ double sk[S::NF][NK], sg[S::NF][NK];
    if (s.done && *s.done) return;

    // brick of this workgroup
    int bi[3] = {0, 0, 0};
    {
        long long w = blockIdx.x;
        for (int a = 0; a < DIM; ++a) {
            const int cnt = s.cls[a] < 0 ? s.nb[a] : (s.nb[a] - s.cls[a] + 1) / 2;
            const int j = (int)(w % cnt);
            w /= cnt;
            bi[a] = s.cls[a] < 0 ? j : 2 * j + s.cls[a];
        }
    }
    const int nmax[3] = {g.nx, g.ny, g.nz};
    int lo[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) lo[a] = bi[a] * B - OV;
    const long long NP = g.NP;
    auto gidx = [&](int i, int j, int k) { return DIM == 2 ? g.idx(i, j) : g.idx(i, j, k); };
    // m^-1/2 at an anchor: m is the product over the axes of the number of
    // extended bricks holding the anchor's index on that axis -- its own
    // brick and, with overlap, the previous one (first index of a brick) or
    // the next one (last index) where that brick exists
    auto weight = [&](int gi, int gj, int gk) {
        if (OV == 0) return 1.0;
        const int id[3] = {gi, gj, gk};
        int m = 1;
        for (int a = 0; a < DIM; ++a) {
            const int J = id[a] / B, t = id[a] % B;
            m *= 1 + ((t == 0 && J >= 1) ? 1 : 0) + ((t == B - 1 && J + 1 < s.nb[a]) ? 1 : 0);
        }
        return 1.0 / sqrt((double)m);
    };

    // this thread's anchor (anchors outside 0..n are absent)
    const int l = threadIdx.x;
    const bool mine = l < NE;
    const int li = l % E, lj = (l / E) % E, lk = DIM == 3 ? l / (E * E) : 0;
    const int gi = lo[0] + li, gj = lo[1] + lj, gk = lo[2] + lk;
    const bool in = mine && gi >= 0 && gi <= nmax[0] && gj >= 0 && gj <= nmax[1] &&
                    (DIM == 2 || (gk >= 0 && gk <= nmax[2]));
    const long long o = in ? gidx(gi, gj, gk) : 0;
    // 3D: a brick whose rows hold no active sample has a zero correction;
    // it skips its loads and its sweep (one thread per (y, z) row of the
    // extended brick reads the row bits of the x tiles it spans)
    if (DIM == 3 && s.rows) {
        int any = 0;
        if (l < E * E) {
            const int rj = lo[1] + l % E, rk = lo[2] + l / E;
            if (rj >= 0 && rj <= nmax[1] && rk >= 0 && rk <= nmax[2]) {
                const int t0 = max(lo[0], 0) / kRow3X, t1 = min(lo[0] + E - 1, nmax[0]) / kRow3X;
                for (int t = t0; t <= t1 && t < s.rntx; ++t)
                    any |= s.rows[t + (long long)s.rntx * (rj + (long long)(nmax[1] + 1) * rk)];
            }
        }
        if (!__syncthreads_or(any)) {
            if (in && !s.accumulate)
                for (int q = 0; q < S::NS; ++q) s.z[q * NP + o] = 0.0;
            return;
        }
    }
    const double w = in ? weight(gi, gj, gk) : 0.0;
    double xv[S::NS], av[S::NS], rv[S::NS], dv[S::NS], cv[S::NS];
#pragma unroll
    for (int q = 0; q < S::NS; ++q) {
        xv[q] = 0.0;
        av[q] = in ? s.a[q * NP + o] : 0.0;
        rv[q] = in ? w * s.r[q * NP + o] : 0.0;
        dv[q] = in ? s.dinv[q * NP + o] : 0.0;
        cv[q] = (in && q > 0) ? s.c[q * NP + o] : 0.0;
    }
    // face coefficients on the extended brick and one anchor beyond (the
    // padded arrays are zero outside each face set)
    for (int e = threadIdx.x; e < NK; e += T) {
        const int ei = e % EK, ej = (e / EK) % EK, ek = DIM == 3 ? e / (EK * EK) : 0;
        const int fi = lo[0] - 1 + ei, fj = lo[1] - 1 + ej, fk = lo[2] - 1 + ek;
        const bool fin = fi >= -1 && fi <= nmax[0] + 1 && fj >= -1 && fj <= nmax[1] + 1 &&
                         (DIM == 2 || (fk >= -1 && fk <= nmax[2] + 1));
        const long long fo = fin ? gidx(fi, fj, fk) : 0;
        for (int f = 0; f < S::NF; ++f) {
            sk[f][e] = fin ? s.K[f * NP + fo] : 0.0;
            sg[f][e] = 0.0;
        }
    }
    __syncthreads();

    // local index of the face anchored at this anchor + (dx, dy, dz)
    auto fidx = [&](const Term& tm) {
        return (li + tm.dx + 1) + EK * ((lj + tm.dy + 1) + EK * (DIM == 3 ? lk + tm.dz + 1 : 0));
    };
    const int par_l = (lo[0] + li + lo[1] + lj + lo[2] + lk) & 1;
    constexpr int NCOL = 2 * S::NS;
#pragma unroll
    for (int sweep = 0; sweep < 2; ++sweep) {
#pragma unroll
        for (int cc = 0; cc < NCOL; ++cc) {
            const int col = sweep == 0 ? cc : NCOL - 1 - cc;
            const int q = col >> 1, par = col & 1;
            // samples of one colour share no face: their updates of the face
            // values below never meet
            if (mine && par_l == par && av[q] != 0.0) {
                double y = 0.0;
#pragma unroll
                for (int t = 0; t < S::ST; ++t) {
                    const Term tm = samp_term<DIM>(q, t);
                    if (tm.s == 0) continue;
                    const int fe = fidx(tm);
                    y += (double)tm.s * sk[tm.q][fe] * sg[tm.q][fe];
                }
                const double aq = av[q];
                y *= aq;
                if (q > 0) y += cv[q] * xv[q];
                if (DIM == 3 && (q == 1 || q == 2)) {
                    const double cross = 0.5 * fmin(cv[1], cv[2]);
                    y += cross * xv[q == 1 ? 2 : 1];
                }
                const double dx = (rv[q] - y) * dv[q];
                xv[q] += dx;
#pragma unroll
                for (int t = 0; t < S::ST; ++t) {
                    const Term tm = samp_term<DIM>(q, t);
                    if (tm.s == 0) continue;
                    sg[tm.q][fidx(tm)] += (double)tm.s * aq * dx;
                }
            }
            __syncthreads();
        }
    }

    // write (or add) the correction of the active samples
    if (in) {
#pragma unroll
        for (int q = 0; q < S::NS; ++q) {
            if (s.accumulate) {
                if (av[q] != 0.0) s.z[q * NP + o] += w * xv[q];
            } else {
                s.z[q * NP + o] = xv[q];
            }
        }
    }
}

// ---- PCG on the padded FP64 vectors (slot sc of the context's scalars) ----
// The vector kernels visit, in 3D, the kRow3X-anchor rows of the sample slices
// whose row bit is set (kRow3X lanes per row, from the compacted list that
// launch_row_list builds; every vector of the solve is zero on the other
// rows) and, in 2D, the whole padded arrays.
template <typename F>
__device__ __forceinline__ void pcg_sweep(const Geo& g, const RowList& rl, F f) {
    if (rl.count >= 0) {
        constexpr int RW = kRow3X;
        const int rntx = (g.nx + RW) / RW;
        const long long nrow = (long long)rntx * (g.ny + 1) * (g.nz + 1);
        const int lane = threadIdx.x % RW;
        const long long stride = (long long)gridDim.x * (NT / RW);
        for (long long w = ((long long)blockIdx.x * NT + threadIdx.x) / RW; w < rl.count; w += stride) {
            const long long u = rl.list[w];
            const int s = (int)(u / nrow);
            const long long row = u - s * nrow;
            const int t = (int)(row % rntx);
            const long long jk = row / rntx;
            const int i = t * RW + lane;
            if (i <= g.nx) f(s * g.NP + g.idx(i, (int)(jk % (g.ny + 1)), (int)(jk / (g.ny + 1))));
        }
    } else {
        const long long n = (long long)g.nsamp() * g.NP;
        for (long long t = (long long)blockIdx.x * NT + threadIdx.x; t < n;
             t += (long long)gridDim.x * NT)
            f(t);
    }
}

// Ordered compaction of the (slice, row) pairs whose row bit is set, item
// u = s * nrow + row: per-chunk counts, one scan of the counts, then each
// chunk writes its items in order (so every sweep of the list, and every dot
// product over it, runs in the same order on every call).
constexpr int RL_PER = 16, RL_CHUNK = NT * RL_PER;

__device__ __forceinline__ bool row_item(const RowBits* __restrict__ rows, long long nrow,
                                         long long u) {
    const int s = (int)(u / nrow);
    const unsigned rb = rows[u - s * nrow];
    return ((rb | (rb >> 6)) >> s) & 1u;
}

__global__ __launch_bounds__(NT) void k_rl_count(const RowBits* __restrict__ rows, long long nrow,
                                                 long long n, int* __restrict__ cnt) {
    const long long base = (long long)blockIdx.x * RL_CHUNK + (long long)threadIdx.x * RL_PER;
    int c = 0;
    for (int e = 0; e < RL_PER; ++e)
        if (base + e < n && row_item(rows, nrow, base + e)) ++c;
    __shared__ int sh[NT];
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[blockIdx.x] = sh[0];
}

// exclusive scan of the nchunk counts in place; the total goes to cnt[nchunk]
__global__ __launch_bounds__(1024) void k_rl_scan(int* __restrict__ cnt, int nchunk) {
    __shared__ int sh[1024];
    const int per = (nchunk + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(nchunk, lo + per);
    int c = 0;
    for (int t = lo; t < hi; ++t) c += cnt[t];
    sh[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int q = 0; q < 1024; ++q) {
            const int v = sh[q];
            sh[q] = run;
            run += v;
        }
        cnt[nchunk] = run;
    }
    __syncthreads();
    int run = sh[threadIdx.x];
    for (int t = lo; t < hi; ++t) {
        const int v = cnt[t];
        cnt[t] = run;
        run += v;
    }
}

__global__ __launch_bounds__(NT) void k_rl_write(const RowBits* __restrict__ rows, long long nrow,
                                                 long long n, const int* __restrict__ off,
                                                 int* __restrict__ list) {
    const long long base = (long long)blockIdx.x * RL_CHUNK + (long long)threadIdx.x * RL_PER;
    int c = 0;
    for (int e = 0; e < RL_PER; ++e)
        if (base + e < n && row_item(rows, nrow, base + e)) ++c;
    __shared__ int sh[NT];
    sh[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int q = 0; q < NT; ++q) {
            const int v = sh[q];
            sh[q] = run;
            run += v;
        }
    }
    __syncthreads();
    int w = off[blockIdx.x] + sh[threadIdx.x];
    for (int e = 0; e < RL_PER; ++e)
        if (base + e < n && row_item(rows, nrow, base + e)) list[w++] = (int)(base + e);
}

__global__ __launch_bounds__(NT) void k_pcg_dot(Geo g, RowList rl, const double* __restrict__ u,
                                                const double* __restrict__ v,
                                                double* __restrict__ part, const int* done) {
    if (done && *done) return;
    double acc = 0.0;
    pcg_sweep(g, rl, [&](long long t) { acc += u[t] * v[t]; });
    double vv[1] = {acc};
    block_partial<1, NT>(vv, part, gridDim.x, blockIdx.x);
}

__device__ double sum_parts(const double* __restrict__ part, int nb) {
    __shared__ double sw[NT / 64];
    double acc = 0.0;
    for (int t = threadIdx.x; t < nb; t += NT) acc += part[t];
    acc = wave_sum64(acc);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < NT / 64; ++w) tot += sw[w];
    return tot;
}

// start: bb = b.b from the partials, iteration 0
// start (keep_bb = 0: bb = b.b from the partials) or restart from the true
// residual (keep_bb = 1: rr from the partials, bb kept)
__global__ __launch_bounds__(NT) void k_pcg_start(const double* part, int nb, Scalars* S,
                                                  double tol, int max_iter, int keep_bb) {
    const double v = sum_parts(part, nb);
    if (threadIdx.x == 0) {
        if (!keep_bb) S->bb = v;
        const double bb = S->bb;
        S->rr = v;
        S->tol2 = tol * tol;
        S->iter = 0;
        S->max_iter = max_iter;
        S->done = bb > 0.0 ? 0 : 1;
        S->rz[0] = S->rz[1] = 0.0;
    }
}

// r.z of this iteration -> beta
__global__ __launch_bounds__(NT) void k_pcg_rz(const double* part, int nb, Scalars* S) {
    if (S->done) return;
    const double rz = sum_parts(part, nb);
    if (threadIdx.x == 0) {
        S->beta = S->iter == 0 ? 0.0 : rz / S->rz[0];
        S->rz[0] = rz;
    }
}

__global__ __launch_bounds__(NT) void k_pcg_dir(Geo g, RowList rl, const double* __restrict__ z,
                                                double* __restrict__ p, const Scalars* S) {
    if (S->done) return;
    const double beta = S->beta;
    pcg_sweep(g, rl, [&](long long t) { p[t] = z[t] + beta * p[t]; });
}

// p.Ap -> alpha (breakdown when p.Ap <= 0 or non-finite)
__global__ __launch_bounds__(NT) void k_pcg_pq(const double* part, int nb, Scalars* S) {
    if (S->done) return;
    const double pq = sum_parts(part, nb);
    if (threadIdx.x == 0) {
        S->pq = pq;
        if (!(pq > 0.0) || !isfinite(pq)) {
            S->done = 3;
        } else {
            S->alpha = S->rz[0] / pq;
        }
    }
}

__global__ __launch_bounds__(NT) void k_pcg_update(Geo g, RowList rl, double* __restrict__ x,
                                                   double* __restrict__ r,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ q, const Scalars* S,
                                                   double* __restrict__ part) {
    if (S->done) return;
    const double alpha = S->alpha;
    double acc = 0.0;
    pcg_sweep(g, rl, [&](long long t) {
        x[t] += alpha * p[t];
        const double rn = r[t] - alpha * q[t];
        r[t] = rn;
        acc += rn * rn;
    });
    double vv[1] = {acc};
    block_partial<1, NT>(vv, part, gridDim.x, blockIdx.x);
}

// r.r -> stop test, next iteration
__global__ __launch_bounds__(NT) void k_pcg_check(const double* part, int nb, Scalars* S) {
    if (S->done) return;
    const double rr = sum_parts(part, nb);
    if (threadIdx.x == 0) {
        S->rr = rr;
        S->iter += 1;
        if (rr <= S->tol2 * S->bb)
            S->done = 1;
        else if (!isfinite(rr))
            S->done = 3;
        else if (S->iter >= S->max_iter)
            S->done = 2;
    }
}

template <int DIM, int B, int OV>
void sgs_launch(const Geo& g, const SgsArgs& base, hipStream_t st) {
    const int n[3] = {g.nx, g.ny, g.nz};
    SgsArgs s = base;
    for (int a = 0; a < 3; ++a) s.nb[a] = a < DIM ? (n[a] + 1 + B - 1) / B : 1;
    if (OV == 0) {
        long long nbk = 1;
        for (int a = 0; a < DIM; ++a) {
            s.cls[a] = -1;
            nbk *= s.nb[a];
        }
        for (int a = DIM; a < 3; ++a) s.cls[a] = -1;
        s.accumulate = 0;
        hipLaunchKernelGGL((k_sgs_bricks<DIM, B, OV>), dim3((unsigned)nbk),
                           dim3(BrickShape<DIM, B, OV>::T), 0, st, g, s);
        return;
    }
    s.accumulate = 1;
    for (int cls = 0; cls < (1 << DIM); ++cls) {
        long long nbk = 1;
        for (int a = 0; a < 3; ++a) {
            if (a < DIM) {
                s.cls[a] = (cls >> a) & 1;
                nbk *= (s.nb[a] - s.cls[a] + 1) / 2;
            } else {
                s.cls[a] = -1;
            }
        }
        if (nbk == 0) continue;
        hipLaunchKernelGGL((k_sgs_bricks<DIM, B, OV>), dim3((unsigned)nbk),
                           dim3(BrickShape<DIM, B, OV>::T), 0, st, g, s);
    }
}

}  // namespace

int schwarz_brick(int dim, int overlap) {
    (void)overlap;
    return dim == 2 ? 16 : 4;
}

void launch_schwarz(const Geo& g, int overlap, const double* r, const double* a, const double* c,
                    const double* dinv, const double* K, const RowBits* rows, double* z,
                    const int* done, hipStream_t st) {
    SgsArgs s{};
    s.rows = g.dim == 3 ? rows : nullptr;
    s.rntx = (g.nx + kRow3X) / kRow3X;
    s.r = r;
    s.a = a;
    s.c = c;
    s.dinv = dinv;
    s.K = K;
    s.z = z;
    s.done = done;
    if (overlap > 0) launch_fill(z, (long long)g.nsamp() * g.NP, 0.0, st);
    if (g.dim == 2) {
        if (overlap > 0)
            sgs_launch<2, 16, 1>(g, s, st);
        else
            sgs_launch<2, 16, 0>(g, s, st);
    } else {
        if (overlap > 0)
            sgs_launch<3, 4, 1>(g, s, st);
        else
            sgs_launch<3, 4, 0>(g, s, st);
    }
}

int pcg_blocks(const Geo& g) { return vec_grid_blocks(g); }

void launch_pcg_dot(const Geo& g, const RowList& rl, const double* u, const double* v,
                    double* part, const int* done, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_dot, dim3(pcg_blocks(g)), dim3(NT), 0, st, g, rl, u, v, part, done);
}
void launch_pcg_start(const double* part, int nb, Scalars* S, double tol, int max_iter,
                      bool keep_bb, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(NT), 0, st, part, nb, S, tol, max_iter,
                       keep_bb ? 1 : 0);
}
void launch_pcg_rz(const double* part, int nb, Scalars* S, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_rz, dim3(1), dim3(NT), 0, st, part, nb, S);
}
void launch_pcg_dir(const Geo& g, const RowList& rl, const double* z, double* p,
                    const Scalars* S, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_dir, dim3(pcg_blocks(g)), dim3(NT), 0, st, g, rl, z, p, S);
}
void launch_pcg_pq(const double* part, int nb, Scalars* S, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_pq, dim3(1), dim3(NT), 0, st, part, nb, S);
}
void launch_pcg_update(const Geo& g, const RowList& rl, double* x, double* r, const double* p,
                       const double* q, const Scalars* S, double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_update, dim3(pcg_blocks(g)), dim3(NT), 0, st, g, rl, x, r, p, q, S,
                       part);
}

long long row_items(const Geo& g) { return row_bytes(g) * g.nsamp(); }

int row_list_chunks(const Geo& g) { return (int)((row_items(g) + RL_CHUNK - 1) / RL_CHUNK); }

void launch_row_list(const Geo& g, const RowBits* rows, int* list, int* cnt, hipStream_t st) {
    const long long nrow = row_bytes(g), n = row_items(g);
    const int nchunk = row_list_chunks(g);
    hipLaunchKernelGGL(k_rl_count, dim3(nchunk), dim3(NT), 0, st, rows, nrow, n, cnt);
    hipLaunchKernelGGL(k_rl_scan, dim3(1), dim3(1024), 0, st, cnt, nchunk);
    hipLaunchKernelGGL(k_rl_write, dim3(nchunk), dim3(NT), 0, st, rows, nrow, n, cnt, list);
}
void launch_pcg_check(const double* part, int nb, Scalars* S, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(NT), 0, st, part, nb, S);
}

}  // namespace vfs
