// Batched 2D solves: many independent problems of different sizes in one
// persistent launch.
//
// Every problem has its own padded arrays (assembled by the single-problem
// kernels).  Work items are (problem, 2D tile) pairs, statically split into
// contiguous chunks per workgroup.  One persistent kernel runs the whole
// mixed-precision solve of every problem: FP32 Jacobi-PCG inner solves and
// FP64 iterative refinement, as a per-problem state machine whose phases are
// separated by a grid barrier.  A problem's reductions use the same
// fence-free partials as the single-problem path (one partial per item,
// summed in a fixed order by every item of that problem; a workgroup caches
// the totals of the problem it is working on).  Each problem retires on its
// own as soon as its FP64 residual meets the tolerance, stamping the device
// wall clock.
//
// Refinement: with the FP64 residual r64 known, an inner solve finds
// A32 d = r64/|r64| in FP32 to the inner tolerance, then x64 += |r64| d and
// r64 = b - A64 x64 (FP64) decide whether the problem needs another one.
//
// The grid barrier spins on a generation counter with a wall-clock deadline:
// on timeout it raises an abort flag that every waiting workgroup also
// observes, so the grid always drains.
#include <algorithm>

#include "vfs_batch.h"
#include "vfs_reduce.h"

namespace vfs {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ bool grid_barrier(BatchCtl* ctl, unsigned nblocks) {
    // every wave's global stores are acknowledged by L2 before thread 0
    // publishes them (agent-scope release: L2 write-back for the other XCDs)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __shared__ int s_abort;
    if (threadIdx.x == 0) {
        // the generation is read (and waited for) before arriving
        const unsigned my_gen =
            __hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned arrived =
            __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int abort = 0;
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctl->bar_gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long deadline = wall_clock64() + ctl->spin_ticks;
            // relaxed polling: coherent loads without cache invalidation
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                   my_gen) {
                if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    abort = 1;
                    break;
                }
                if (wall_clock64() > deadline) {
                    __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    abort = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) abort = 1;
        // one acquire for the whole workgroup (invalidates this CU's caches)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_abort = abort;
    }
    __syncthreads();
    return s_abort == 0;
}

// Sum of nv-vector partials [p.item0, p.item0 + p.nt) (layout part[w * nv + q]).
template <int NV>
__device__ __forceinline__ void problem_total(const double* __restrict__ part, int item0, int nt,
                                              double (&tot)[NV]) {
    constexpr int NW = NT / 64;
    __shared__ double sr[NV][NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nt; b += NT) s += part[(long long)(item0 + b) * NV + q];
        s = wave_sum64(s);
        if (lane == 0) sr[q][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = sr[q][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += sr[q][w];
        tot[q] = s;
    }
    __syncthreads();
}

template <int NV>
__device__ __forceinline__ void item_partial(double (&v)[NV], double* __restrict__ part, int w) {
    constexpr int NW = NT / 64;
    __shared__ double sw[NV][NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum64(v[q]);
        if (lane == 0) sw[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = sw[q][0];
#pragma unroll
            for (int w2 = 1; w2 < NW; ++w2) s += sw[q][w2];
            part[(long long)w * NV + q] = s;
        }
    }
    __syncthreads();
}

// One 2D tile of the fused apply on problem pb (same arithmetic as the
// single-problem kernel).  MODE 0: direction p = z + beta p_in, q = A p,
// returns this thread's share of p.q.  MODE 2: r = b - A x (FP64), returns r.r.
template <typename T, int BX, int BY, int MODE>
__device__ double tile_apply(const Geo& g, int i0, int j0, const T* __restrict__ r,
                             const T* __restrict__ dinv, const T* __restrict__ pin,
                             T* __restrict__ pout, T* __restrict__ q, const T* __restrict__ a,
                             const T* __restrict__ c, const T* __restrict__ K,
                             const T* __restrict__ bv, T beta, bool first, T* lds) {
    // lds layout: sW[3][BY+2][BX+2], sV[3][BY+2][BX+2], sG[2][BY+1][BX+1]
    constexpr int HX = BX + 2, HY = BY + 2, FX = BX + 1, FY = BY + 1;
    T* sW = lds;
    T* sV = lds + 3 * HX * HY;
    T* sG = lds + 6 * HX * HY;
    const long long NP = g.NP;
    const int tid = threadIdx.x;
    for (int e = tid; e < HX * HY; e += NT) {
        const int li = e % HX, lj = e / HX;
        const int i = i0 - 1 + li, j = j0 - 1 + lj;
        T v[3] = {T(0), T(0), T(0)};
        T w[3] = {T(0), T(0), T(0)};
        if (i <= g.nx + 1 && j <= g.ny + 1) {
            const long long o = g.idx(i, j);
            const bool own = li >= 1 && li <= BX && lj >= 1 && lj <= BY && i <= g.nx && j <= g.ny;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const long long os = o + s * NP;
                T val;
                if (MODE == 0) {
                    const T z = dinv[os] * r[os];
                    val = first ? z : z + beta * pin[os];
                    if (own) pout[os] = val;
                } else {
                    val = pin[os];
                }
                v[s] = val;
                w[s] = a[os] * val;
            }
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            sV[(s * HY + lj) * HX + li] = v[s];
            sW[(s * HY + lj) * HX + li] = w[s];
        }
    }
    __syncthreads();
#define W_(s, y, x) sW[((s) * HY + (y)) * HX + (x)]
    for (int e = tid; e < FX * FY; e += NT) {
        const int li = e % FX, lj = e / FX;
        {
            const int i = i0 + li, j = j0 - 1 + lj;
            T gv = T(0);
            if (i <= g.nx && j >= 0 && j < g.ny) {
                const T k = K[g.idx(i, j)];
                gv = k * ((W_(0, lj, li + 1) - W_(0, lj, li)) + (W_(1, lj, li) - W_(1, lj, li + 1)) +
                          (W_(2, lj, li + 1) - W_(2, lj + 1, li + 1)));
            }
            sG[(0 * FY + lj) * FX + li] = gv;
        }
        {
            const int i = i0 - 1 + li, j = j0 + lj;
            T gv = T(0);
            if (i >= 0 && i < g.nx && j <= g.ny) {
                const T k = K[NP + g.idx(i, j)];
                gv = k * ((W_(0, lj + 1, li) - W_(0, lj, li)) + (W_(1, lj + 1, li) - W_(1, lj, li)) +
                          (W_(2, lj + 1, li) - W_(2, lj + 1, li + 1)));
            }
            sG[(1 * FY + lj) * FX + li] = gv;
        }
    }
#undef W_
    __syncthreads();
    double acc = 0.0;
    for (int e = tid; e < BX * BY; e += NT) {
        const int tx = e % BX, ty = e / BX;
        const int i = i0 + tx, j = j0 + ty;
        if (i > g.nx || j > g.ny) continue;
        const long long o = g.idx(i, j);
#define G_(f, y, x) sG[((f) * FY + (y)) * FX + (x)]
        const T gu0 = G_(0, ty + 1, tx), gu1 = G_(0, ty + 1, tx + 1), gum = G_(0, ty, tx);
        const T gv0 = G_(1, ty, tx + 1), gv1 = G_(1, ty + 1, tx + 1), gvm = G_(1, ty, tx);
#undef G_
        const T v0 = sV[(0 * HY + ty + 1) * HX + tx + 1];
        const T v1 = sV[(1 * HY + ty + 1) * HX + tx + 1];
        const T v2 = sV[(2 * HY + ty + 1) * HX + tx + 1];
        const T y0 = a[o] * ((gu0 - gu1) + (gv0 - gv1));
        const T y1 = a[NP + o] * ((gu1 - gu0) + (gv0 - gv1)) + c[NP + o] * v1;
        const T y2 = a[2 * NP + o] * ((gu0 - gum) + (gv0 - gvm)) + c[2 * NP + o] * v2;
        if (MODE == 2) {
            const T r0 = bv[o] - y0, r1 = bv[NP + o] - y1, r2 = bv[2 * NP + o] - y2;
            q[o] = r0;
            q[NP + o] = r1;
            q[2 * NP + o] = r2;
            acc += (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2;
        } else {
            q[o] = y0;
            q[NP + o] = y1;
            q[2 * NP + o] = y2;
            acc += (double)v0 * y0 + (double)v1 * y1 + (double)v2 * y2;
        }
    }
    __syncthreads();   // LDS reuse by the next tile
    return acc;
}

__device__ __forceinline__ void item_of(const BatchArgs& A, int w, int& p, int& i0, int& j0,
                                        int bx, int by) {
    p = A.item_prob[w];
    const int t = w - A.prob[p].item0;
    const int ntx = A.prob[p].ntx;
    i0 = (t % ntx) * bx;
    j0 = (t / ntx) * by;
}

// FP64 residual r64 = b - A64 x64 per item, partial r.r per item.
template <int BX, int BY>
__global__ __launch_bounds__(NT) void k_batch_resid(BatchArgs A) {
    extern __shared__ double lds_dyn[];
    double* lds64 = lds_dyn;
    for (int w = blockIdx.x; w < A.nitems; w += gridDim.x) {
        int p, i0, j0;
        item_of(A, w, p, i0, j0, BX, BY);
        const BProb& P = A.prob[p];
        double acc = 0.0;
        if (A.state[p].needs || A.first_pass)
            acc = tile_apply<double, BX, BY, 2>(P.g, i0, j0, nullptr, nullptr, P.x64, nullptr,
                                                P.r64, P.a64, P.c64, P.K64, P.b64, 0.0, true,
                                                lds64);
        double v[1] = {acc};
        item_partial<1>(v, A.partR, w);
    }
}

// one workgroup per problem: |r64|^2 -> state; decides whether it needs a pass
__global__ __launch_bounds__(NT) void k_batch_finalize(BatchArgs A) {
    const int p = blockIdx.x;
    if (p >= A.nprob) return;
    BState& S = A.state[p];
    if (!(S.needs || A.first_pass)) return;
    double tot[1];
    problem_total<1>(A.partR, A.prob[p].item0, A.prob[p].nt, tot);
    if (threadIdx.x == 0) {
        const double rho2 = tot[0];
        if (A.first_pass) {
            S.bb64 = rho2;
            S.iters_total = 0;
            S.passes = 0;
            S.t_done = 0;
        }
        S.rho2 = rho2;
        const double rel = S.bb64 > 0.0 ? sqrt(rho2 / S.bb64) : 0.0;
        S.rel = rel;
        const int need = (rel > A.tol && S.passes < A.max_passes && S.iters_total < A.max_iter &&
                          isfinite(rel)) ? 1 : 0;
        if (!need && S.t_done == 0) S.t_done = wall_clock64();
        S.needs = need;
        // inner tolerance of the next pass, relative to |r64|
        double ti = rel > 0.0 ? 0.5 * A.tol / rel : 0.5;
        ti = ti < 1e-5 ? 1e-5 : (ti > 0.5 ? 0.5 : ti);
        S.tol_in2 = ti * ti;
    }
}

// x64 = 0 for every problem (first pass)
__global__ __launch_bounds__(NT) void k_batch_zero_x(BatchArgs A) {
    for (int w = blockIdx.x; w < A.nitems; w += gridDim.x) {
        int p, i0, j0;
        item_of(A, w, p, i0, j0, A.bx, A.by);
        const BProb& P = A.prob[p];
        if (w == P.item0 && threadIdx.x == 0) {
            A.state[p].t_start = wall_clock64();
            A.state[p].needs = 0;
        }
        for (int e = threadIdx.x; e < A.bx * A.by; e += NT) {
            const int i = i0 + e % A.bx, j = j0 + e / A.bx;
            if (i > P.g.nx || j > P.g.ny) continue;
            const long long o = P.g.idx(i, j);
            for (int s = 0; s < 3; ++s) P.x64[o + s * P.g.NP] = 0.0;
        }
    }
}

// Resets the barrier / counters of the persistent kernel (a kernel, not a
// memset, so that it can live in a captured graph).
__global__ void k_batch_reset_ctl(BatchCtl* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->bar_count = 0;
        ctl->abort = 0;
        ctl->n_done = 0;
        ctl->n_need = 0;
    }
}

// The persistent solve of every problem, refinement included.  Global
// phases alternate A (even) and B (odd), separated by grid barriers.  Per
// problem, by mode:
//   CG      A: r.z / r.r totals, stop test, direction + FP32 apply, p.q partial
//           B: p.q total, alpha, FP32 update, r.z / r.r partials
//   stop -> AXPY (B: x64 += |r64| x32) -> RESID (A: r64 = b - A64 x64, FP64,
//           |r64|^2 partial) -> DECIDE (B: |r64| total; DONE if it meets tol,
//           else r32 = r64/|r64|, x32 = 0, r.z / r.r partials, back to CG).
// Problems therefore retire independently; their completion time is the
// device wall clock at DONE.
template <int BX, int BY>
__global__ __launch_bounds__(NT) void k_batch_pcg(BatchArgs A) {
    extern __shared__ double lds_dyn[];
    float* lds32 = reinterpret_cast<float*>(lds_dyn);
    double* lds64 = lds_dyn;
    BatchCtl* ctl = A.ctl;
    const unsigned G = gridDim.x;
    const int per = (A.nitems + G - 1) / G;
    const int w0 = min(A.nitems, (int)blockIdx.x * per), w1 = min(A.nitems, w0 + per);

    // initialise the r32 of problems that need a solve (first inner solve)
    auto init_inner = [&](const BProb& P, int i0, int j0, double rho2, double (&v)[2]) {
        const double inv = rho2 > 0.0 ? 1.0 / sqrt(rho2) : 0.0;
        for (int e = threadIdx.x; e < BX * BY; e += NT) {
            const int i = i0 + e % BX, j = j0 + e / BX;
            if (i > P.g.nx || j > P.g.ny) continue;
            const long long o = P.g.idx(i, j);
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const long long os = o + s * P.g.NP;
                const float ri = (float)(P.r64[os] * inv);
                const float zi = P.dinv[os] * ri;
                P.r32[os] = ri;
                P.x32[os] = 0.f;
                v[0] += (double)ri * (double)zi;
                v[1] += (double)ri * (double)ri;
            }
        }
    };

    // phase "-1": initial modes
    for (int w = w0; w < w1; ++w) {
        int p, i0, j0;
        item_of(A, w, p, i0, j0, BX, BY);
        const BProb& P = A.prob[p];
        BState& S = A.state[p];
        double v[2] = {0.0, 0.0};
        if (S.needs) init_inner(P, i0, j0, S.rho2, v);
        if (w == P.item0 && threadIdx.x == 0) {
            S.ph[0].mode = S.needs ? BM_CG : BM_DONE;
            S.ph[0].kloc = 0;
            if (S.needs)
                __hip_atomic_fetch_add(&ctl->n_need, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        item_partial<2>(v, A.partB, w);
    }
    if (!grid_barrier(ctl, G)) return;
    const int n_need = __hip_atomic_load(&ctl->n_need, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n_need == 0) return;

    for (int phi = 0;; phi += 2) {
        // ------------------------------------------------------------ phase A
        {
            const int cs = phi & 1, ns = cs ^ 1;
            int cached = -1;
            double rzk = 0.0, rrk = 0.0;
            for (int w = w0; w < w1; ++w) {
                int p, i0, j0;
                item_of(A, w, p, i0, j0, BX, BY);
                const BProb& P = A.prob[p];
                BState& S = A.state[p];
                const BPhase cur = S.ph[cs];
                const bool owner = w == P.item0 && threadIdx.x == 0;
                BPhase nxt = cur;
                if (cur.mode == BM_CG) {
                    const int k = cur.kloc;
                    if (p != cached) {
                        double tot[2];
                        problem_total<2>(A.partB, P.item0, P.nt, tot);
                        rzk = tot[0];
                        rrk = tot[1];
                        cached = p;
                    }
                    const double bb = k == 0 ? rrk : S.bb;
                    const bool stop = !isfinite(rzk) || !isfinite(rrk) || rrk <= S.tol_in2 * bb ||
                                      k >= A.max_iter_pass || S.iters_total + k >= A.max_iter;
                    const double beta = k == 0 ? 0.0 : rzk / S.rz[(k + 1) & 1];
                    double v[1] = {0.0};
                    if (!stop) {
                        float* pin = (k & 1) ? P.p1 : P.p0;
                        float* pout = (k & 1) ? P.p0 : P.p1;
                        v[0] = tile_apply<float, BX, BY, 0>(P.g, i0, j0, P.r32, P.dinv, pin, pout,
                                                            P.q32, P.a, P.c, P.K, nullptr,
                                                            (float)beta, k == 0, lds32);
                    }
                    item_partial<1>(v, A.partA, w);
                    if (owner) {
                        S.rz[k & 1] = rzk;
                        if (k == 0) S.bb = bb;
                        if (stop) {
                            S.last_iter = k;
                            nxt.mode = BM_AXPY;
                        }
                    }
                } else if (cur.mode == BM_RESID) {
                    double v[1];
                    v[0] = tile_apply<double, BX, BY, 2>(P.g, i0, j0, nullptr, nullptr, P.x64,
                                                         nullptr, P.r64, P.a64, P.c64, P.K64,
                                                         P.b64, 0.0, true, lds64);
                    item_partial<1>(v, A.partR, w);
                    nxt.mode = BM_DECIDE;
                }
                if (owner) S.ph[ns] = nxt;
            }
        }
        // stops are counted only in phase B, so n_done is stable during phase A
        const int nd = __hip_atomic_load(&ctl->n_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!grid_barrier(ctl, G)) return;
        if (nd >= n_need) break;
        // ------------------------------------------------------------ phase B
        {
            const int cs = (phi + 1) & 1, ns = cs ^ 1;
            int cached = -1;
            double pq = 0.0;
            for (int w = w0; w < w1; ++w) {
                int p, i0, j0;
                item_of(A, w, p, i0, j0, BX, BY);
                const BProb& P = A.prob[p];
                BState& S = A.state[p];
                const BPhase cur = S.ph[cs];
                const bool owner = w == P.item0 && threadIdx.x == 0;
                BPhase nxt = cur;
                if (cur.mode == BM_CG) {
                    const int k = cur.kloc;
                    if (p != cached) {
                        double tot[1];
                        problem_total<1>(A.partA, P.item0, P.nt, tot);
                        pq = tot[0];
                        cached = p;
                    }
                    const float alpha = (pq > 0.0 && isfinite(pq)) ? (float)(S.rz[k & 1] / pq) : 0.f;
                    const float* pk = (k & 1) ? P.p0 : P.p1;
                    double v[2] = {0.0, 0.0};
                    for (int e = threadIdx.x; e < BX * BY; e += NT) {
                        const int i = i0 + e % BX, j = j0 + e / BX;
                        if (i > P.g.nx || j > P.g.ny) continue;
                        const long long o = P.g.idx(i, j);
#pragma unroll
                        for (int s = 0; s < 3; ++s) {
                            const long long os = o + s * P.g.NP;
                            const float ri = P.r32[os] - alpha * P.q32[os];
                            const float zi = P.dinv[os] * ri;
                            P.x32[os] = P.x32[os] + alpha * pk[os];
                            P.r32[os] = ri;
                            v[0] += (double)ri * (double)zi;
                            v[1] += (double)ri * (double)ri;
                        }
                    }
                    item_partial<2>(v, A.partB, w);
                    nxt.kloc = k + 1;
                } else if (cur.mode == BM_AXPY) {
                    const double rho = sqrt(S.rho2);
                    for (int e = threadIdx.x; e < BX * BY; e += NT) {
                        const int i = i0 + e % BX, j = j0 + e / BX;
                        if (i > P.g.nx || j > P.g.ny) continue;
                        const long long o = P.g.idx(i, j);
#pragma unroll
                        for (int s = 0; s < 3; ++s)
                            P.x64[o + s * P.g.NP] += rho * (double)P.x32[o + s * P.g.NP];
                    }
                    if (owner) {
                        S.iters_total += S.last_iter;
                        S.passes += 1;
                    }
                    nxt.mode = BM_RESID;
                } else if (cur.mode == BM_DECIDE) {
                    double tot[1];
                    problem_total<1>(A.partR, P.item0, P.nt, tot);
                    const double rho2 = tot[0];
                    const double rel = S.bb64 > 0.0 ? sqrt(rho2 / S.bb64) : 0.0;
                    const bool fin = !(rel > A.tol) || !isfinite(rel) || S.passes >= A.max_passes ||
                                     S.iters_total >= A.max_iter;
                    double v[2] = {0.0, 0.0};
                    if (!fin) init_inner(P, i0, j0, rho2, v);
                    item_partial<2>(v, A.partB, w);
                    if (owner) {
                        S.rho2 = rho2;
                        S.rel = rel;
                        if (fin) {
                            nxt.mode = BM_DONE;
                            S.t_done = wall_clock64();
                            S.needs = 0;
                            __hip_atomic_fetch_add(&ctl->n_done, 1, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        } else {
                            double ti = rel > 0.0 ? 0.5 * A.tol / rel : 0.5;
                            ti = ti < 1e-5 ? 1e-5 : (ti > 0.5 ? 0.5 : ti);
                            S.tol_in2 = ti * ti;
                            nxt.mode = BM_CG;
                            nxt.kloc = 0;
                        }
                    }
                }
                if (owner) S.ph[ns] = nxt;
            }
        }
        if (!grid_barrier(ctl, G)) return;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// variants: (BX, BY) tile shapes
// ---------------------------------------------------------------------------
static const int kVar[kBatchVariants][2] = {{64, 4}, {64, 8}, {32, 8}, {128, 2}};

void batch_tile_shape(int variant, int* bx, int* by) {
    *bx = kVar[variant][0];
    *by = kVar[variant][1];
}

size_t batch_lds_bytes(int variant, int word) {
    const int bx = kVar[variant][0], by = kVar[variant][1];
    return (size_t)word * (6 * (bx + 2) * (by + 2) + 2 * (bx + 1) * (by + 1));
}

template <int BX, int BY>
static void launch_variant(int which, const BatchArgs& A, int grid, hipStream_t s) {
    const size_t l32 = (size_t)4 * (6 * (BX + 2) * (BY + 2) + 2 * (BX + 1) * (BY + 1));
    const size_t l64 = 2 * l32;
    switch (which) {
        case 0: hipLaunchKernelGGL((k_batch_pcg<BX, BY>), dim3(grid), dim3(NT), l64, s, A); break;
        case 1: hipLaunchKernelGGL((k_batch_resid<BX, BY>), dim3(grid), dim3(NT), l64, s, A); break;
    }
}

void launch_batch_pcg(int variant, const BatchArgs& A, int grid, hipStream_t s) {
    switch (variant) {
        case 0: launch_variant<64, 4>(0, A, grid, s); break;
        case 1: launch_variant<64, 8>(0, A, grid, s); break;
        case 2: launch_variant<32, 8>(0, A, grid, s); break;
        default: launch_variant<128, 2>(0, A, grid, s); break;
    }
}

void launch_batch_resid(int variant, const BatchArgs& A, int grid, hipStream_t s) {
    switch (variant) {
        case 0: launch_variant<64, 4>(1, A, grid, s); break;
        case 1: launch_variant<64, 8>(1, A, grid, s); break;
        case 2: launch_variant<32, 8>(1, A, grid, s); break;
        default: launch_variant<128, 2>(1, A, grid, s); break;
    }
}

void launch_batch_finalize(const BatchArgs& A, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_finalize, dim3(A.nprob), dim3(NT), 0, s, A);
}

void launch_batch_zero_x(const BatchArgs& A, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_zero_x, dim3(grid), dim3(NT), 0, s, A);
}

void launch_batch_reset_ctl(BatchCtl* ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset_ctl, dim3(1), dim3(64), 0, s, ctl);
}

int batch_pcg_occupancy(int variant, int* blocks_per_cu) {
    hipError_t e;
    int nb = 0;
    const size_t l32 = batch_lds_bytes(variant, 8);
    switch (variant) {
        case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pcg<64, 4>, NT, l32); break;
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pcg<64, 8>, NT, l32); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pcg<32, 8>, NT, l32); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pcg<128, 2>, NT, l32); break;
    }
    *blocks_per_cu = nb;
    return e == hipSuccess ? 0 : -1;
}

}  // namespace vfs
