// Batched 2D solves: many independent problems of different sizes in one
// persistent launch.
//
// Every problem has its own padded arrays (assembled by the single-problem
// kernels).  Work items are (problem, 2D tile) pairs over the tiles holding
// an active sample, rebuilt after each assembly and dealt round-robin over
// the workgroups; the other tiles' vectors are zeroed at the start of the
// solve and never touched.  One persistent kernel runs the whole
// mixed-precision solve of every problem: FP32 Jacobi-PCG inner solves and
// FP64 iterative refinement, as a per-problem state machine whose phases are
// separated by a grid barrier.  An inner CG iteration takes one phase: the
// one-reduction form of the fused single-problem kernel (the update of the
// previous iteration carried out lazily on each tile and its halo, the next
// r.z from the expansion r.z - 2 alpha q.D^-1 r + alpha^2 q.D^-1 q), with r,
// p and q double-buffered by iteration parity and the five partials of a
// problem alternating between two regions.  A problem's reductions use the
// same fence-free partials as the single-problem path (one partial per item,
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
    // publishes them
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __shared__ int s_abort;
    if (threadIdx.x == 0) {
        // the generation is read (and waited for) before arriving
        const unsigned my_gen =
            __hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        // two-level arrival: group counter, then (last of the group) the top
        // counter; acquire-release RMWs chain every workgroup's writes to the
        // one that advances the generation (agent scope: L2 write-back for
        // the other XCDs)
        const unsigned gi = blockIdx.x % kBarGroups;
        const unsigned ngrp = nblocks < (unsigned)kBarGroups ? nblocks : (unsigned)kBarGroups;
        const unsigned gsz = (nblocks - gi + kBarGroups - 1) / kBarGroups;
        unsigned* grp = &ctl->bar_grp[gi * kBarStride];
        int abort = 0;
        bool advanced = false;
        if (__hip_atomic_fetch_add(grp, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gsz - 1) {
            __hip_atomic_store(grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL,
                                       __HIP_MEMORY_SCOPE_AGENT) == ngrp - 1) {
                __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&ctl->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                advanced = true;
            }
        }
        if (!advanced) {
            const long long deadline = wall_clock64() + (long long)ctl->spin_ticks;
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

// One 2D tile of the FP64 residual r = b - A x (the single-problem apply's
// arithmetic); returns this thread's share of r.r.
template <int BX, int BY>
__device__ double tile_resid(const Geo& g, int i0, int j0, const double* __restrict__ xin,
                             double* __restrict__ rout, const double* __restrict__ a,
                             const double* __restrict__ c, const double* __restrict__ K,
                             const double* __restrict__ bv, double* lds) {
    using T = double;
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
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const long long os = o + s * NP;
                v[s] = xin[os];
                w[s] = a[os] * v[s];
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
        const T v1 = sV[(1 * HY + ty + 1) * HX + tx + 1];
        const T v2 = sV[(2 * HY + ty + 1) * HX + tx + 1];
        const T y0 = a[o] * ((gu0 - gu1) + (gv0 - gv1));
        const T y1 = a[NP + o] * ((gu1 - gu0) + (gv0 - gv1)) + c[NP + o] * v1;
        const T y2 = a[2 * NP + o] * ((gu0 - gum) + (gv0 - gvm)) + c[2 * NP + o] * v2;
        const T r0 = bv[o] - y0, r1 = bv[NP + o] - y1, r2 = bv[2 * NP + o] - y2;
        rout[o] = r0;
        rout[NP + o] = r1;
        rout[2 * NP + o] = r2;
        acc += r0 * r0 + r1 * r1 + r2 * r2;
    }
    __syncthreads();   // LDS reuse by the next tile
    return acc;
}

// One 2D tile of the fused CG iteration k on problem P (the arithmetic of the
// single-problem fused kernel).  INIT (k = 0): z = D^-1 r, p = z, q = A p.
// Otherwise r = r_{k-1} - alpha q_{k-1} on the tile and its halo, x += alpha
// p_{k-1} at the own anchors, z = D^-1 r, p = z + beta p_{k-1}, q = A p.
// Adds this thread's shares of (r.z, p.q, q.z, q.D^-1 q, r.r) to v.
//
// The faces need a p at every position of the tile and its halo, so the
// vectors are kept weighted, as in the fused 3D iteration: the direction as
// P = a p, the residual and A p as R = e r and Q = e q with e = a D^-1.
// Then a p_k = R_{k-1} - alpha Q_{k-1} + beta P_{k-1} takes three loads per
// halo position (R, Q, P) instead of five (r, q, p, D^-1, a).  The own
// anchors read e and a as well and form r = R / e, z = R / a, p = P / a and
// D^-1 = e / a.  INIT reads the plain residual r_0 from the second r buffer
// and writes R_0 = e r_0 to the first.
template <int BX, int BY, bool INIT>
__device__ void tile_fused(const BProb& P, int i0, int j0, float alpha, float beta, int k,
                           float* lds, double (&v)[5]) {
    constexpr int HX = BX + 2, HY = BY + 2, FX = BX + 1, FY = BY + 1;
    constexpr int RPT = BY * BX / NT;             // own anchors per thread
    constexpr int NH = 2 * HX + 2 * BY;           // halo ring of the tile
    constexpr int NHR = (NH + NT - 1) / NT;
    constexpr int NE2 = (FX * FY + NT - 1) / NT;
    static_assert(RPT * NT == BX * BY && NT % BX == 0, "tile must be a multiple of the workgroup");
    const Geo& g = P.g;
    const int pin = (k + 1) & 1, pout = k & 1;
    float* const rv[2] = {P.r32, P.r32b};
    float* const pv[2] = {P.p0, P.p1};
    float* const qv[2] = {P.q32, P.q32b};
    const float* __restrict__ r_in = rv[INIT ? 1 : pin];
    const float* __restrict__ q_in = qv[pin];
    const float* __restrict__ p_in = pv[pin];
    float* __restrict__ r_out = rv[pout];
    float* __restrict__ p_out = pv[pout];
    float* __restrict__ q_out = qv[pout];
    float* __restrict__ x = P.x32;
    const float* __restrict__ ead = P.ead;   // e = a D^-1
    const float* __restrict__ a = P.a;
    const float* __restrict__ c = P.c;
    const float* __restrict__ K = P.K;
    float* sW = lds;                     // a p      [3][HY][HX]
    float* sG = sW + 3 * HY * HX;        // faces    [2][FY][FX]
    const long long NP = g.NP;
    const int tid = threadIdx.x;
    const int tx = tid % BX;
#define L3(arr, s_, y_, x_) arr[((s_) * HY + (y_)) * HX + (x_)]
#define G2(f_, y_, x_) sG[((f_) * FY + (y_)) * FX + (x_)]
    // own anchors (i0 + tx, j0 + ty): the thread that forms p, z there also
    // forms q there, so only a p crosses threads (through LDS)
    float Rr[RPT][3], Ee[RPT][3], Qq[RPT][3], Pp[RPT][3], Aa[RPT][3], Xx[RPT][3], Co[RPT][2];
    bool own[RPT];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + tx, j = j0 + tid / BX + rr * (NT / BX);
        const bool in = i <= g.nx + 1 && j <= g.ny + 1;
        own[rr] = i <= g.nx && j <= g.ny;
        const long long o = in ? g.idx(i, j) : 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const long long os = o + s * NP;
            Rr[rr][s] = Ee[rr][s] = Qq[rr][s] = Pp[rr][s] = Aa[rr][s] = Xx[rr][s] = 0.f;
            if (in) {
                Rr[rr][s] = r_in[os];
                Ee[rr][s] = ead[os];
                Aa[rr][s] = a[os];
                if (!INIT) {
                    Qq[rr][s] = q_in[os];
                    Pp[rr][s] = p_in[os];
                }
            }
            if (!INIT && own[rr]) Xx[rr][s] = x[os];
        }
        Co[rr][0] = own[rr] ? c[NP + o] : 0.f;
        Co[rr][1] = own[rr] ? c[2 * NP + o] : 0.f;
    }
    // halo ring: rows lj = 0 and HY - 1 (corners included), then columns
    // li = 0 and HX - 1; position h = tid + m NT
    float Rh[NHR][3], Eh[NHR][3], Qh[NHR][3], Ph[NHR][3];
    int hli[NHR], hlj[NHR];
#pragma unroll
    for (int m = 0; m < NHR; ++m) {
        const int h = tid + m * NT;
        int li = 0, lj = 0;
        if (h < HX) {
            li = h;
        } else if (h < 2 * HX) {
            li = h - HX;
            lj = HY - 1;
        } else {
            const int e = h - 2 * HX;
            lj = 1 + (e >> 1);
            li = (e & 1) ? HX - 1 : 0;
        }
        hli[m] = li;
        hlj[m] = lj;
        const int i = i0 - 1 + li, j = j0 - 1 + lj;
        const bool in = h < NH && i <= g.nx + 1 && j <= g.ny + 1;
        const long long o = in ? g.idx(i, j) : 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const long long os = o + s * NP;
            Rh[m][s] = Eh[m][s] = Qh[m][s] = Ph[m][s] = 0.f;
            if (in) {
                Rh[m][s] = r_in[os];
                if (INIT) {
                    Eh[m][s] = ead[os];   // to weight the plain residual
                } else {
                    Qh[m][s] = q_in[os];
                    Ph[m][s] = p_in[os];
                }
            }
        }
    }
    float Ku[NE2], Kv[NE2];
#pragma unroll
    for (int m = 0; m < NE2; ++m) {
        const int e = tid + m * NT;
        const int li = e % FX, lj = e / FX;
        Ku[m] = Kv[m] = 0.f;
        if (e < FX * FY) {
            const int iu = i0 + li, ju = j0 - 1 + lj;
            if (iu <= g.nx && ju >= 0 && ju < g.ny) Ku[m] = K[g.idx(iu, ju)];
            const int iv = i0 - 1 + li, jv = j0 + lj;
            if (iv >= 0 && iv < g.nx && jv <= g.ny) Kv[m] = K[NP + g.idx(iv, jv)];
        }
    }
    // R_k and a p_k on the tile and its halo; own anchors also store R, x, P
    // and keep p, z, D^-1
    float Vo[RPT][3], Zo[RPT][3], Dd[RPT][3];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int ty = tid / BX + rr * (NT / BX);
        const long long o = own[rr] ? g.idx(i0 + tx, j0 + ty) : 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const float Rn = INIT ? Ee[rr][s] * Rr[rr][s] : Rr[rr][s] - alpha * Qq[rr][s];
            const float W = INIT ? Rn : Rn + beta * Pp[rr][s];   // a p_k
            const float ia = Aa[rr][s] != 0.f ? 1.f / Aa[rr][s] : 0.f;
            const float ie = Ee[rr][s] != 0.f ? __builtin_amdgcn_rcpf(Ee[rr][s]) : 0.f;
            const float rn = INIT ? Rr[rr][s] : Rn * ie;   // r_k (for the partials only)
            const float zn = Rn * ia;
            if (own[rr]) {
                const long long os = o + s * NP;
                r_out[os] = Rn;
                if (!INIT) x[os] = Xx[rr][s] + alpha * (Pp[rr][s] * ia);
                p_out[os] = W;
                v[0] += (double)rn * (double)zn;
                v[4] += (double)rn * (double)rn;
            }
            Vo[rr][s] = W * ia;
            Zo[rr][s] = zn;
            Dd[rr][s] = Ee[rr][s] * ia;
            L3(sW, s, ty + 1, tx + 1) = W;
        }
    }
#pragma unroll
    for (int m = 0; m < NHR; ++m) {
        if (tid + m * NT >= NH) continue;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const float Rn = INIT ? Eh[m][s] * Rh[m][s] : Rh[m][s] - alpha * Qh[m][s];
            L3(sW, s, hlj[m], hli[m]) = INIT ? Rn : Rn + beta * Ph[m][s];
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NE2; ++m) {
        const int e = tid + m * NT;
        if (e >= FX * FY) continue;
        const int li = e % FX, lj = e / FX;
        G2(0, lj, li) = Ku[m] * ((L3(sW, 0, lj, li + 1) - L3(sW, 0, lj, li)) +
                                 (L3(sW, 1, lj, li) - L3(sW, 1, lj, li + 1)) +
                                 (L3(sW, 2, lj, li + 1) - L3(sW, 2, lj + 1, li + 1)));
        G2(1, lj, li) = Kv[m] * ((L3(sW, 0, lj + 1, li) - L3(sW, 0, lj, li)) +
                                 (L3(sW, 1, lj + 1, li) - L3(sW, 1, lj, li)) +
                                 (L3(sW, 2, lj + 1, li) - L3(sW, 2, lj + 1, li + 1)));
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int ty = tid / BX + rr * (NT / BX);
        if (own[rr]) {
            const long long o = g.idx(i0 + tx, j0 + ty);
            const float gu0 = G2(0, ty + 1, tx), gu1 = G2(0, ty + 1, tx + 1), gum = G2(0, ty, tx);
            const float gv0 = G2(1, ty, tx + 1), gv1 = G2(1, ty + 1, tx + 1), gvm = G2(1, ty, tx);
            float y[3];
            y[0] = Aa[rr][0] * ((gu0 - gu1) + (gv0 - gv1));
            y[1] = Aa[rr][1] * ((gu1 - gu0) + (gv0 - gv1)) + Co[rr][0] * Vo[rr][1];
            y[2] = Aa[rr][2] * ((gu0 - gum) + (gv0 - gvm)) + Co[rr][1] * Vo[rr][2];
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                q_out[o + s * NP] = (Dd[rr][s] * Aa[rr][s]) * y[s];   // e q
                const double yd = y[s];
                v[1] += (double)Vo[rr][s] * yd;
                v[2] += (double)Zo[rr][s] * yd;
                v[3] += (double)Dd[rr][s] * yd * yd;
            }
        }
    }
#undef L3
#undef G2
    __syncthreads();   // LDS reuse by the next tile
}

__device__ __forceinline__ void item_of(const BatchArgs& A, int w, int& p, int& i0, int& j0,
                                        int bx, int by) {
    p = A.item_prob[w];
    const int t = A.item_tile[w];
    const int ntx = A.prob[p].ntx;
    i0 = (t % ntx) * bx;
    j0 = (t / ntx) * by;
}

// FP64 residual r64 = b - A64 x64 per item, partial r.r per item.
template <int BX, int BY>
__global__ __launch_bounds__(NT) void k_batch_resid(BatchArgs A) {
    extern __shared__ double lds_dyn[];
    double* lds64 = lds_dyn;
    const int nitems = *A.nlive;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        int p, i0, j0;
        item_of(A, w, p, i0, j0, BX, BY);
        const BProb& P = A.prob[p];
        double acc = 0.0;
        if (A.state[p].needs || A.first_pass)
            acc = tile_resid<BX, BY>(P.g, i0, j0, P.x64, P.r64, P.a64, P.c64, P.K64, P.b64, lds64);
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
// Start of a solve: zeroes the solution and every CG vector of problem
// blockIdx.y over its whole arrays, so that tiles outside the active list
// (read as halo by their active neighbours) hold zeros, and stamps the start
// time.
__global__ __launch_bounds__(NT) void k_batch_zero(BatchArgs A) {
    const int p = blockIdx.y;
    const BProb& P = A.prob[p];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.state[p].t_start = wall_clock64();
        A.state[p].needs = 0;
    }
    const long long n = 3 * P.g.NP;
    for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < n;
         e += (long long)gridDim.x * NT) {
        P.x64[e] = 0.0;
        P.r64[e] = 0.0;
        P.x32[e] = 0.f;
        P.r32[e] = 0.f;
        P.r32b[e] = 0.f;
        P.p0[e] = 0.f;
        P.p1[e] = 0.f;
        P.q32[e] = 0.f;
        P.q32b[e] = 0.f;
    }
}

// Tile f of the list of all tiles is active if any sample anchored in it has
// a != 0 (the same test as the single-problem tile lists).
__global__ __launch_bounds__(NT) void k_batch_tile_flags(const BProb* __restrict__ prob,
                                                         const int* __restrict__ full_prob,
                                                         int nfull, int bx, int by,
                                                         int* __restrict__ flags) {
    for (int f = blockIdx.x; f < nfull; f += gridDim.x) {
        const BProb& P = prob[full_prob[f]];
        const int t = f - P.full0;
        const int i0 = (t % P.ntx) * bx, j0 = (t / P.ntx) * by;
        int any = 0;
        for (int e = threadIdx.x; e < bx * by; e += NT) {
            const int i = i0 + e % bx, j = j0 + e / bx;
            if (i <= P.g.nx && j <= P.g.ny)
                for (int s = 0; s < 3; ++s) any |= P.a64[s * P.g.NP + P.g.idx(i, j)] != 0.0;
        }
        any = __syncthreads_or(any);
        if (threadIdx.x == 0) flags[f] = any;
    }
}

// Resets the barrier / counters of the persistent kernel (a kernel, not a
// memset, so that it can live in a captured graph).
__global__ void k_batch_reset_ctl(BatchCtl* ctl) {
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0) {
        ctl->bar_count = 0;
        ctl->abort = 0;
        ctl->n_done = 0;
        ctl->n_need = 0;
    }
    if (threadIdx.x < kBarGroups) ctl->bar_grp[threadIdx.x * kBarStride] = 0;
}

// The persistent solve of every problem, refinement included.  One phase per
// step, a grid barrier after each.  Per problem, by mode:
//   CG      kloc 0: r32 given, z = D^-1 r, p = z, q = A p, five partials;
//           kloc k >= 1: totals of iteration k-1 -> stop test, alpha_{k-1},
//           beta_k; lazy update, direction, q = A p, five partials
//   stop -> AXPY (x64 += |r64| x32) -> RESID (r64 = b - A64 x64, FP64,
//           |r64|^2 partial) -> DECIDE (|r64| total; DONE if it meets tol,
//           else r32 = r64/|r64|, x32 = 0 and back to CG at kloc 0).
// DECIDE acts only in odd phases, so the count of retired problems changes
// only there and every workgroup reads the same value of it in the even
// phases, where the loop may end.  Problems therefore retire independently;
// their completion time is the device wall clock at DONE.
template <int BX, int BY>
__global__ __launch_bounds__(NT, 2) void k_batch_pcg(BatchArgs A) {
    extern __shared__ double lds_dyn[];
    float* lds32 = reinterpret_cast<float*>(lds_dyn);
    double* lds64 = lds_dyn;
    BatchCtl* ctl = A.ctl;
    const unsigned G = gridDim.x;
    // items are dealt round-robin (item w to workgroup w mod G), so every
    // problem's tiles are spread over the whole grid and the problems still
    // iterating near the end of a solve keep every workgroup busy
    const int wb = (int)blockIdx.x, ws = (int)G;
    const int nitems = *A.nlive;

    // r = r64 / |r64| into the second r buffer (the INIT iteration weights it
    // into the first), x32 = 0 on the tile (start of an inner solve)
    auto init_inner = [&](const BProb& P, int i0, int j0, double rho2) {
        const double inv = rho2 > 0.0 ? 1.0 / sqrt(rho2) : 0.0;
        for (int e = threadIdx.x; e < BX * BY; e += NT) {
            const int i = i0 + e % BX, j = j0 + e / BX;
            if (i > P.g.nx || j > P.g.ny) continue;
            const long long o = P.g.idx(i, j);
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const long long os = o + s * P.g.NP;
                P.r32b[os] = (float)(P.r64[os] * inv);
                P.x32[os] = 0.f;
            }
        }
    };

    // phase "-1": initial modes
    for (int w = wb; w < nitems; w += ws) {
        int p, i0, j0;
        item_of(A, w, p, i0, j0, BX, BY);
        const BProb& P = A.prob[p];
        BState& S = A.state[p];
        if (S.needs) init_inner(P, i0, j0, S.rho2);
        if (w == P.item0 && threadIdx.x == 0) {
            S.ph[0].mode = S.needs ? BM_CG : BM_DONE;
            S.ph[0].kloc = 0;
            S.retired = S.needs ? 0 : 1;
            if (S.needs)
                __hip_atomic_fetch_add(&ctl->n_need, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (!grid_barrier(ctl, G)) return;
    const int n_need = __hip_atomic_load(&ctl->n_need, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n_need == 0) return;

    __shared__ int s_list[NT];
    __shared__ int s_wcnt[NT / 64];
    for (int phi = 0;; ++phi) {
        const int cs = phi & 1, ns = cs ^ 1;
        const bool retire_phase = (phi & 1) != 0;
        int cached = -1;
        double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        // gather this workgroup's items of problems that have not retired (up
        // to NT per round, in item order): the mode reads of all items are in
        // flight together instead of one dependent chain per item
        for (int r0 = 0; wb + r0 * ws < nitems; r0 += NT) {
            const int wt = wb + (r0 + (int)threadIdx.x) * ws;
            const bool act = wt < nitems && !A.state[A.item_prob[wt]].retired;
            const unsigned long long bal = __ballot(act);
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
            if (lane == 0) s_wcnt[wid] = __popcll(bal);
            __syncthreads();
            int off = 0, nact = 0;
#pragma unroll
            for (int q = 0; q < NT / 64; ++q) {
                off += q < wid ? s_wcnt[q] : 0;
                nact += s_wcnt[q];
            }
            if (act) s_list[off + __popcll(bal & ((1ull << lane) - 1ull))] = wt;
            __syncthreads();
            for (int e = 0; e < nact; ++e) {
                const int w = s_list[e];
                int p, i0, j0;
                item_of(A, w, p, i0, j0, BX, BY);
                const BProb& P = A.prob[p];
                BState& S = A.state[p];
                const BPhase cur = S.ph[cs];
                const bool owner = w == P.item0 && threadIdx.x == 0;
                BPhase nxt = cur;
                if (cur.mode == BM_CG) {
                    const int k = cur.kloc;
                    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                    if (k == 0) {
                        tile_fused<BX, BY, true>(P, i0, j0, 0.f, 0.f, 0, lds32, v);
                        item_partial<5>(v, A.partF[0], w);
                        nxt.kloc = 1;
                    } else {
                        if (p != cached) {
                            problem_total<5>(A.partF[(k + 1) & 1], P.item0, P.nt, tot);
                            cached = p;
                        }
                        const double rz = tot[0], pq = tot[1], qdr = tot[2], qdq = tot[3], rrk = tot[4];
                        const double bb = k == 1 ? rrk : S.bb;
                        const bool stop = !isfinite(rz) || !isfinite(rrk) || !isfinite(pq) ||
                                          rrk <= S.tol_in2 * bb || k - 1 >= A.max_iter_pass ||
                                          S.iters_total + k - 1 >= A.max_iter || !(pq > 0.0);
                        if (stop) {
                            if (owner) {
                                S.last_iter = k - 1;
                                nxt.mode = BM_AXPY;
                            }
                        } else {
                            const double ad = rz / pq;
                            const double rzn = rz - 2.0 * ad * qdr + ad * ad * qdq;
                            const double bd = rz > 0.0 ? rzn / rz : 0.0;
                            tile_fused<BX, BY, false>(P, i0, j0, (float)ad, (float)bd, k, lds32, v);
                            item_partial<5>(v, A.partF[k & 1], w);
                            if (owner && k == 1) S.bb = bb;
                            nxt.kloc = k + 1;
                        }
                    }
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
                } else if (cur.mode == BM_RESID) {
                    double v[1];
                    v[0] = tile_resid<BX, BY>(P.g, i0, j0, P.x64, P.r64, P.a64, P.c64, P.K64, P.b64,
                                              lds64);
                    item_partial<1>(v, A.partR, w);
                    nxt.mode = BM_DECIDE;
                } else if (cur.mode == BM_DECIDE && retire_phase) {
                    double t1[1];
                    problem_total<1>(A.partR, P.item0, P.nt, t1);
                    const double rho2 = t1[0];
                    const double rel = S.bb64 > 0.0 ? sqrt(rho2 / S.bb64) : 0.0;
                    const bool fin = !(rel > A.tol) || !isfinite(rel) || S.passes >= A.max_passes ||
                                     S.iters_total >= A.max_iter;
                    if (!fin) init_inner(P, i0, j0, rho2);
                    if (owner) {
                        S.rho2 = rho2;
                        S.rel = rel;
                        if (fin) {
                            nxt.mode = BM_DONE;
                            S.t_done = wall_clock64();
                            S.needs = 0;
                            S.retired = 1;
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
            __syncthreads();   // s_list and s_wcnt are rewritten by the next round
        }
        // retirements happen only in odd phases: the count is stable in even ones
        const int nd = retire_phase ? 0
                                    : __hip_atomic_load(&ctl->n_done, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        if (!grid_barrier(ctl, G)) return;
        if (!retire_phase && nd >= n_need) break;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// variants: (BX, BY) tile shapes
// ---------------------------------------------------------------------------
static const int kVar[kBatchVariants][2] = {{64, 4}, {64, 8}, {32, 8}, {128, 2}, {64, 12}, {64, 16}};

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
        case 3: launch_variant<128, 2>(0, A, grid, s); break;
        case 4: launch_variant<64, 12>(0, A, grid, s); break;
        default: launch_variant<64, 16>(0, A, grid, s); break;
    }
}

void launch_batch_resid(int variant, const BatchArgs& A, int grid, hipStream_t s) {
    switch (variant) {
        case 0: launch_variant<64, 4>(1, A, grid, s); break;
        case 1: launch_variant<64, 8>(1, A, grid, s); break;
        case 2: launch_variant<32, 8>(1, A, grid, s); break;
        case 3: launch_variant<128, 2>(1, A, grid, s); break;
        case 4: launch_variant<64, 12>(1, A, grid, s); break;
        default: launch_variant<64, 16>(1, A, grid, s); break;
    }
}

void launch_batch_finalize(const BatchArgs& A, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_finalize, dim3(A.nprob), dim3(NT), 0, s, A);
}

void launch_batch_zero(const BatchArgs& A, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_zero, dim3(64, A.nprob), dim3(NT), 0, s, A);
}

void launch_batch_tile_flags(const BProb* prob, const int* full_prob, int nfull, int bx, int by,
                             int* flags, hipStream_t s) {
    if (nfull <= 0) return;
    hipLaunchKernelGGL(k_batch_tile_flags, dim3(std::min(nfull, 8192)), dim3(NT), 0, s, prob,
                       full_prob, nfull, bx, by, flags);
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
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pcg<128, 2>, NT, l32); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pcg<64, 12>, NT, l32); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pcg<64, 16>, NT, l32); break;
    }
    *blocks_per_cu = nb;
    return e == hipSuccess ? 0 : -1;
}

}  // namespace vfs
