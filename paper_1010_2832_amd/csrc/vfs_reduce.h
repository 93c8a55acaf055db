// Deterministic FP64 reductions across workgroups without atomics or fences.
//
// A producer kernel writes one partial sum per workgroup (plain stores).  The
// consumer is the *next* kernel on the stream: the kernel boundary makes the
// partials visible, and every consumer workgroup sums all partials itself in
// a fixed order (strided per thread, wave-xor tree, waves in order), so every
// workgroup obtains bit-identical totals and may act on them uniformly.
// This avoids the device-scope release/acquire of a "last workgroup" scheme,
// which on a multi-XCD part writes back the whole L2 per workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include "vfs_internal.h"

namespace vfs {

// DPP move of a double (both 32-bit halves) with the given control word; lanes
// whose source lies outside their row, or rows outside ROWS, receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (all lanes active), returned in every lane.
// Row prefix sums by row_shr 1, 2, 4, 8 leave each 16-lane row's sum in its
// lane 15; row_bcast 15 adds row 0 into row 1 and row 2 into row 3, and
// row_bcast 31 adds lane 31 into rows 2 and 3, so lane 63 holds the total.
// Register moves only (no LDS crossbar), in a fixed order.
__device__ __forceinline__ double wave_sum64(double v) {
    v += dpp_move<0x111, 0xf>(v);   // row_shr:1
    v += dpp_move<0x112, 0xf>(v);   // row_shr:2
    v += dpp_move<0x114, 0xf>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v);   // row_shr:8
    v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Writes this workgroup's sums of v[] to part[q * nb + bid].
template <int NV, int NT>
__device__ __forceinline__ void block_partial(double (&v)[NV], double* __restrict__ part, int nb,
                                              int bid) {
    constexpr int NW = NT / 64;
    __shared__ double sw[NV][NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum64(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) sw[q][wid] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = sw[q][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) s += sw[q][w];
            part[(long long)q * nb + bid] = s;
        }
    }
}

// Every thread of the workgroup receives the totals of part[q * nb + 0..nb).
template <int NV, int NT>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nb,
                                                double (&tot)[NV]) {
    constexpr int NW = NT / 64;
    __shared__ double sr[NV][NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += NT) s += part[(long long)q * nb + b];
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

// Split form of reduce_partials for latency hiding: load the (at most
// MAXP * NT per value) partials into registers first, issue independent
// global loads, then finish.  Same order of additions as reduce_partials.
template <int NV, int NT, int MAXP>
struct PartialLoads {
    double v[NV][MAXP];
    const double* src = nullptr;
    int n = 0;
    __device__ __forceinline__ void load(const double* __restrict__ part, int nb) {
        src = part;
        n = nb;
#pragma unroll
        for (int m = 0; m < MAXP; ++m) {
            const int b = threadIdx.x + m * NT;
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q][m] = b < nb ? part[(long long)q * nb + b] : 0.0;
        }
    }
    __device__ __forceinline__ void finish(double (&tot)[NV]) {
        constexpr int NW = NT / 64;
        __shared__ double sr[NV][NW];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < MAXP; ++m) s += v[q][m];
            // partials beyond the register window (large grids)
            for (int b = threadIdx.x + MAXP * NT; b < n; b += NT) s += src[(long long)q * n + b];
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
};

// Decision of a MODE_DIR apply from the r.z / r.r totals: returns false if
// the solve stops here (converged, iteration cap, non-finite); sets beta.
__device__ __forceinline__ bool cg_direction_decide(const RedArgs& ra, int bid, double rzk,
                                                    double rrk, double& beta) {
    Scalars* sc = ra.sc;
    const double bb = ra.set_bb ? rrk : sc->bb;
    int stop = 0;
    if (!isfinite(rzk) || !isfinite(rrk))
        stop = 3;
    else if (rrk <= sc->tol2 * bb)
        stop = 1;
    else if (ra.kidx >= sc->max_iter)
        stop = 2;
    beta = ra.kidx == 0 ? 0.0 : rzk / sc->rz[(ra.kidx + 1) & 1];
    if (bid == 0 && threadIdx.x == 0) {
        sc->rz[ra.kidx & 1] = rzk;
        sc->rr = rrk;
        sc->beta = beta;
        if (ra.set_bb) sc->bb = bb;
        if (stop) {
            sc->done = stop;
            sc->iter = ra.kidx;
        }
    }
    return stop == 0;
}

// Shared preamble of a MODE_DIR apply: returns false if the solve stops here
// (converged, iteration cap, non-finite); sets beta.
template <int NT>
__device__ __forceinline__ bool cg_direction_preamble(const RedArgs& ra, int bid, double& beta) {
    Scalars* sc = ra.sc;
    double tot[2];
    reduce_partials<2, NT>(ra.part_in, ra.nb_in, tot);
    const double rzk = tot[0], rrk = tot[1];
    const double bb = ra.set_bb ? rrk : sc->bb;
    int stop = 0;
    if (!isfinite(rzk) || !isfinite(rrk))
        stop = 3;
    else if (rrk <= sc->tol2 * bb)
        stop = 1;
    else if (ra.kidx >= sc->max_iter)
        stop = 2;
    beta = ra.kidx == 0 ? 0.0 : rzk / sc->rz[(ra.kidx + 1) & 1];
    if (bid == 0 && threadIdx.x == 0) {
        sc->rz[ra.kidx & 1] = rzk;
        sc->rr = rrk;
        sc->beta = beta;
        if (ra.set_bb) sc->bb = bb;
        if (stop) {
            sc->done = stop;
            sc->iter = ra.kidx;
        }
    }
    return stop == 0;
}

// Preamble of a truncated flexible-CG direction (Notay 2000): the new
// direction is p = z - sum_i beta_i P_i over the mk previous directions with
// beta_i = z.Q_i / P_i.Q_i (Q_i = A P_i), which makes it A-orthogonal to
// them; with mk = 1 this is the Polak-Ribiere flexible CG (Golub and Ye).
// Inputs: partials (z.r, then z.Q_i and r.D^-1 Q_i for i = 1..kFcgMax) of the
// preconditioner output z and partials (r.D^-1 r, r.r) of the update.  When
// z is not a descent direction (z.r <= 0 or non-finite) the Jacobi direction
// D^-1 r is used instead (fb = true).  beta[i] receives beta_{i+1}.
template <int NT>
__device__ __forceinline__ bool fcg_direction_preamble(const RedArgs& ra, int bid,
                                                       double (&beta)[kFcgMax], bool& fb) {
    Scalars* sc = ra.sc;
    constexpr int NV = 1 + 2 * kFcgMax;
    double tz[NV], t2[2];
    reduce_partials<NV, NT>(ra.part_in, ra.nb_in, tz);
    reduce_partials<2, NT>(ra.part_in2, ra.nb_in2, t2);
    const double zr = tz[0], rdr = t2[0], rr = t2[1];
    const int mk = ra.fh.mk;
    bool bad = !(zr > 0.0) || !isfinite(zr);
    for (int i = 0; i < mk; ++i) bad = bad || !isfinite(tz[1 + 2 * i]);
    fb = bad;
    const double rz = fb ? rdr : zr;
    const double bb = ra.set_bb ? rr : sc->bb;
    int stop = 0;
    if (!isfinite(rdr) || !isfinite(rr))
        stop = 3;
    else if (rr <= sc->tol2 * bb)
        stop = 1;
    else if (ra.kidx >= sc->max_iter)
        stop = 2;
#pragma unroll
    for (int i = 0; i < kFcgMax; ++i) {
        const double pq = i < mk ? sc->pqh[(ra.kidx - 1 - i) & 7] : 0.0;
        const double zq = fb ? tz[2 + 2 * i] : tz[1 + 2 * i];
        beta[i] = (i < mk && pq > 0.0) ? zq / pq : 0.0;
    }
    if (bid == 0 && threadIdx.x == 0) {
        sc->rz[ra.kidx & 1] = rz;
        sc->rr = rr;
        sc->beta = beta[0];
        if (ra.set_bb) sc->bb = bb;
        if (fb && !stop) sc->fallbacks += 1;
        if (stop) {
            sc->done = stop;
            sc->iter = ra.kidx;
        }
    }
    return stop == 0;
}

}  // namespace vfs
