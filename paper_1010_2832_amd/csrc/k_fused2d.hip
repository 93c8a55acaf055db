// 2D Jacobi-preconditioned CG with one fused kernel per iteration.
//
// Plain PCG (the update x += alpha p, r -= alpha q, then z = D^-1 r, then
// p = z + beta p, q = A p) needs two global reductions per iteration: p.q
// before the update and r.z before the next direction.  Here the update of
// iteration k-1 is carried out lazily by launch k, and r_k.z_k is obtained
// one launch early from quantities reduced together with p.q:
//   r_k.z_k = r_{k-1}.z_{k-1} - 2 alpha q_{k-1}.D^-1 r_{k-1}
//             + alpha^2 q_{k-1}.D^-1 q_{k-1},
// re-anchored every step on the directly summed r_{k-1}.z_{k-1}, so the
// expansion error does not accumulate.  q = A p is always applied
// explicitly (no recurrence for A p), so the iterates are those of plain PCG
// up to the rounding of beta.  The matrix is the paper's
// A = dt B^T K B + Dg (eq. stokesmixedsystemspd, factored form of Section 7),
// applied with the same LDS-tiled stencil as k_apply2d.
//
// Launch k >= 1, from the partials (r.z, p.q, q.D^-1 r, q.D^-1 q, r.r) of
// launch k-1:
//   stop test on r_{k-1}.r_{k-1};  alpha = r.z / p.q;  beta from the
//   expansion;  on the tile and its halo: r_k = r_{k-1} - alpha q_{k-1},
//   z_k = D^-1 r_k, p_k = z_k + beta p_{k-1}; at the own anchors also
//   x_k = x_{k-1} + alpha p_{k-1}; then q_k = A p_k and the partials of
//   iteration k.
// Launch 0 (init) forms z_0 = D^-1 r_0, p_0 = z_0, q_0 = A p_0 and the first
// partials.  r, p and q are double-buffered by launch parity because the
// halo of launch k reads the values of launch k-1 that neighbouring
// workgroups overwrite; x is read and written only at the own anchors.
#include "vfs_internal.h"
#include "vfs_reduce.h"

#include <algorithm>

namespace vfs {
namespace {

constexpr int NT = 384;
constexpr int NV = 5;   // r.z, p.q, q.D^-1 r, q.D^-1 q, r.r

// Tile of workgroup b (one tile per workgroup).  Workgroups are dispatched
// round-robin over the 8 XCDs of the chip (b runs on XCD b % 8); XCD x takes
// the contiguous part [start_x, start_x + n_x) of the tile list, so tiles
// that are neighbours in x share their boundary cache lines in one L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    if (G < 8) return b;
    const int x = b & 7, slot = b >> 3;
    const int q = G >> 3, rem = G & 7;
    return x * q + min(x, rem) + slot;
}

// Base address of every slice the launch reads or writes, passed as kernel
// arguments (the parity buffers are picked on the host).  Each load or store
// then takes its base in scalar registers and one 32-bit byte offset per lane,
// shared by every slice read at that position, instead of a 64-bit address
// per lane and access (slice bases computed inside the kernel get folded into
// the per-lane addresses).  Offsets stay within one slice (at most about
// 2.7e8 elements for the largest 2D grid, 16384^2), far below 4 GiB.
template <typename T>
struct Slices2d {
    const T* r[3];   // r_{k-1} (launch 0: r_0)
    const T* q[3];   // q_{k-1}
    const T* p[3];   // p_{k-1}
    const T* d[3];   // D^-1
    const T* a[3];   // sample weights
    T* x[3];         // x, read and written in place
    const T* c[2];   // diagonal coefficients of slices 1 and 2
    const T* K[2];   // face coefficients (u, v)
    T* ro[3];        // r_k
    T* po[3];        // p_k
    T* qo[3];        // q_k
};

// Byte offset of anchor (i, j) in a slice, or 0 (the slice's zero pad) when
// ok is false; computed in 32 bits with a mask rather than a select (which
// the compiler turns into a branch), so that every load sees a zero-extended
// 32-bit offset.
template <typename T>
__device__ __forceinline__ unsigned boff2d(const Geo& g, int i, int j, bool ok) {
    const unsigned e = (unsigned)kFront + (unsigned)(j + 1) * (unsigned)g.PX + (unsigned)i;
    unsigned b = (e * (unsigned)sizeof(T)) & (0u - (unsigned)ok);
    // opaque to the optimizer (no instruction is emitted; not volatile, so it
    // does not pin the schedule): it would otherwise widen the mask to 64
    // bits and the loads would lose the 32-bit offset form
    asm("" : "+v"(b));
    return b;
}

// Element at byte offset boff of a slice.
template <typename T>
__device__ __forceinline__ T ldo(const T* __restrict__ base, unsigned boff) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename T>
__device__ __forceinline__ void sto(T* __restrict__ base, unsigned boff, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff) = v;
}

// Launched over the compacted list of tiles that hold an active sample;
// the vectors of the other tiles stay zero (they hold no active sample), so
// their values read as halo are correct.
template <typename T, bool INIT, int BX, int BY>
__global__ __launch_bounds__(NT) void k_fused2d(Geo g, Slices2d<T> S, const int* __restrict__ tiles,
                                                int ntx, RedArgs ra) {
    constexpr int RPT = BY * BX / NT;              // own anchors per thread
    constexpr int NH = 2 * (BX + 2) + 2 * BY;      // halo ring of the tile
    constexpr int NE2 = ((BX + 1) * (BY + 1) + NT - 1) / NT;
    static_assert(RPT * NT == BX * BY && NH <= NT, "tile shape");
    const int bid = blockIdx.x;
    Scalars* sc = ra.sc;
    const int k = ra.kidx;
    __shared__ T sW[3][BY + 2][BX + 2];   // a p_k on the tile and its halo
    __shared__ T sG[2][BY + 1][BX + 1];
    const int tile = tiles[xcd_tile(bid, gridDim.x)];
    const int i0 = (tile % ntx) * BX, j0 = (tile / ntx) * BY;
    const int tid = threadIdx.x;
    // own anchors (i0 + tx, j0 + ty(rr)); the same thread forms p, z and q
    // there, so only a p crosses threads (through LDS)
    const int tx = tid % BX;
    auto own_row = [&](int rr) { return tid / BX + rr * (NT / BX); };
    // halo ring position of thread tid < NH: rows lj = 0 and BY + 1 (corners
    // included), then columns li = 0 and BX + 1
    const bool hrole = tid < NH;
    int hli = 0, hlj = 0;
    if (tid < BX + 2) {
        hli = tid;
    } else if (tid < 2 * (BX + 2)) {
        hli = tid - (BX + 2);
        hlj = BY + 1;
    } else if (hrole) {
        const int e = tid - 2 * (BX + 2);
        hlj = 1 + (e >> 1);
        hli = (e & 1) ? BX + 1 : 0;
    }

    // (1) partials of the previous launch (one per thread in registers; a
    // longer list is finished by a loop)
    PartialLoads<NV, NT, 1> pl;
    if (!INIT) pl.load(ra.part_in, ra.nb_in);

    // (2) loads that do not depend on the totals.  Positions outside the grid
    // read offset 0 of each slice, its zero pad, so no load is guarded.
    T Rr[RPT][3], Dd[RPT][3], Qq[RPT][3], Pp[RPT][3], Aa[RPT][3], Xx[RPT][3], Co[RPT][2];
    bool own[RPT];
    unsigned Ob[RPT];   // byte offset of the own anchor in a slice (0 outside the grid)
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + tx, j = j0 + own_row(rr);
        own[rr] = i <= g.nx && j <= g.ny;
        const unsigned ob = boff2d<T>(g, i, j, i <= g.nx + 1 && j <= g.ny + 1);
        unsigned oxb = ob & (0u - (unsigned)own[rr]);
        asm("" : "+v"(oxb));   // keeps the 32-bit offset form (see boff2d)
        Ob[rr] = oxb;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            Rr[rr][s] = ldo(S.r[s], ob);
            Dd[rr][s] = ldo(S.d[s], ob);
            Aa[rr][s] = ldo(S.a[s], ob);
            Qq[rr][s] = INIT ? T(0) : ldo(S.q[s], ob);
            Pp[rr][s] = INIT ? T(0) : ldo(S.p[s], ob);
            Xx[rr][s] = INIT ? T(0) : ldo<T>(S.x[s], oxb);
        }
        Co[rr][0] = ldo(S.c[0], oxb);
        Co[rr][1] = ldo(S.c[1], oxb);
    }
    // halo loads only in the waves that hold halo positions
    T Rh[3] = {}, Dh[3] = {}, Qh[3] = {}, Ph[3] = {}, Ah[3] = {};
    if (hrole) {
        const int i = i0 - 1 + hli, j = j0 - 1 + hlj;
        const unsigned ob = boff2d<T>(g, i, j, i <= g.nx + 1 && j <= g.ny + 1);
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            Rh[s] = ldo(S.r[s], ob);
            Dh[s] = ldo(S.d[s], ob);
            Ah[s] = ldo(S.a[s], ob);
            Qh[s] = INIT ? T(0) : ldo(S.q[s], ob);
            Ph[s] = INIT ? T(0) : ldo(S.p[s], ob);
        }
    }
    T Ku[NE2], Kv[NE2];
#pragma unroll
    for (int m = 0; m < NE2; ++m) {
        const int e = tid + m * NT;
        const int li = e % (BX + 1), lj = e / (BX + 1);
        const bool fe = e < (BX + 1) * (BY + 1);
        const int iu = i0 + li, ju = j0 - 1 + lj;
        const int iv = i0 - 1 + li, jv = j0 + lj;
        const bool okU = fe && iu <= g.nx && ju >= 0 && ju < g.ny;
        const bool okV = fe && iv >= 0 && iv < g.nx && jv <= g.ny;
        Ku[m] = ldo(S.K[0], boff2d<T>(g, iu, ju, okU));
        Kv[m] = ldo(S.K[1], boff2d<T>(g, iv, jv, okV));
    }

    // (3) totals of iteration k-1 -> stop decision, alpha_{k-1}, beta_k.  The
    // flag of a solve that has already stopped is read only now, so that its
    // round trip overlaps the loads above (all of which are in bounds
    // whether or not the solve goes on).
    T alpha = T(0), beta = T(0);
    if (!INIT && sc->done) return;
    if (!INIT) {
        double t[NV];
        pl.finish(t);
        const double rz = t[0], pq = t[1], qdr = t[2], qdq = t[3], rrk = t[4];
        const double bb = ra.set_bb ? rrk : sc->bb;
        int stop = 0;
        if (!isfinite(rz) || !isfinite(rrk) || !isfinite(pq))
            stop = 3;
        else if (rrk <= sc->tol2 * bb)
            stop = 1;
        else if (k - 1 >= sc->max_iter)
            stop = 2;
        else if (!(pq > 0.0))
            stop = 3;
        const double ad = stop ? 0.0 : rz / pq;
        const double rzn = rz - 2.0 * ad * qdr + ad * ad * qdq;
        const double bd = (rz > 0.0) ? rzn / rz : 0.0;
        if (bid == 0 && tid == 0) {
            sc->rz[k & 1] = rz;
            sc->rr = rrk;
            sc->pq = pq;
            sc->alpha = ad;
            sc->beta = bd;
            if (ra.set_bb) sc->bb = bb;
            if (stop) {
                sc->done = stop;
                sc->iter = k - 1;
            }
        }
        if (stop) return;
        alpha = (T)ad;
        beta = (T)bd;
    }

    // (4) tile and halo: r_k, z_k, p_k; own anchors also x_k
    double rz_n = 0.0, rr_n = 0.0;
    T Vo[RPT][3], Zo[RPT][3];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int ty = own_row(rr);
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const T rn = INIT ? Rr[rr][s] : Rr[rr][s] - alpha * Qq[rr][s];
            const T zn = Dd[rr][s] * rn;
            const T pn = INIT ? zn : zn + beta * Pp[rr][s];
            if (own[rr]) {
                unsigned ob = Ob[rr];
                asm("" : "+v"(ob));   // 32-bit offset form in this block too
                if (!INIT) {
                    sto(S.ro[s], ob, rn);
                    sto(S.x[s], ob, Xx[rr][s] + alpha * Pp[rr][s]);
                }
                sto(S.po[s], ob, pn);
                rz_n += (double)rn * (double)zn;
                rr_n += (double)rn * (double)rn;
            }
            Vo[rr][s] = pn;
            Zo[rr][s] = zn;
            sW[s][ty + 1][tx + 1] = Aa[rr][s] * pn;
        }
    }
    if (hrole) {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const T rn = INIT ? Rh[s] : Rh[s] - alpha * Qh[s];
            const T pn = INIT ? Dh[s] * rn : Dh[s] * rn + beta * Ph[s];
            sW[s][hlj][hli] = Ah[s] * pn;
        }
    }
    __syncthreads();

    // (5) faces: g = K (B p)
#pragma unroll
    for (int m = 0; m < NE2; ++m) {
        const int e = tid + m * NT;
        if (e >= (BX + 1) * (BY + 1)) continue;
        const int li = e % (BX + 1), lj = e / (BX + 1);
        sG[0][lj][li] = Ku[m] * ((sW[0][lj][li + 1] - sW[0][lj][li]) +
                                 (sW[1][lj][li] - sW[1][lj][li + 1]) +
                                 (sW[2][lj][li + 1] - sW[2][lj + 1][li + 1]));
        sG[1][lj][li] = Kv[m] * ((sW[0][lj + 1][li] - sW[0][lj][li]) +
                                 (sW[1][lj + 1][li] - sW[1][lj][li]) +
                                 (sW[2][lj + 1][li] - sW[2][lj + 1][li + 1]));
    }
    __syncthreads();

    // (6) q_k = B^T g + Dg p at the anchors; partials of p.q, q.z, q.D^-1 q
    double pq_n = 0.0, qz_n = 0.0, qdq_n = 0.0;
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int ty = own_row(rr);
        if (own[rr]) {
            unsigned ob = Ob[rr];
            asm("" : "+v"(ob));
            const T gu0 = sG[0][ty + 1][tx], gu1 = sG[0][ty + 1][tx + 1], gum = sG[0][ty][tx];
            const T gv0 = sG[1][ty][tx + 1], gv1 = sG[1][ty + 1][tx + 1], gvm = sG[1][ty][tx];
            T y[3];
            y[0] = Aa[rr][0] * ((gu0 - gu1) + (gv0 - gv1));
            y[1] = Aa[rr][1] * ((gu1 - gu0) + (gv0 - gv1)) + Co[rr][0] * Vo[rr][1];
            y[2] = Aa[rr][2] * ((gu0 - gum) + (gv0 - gvm)) + Co[rr][1] * Vo[rr][2];
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                sto(S.qo[s], ob, y[s]);
                const double yd = y[s];
                pq_n += (double)Vo[rr][s] * yd;
                qz_n += (double)Zo[rr][s] * yd;
                qdq_n += (double)Dd[rr][s] * yd * yd;
            }
        }
    }
    double vv[NV] = {rz_n, pq_n, qz_n, qdq_n, rr_n};
    block_partial<NV, NT>(vv, ra.part_out, gridDim.x, bid);
}

// tile t (BX x BY anchors) is active if any of its samples has a != 0
template <int BX, int BY>
__global__ __launch_bounds__(NT) void k_tiles2d_flags(Geo g, int ntx, const double* __restrict__ a,
                                                      int* __restrict__ flags) {
    const int t = blockIdx.x;
    const int i0 = (t % ntx) * BX, j0 = (t / ntx) * BY;
    int any = 0;
    for (int e = threadIdx.x; e < BX * BY; e += NT) {
        const int i = i0 + e % BX, j = j0 + e / BX;
        if (i <= g.nx && j <= g.ny)
            for (int s = 0; s < 3; ++s) any |= a[s * g.NP + g.idx(i, j)] != 0.0;
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) flags[t] = any;
}

// ordered compaction of the active tile ids (one workgroup)
__global__ __launch_bounds__(1024) void k_tiles2d_compact(int n, const int* __restrict__ flags,
                                                          int* __restrict__ list,
                                                          int* __restrict__ count) {
    __shared__ int s_cnt[1024];
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    int c = 0;
    for (int t = lo; t < hi; ++t) c += flags[t];
    s_cnt[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int q = 0; q < 1024; ++q) {
            const int v = s_cnt[q];
            s_cnt[q] = run;
            run += v;
        }
        *count = run;
    }
    __syncthreads();
    int w = s_cnt[threadIdx.x];
    for (int t = lo; t < hi; ++t)
        if (flags[t]) list[w++] = t;
}

// tile shape and workgroup size: 64 x 12 anchors with 384 threads (two own
// anchors per thread) was the fastest of the shapes swept on the 512^2
// workload: about one tile per compute unit (310.4 ms per solve against 318.1
// for 64 x 16 with 512 threads, 316.6 for 64 x 14, 325.1 for 64 x 12 with 256
// threads)
constexpr int kBX = 64, kBY = 12;

}  // namespace

int tile2d_anchors() { return kBX * kBY; }

void fused2d_tile_dims(const Geo& g, int& ntx, int& nty) {
    ntx = (g.nx + 1 + kBX - 1) / kBX;
    nty = (g.ny + 1 + kBY - 1) / kBY;
}

void launch_tiles2d(const Geo& g, const double* a, int* flags, int* list, int* count,
                    hipStream_t s) {
    int ntx, nty;
    fused2d_tile_dims(g, ntx, nty);
    const int n = ntx * nty;
    hipLaunchKernelGGL((k_tiles2d_flags<kBX, kBY>), dim3(n), dim3(NT), 0, s, g, ntx, a, flags);
    hipLaunchKernelGGL(k_tiles2d_compact, dim3(1), dim3(1024), 0, s, n, flags, list, count);
}

template <typename T>
void launch_fused2d(const Geo& g, bool init, const FusedVecs& v, const T* dinv, const T* a,
                    const T* c, const T* K, const int* tiles, int count, const RedArgs& ra,
                    hipStream_t s) {
    if (count <= 0) return;
    int ntx, nty;
    fused2d_tile_dims(g, ntx, nty);
    // launch k reads the slot (k-1)&1 of r, p, q and writes slot k&1
    const int pin = (ra.kidx + 1) & 1, pout = ra.kidx & 1;
    const long long NP = g.NP;
    Slices2d<T> S{};
    for (int q = 0; q < 3; ++q) {
        S.r[q] = static_cast<const T*>(v.r[init ? 0 : pin]) + q * NP;
        S.q[q] = static_cast<const T*>(v.q[pin]) + q * NP;
        S.p[q] = static_cast<const T*>(v.p[pin]) + q * NP;
        S.d[q] = dinv + q * NP;
        S.a[q] = a + q * NP;
        S.x[q] = static_cast<T*>(v.x) + q * NP;
        S.ro[q] = static_cast<T*>(v.r[pout]) + q * NP;
        S.po[q] = static_cast<T*>(v.p[pout]) + q * NP;
        S.qo[q] = static_cast<T*>(v.q[pout]) + q * NP;
    }
    S.c[0] = c + NP;
    S.c[1] = c + 2 * NP;
    S.K[0] = K;
    S.K[1] = K + NP;
    if (init)
        hipLaunchKernelGGL((k_fused2d<T, true, kBX, kBY>), dim3(count), dim3(NT), 0, s, g, S, tiles,
                           ntx, ra);
    else
        hipLaunchKernelGGL((k_fused2d<T, false, kBX, kBY>), dim3(count), dim3(NT), 0, s, g, S, tiles,
                           ntx, ra);
}

template void launch_fused2d<float>(const Geo&, bool, const FusedVecs&, const float*, const float*,
                                    const float*, const float*, const int*, int, const RedArgs&,
                                    hipStream_t);

}  // namespace vfs
