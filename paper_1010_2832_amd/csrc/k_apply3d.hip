// 3D CG kernels on the padded grid, launched over a compacted list of
// active tiles (64 x 4 anchors in x,y times 8 planes in z).  Tiles without
// any active sample hold zeros in every solver vector and are skipped.
//
// Apply (paper eq. stokesmixedsystemspd, factored form of Section 7):
// g = K (B x) on faces, y = B^T g + Dg x on samples.  A workgroup marches its
// 8 z-planes keeping two planes of weighted samples (halo 1 in x,y) and two
// planes of each face field in LDS, so every face value is formed once and
// every sample is read once per plane (plus the x,y halo ring).
//
// Face rows (numerators; K carries dt/h^2), with X = W tau_xx, Y = W tau_yy,
// E = W tau_xy (z-edges), F = W tau_xz (y-edges), H = W tau_yz (x-edges):
//   u(i,j,k): P(i)-P(i-1) + X(i-1)-X(i) + E(i,j,k)-E(i,j+1,k) + F(i,j,k)-F(i,j,k+1)
//   v(i,j,k): P(j)-P(j-1) + Y(j-1)-Y(j) + E(i,j,k)-E(i+1,j,k) + H(i,j,k)-H(i,j,k+1)
//   w(i,j,k): P(k)-P(k-1) + X(k)-X(k-1) + Y(k)-Y(k-1) + F(i,j,k)-F(i+1,j,k)
//             + H(i,j,k)-H(i,j+1,k)
#include "vfs_internal.h"
#include "vfs_reduce.h"

#include <algorithm>

namespace vfs {
namespace {

constexpr int TX = kTile3X, TY = kTile3Y, KZ = kTile3Z, NT = 256;
constexpr int HX = TX + 2, HY = TY + 2;
constexpr int FX = TX + 1, FY = TY + 1;

// XCD-aware assignment of the active-tile list to workgroups.  Workgroups
// are dispatched round-robin over the 8 XCDs of the chip, so workgroup b runs
// on XCD b % 8.  Each XCD takes one contiguous eighth of the list (tiles in
// x order, then y, then z), so tiles that share halo cache lines, and the
// apply and the update of the same tile, stay within one XCD's L2.  With
// fewer than 8 workgroups the list is simply strided.
struct TileRange {
    int first, step, end;
};

__device__ __forceinline__ TileRange tile_range(int count) {
    const int G = gridDim.x, b = blockIdx.x;
    if (G < 8) return TileRange{b, G, count};
    const int x = b & 7, slot = b >> 3;
    const int nblk = (G - x + 7) >> 3;   // workgroups on this XCD
    const int t0 = (int)((long long)count * x / 8), t1 = (int)((long long)count * (x + 1) / 8);
    return TileRange{t0 + slot, nblk, t1};
}

// Anchors of work item u: x from i0, y from j0, planes [k0, kend).
__device__ __forceinline__ void tile_origin(const Tiles& t, const Geo& g, int u, int& i0, int& j0,
                                            int& k0, int& kend) {
    const int id = t.list[u / t.split];
    const int tx = id % t.ntx;
    const int ty = (id / t.ntx) % t.nty;
    const int tz = id / (t.ntx * t.nty);
    const int kz = KZ / t.split;
    i0 = tx * TX;
    j0 = ty * TY;
    k0 = tz * KZ + (u % t.split) * kz;
    kend = min(k0 + kz, g.nz + 1);
}

template <typename T, int MODE, bool ZIN>
struct Loader {
    const Geo& g;
    const T* r;
    const T* zs;
    const T* dinv;
    const T* pin;
    T* pout;
    const T* a;
    T beta;
    bool first;
    bool fb;   // MODE_FDIR: use the Jacobi z instead of zs
    int mk;    // MODE_FDIR: previous directions subtracted
    T bet[kFcgMax];
    const T* prev[kFcgMax];

    // value of slice s at offset os (direction update in MODE_DIR / MODE_FDIR)
    __device__ __forceinline__ T value(long long os, bool own) const {
        if (MODE == MODE_JDIR) {
            const T z = ZIN ? zs[os] : dinv[os] * r[os];
            if (own && pout) pout[os] = z;
            return z;
        }
        if (MODE == MODE_FDIR) {
            T val = fb ? dinv[os] * r[os] : zs[os];
#pragma unroll
            for (int i = 0; i < kFcgMax; ++i)
                if (i < mk) val -= bet[i] * prev[i][os];
            if (own) pout[os] = val;
            return val;
        }
        if (MODE == MODE_DIR) {
            const T z = ZIN ? zs[os] : dinv[os] * r[os];
            const T val = first ? z : z + beta * pin[os];
            if (own) pout[os] = val;
            return val;
        }
        return pin[os];
    }
};

template <typename T, int MODE, bool ZIN>
__global__ __launch_bounds__(NT) void k_apply3d(Geo g, Tiles tl, const T* __restrict__ r,
                                                const T* __restrict__ zs,
                                                const T* __restrict__ dinv,
                                                const T* __restrict__ pin, T* __restrict__ pout,
                                                T* __restrict__ q, const T* __restrict__ a,
                                                const T* __restrict__ c, const T* __restrict__ K,
                                                const T* __restrict__ bv, RedArgs ra) {
    T beta = T(0);
    bool first = true, fb = false;
    T bet[kFcgMax] = {};
    if (MODE == MODE_DIR) {
        if (ra.sc->done) return;
        double bd;
        if (!cg_direction_preamble<NT>(ra, blockIdx.x, bd)) return;
        first = ra.kidx == 0;
        beta = (T)bd;
    } else if (MODE == MODE_JDIR) {
        if (ra.skip && *ra.skip) return;
    } else if (MODE == MODE_FDIR) {
        if (ra.sc->done) return;
        double bd[kFcgMax];
        if (!fcg_direction_preamble<NT>(ra, blockIdx.x, bd, fb)) return;
#pragma unroll
        for (int i = 0; i < kFcgMax; ++i) bet[i] = (T)bd[i];
    }
    __shared__ T sW[2][6][HY][HX];
    __shared__ T gU[2][FY][FX];
    __shared__ T gV[2][FY][FX];
    __shared__ T gW[2][FY][FX];
    const long long NP = g.NP;
    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    Loader<T, MODE, ZIN> ld{g, r, zs, dinv, pin, pout, a, beta, first, fb, ra.fh.mk, {}, {}};
#pragma unroll
    for (int i = 0; i < kFcgMax; ++i) {
        ld.bet[i] = bet[i];
        ld.prev[i] = static_cast<const T*>(ra.fh.P[i]);
    }
    double acc = 0.0;
  const TileRange tr = tile_range(tl.items());
  for (int wtile = tr.first; wtile < tr.end; wtile += tr.step) {
    int i0, j0, k0, kend;
    tile_origin(tl, g, wtile, i0, j0, k0, kend);
    T vcur[6], acur[6], vnext[6], anext[6];
    __syncthreads();   // LDS of the previous tile is no longer read
    // load weighted plane kk into ring slot kk&1; own anchor values -> vo, ao
    auto load_plane = [&](int kk, T (&vo)[6], T (&ao)[6]) {
        const int sl = kk & 1;
        {   // own interior anchor
            const int i = i0 + tx, j = j0 + ty;
            const bool in = i <= g.nx + 1 && j <= g.ny + 1 && kk <= g.nz + 1;
            const bool own = in && i <= g.nx && j <= g.ny && kk >= k0 && kk < kend;
            const long long o = in ? g.idx(i, j, kk) : 0;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                T val = T(0), aw = T(0);
                if (in) {
                    const long long os = o + s * NP;
                    val = ld.value(os, own);
                    aw = a[os];
                }
                vo[s] = val;
                ao[s] = aw;
                sW[sl][s][ty + 1][tx + 1] = aw * val;
            }
        }
        // halo ring: rows lj = 0 and HY-1 (HX each), columns li = 0 and HX-1 (TY each)
        if (tid < 2 * HX + 2 * TY) {
            int li, lj;
            if (tid < HX) {
                li = tid;
                lj = 0;
            } else if (tid < 2 * HX) {
                li = tid - HX;
                lj = HY - 1;
            } else {
                const int e = tid - 2 * HX;
                lj = 1 + (e >> 1);
                li = (e & 1) ? HX - 1 : 0;
            }
            const int i = i0 - 1 + li, j = j0 - 1 + lj;
            const bool in = i <= g.nx + 1 && j <= g.ny + 1 && kk <= g.nz + 1;
            const long long o = in ? g.idx(i, j, kk) : 0;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                T w = T(0);
                if (in) {
                    const long long os = o + s * NP;
                    w = a[os] * ld.value(os, false);
                }
                sW[sl][s][lj][li] = w;
            }
        }
    };

    // faces: g_u(kk), g_v(kk) from planes kk, kk+1; g_w(kk+1) from planes kk, kk+1
    auto faces = [&](int kk, bool uv, bool w) {
        const int s0 = kk & 1, s1 = (kk + 1) & 1;
        for (int e = tid; e < FX * FY; e += NT) {
            const int li = e % FX, lj = e / FX;
            if (uv) {
                {   // u face (i0+li, j0-1+lj, kk): weighted indices li (i-1), li+1 (i), lj+...
                    const int i = i0 + li, j = j0 - 1 + lj;
                    T gv = T(0);
                    if (i <= g.nx && j >= 0 && j < g.ny && kk >= 0 && kk < g.nz) {
                        const T kf = K[g.idx(i, j, kk)];
                        // P,X at (i-1): [lj][li], (i): [lj][li+1]; E at j: [lj][li+1], j+1: [lj+1][li+1]
                        const T d = (sW[s0][0][lj][li + 1] - sW[s0][0][lj][li]) +
                                    (sW[s0][1][lj][li] - sW[s0][1][lj][li + 1]) +
                                    (sW[s0][3][lj][li + 1] - sW[s0][3][lj + 1][li + 1]) +
                                    (sW[s0][4][lj][li + 1] - sW[s1][4][lj][li + 1]);
                        gv = kf * d;
                    }
                    gU[s0][lj][li] = gv;
                }
                {   // v face (i0-1+li, j0+lj, kk)
                    const int i = i0 - 1 + li, j = j0 + lj;
                    T gv = T(0);
                    if (i >= 0 && i < g.nx && j <= g.ny && kk >= 0 && kk < g.nz) {
                        const T kf = K[NP + g.idx(i, j, kk)];
                        // weighted (i): li, (i+1): li+1; (j): lj+1, (j-1): lj
                        const T d = (sW[s0][0][lj + 1][li] - sW[s0][0][lj][li]) +
                                    (sW[s0][2][lj][li] - sW[s0][2][lj + 1][li]) +
                                    (sW[s0][3][lj + 1][li] - sW[s0][3][lj + 1][li + 1]) +
                                    (sW[s0][5][lj + 1][li] - sW[s1][5][lj + 1][li]);
                        gv = kf * d;
                    }
                    gV[s0][lj][li] = gv;
                }
            }
            if (w) {   // w face (i0-1+li, j0-1+lj, kk+1): weighted (i): li, (j): lj
                const int i = i0 - 1 + li, j = j0 - 1 + lj, kw = kk + 1;
                T gv = T(0);
                if (i >= 0 && i < g.nx && j >= 0 && j < g.ny && kw >= 0 && kw <= g.nz) {
                    const T kf = K[2 * NP + g.idx(i, j, kw)];
                    const T d = (sW[s1][0][lj][li] - sW[s0][0][lj][li]) +
                                (sW[s1][1][lj][li] - sW[s0][1][lj][li]) +
                                (sW[s1][2][lj][li] - sW[s0][2][lj][li]) +
                                (sW[s1][4][lj][li] - sW[s1][4][lj][li + 1]) +
                                (sW[s1][5][lj][li] - sW[s1][5][lj + 1][li]);
                    gv = kf * d;
                }
                gW[s1][lj][li] = gv;
            }
        }
    };

    // prologue: planes k0-1 and k0, faces u,v at k0-1 and w at k0
    load_plane(k0 - 1, vnext, anext);
    load_plane(k0, vcur, acur);
    __syncthreads();
    faces(k0 - 1, true, true);
    __syncthreads();

    for (int k = k0; k < kend; ++k) {
        load_plane(k + 1, vnext, anext);
        __syncthreads();
        faces(k, true, true);
        __syncthreads();
        const int i = i0 + tx, j = j0 + ty;
        if (i <= g.nx && j <= g.ny) {
            const int sk = k & 1, sp = (k - 1) & 1, sn = (k + 1) & 1;
            const T gu0 = gU[sk][ty + 1][tx], gu1 = gU[sk][ty + 1][tx + 1];
            const T gum = gU[sk][ty][tx], guz = gU[sp][ty + 1][tx];
            const T gv0 = gV[sk][ty][tx + 1], gv1 = gV[sk][ty + 1][tx + 1];
            const T gvm = gV[sk][ty][tx], gvz = gV[sp][ty][tx + 1];
            const T gw0 = gW[sk][ty + 1][tx + 1], gw1 = gW[sn][ty + 1][tx + 1];
            const T gwx = gW[sk][ty + 1][tx], gwy = gW[sk][ty][tx + 1];
            const long long o = g.idx(i, j, k);
            const T c1 = c[NP + o], c2 = c[2 * NP + o];
            const T cross = T(0.5) * fmin(c1, c2);
            T y[6];
            y[0] = acur[0] * ((gu0 - gu1) + (gv0 - gv1) + (gw0 - gw1));
            y[1] = acur[1] * ((gu1 - gu0) + (gw0 - gw1)) + c1 * vcur[1] + cross * vcur[2];
            y[2] = acur[2] * ((gv1 - gv0) + (gw0 - gw1)) + c2 * vcur[2] + cross * vcur[1];
            y[3] = acur[3] * ((gu0 - gum) + (gv0 - gvm)) + c[3 * NP + o] * vcur[3];
            y[4] = acur[4] * ((gu0 - guz) + (gw0 - gwx)) + c[4 * NP + o] * vcur[4];
            y[5] = acur[5] * ((gv0 - gvz) + (gw0 - gwy)) + c[5 * NP + o] * vcur[5];
            if (MODE == MODE_RESID) {
#pragma unroll
                for (int s = 0; s < 6; ++s) {
                    const T rr = bv[s * NP + o] - y[s];
                    q[s * NP + o] = rr;
                    acc += (double)rr * (double)rr;
                }
            } else {
#pragma unroll
                for (int s = 0; s < 6; ++s) {
                    q[s * NP + o] = y[s];
                    if (MODE == MODE_DIR || MODE == MODE_FDIR || MODE == MODE_JDIR)
                        acc += (double)vcur[s] * (double)y[s];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            vcur[s] = vnext[s];
            acur[s] = anext[s];
        }
    }
  }
    if (MODE == MODE_APPLY) return;
    double vv[1] = {acc};
    block_partial<1, NT>(vv, ra.part_out, gridDim.x, blockIdx.x);
}

// MODE_DIR (Jacobi PCG direction + apply) with software pipelining: the raw
// inputs (r, D^-1, p_old, a) of plane k+2 are loaded into registers while
// plane k's faces and outputs are computed, and the face K and output c
// values one plane ahead, so no plane waits for a full memory round trip.
// Same arithmetic, same order and same partials as k_apply3d<T, MODE_DIR>.
template <typename T>
struct RawPlane {
    T r[6], d[6], p[6], a[6];
};

template <typename T>
__global__ __launch_bounds__(NT) void k_dir3d_pipe(Geo g, Tiles tl, const T* __restrict__ r,
                                                   const T* __restrict__ dinv,
                                                   const T* __restrict__ pin, T* __restrict__ pout,
                                                   T* __restrict__ q, const T* __restrict__ a,
                                                   const T* __restrict__ c,
                                                   const T* __restrict__ K, RedArgs ra) {
    if (ra.sc->done) return;
    double bd;
    if (!cg_direction_preamble<NT>(ra, blockIdx.x, bd)) return;
    const bool first = ra.kidx == 0;
    const T beta = (T)bd;
    __shared__ T sW[2][6][HY][HX];
    __shared__ T gU[2][FY][FX];
    __shared__ T gV[2][FY][FX];
    __shared__ T gW[2][FY][FX];
    const long long NP = g.NP;
    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    // this thread's halo-ring position (rows lj = 0 and HY-1, columns li = 0 and HX-1)
    const bool hrole = tid < 2 * HX + 2 * TY;
    int hli = 0, hlj = 0;
    if (tid < HX) {
        hli = tid;
        hlj = 0;
    } else if (tid < 2 * HX) {
        hli = tid - HX;
        hlj = HY - 1;
    } else if (hrole) {
        const int e = tid - 2 * HX;
        hlj = 1 + (e >> 1);
        hli = (e & 1) ? HX - 1 : 0;
    }
    constexpr int NF = (FX * FY + NT - 1) / NT;
    double acc = 0.0;
    const TileRange trg = tile_range(tl.items());
    for (int wtile = trg.first; wtile < trg.end; wtile += trg.step) {
        int i0, j0, k0, kend;
        tile_origin(tl, g, wtile, i0, j0, k0, kend);
        const int io = i0 + tx, jo = j0 + ty;
        const int ih = i0 - 1 + hli, jh = j0 - 1 + hlj;

        auto fetch = [&](int kk, RawPlane<T>& o, RawPlane<T>& h) {
            const bool ino = io <= g.nx + 1 && jo <= g.ny + 1 && kk <= g.nz + 1;
            const long long oo = ino ? g.idx(io, jo, kk) : 0;
            const bool inh = hrole && ih <= g.nx + 1 && jh <= g.ny + 1 && kk <= g.nz + 1;
            const long long oh = inh ? g.idx(ih, jh, kk) : 0;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const long long so = oo + s * NP, sh = oh + s * NP;
                o.r[s] = ino ? r[so] : T(0);
                o.d[s] = ino ? dinv[so] : T(0);
                o.p[s] = (ino && !first) ? pin[so] : T(0);
                o.a[s] = ino ? a[so] : T(0);
                h.r[s] = inh ? r[sh] : T(0);
                h.d[s] = inh ? dinv[sh] : T(0);
                h.p[s] = (inh && !first) ? pin[sh] : T(0);
                h.a[s] = inh ? a[sh] : T(0);
            }
        };
        // direction values of plane kk into the ring slot; own anchor values out
        auto commit = [&](int kk, const RawPlane<T>& o, const RawPlane<T>& h, T (&vo)[6],
                          T (&ao)[6]) {
            const int sl = kk & 1;
            const bool own = io <= g.nx && jo <= g.ny && kk >= k0 && kk < kend;
            const long long oo = own ? g.idx(io, jo, kk) : 0;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const T z = o.d[s] * o.r[s];
                const T val = first ? z : z + beta * o.p[s];
                if (own) pout[oo + s * NP] = val;
                vo[s] = val;
                ao[s] = o.a[s];
                sW[sl][s][ty + 1][tx + 1] = o.a[s] * val;
            }
            if (hrole) {
#pragma unroll
                for (int s = 0; s < 6; ++s) {
                    const T z = h.d[s] * h.r[s];
                    const T val = first ? z : z + beta * h.p[s];
                    sW[sl][s][hlj][hli] = h.a[s] * val;
                }
            }
        };
        // K of the faces formed at plane kk: u, v at kk and w at kk + 1
        auto fetchK = [&](int kk, T (&ku)[NF], T (&kv)[NF], T (&kw)[NF]) {
#pragma unroll
            for (int m = 0; m < NF; ++m) {
                const int e = tid + m * NT;
                const int li = e % FX, lj = e / FX;
                ku[m] = kv[m] = kw[m] = T(0);
                if (e < FX * FY) {
                    const int iu = i0 + li, ju = j0 - 1 + lj;
                    if (iu <= g.nx && ju >= 0 && ju < g.ny && kk >= 0 && kk < g.nz)
                        ku[m] = K[g.idx(iu, ju, kk)];
                    const int iv = i0 - 1 + li, jv = j0 + lj;
                    if (iv >= 0 && iv < g.nx && jv <= g.ny && kk >= 0 && kk < g.nz)
                        kv[m] = K[NP + g.idx(iv, jv, kk)];
                    const int iw = i0 - 1 + li, jw = j0 - 1 + lj, kw2 = kk + 1;
                    if (iw >= 0 && iw < g.nx && jw >= 0 && jw < g.ny && kw2 >= 0 && kw2 <= g.nz)
                        kw[m] = K[2 * NP + g.idx(iw, jw, kw2)];
                }
            }
        };
        auto faces = [&](int kk, const T (&ku)[NF], const T (&kv)[NF], const T (&kw)[NF]) {
            const int s0 = kk & 1, s1 = (kk + 1) & 1;
#pragma unroll
            for (int m = 0; m < NF; ++m) {
                const int e = tid + m * NT;
                if (e >= FX * FY) continue;
                const int li = e % FX, lj = e / FX;
                gU[s0][lj][li] = ku[m] * ((sW[s0][0][lj][li + 1] - sW[s0][0][lj][li]) +
                                          (sW[s0][1][lj][li] - sW[s0][1][lj][li + 1]) +
                                          (sW[s0][3][lj][li + 1] - sW[s0][3][lj + 1][li + 1]) +
                                          (sW[s0][4][lj][li + 1] - sW[s1][4][lj][li + 1]));
                gV[s0][lj][li] = kv[m] * ((sW[s0][0][lj + 1][li] - sW[s0][0][lj][li]) +
                                          (sW[s0][2][lj][li] - sW[s0][2][lj + 1][li]) +
                                          (sW[s0][3][lj + 1][li] - sW[s0][3][lj + 1][li + 1]) +
                                          (sW[s0][5][lj + 1][li] - sW[s1][5][lj + 1][li]));
                gW[s1][lj][li] = kw[m] * ((sW[s1][0][lj][li] - sW[s0][0][lj][li]) +
                                          (sW[s1][1][lj][li] - sW[s0][1][lj][li]) +
                                          (sW[s1][2][lj][li] - sW[s0][2][lj][li]) +
                                          (sW[s1][4][lj][li] - sW[s1][4][lj][li + 1]) +
                                          (sW[s1][5][lj][li] - sW[s1][5][lj + 1][li]));
            }
        };
        auto fetchC = [&](int kk, T (&cc)[5]) {
            const bool ok = io <= g.nx && jo <= g.ny && kk >= k0 && kk < kend;
            const long long o = ok ? g.idx(io, jo, kk) : 0;
#pragma unroll
            for (int s = 0; s < 5; ++s) cc[s] = ok ? c[(s + 1) * NP + o] : T(0);
        };

        T vcur[6], acur[6], vnext[6], anext[6];
        RawPlane<T> Fo, Fh;
        T Ku[NF], Kv[NF], Kw[NF], Cc[5];
        __syncthreads();   // LDS of the previous tile is no longer read
        // prologue: planes k0-1 and k0, faces at k0-1
        fetch(k0 - 1, Fo, Fh);
        fetchK(k0 - 1, Ku, Kv, Kw);
        commit(k0 - 1, Fo, Fh, vnext, anext);
        fetch(k0, Fo, Fh);
        commit(k0, Fo, Fh, vcur, acur);
        fetch(k0 + 1, Fo, Fh);            // in flight during the prologue faces
        __syncthreads();
        faces(k0 - 1, Ku, Kv, Kw);
        fetchK(k0, Ku, Kv, Kw);
        fetchC(k0, Cc);
        __syncthreads();

        for (int k = k0; k < kend; ++k) {
            commit(k + 1, Fo, Fh, vnext, anext);
            if (k + 2 <= kend) fetch(k + 2, Fo, Fh);
            __syncthreads();
            faces(k, Ku, Kv, Kw);
            T Cn[5];
            if (k + 1 < kend) fetchK(k + 1, Ku, Kv, Kw);   // no faces after the last plane
            fetchC(k + 1, Cn);
            __syncthreads();
            if (io <= g.nx && jo <= g.ny) {
                const int sk = k & 1, sp = (k - 1) & 1, sn = (k + 1) & 1;
                const T gu0 = gU[sk][ty + 1][tx], gu1 = gU[sk][ty + 1][tx + 1];
                const T gum = gU[sk][ty][tx], guz = gU[sp][ty + 1][tx];
                const T gv0 = gV[sk][ty][tx + 1], gv1 = gV[sk][ty + 1][tx + 1];
                const T gvm = gV[sk][ty][tx], gvz = gV[sp][ty][tx + 1];
                const T gw0 = gW[sk][ty + 1][tx + 1], gw1 = gW[sn][ty + 1][tx + 1];
                const T gwx = gW[sk][ty + 1][tx], gwy = gW[sk][ty][tx + 1];
                const long long o = g.idx(io, jo, k);
                const T c1 = Cc[0], c2 = Cc[1];
                const T cross = T(0.5) * fmin(c1, c2);
                T y[6];
                y[0] = acur[0] * ((gu0 - gu1) + (gv0 - gv1) + (gw0 - gw1));
                y[1] = acur[1] * ((gu1 - gu0) + (gw0 - gw1)) + c1 * vcur[1] + cross * vcur[2];
                y[2] = acur[2] * ((gv1 - gv0) + (gw0 - gw1)) + c2 * vcur[2] + cross * vcur[1];
                y[3] = acur[3] * ((gu0 - gum) + (gv0 - gvm)) + Cc[2] * vcur[3];
                y[4] = acur[4] * ((gu0 - guz) + (gw0 - gwx)) + Cc[3] * vcur[4];
                y[5] = acur[5] * ((gv0 - gvz) + (gw0 - gwy)) + Cc[4] * vcur[5];
#pragma unroll
                for (int s = 0; s < 6; ++s) {
                    q[s * NP + o] = y[s];
                    acc += (double)vcur[s] * (double)y[s];
                }
            }
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                vcur[s] = vnext[s];
                acur[s] = anext[s];
            }
#pragma unroll
            for (int s = 0; s < 5; ++s) Cc[s] = Cn[s];
        }
    }
    double vv[1] = {acc};
    block_partial<1, NT>(vv, ra.part_out, gridDim.x, blockIdx.x);
}

// One launch per Jacobi-PCG iteration in 3D (mixed precision), the plane-
// marching form of the fused 2D iteration: launch k carries out iteration
// k-1's update lazily (r_k = r_{k-1} - alpha q_{k-1} on the tile and its
// halo, x_k = x_{k-1} + alpha p_{k-1} at the own anchors), forms z_k = D^-1 r_k
// and p_k = z_k + beta p_{k-1}, applies q_k = A p_k and reduces (r.z, p.q,
// q.D^-1 r, q.D^-1 q, r.r).  beta_k comes from the expansion
// r_k.z_k = r.z - 2 alpha q.D^-1 r + alpha^2 q.D^-1 q of the previous
// launch's totals (re-anchored every launch on the directly summed r.z), so
// one global reduction per iteration suffices.  r, p and q alternate between
// two buffers by launch parity because the halo of launch k reads the values
// of launch k-1 that neighbouring workgroups overwrite.  The raw inputs of
// plane k+2 are loaded while plane k is computed, as in k_dir3d_pipe.
//
// Work tiles are FTX x FTY anchors marching FKZ planes (a part of one list
// tile in x, FTY / 4 x FKZ / 8 list tiles in y and z), so the halo ring costs
// 2 rows per FTY, 2 columns per FTX and 2 planes per FKZ.  Every solver vector
// is zero on a sample with a = 0 (inactive samples have a = c = D^-1 = 0, the
// solve starts from zero there and nothing is ever stored there), so a half
// row of one sample slice whose row bit is clear is neither loaded nor
// stored: its values are known to be 0.
//
// The faces need a p_k at every position of the tile and its halo.  The
// direction is kept weighted, P = a p (a = W_L), and so are the residual and
// A p, R = e r and Q = e q with e = a D^-1 (ead): then
// a p_k = e (r_{k-1} - alpha q_{k-1}) + beta P_{k-1} = R_{k-1} - alpha Q_{k-1}
// + beta P_{k-1} takes three loads per halo position (R, Q and P, where the
// unweighted vectors took r, q, p, D^-1 and a).  The own anchors also read e
// and a, and form r = R / e, z = D^-1 r = R / a, p = P / a and D^-1 = e / a
// for the partials, the update of x and the compliance term; their A p is
// stored as Q = (D^-1 a) A p.  The launch that starts a solve reads the plain
// residual from the second r buffer and writes R_0 = e r_0 to the first.
//
// When nx is a multiple of FTX the anchors i = 0..nx need one x tile more than
// nx / FTX, and that tile holds only the column i = nx, where only tau_xy and
// tau_xz exist (on the wall x = nx h).  The fused work tiles then stop one x
// tile earlier and the last of them also owns that column: the threads that
// load its x halo at i = nx (rows j0 .. j0 + FTY - 1) carry out the update of
// those two samples and form their outputs from the face values already in
// LDS (the v and w faces at i = nx do not exist and count as 0).
#ifndef VFS_FUSED3_FOLD
#define VFS_FUSED3_FOLD 1
#endif
// The kernel runs with G = 1 or 2 threads per anchor.  With G = 2, slice
// group 0 (p, tau_xx, tau_yy) and slice group 1 (tau_xy, tau_xz, tau_yz) are
// waves 0-3 and 4-7 of the workgroup; each thread keeps the prefetched plane
// of three slices only, so the kernel fits in 128 VGPRs and 16 waves run per
// CU instead of 8.  The bytes in flight per CU stay the same (two workgroups
// of one tile each), so G = 2 pays off where a workgroup has few planes to
// march (short tile lists split in z), and G = 1 where the sweep is long.
constexpr int FTX = kFused3X, FTY = kFused3Y, FKZ = kFused3Z;
constexpr int FNA = FTX * FTY;
// a tile list split into at least this many z parts runs with G = 2
#ifndef VFS_FUSED3_PAIR_SPLIT
#define VFS_FUSED3_PAIR_SPLIT 2
#endif
constexpr int FHX = FTX + 2, FHY = FTY + 2, FFX = FTX + 1, FFY = FTY + 1;

// the last x tile is folded into the one before it (nx a multiple of FTX)
__host__ __device__ __forceinline__ bool fused_fold(int nx) {
    return VFS_FUSED3_FOLD && nx >= FTX && nx % FTX == 0;
}

// row bits of x tile t, row (j, k); 0 outside the anchors of the grid
__device__ __forceinline__ unsigned row_bits_at(const Geo& g, const RowBits* __restrict__ rows,
                                                int ntx, int t, int j, int k) {
    if (t < 0 || t >= ntx || j < 0 || j > g.ny || k < 0 || k > g.nz) return 0u;
    return rows[t + (long long)ntx * (j + (long long)(g.ny + 1) * k)];
}

// slice bits of the half row holding anchor `lane` (0 .. kRow3X - 1) of a row
__device__ __forceinline__ unsigned half_bits(unsigned rb, int lane) {
    return (lane >= kRow3X / 2 ? rb >> 6 : rb) & 63u;
}

// Byte offset of anchor (i, j, k) within a sample slice of FP32 values, or 0
// (the slice's zero pad) when ok is false.  The fused iteration adds the
// slice's offset s * NP * 4 and addresses every array from its base, so all
// six slices must lie within 4 GiB (checked before its launch); the mask
// replaces a select and the empty asm hides the value from the optimizer, so
// that every access keeps the scalar-base form (array base in SGPRs, 32-bit
// offset in one VGPR).
__device__ __forceinline__ unsigned boff3(const Geo& g, int i, int j, int k, bool ok) {
    const unsigned e = (unsigned)kFront +
                       ((unsigned)(k + 1) * (unsigned)g.PY + (unsigned)(j + 1)) * (unsigned)g.PX +
                       (unsigned)i;
    unsigned b = (e * 4u) & (0u - (unsigned)ok);
    asm("" : "+v"(b));
    return b;
}
template <typename T>
__device__ __forceinline__ T ld_at(const T* __restrict__ base, unsigned boff) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename T>
__device__ __forceinline__ void st_at(T* __restrict__ base, unsigned boff, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff) = v;
}

// Anchors of fused work item u: x from i0, y from j0, planes [k0, kend).
__device__ __forceinline__ void fused_origin(const Tiles& t, const Geo& g, int u, int& tx, int& j0,
                                             int& k0, int& kend) {
    const int id = t.list[u / t.split];
    tx = id % t.ntx;
    const int ty = (id / t.ntx) % t.nty;
    const int tz = id / (t.ntx * t.nty);
    const int kz = FKZ / t.split;
    j0 = ty * FTY;
    k0 = tz * FKZ + (u % t.split) * kz;
    kend = min(k0 + kz, g.nz + 1);
}

// Work items of one fused launch.  As in tile_range, XCD x (workgroups
// b = x mod 8) takes one contiguous eighth [t0, t1) of the item list.  A
// workgroup's first two items are fixed (items t0 + slot and t0 + slot + nblk,
// slot = b / 8, nblk workgroups on the XCD); its later items come from its
// XCD's counter in list order, so that the workgroups whose items hold few
// active rows take more of them (a fixed stride left the busiest workgroup
// with about 1.3x the mean work at 256^3).  The first claim is made during
// the second item, when the workgroups no longer start in step, and a short
// list never touches the counter.  The counters
// alternate by launch parity: launch k takes from slot k & 1 and clears slot
// (k + 1) & 1, which launch k - 1 used and launch k + 1 takes from.  The
// first launch of a solve keeps the fixed stride, so a solve never depends on
// counters left by an earlier one; so do grids of fewer than 8 workgroups.
struct FusedQueue {
    int t0, t1, first, step;   // the XCD's range, first item and stride (nblk)
    unsigned* ctr;             // the XCD's counter, or null: fixed stride
};
__device__ __forceinline__ FusedQueue fused_queue(int count, unsigned* wq, int kidx, bool dyn) {
    const int G = gridDim.x, b = blockIdx.x;
    if (G < 8) return FusedQueue{0, count, b, G, nullptr};
    const int x = b & 7, slot = b >> 3;
    const int nblk = (G - x + 7) >> 3;
    const int t0 = (int)((long long)count * x / 8), t1 = (int)((long long)count * (x + 1) / 8);
    return FusedQueue{t0, t1, t0 + slot, nblk, dyn ? wq + 8 * (kidx & 1) + x : nullptr};
}

template <typename T, int NS>
struct FusedOwn {
    T r[NS], q[NS], P[NS], e[NS], a[NS], x[NS];   // P = a p, e = a D^-1
    T c[NS];      // compliance coefficients of the own anchor one plane below
    unsigned m;   // row bits of the plane (this thread's slices)
};
template <typename T, int NS>
struct FusedHalo {
    T r[NS], q[NS], P[NS], e[NS];
    T x3, x4, c3, c4, a3, a4;   // x, c and a of tau_xy, tau_xz in the folded column i = nx
    unsigned m;
};

// R, Q and P of one plane: all that a p = R - alpha Q + beta P needs
template <typename T, int NS>
struct FusedW {
    T r[NS], q[NS], P[NS];
};

template <typename T, bool INIT, int G>
__global__ __launch_bounds__(G * FNA, 2 * G) void k_fused3d(Geo g, Tiles ft, FusedVecs v,
                                                    const T* __restrict__ ead,
                                                    const T* __restrict__ a,
                                                    const T* __restrict__ c,
                                                    const T* __restrict__ K,
                                                    const RowBits* __restrict__ rows,
                                                    unsigned* __restrict__ wq, RedArgs ra) {
    constexpr int FNS = 6 / G, FNT = G * FNA;   // slices and threads per anchor / workgroup
    Scalars* sc = ra.sc;
    const int kidx = ra.kidx;
    const int pin = (kidx + 1) & 1, pout = kidx & 1;   // launch k reads (k-1)&1, writes k&1
    const T* __restrict__ r_in = static_cast<const T*>(v.r[INIT ? 1 : pin]);
    const T* __restrict__ q_in = static_cast<const T*>(v.q[pin]);
    const T* __restrict__ p_in = static_cast<const T*>(v.p[pin]);
    T* __restrict__ r_out = static_cast<T*>(v.r[pout]);
    T* __restrict__ p_out = static_cast<T*>(v.p[pout]);
    T* __restrict__ q_out = static_cast<T*>(v.q[pout]);
    T* __restrict__ x = static_cast<T*>(v.x);

    // clear the work-queue slot of the next launch (before any early return)
    if (blockIdx.x == 0 && threadIdx.x < 8) wq[8 * ((kidx + 1) & 1) + threadIdx.x] = 0u;
    // totals of the previous launch -> stop decision, alpha_{k-1}, beta_k
    PartialLoads<5, FNT, 2 / G> pl;
    if (!INIT) pl.load(ra.part_in, ra.nb_in);
    if (!INIT && sc->done) return;
    T alpha = T(0), beta = T(0);
    if (!INIT) {
        double t[5];
        pl.finish(t);
        const double rz = t[0], pq = t[1], qdr = t[2], qdq = t[3], rrk = t[4];
        const double bb = ra.set_bb ? rrk : sc->bb;
        int stop = 0;
        if (!isfinite(rz) || !isfinite(rrk) || !isfinite(pq))
            stop = 3;
        else if (rrk <= sc->tol2 * bb)
            stop = 1;
        else if (kidx - 1 >= sc->max_iter)
            stop = 2;
        else if (!(pq > 0.0))
            stop = 3;
        const double ad = stop ? 0.0 : rz / pq;
        const double rzn = rz - 2.0 * ad * qdr + ad * ad * qdq;
        const double bd = (rz > 0.0) ? rzn / rz : 0.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rz[kidx & 1] = rz;
            sc->rr = rrk;
            sc->pq = pq;
            sc->alpha = ad;
            sc->beta = bd;
            if (ra.set_bb) sc->bb = bb;
            if (stop) {
                sc->done = stop;
                sc->iter = kidx - 1;
            }
        }
        if (stop) return;
        alpha = (T)ad;
        beta = (T)bd;
    }

    __shared__ T sW[2][6][FHY][FHX];
    __shared__ T gU[2][FFY][FFX];
    __shared__ T gV[2][FFY][FFX];
    __shared__ T gW[2][FFY][FFX];
    __shared__ T sXF[2][FTY][2][5];     // folded column: p, a, z, D^-1, c per plane parity
    __shared__ unsigned sXM[2][FTY];    // and its row bits
    // row bits of the work item's planes k0 - 1 .. kend, rows j0 - 1 .. j0 + FTY,
    // x tiles xt - 1, xt, xt + 1 (read once per item, so that no plane waits
    // on a global load before it can issue its own)
    __shared__ RowBits sRB[FKZ + 2][FHY][3];
    // p, a, z and D^-1 of a thread's own samples, from the commit of a plane to
    // the outputs of that plane: registers with G = 1, per-thread LDS slots by
    // plane parity with G = 2 (128 VGPRs leave no room for them)
    constexpr int NOWN = G == 2 ? FNT : 1;
    __shared__ T sOwn[2][4][FNS][NOWN];
    __shared__ int sNext;   // the item claimed from the work queue
    const unsigned NPB = (unsigned)g.NP * 4u;   // bytes of a slice (6 slices < 4 GiB)
    const int tid = threadIdx.x;
    // slice group (uniform per wave) and anchor of the plane
    const int grp = G == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid / FNA);
    const int ot = G == 1 ? tid : tid % FNA;
    const int s0 = grp * FNS;                    // first slice of this thread
    const unsigned gmask = ((1u << FNS) - 1u) << s0;
    const int tx = ot % FTX, ty = ot / FTX;
    const bool hrole = ot < 2 * FHX + 2 * FTY;
    int hli = 0, hlj = 0;
    if (ot < FHX) {
        hli = ot;
        hlj = 0;
    } else if (ot < 2 * FHX) {
        hli = ot - FHX;
        hlj = FHY - 1;
    } else if (hrole) {
        const int e = ot - 2 * FHX;
        hlj = 1 + (e >> 1);
        hli = (e & 1) ? FHX - 1 : 0;
    }
    // x tile of the halo position relative to the work tile's (-1, 0, +1),
    // and its anchor within that tile's rows
    const int hdt = hli == 0 ? -1 : (hli == FHX - 1 ? 1 : 0);
    const int hlane = hdt < 0 ? FTX - 1 : (hdt > 0 ? 0 : hli - 1);
    const int rntx = (g.nx + kRow3X) / kRow3X;   // x parts of the row bits
    const bool fold = fused_fold(g.nx);
    // right x-halo threads of the own rows that hold tau_xy, tau_xz: owners
    // of the folded column (its two slices are q = qx, qx + 1 of the thread)
    const bool xrole = fold && s0 + FNS > 4 && hrole && ot >= 2 * FHX && hli == FHX - 1;
    constexpr int qx = FNS - 3;
    constexpr int NF = (FFX * FFY + FNT - 1) / FNT;
    double rz_n = 0.0, rr_n = 0.0, pq_n = 0.0, qz_n = 0.0, qdq_n = 0.0;
    // with two threads per anchor the list is split in z and holds at most one
    // item per workgroup, so that shape never claims
    const FusedQueue fq = fused_queue(ft.items(), wq, kidx, !INIT && G == 1);
    for (int wtile = fq.first; wtile < fq.t1;) {
        int xt, j0, k0, kend;
        fused_origin(ft, g, wtile, xt, j0, k0, kend);
        const int i0 = xt * FTX;
        const int io = i0 + tx, jo = j0 + ty;
        const int ih = i0 - 1 + hli, jh = j0 - 1 + hlj;
        // this thread also owns anchor (nx, jh) of the folded column
        const bool xown = xrole && xt == ft.ntx - 1 && jh <= g.ny;
        const bool first_round = wtile < fq.t0 + fq.step;   // the next item is fixed
        __syncthreads();   // LDS of the previous item is no longer read
        for (int e = tid; e < (kend - k0 + 2) * FHY * 3; e += FNT) {
            const int pl = e / (FHY * 3), rw = (e / 3) % FHY, part = e % 3;
            sRB[pl][rw][part] =
                (RowBits)row_bits_at(g, rows, rntx, xt + part - 1, j0 - 1 + rw, k0 - 1 + pl);
        }

        auto fetch = [&](int kk, FusedOwn<T, FNS>& o, FusedHalo<T, FNS>& h) {
            const bool own = io <= g.nx && jo <= g.ny && kk >= k0 && kk < kend;
            const int pl = kk - k0 + 1;
            o.m = io <= g.nx + 1 ? half_bits(sRB[pl][ty + 1][1], tx) & gmask : 0u;
            const unsigned oo = boff3(g, io, jo, kk, o.m != 0u);
            h.m = (hrole && ih <= g.nx + 1) ? half_bits(sRB[pl][hlj][hdt + 1], hlane) & gmask : 0u;
            const unsigned oh = boff3(g, ih, jh, kk, h.m != 0u);
            // c of the own anchor at plane kk - 1 (the plane whose outputs are
            // formed while this one is being committed); p has none
            const bool ownb = io <= g.nx && jo <= g.ny && kk - 1 >= k0 && kk - 1 < kend;
            const unsigned mb = ownb ? half_bits(sRB[pl - 1][ty + 1][1], tx) & gmask & ~1u : 0u;
            const unsigned ob = boff3(g, io, jo, kk - 1, mb != 0u);
#pragma unroll
            for (int q = 0; q < FNS; ++q) {
                const int s = s0 + q;
                o.c[q] = ((mb >> s) & 1u) ? ld_at(c, ob + (unsigned)s * NPB) : T(0);
            }
            const bool hx = xown && kk >= k0 && kk < kend;
            const bool h3 = hx && ((h.m >> 3) & 1u), h4 = hx && ((h.m >> 4) & 1u);
            h.x3 = (h3 && !INIT) ? ld_at(x, oh + 3u * NPB) : T(0);
            h.x4 = (h4 && !INIT) ? ld_at(x, oh + 4u * NPB) : T(0);
            h.c3 = h3 ? ld_at(c, oh + 3u * NPB) : T(0);
            h.c4 = h4 ? ld_at(c, oh + 4u * NPB) : T(0);
            h.a3 = h3 ? ld_at(a, oh + 3u * NPB) : T(0);
            h.a4 = h4 ? ld_at(a, oh + 4u * NPB) : T(0);
#pragma unroll
            for (int q = 0; q < FNS; ++q) {
                const int s = s0 + q;
                const unsigned sb = (unsigned)s * NPB;   // slice offset in bytes (uniform)
                const bool lo = (o.m >> s) & 1u, lh = (h.m >> s) & 1u;
                o.r[q] = lo ? ld_at(r_in, oo + sb) : T(0);
                // a p needs neither a nor e outside the item's own anchors (its
                // z-halo planes, the rows past the grid), except to weight the
                // plain residual of the first launch
                o.e[q] = (lo && (INIT || own)) ? ld_at(ead, oo + sb) : T(0);
                o.a[q] = (lo && own) ? ld_at(a, oo + sb) : T(0);
                o.q[q] = (lo && !INIT) ? ld_at(q_in, oo + sb) : T(0);
                o.P[q] = (lo && !INIT) ? ld_at(p_in, oo + sb) : T(0);
                o.x[q] = (lo && own && !INIT) ? ld_at(x, oo + sb) : T(0);
                h.r[q] = lh ? ld_at(r_in, oh + sb) : T(0);
                // the halo needs e only to weight the plain residual of the
                // first launch, and for the own samples of the folded column
                h.e[q] = (lh && (INIT || (hx && (s == 3 || s == 4)))) ? ld_at(ead, oh + sb) : T(0);
                h.q[q] = (lh && !INIT) ? ld_at(q_in, oh + sb) : T(0);
                h.P[q] = (lh && !INIT) ? ld_at(p_in, oh + sb) : T(0);
            }
        };
        // a p_k of plane kk into the ring slot; own anchors also store R_k,
        // x_k, P_k and add to r.z, r.r; own p, a, z, D^-1, c and row bits out
        auto commit = [&](int kk, const FusedOwn<T, FNS>& o, const FusedHalo<T, FNS>& h,
                          T (&vo)[FNS], T (&ao)[FNS], T (&zo)[FNS], T (&dq)[FNS], unsigned& mo,
                          T (&cb)[FNS]) {
            const int sl = kk & 1;
#pragma unroll
            for (int q = 0; q < FNS; ++q) cb[q] = o.c[q];
            const bool own = io <= g.nx && jo <= g.ny && kk >= k0 && kk < kend;
            mo = own ? o.m : 0u;
            const unsigned oo = boff3(g, io, jo, kk, mo != 0u);
#pragma unroll
            for (int q = 0; q < FNS; ++q) {
                const int s = s0 + q;
                const T Rn = INIT ? o.e[q] * o.r[q] : o.r[q] - alpha * o.q[q];   // e r_k
                const T W = INIT ? Rn : Rn + beta * o.P[q];                         // a p_k
                const T ia = o.a[q] != T(0) ? T(1) / o.a[q] : T(0);
                const T ie = o.e[q] != T(0) ? __builtin_amdgcn_rcpf(o.e[q]) : T(0);
                const T rn = INIT ? o.r[q] : Rn * ie;   // r_k (for the partials only)
                const T dd = o.e[q] * ia;               // D^-1
                const T zn = Rn * ia;                   // z_k = D^-1 r_k
                if ((mo >> s) & 1u) {
                    const unsigned sb = (unsigned)s * NPB;
                    st_at(r_out, oo + sb, Rn);
                    if (!INIT) st_at(x, oo + sb, o.x[q] + alpha * (o.P[q] * ia));
                    st_at(p_out, oo + sb, W);
                    rz_n += (double)rn * (double)zn;
                    rr_n += (double)rn * (double)rn;
                }
                if constexpr (G == 1) {
                    vo[q] = W * ia;
                    ao[q] = o.a[q];
                    zo[q] = zn;
                    dq[q] = dd;
                } else {
                    sOwn[sl][0][q][tid] = W * ia;
                    sOwn[sl][1][q][tid] = o.a[q];
                    sOwn[sl][2][q][tid] = zn;
                    sOwn[sl][3][q][tid] = dd;
                }
                sW[sl][s][ty + 1][tx + 1] = W;
            }
            if (hrole) {
#pragma unroll
                for (int q = 0; q < FNS; ++q) {
                    const T Rn = INIT ? h.e[q] * h.r[q] : h.r[q] - alpha * h.q[q];
                    sW[sl][s0 + q][hlj][hli] = INIT ? Rn : Rn + beta * h.P[q];
                }
            }
            // the folded column: tau_xy (slice 3, q 0) and tau_xz (slice 4,
            // q 1) at (nx, jh); what its outputs need later waits in this
            // thread's LDS slots
            if (xown) {
                const unsigned xm = (kk >= k0 && kk < kend) ? (h.m & 0x18u) : 0u;
                sXM[sl][hlj - 1] = xm;
                const unsigned oh = boff3(g, ih, jh, kk, xm != 0u);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int s = 3 + e;
                    if (!((xm >> s) & 1u)) continue;
                    const T es = h.e[qx + e];
                    const T Rn = INIT ? es * h.r[qx + e] : h.r[qx + e] - alpha * h.q[qx + e];
                    const T W = INIT ? Rn : Rn + beta * h.P[qx + e];
                    const T as = e ? h.a4 : h.a3;
                    const T ia = as != T(0) ? T(1) / as : T(0);
                    const T ie = es != T(0) ? __builtin_amdgcn_rcpf(es) : T(0);
                    const T rn = INIT ? h.r[qx + e] : Rn * ie;
                    const T dd = es * ia;
                    const T zn = Rn * ia;
                    T* f = sXF[sl][hlj - 1][e];
                    f[0] = W * ia;
                    f[1] = as;
                    f[2] = zn;
                    f[3] = dd;
                    f[4] = e ? h.c4 : h.c3;
                    const unsigned sb = (unsigned)s * NPB;
                    st_at(r_out, oh + sb, Rn);
                    if (!INIT) st_at(x, oh + sb, (e ? h.x4 : h.x3) + alpha * (h.P[qx + e] * ia));
                    st_at(p_out, oh + sb, W);
                    rz_n += (double)rn * (double)zn;
                    rr_n += (double)rn * (double)rn;
                }
            }
        };
        // the plane below the item: outside the first launch only a p is formed
        // there, from three loads per sample, so its loads need not wait for
        // those of plane k0
        auto fetchW = [&](int kk, FusedW<T, FNS>& o, FusedW<T, FNS>& h) {
            const int pl = kk - k0 + 1;
            const unsigned mo = io <= g.nx + 1 ? half_bits(sRB[pl][ty + 1][1], tx) & gmask : 0u;
            const unsigned oo = boff3(g, io, jo, kk, mo != 0u);
            const unsigned mh =
                (hrole && ih <= g.nx + 1) ? half_bits(sRB[pl][hlj][hdt + 1], hlane) & gmask : 0u;
            const unsigned oh = boff3(g, ih, jh, kk, mh != 0u);
#pragma unroll
            for (int q = 0; q < FNS; ++q) {
                const int s = s0 + q;
                const unsigned sb = (unsigned)s * NPB;
                const bool lo = (mo >> s) & 1u, lh = (mh >> s) & 1u;
                o.r[q] = lo ? ld_at(r_in, oo + sb) : T(0);
                o.q[q] = lo ? ld_at(q_in, oo + sb) : T(0);
                o.P[q] = lo ? ld_at(p_in, oo + sb) : T(0);
                h.r[q] = lh ? ld_at(r_in, oh + sb) : T(0);
                h.q[q] = lh ? ld_at(q_in, oh + sb) : T(0);
                h.P[q] = lh ? ld_at(p_in, oh + sb) : T(0);
            }
        };
        auto commitW = [&](int kk, const FusedW<T, FNS>& o, const FusedW<T, FNS>& h) {
            const int sl = kk & 1;
#pragma unroll
            for (int q = 0; q < FNS; ++q) {
                sW[sl][s0 + q][ty + 1][tx + 1] = (o.r[q] - alpha * o.q[q]) + beta * o.P[q];
                if (hrole) sW[sl][s0 + q][hlj][hli] = (h.r[q] - alpha * h.q[q]) + beta * h.P[q];
            }
        };
        auto fetchK = [&](int kk, T (&ku)[NF], T (&kv)[NF], T (&kw)[NF]) {
#pragma unroll
            for (int m = 0; m < NF; ++m) {
                const int e = tid + m * FNT;
                const int li = e % FFX, lj = e / FFX;
                ku[m] = kv[m] = kw[m] = T(0);
                if (e < FFX * FFY) {
                    const int iu = i0 + li, ju = j0 - 1 + lj;
                    const bool bu = iu <= g.nx && ju >= 0 && ju < g.ny && kk >= 0 && kk < g.nz;
                    const unsigned fu = boff3(g, iu, ju, kk, bu);
                    if (bu) ku[m] = ld_at(K, fu);
                    const int iv = i0 - 1 + li, jv = j0 + lj;
                    const bool bv = iv >= 0 && iv < g.nx && jv <= g.ny && kk >= 0 && kk < g.nz;
                    const unsigned fv = boff3(g, iv, jv, kk, bv);
                    if (bv) kv[m] = ld_at(K, fv + NPB);
                    const int iw = i0 - 1 + li, jw = j0 - 1 + lj, kw2 = kk + 1;
                    const bool bw = iw >= 0 && iw < g.nx && jw >= 0 && jw < g.ny && kw2 >= 0 &&
                                    kw2 <= g.nz;
                    const unsigned fw = boff3(g, iw, jw, kw2, bw);
                    if (bw) kw[m] = ld_at(K, fw + 2u * NPB);
                }
            }
        };
        auto faces = [&](int kk, const T (&ku)[NF], const T (&kv)[NF], const T (&kw)[NF]) {
            const int s0f = kk & 1, s1f = (kk + 1) & 1;
#pragma unroll
            for (int m = 0; m < NF; ++m) {
                const int e = tid + m * FNT;
                if (e >= FFX * FFY) continue;
                const int li = e % FFX, lj = e / FFX;
                gU[s0f][lj][li] = ku[m] * ((sW[s0f][0][lj][li + 1] - sW[s0f][0][lj][li]) +
                                           (sW[s0f][1][lj][li] - sW[s0f][1][lj][li + 1]) +
                                           (sW[s0f][3][lj][li + 1] - sW[s0f][3][lj + 1][li + 1]) +
                                           (sW[s0f][4][lj][li + 1] - sW[s1f][4][lj][li + 1]));
                gV[s0f][lj][li] = kv[m] * ((sW[s0f][0][lj + 1][li] - sW[s0f][0][lj][li]) +
                                           (sW[s0f][2][lj][li] - sW[s0f][2][lj + 1][li]) +
                                           (sW[s0f][3][lj + 1][li] - sW[s0f][3][lj + 1][li + 1]) +
                                           (sW[s0f][5][lj + 1][li] - sW[s1f][5][lj + 1][li]));
                gW[s1f][lj][li] = kw[m] * ((sW[s1f][0][lj][li] - sW[s0f][0][lj][li]) +
                                           (sW[s1f][1][lj][li] - sW[s0f][1][lj][li]) +
                                           (sW[s1f][2][lj][li] - sW[s0f][2][lj][li]) +
                                           (sW[s1f][4][lj][li] - sW[s1f][4][lj][li + 1]) +
                                           (sW[s1f][5][lj][li] - sW[s1f][5][lj + 1][li]));
            }
        };

        T vcur[FNS], acur[FNS], zcur[FNS], dcur[FNS], vnext[FNS], anext[FNS], znext[FNS],
            dnext[FNS];
        unsigned mcur, mnext;
        FusedOwn<T, FNS> Fo;
        FusedHalo<T, FNS> Fh;
        T Ku[NF], Kv[NF], Kw[NF], Cc[FNS];
        __syncthreads();   // row bits of this item in LDS
        // claim the next item now: the reply arrives with the prologue's loads
        unsigned claim = 0u;
        if (fq.ctr && !first_round && tid == 0) claim = atomicAdd(fq.ctr, 1u);
        if constexpr (INIT) {   // e weights the plain residual of plane k0 - 1 too
            fetch(k0 - 1, Fo, Fh);
            fetchK(k0 - 1, Ku, Kv, Kw);
            commit(k0 - 1, Fo, Fh, vnext, anext, znext, dnext, mnext, Cc);
            fetch(k0, Fo, Fh);
        } else {
            FusedW<T, FNS> Wo, Wh;
            fetchW(k0 - 1, Wo, Wh);
            fetchK(k0 - 1, Ku, Kv, Kw);
            fetch(k0, Fo, Fh);
            commitW(k0 - 1, Wo, Wh);
        }
        commit(k0, Fo, Fh, vcur, acur, zcur, dcur, mcur, Cc);
        fetch(k0 + 1, Fo, Fh);
        if (fq.ctr && tid == 0) sNext = (int)claim;
        __syncthreads();
        faces(k0 - 1, Ku, Kv, Kw);
        fetchK(k0, Ku, Kv, Kw);
        __syncthreads();

        for (int k = k0; k < kend; ++k) {
            // c of plane k arrives with the raw inputs of plane k + 1
            commit(k + 1, Fo, Fh, vnext, anext, znext, dnext, mnext, Cc);
            if (k + 2 <= kend) fetch(k + 2, Fo, Fh);
            __syncthreads();
            faces(k, Ku, Kv, Kw);
            if (k + 1 < kend) fetchK(k + 1, Ku, Kv, Kw);   // no faces after the last plane
            __syncthreads();
            if (mcur) {
                const int sk = k & 1, sp = (k - 1) & 1, sn = (k + 1) & 1;
                if constexpr (G == 2) {
#pragma unroll
                    for (int q = 0; q < FNS; ++q) {
                        vcur[q] = sOwn[sk][0][q][tid];
                        acur[q] = sOwn[sk][1][q][tid];
                    }
                }
                const T gu0 = gU[sk][ty + 1][tx], gv0 = gV[sk][ty][tx + 1];
                const T gw0 = gW[sk][ty + 1][tx + 1];
                T y[FNS];
                if (G == 1 || grp == 0) {   // p, tau_xx, tau_yy: q = 0, 1, 2
                    const T gu1 = gU[sk][ty + 1][tx + 1], gv1 = gV[sk][ty + 1][tx + 1];
                    const T gw1 = gW[sn][ty + 1][tx + 1];
                    const T c1 = Cc[1], c2 = Cc[2];
                    const T cross = T(0.5) * fmin(c1, c2);
                    y[0] = acur[0] * ((gu0 - gu1) + (gv0 - gv1) + (gw0 - gw1));
                    y[1] = acur[1] * ((gu1 - gu0) + (gw0 - gw1)) + c1 * vcur[1] + cross * vcur[2];
                    y[2] = acur[2] * ((gv1 - gv0) + (gw0 - gw1)) + c2 * vcur[2] + cross * vcur[1];
                }
                if (G == 1 || grp == 1) {   // tau_xy, tau_xz, tau_yz: q = b, b + 1, b + 2
                    constexpr int b = FNS - 3;
                    const T gum = gU[sk][ty][tx], guz = gU[sp][ty + 1][tx];
                    const T gvm = gV[sk][ty][tx], gvz = gV[sp][ty][tx + 1];
                    const T gwx = gW[sk][ty + 1][tx], gwy = gW[sk][ty][tx + 1];
                    y[b] = acur[b] * ((gu0 - gum) + (gv0 - gvm)) + Cc[b] * vcur[b];
                    y[b + 1] = acur[b + 1] * ((gu0 - guz) + (gw0 - gwx)) + Cc[b + 1] * vcur[b + 1];
                    y[b + 2] = acur[b + 2] * ((gv0 - gvz) + (gw0 - gwy)) + Cc[b + 2] * vcur[b + 2];
                }
                const unsigned o = boff3(g, io, jo, k, true);
#pragma unroll
                for (int q = 0; q < FNS; ++q) {
                    const int s = s0 + q;
                    if (!((mcur >> s) & 1u)) continue;
                    if constexpr (G == 2) {
                        zcur[q] = sOwn[sk][2][q][tid];
                        dcur[q] = sOwn[sk][3][q][tid];
                    }
                    st_at(q_out, o + (unsigned)s * NPB, (dcur[q] * acur[q]) * y[q]);   // e q
                    const double yd = y[q];
                    pq_n += (double)vcur[q] * yd;
                    qz_n += (double)zcur[q] * yd;
                    qdq_n += (double)dcur[q] * yd * yd;
                }
            }
            const unsigned xmc = xown ? sXM[k & 1][hlj - 1] : 0u;
            if (xmc) {   // anchor (nx, jh): faces u at li = FTX, v and w at li = FTX - 1
                const int sk = k & 1, sp = (k - 1) & 1;
                const T gu0 = gU[sk][hlj][FTX], gum = gU[sk][hlj - 1][FTX];
                const T guz = gU[sp][hlj][FTX];
                const T gvm = gV[sk][hlj - 1][FTX], gwx = gW[sk][hlj][FTX];
                const T fl[2] = {(gu0 - gum) - gvm, (gu0 - guz) - gwx};
                const unsigned o = boff3(g, ih, jh, k, true);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    if (!((xmc >> (3 + e)) & 1u)) continue;
                    const T* f = sXF[sk][hlj - 1][e];
                    const T yv = f[1] * fl[e] + f[4] * f[0];
                    st_at(q_out, o + (unsigned)(3 + e) * NPB, (f[3] * f[1]) * yv);
                    const double yd = yv;
                    pq_n += (double)f[0] * yd;
                    qz_n += (double)f[2] * yd;
                    qdq_n += (double)f[3] * yd * yd;
                }
            }
            if constexpr (G == 1) {
#pragma unroll
                for (int q = 0; q < FNS; ++q) {
                    vcur[q] = vnext[q];
                    acur[q] = anext[q];
                    zcur[q] = znext[q];
                    dcur[q] = dnext[q];
                }
            }
            mcur = mnext;
        }
        // next item: the fixed stride, or the claimed one after the XCD's two
        // fixed rounds (sNext is rewritten only after the next item's first
        // barrier)
        wtile = (!fq.ctr || first_round) ? wtile + fq.step : fq.t0 + 2 * fq.step + sNext;
    }
    double vv[5] = {rz_n, pq_n, qz_n, qdq_n, rr_n};
    block_partial<5, FNT>(vv, ra.part_out, gridDim.x, blockIdx.x);
}

// x += alpha p; r -= alpha q; z = D^-1 r; r.z, r.r over the active tiles
template <typename T>
__global__ __launch_bounds__(NT) void k_update3d(Geo g, Tiles tl, T* __restrict__ x,
                                                 const T* __restrict__ p, T* __restrict__ r,
                                                 const T* __restrict__ q,
                                                 const T* __restrict__ dinv, T* __restrict__ z,
                                                 RedArgs ra) {
    Scalars* sc = ra.sc;
    if (sc->done) return;
    double tot[1];
    reduce_partials<1, NT>(ra.part_in, ra.nb_in, tot);
    const double pq = tot[0];
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->done = 3;
            sc->iter = ra.kidx;
        }
        return;
    }
    const double alpha_d = sc->rz[ra.kidx & 1] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = alpha_d;
        sc->pqh[ra.kidx & 7] = pq;
    }
    const T alpha = (T)alpha_d;
    const long long NP = g.NP;
    double rz = 0.0, rr = 0.0;
    const TileRange tr = tile_range(tl.items());
  for (int wtile = tr.first; wtile < tr.end; wtile += tr.step) {
        int i0, j0, k0, kend;
        tile_origin(tl, g, wtile, i0, j0, k0, kend);
        const int i = i0 + (threadIdx.x & 63), j = j0 + (threadIdx.x >> 6);
        if (!(i <= g.nx && j <= g.ny)) continue;
        for (int k = k0; k < kend; ++k) {
            const long long o = g.idx(i, j, k);
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const long long t = o + s * NP;
                const T ri = r[t] - alpha * q[t];
                const T zi = dinv[t] * ri;
                x[t] = x[t] + alpha * p[t];
                r[t] = ri;
                if (z) z[t] = zi;
                rz += (double)ri * (double)zi;
                rr += (double)ri * (double)ri;
            }
        }
    }
    double vv[2] = {rz, rr};
    block_partial<2, NT>(vv, ra.part_out, gridDim.x, blockIdx.x);
}

// tile t is active if any sample anchored in it has a != 0
__global__ __launch_bounds__(NT) void k_tile_flags(Geo g, int ntx, int nty, int ntz,
                                                   const double* __restrict__ a,
                                                   int* __restrict__ flags) {
    const int id = blockIdx.x;
    const int tx = id % ntx, ty = (id / ntx) % nty, tz = id / (ntx * nty);
    const int i = tx * TX + (threadIdx.x & 63), j = ty * TY + (threadIdx.x >> 6);
    const int k0 = tz * KZ, kend = min(k0 + KZ, g.nz + 1);
    int any = 0;
    if (i <= g.nx && j <= g.ny)
        for (int k = k0; k < kend; ++k)
            for (int s = 0; s < 6; ++s) any |= a[s * g.NP + g.idx(i, j, k)] != 0.0;
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) flags[id] = any ? 1 : 0;
}

// ordered compaction of the active tile ids (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void k_tile_compact(int n, const int* __restrict__ flags,
                                                       int* __restrict__ list,
                                                       int* __restrict__ count) {
    __shared__ int s_cnt[1024];
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    int c = 0;
    for (int t = lo; t < hi; ++t) c += flags[t];
    s_cnt[threadIdx.x] = c;
    __syncthreads();
    // sequential-in-thread-0 exclusive scan is enough for 1024 entries
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

// a fused work tile (fx, fy, fz) is active if one of the list tiles it
// overlaps is (with the folded column i = nx for the last fused x tile)
__global__ void k_fused_flags(int ntx, int nty, int ntz, int fnx, int fny, int fnz,
                              const int* __restrict__ tflags, int* __restrict__ fflags) {
    constexpr int SY = FTY / TY, SZ = FKZ / KZ;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= fnx * fny * fnz) return;
    const int fx = id % fnx, fy = (id / fnx) % fny, fz = id / (fnx * fny);
    const int tx0 = fx * FTX / TX;
    const int tx1 = fx == fnx - 1 ? ntx - 1 : (fx * FTX + FTX - 1) / TX;
    int any = 0;
    for (int tx = tx0; tx <= tx1; ++tx)
        for (int dz = 0; dz < SZ; ++dz)
            for (int dy = 0; dy < SY; ++dy) {
                const int ty = fy * SY + dy, tz = fz * SZ + dz;
                if (ty < nty && tz < ntz) any |= tflags[tx + ntx * (ty + nty * tz)];
            }
    fflags[id] = any ? 1 : 0;
}

// kRow3X lanes per row (x part t, y, z): bit s (bit 6 + s) of the row's word
// is set if an anchor i <= nx of the first (second) half of RW t .. RW t +
// RW - 1 has a != 0 in sample slice s.
__global__ __launch_bounds__(256) void k_row_bits(Geo g, int ntx, const double* __restrict__ a,
                                                  RowBits* __restrict__ rows, long long nrows) {
    constexpr int RW = kRow3X;
    const long long row = ((long long)blockIdx.x * 256 + threadIdx.x) / RW;
    const int lane = threadIdx.x % RW;
    int bits = 0;
    if (row < nrows) {
        const int t = (int)(row % ntx);
        const long long jk = row / ntx;
        const int j = (int)(jk % (g.ny + 1)), k = (int)(jk / (g.ny + 1));
        const int i = t * RW + lane;
        if (i <= g.nx) {
            const long long o = g.idx(i, j, k);
            for (int s = 0; s < 6; ++s)
                if (a[s * g.NP + o] != 0.0) bits |= 1 << s;
        }
    }
#pragma unroll
    for (int off = RW / 4; off > 0; off >>= 1) bits |= __shfl_xor(bits, off);   // each half
    const int other = __shfl_xor(bits, RW / 2);   // the other half's bits
    if (lane == 0 && row < nrows) rows[row] = (RowBits)(bits | (other << 6));
}

}  // namespace

void tile_dims(const Geo& g, int& ntx, int& nty, int& ntz) {
    ntx = (g.nx + 1 + TX - 1) / TX;
    nty = (g.ny + 1 + TY - 1) / TY;
    ntz = (g.nz + 1 + KZ - 1) / KZ;
}

void launch_tiles(const Geo& g, const double* a, int* flags, int* list, int* count,
                  hipStream_t s) {
    int ntx, nty, ntz;
    tile_dims(g, ntx, nty, ntz);
    const int n = ntx * nty * ntz;
    hipLaunchKernelGGL(k_tile_flags, dim3(n), dim3(NT), 0, s, g, ntx, nty, ntz, a, flags);
    hipLaunchKernelGGL(k_tile_compact, dim3(1), dim3(1024), 0, s, n, flags, list, count);
}

void fused_tile_dims(const Geo& g, int& ntx, int& nty, int& ntz) {
    ntx = (g.nx + 1 + FTX - 1) / FTX - (fused_fold(g.nx) ? 1 : 0);
    nty = (g.ny + 1 + FTY - 1) / FTY;
    ntz = (g.nz + 1 + FKZ - 1) / FKZ;
}

void launch_fused_tiles(const Geo& g, const int* tile_flags, int* flags, int* list, int* count,
                        hipStream_t s) {
    int ntx, nty, ntz, fx, fy, fz;
    tile_dims(g, ntx, nty, ntz);
    fused_tile_dims(g, fx, fy, fz);
    const int n = fx * fy * fz;
    hipLaunchKernelGGL(k_fused_flags, dim3((n + 255) / 256), dim3(256), 0, s, ntx, nty, ntz, fx,
                       fy, fz, tile_flags, flags);
    hipLaunchKernelGGL(k_tile_compact, dim3(1), dim3(1024), 0, s, n, flags, list, count);
}

long long row_bytes(const Geo& g) {
    const int rntx = (g.nx + kRow3X) / kRow3X;
    return (long long)rntx * (g.ny + 1) * (g.nz + 1);
}

void launch_row_bits(const Geo& g, const double* a, RowBits* rows, hipStream_t s) {
    const int rntx = (g.nx + kRow3X) / kRow3X;
    const long long n = row_bytes(g);
    const long long per = 256 / kRow3X;   // rows per workgroup
    hipLaunchKernelGGL(k_row_bits, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0, s, g, rntx,
                       a, rows, n);
}

// Workgroups of a 3D apply launch: no more than can be resident at once
// (occupancy x compute units, queried once per device and precision), so no
// tail wave runs after the first, and at most kMaxTileBlocks.  The pipelined
// Jacobi direction kernel holds more registers than the generic kernel and
// gets its own figure (dir3d_grid); a consumer of an apply's partials uses
// the figure of the kernel that produced them.
static int resident_grid(int count, int word, bool pipelined) {
    static int cache[2][2][16] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int& c = cache[pipelined ? 1 : 0][word == 8 ? 1 : 0][dev & 15];
    if (c == 0) {
        int nb = 0, ncu = 0;
        hipError_t e;
        if (pipelined)
            e = word == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dir3d_pipe<double>, NT, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dir3d_pipe<float>, NT, 0);
        else
            e = word == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &nb, k_apply3d<double, MODE_DIR, true>, NT, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &nb, k_apply3d<float, MODE_DIR, true>, NT, 0);
        if (e != hipSuccess || nb < 1) nb = 1;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            ncu < 1)
            ncu = 1;
        c = nb * ncu;
    }
    return std::max(1, std::min(std::min(count, kMaxTileBlocks), c));
}

int tile3d_anchors() { return TX * TY * KZ; }

// Plane split of a tile list of `count` tiles: the largest power of two (at
// most KZ) whose work items all fit in one round of `capacity` resident
// workgroups (the grid of the solve's main kernel), so that no workgroup
// runs a second item after the others are done.  Measured on a 128^3 column
// (92 active tiles): split 8 (736 items) took 26.5 / 46.6 us per mixed / FP64
// iteration, the fitting splits 4 (mixed, 512 resident) and 2 (FP64, 256
// resident) 23.7 / 40.1 us.
int tile_split(int count, int capacity) {
    int split = 1;
    while (split < KZ && (long long)count * split * 2 <= capacity) split *= 2;
    return split;
}

// the same rule for the fused work tiles (at most FKZ parts)
int fused_split(int count, int capacity) {
    int split = 1;
    while (split < FKZ && (long long)count * split * 2 <= capacity) split *= 2;
    return split;
}

// The update is elementwise, with no halo and no plane-to-plane dependence:
// a short tile list gives it one plane per work item (split KZ), as long as
// that does not exceed the grid cap, whatever split the applies use.
Tiles update3d_tiles(const Tiles& tl) {
    Tiles tu = tl;
    while (tu.split < KZ && (long long)tl.count * tu.split * 2 <= kMaxTileBlocks) tu.split *= 2;
    return tu;
}

int apply3d_grid(int count, int word) { return resident_grid(count, word, false); }

int dir3d_grid(int count, int word) { return resident_grid(count, word, true); }

// Workgroups of the fused 3D iteration (FP32): its occupancy x compute units.
int fused3d_grid(int count) {
    static int cache[16] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int& c = cache[dev & 15];
    if (c == 0) {
        // the smaller residency of the two shapes (both hold two workgroups per CU)
        int nb = 0, nb1 = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused3d<float, false, 2>,
                                                         2 * FNA, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb1, k_fused3d<float, false, 1>, FNA,
                                                         0) != hipSuccess)
            nb = nb1 = 1;
        nb = std::max(1, std::min(nb, nb1));
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            ncu < 1)
            ncu = 1;
        c = nb * ncu;
    }
    return std::max(1, std::min(std::min(count, kMaxTileBlocks), c));
}

void launch_fused3d(const Geo& g, const Tiles& ft, bool init, const FusedVecs& v,
                    const float* ead, const float* a, const float* c, const float* K,
                    const RowBits* rows, unsigned* wq, const RedArgs& ra, hipStream_t s) {
    if (ft.count <= 0) return;
    const dim3 gs(fused3d_grid(ft.items()));
    if (ft.split >= VFS_FUSED3_PAIR_SPLIT) {
        if (init)
            hipLaunchKernelGGL((k_fused3d<float, true, 2>), gs, dim3(2 * FNA), 0, s, g, ft, v,
                               ead, a, c, K, rows, wq, ra);
        else
            hipLaunchKernelGGL((k_fused3d<float, false, 2>), gs, dim3(2 * FNA), 0, s, g, ft, v,
                               ead, a, c, K, rows, wq, ra);
    } else {
        if (init)
            hipLaunchKernelGGL((k_fused3d<float, true, 1>), gs, dim3(FNA), 0, s, g, ft, v, ead,
                               a, c, K, rows, wq, ra);
        else
            hipLaunchKernelGGL((k_fused3d<float, false, 1>), gs, dim3(FNA), 0, s, g, ft, v, ead,
                               a, c, K, rows, wq, ra);
    }
}

template <typename T>
void launch_apply3d(const Geo& g, const Tiles& tl, int mode, bool zin, const T* r, const T* zsrc,
                    const T* dinv, const T* pin, T* pout, T* q, const T* a, const T* c,
                    const T* K, const T* bvec, const RedArgs& ra, hipStream_t s) {
    if (tl.count <= 0) return;
    const dim3 gs(apply3d_grid(tl.items(), (int)sizeof(T)));
    if (mode == MODE_DIR) {
        if (zin)
            hipLaunchKernelGGL((k_apply3d<T, MODE_DIR, true>), gs, dim3(NT), 0, s, g, tl, r, zsrc,
                               dinv, pin, pout, q, a, c, K, bvec, ra);
        else
            hipLaunchKernelGGL((k_dir3d_pipe<T>), dim3(dir3d_grid(tl.items(), (int)sizeof(T))),
                               dim3(NT), 0, s, g, tl, r, dinv, pin, pout, q, a, c, K, ra);
    } else if (mode == MODE_FDIR) {
        hipLaunchKernelGGL((k_apply3d<T, MODE_FDIR, false>), gs, dim3(NT), 0, s, g, tl, r, zsrc,
                           dinv, pin, pout, q, a, c, K, bvec, ra);
    } else if (mode == MODE_JDIR) {
        if (zin)
            hipLaunchKernelGGL((k_apply3d<T, MODE_JDIR, true>), gs, dim3(NT), 0, s, g, tl, r, zsrc,
                               dinv, pin, pout, q, a, c, K, bvec, ra);
        else
            hipLaunchKernelGGL((k_apply3d<T, MODE_JDIR, false>), gs, dim3(NT), 0, s, g, tl, r,
                               zsrc, dinv, pin, pout, q, a, c, K, bvec, ra);
    } else if (mode == MODE_APPLY) {
        hipLaunchKernelGGL((k_apply3d<T, MODE_APPLY, false>), gs, dim3(NT), 0, s, g, tl, r, zsrc,
                           dinv, pin, pout, q, a, c, K, bvec, ra);
    } else {
        hipLaunchKernelGGL((k_apply3d<T, MODE_RESID, false>), gs, dim3(NT), 0, s, g, tl, r, zsrc,
                           dinv, pin, pout, q, a, c, K, bvec, ra);
    }
}

template <typename T>
void launch_update3d(const Geo& g, const Tiles& tl, T* x, const T* p, T* r, const T* q,
                     const T* dinv, T* z, const RedArgs& ra, hipStream_t s) {
    if (tl.count <= 0) return;
    const Tiles tu = update3d_tiles(tl);
    hipLaunchKernelGGL((k_update3d<T>), dim3(std::min(tu.items(), kMaxTileBlocks)), dim3(NT), 0, s,
                       g, tu, x, p, r, q, dinv, z, ra);
}

#define VFS_INST3(T)                                                                           \
    template void launch_apply3d<T>(const Geo&, const Tiles&, int, bool, const T*, const T*,   \
                                    const T*, const T*, T*, T*, const T*, const T*, const T*,   \
                                    const T*, const RedArgs&, hipStream_t);                    \
    template void launch_update3d<T>(const Geo&, const Tiles&, T*, const T*, T*, const T*,      \
                                     const T*, T*, const RedArgs&, hipStream_t);
VFS_INST3(double)
VFS_INST3(float)

}  // namespace vfs
