// HIP kernels of the FEWHA hot path for gfx950 (CDNA4, wave64).
//
// Every stage is bandwidth/latency bound (no dense contraction anywhere), so the kernels are
// gather-only stencils: each output element is written by exactly one lane, nothing uses
// atomics except the last-block-done counter of the reductions, and results are bitwise
// reproducible run to run.
//
//   k_idwt         W^T (= W^-1) of every layer, all J levels in one launch: each workgroup owns a
//                  square output tile and rebuilds, level by level from the coarsest, only the
//                  cone of approximation coefficients that tile depends on (LDS resident);
//                  optionally scales coefficients by the Jacobi preconditioner on load (z = J^-1 r).
//   k_nodes        per WFS node tile: P (bilinear ray gather from all layers through per-axis
//                  cell tables, LGS cone included), Gamma, C_eta^-1 and Gamma^T fused through LDS
//                  (the paper's Kernel-2 stage), or Gamma^T C s / Gamma^T mask s.
//   k_slopes       mask Gamma P u on subaperture tiles (forward operator A).
//   k_pt           P^T as a gather per layer node over the contiguous ranges of sensor nodes whose
//                  cells touch it, with the very table entries the forward uses: the exact
//                  transpose of P without atomics.
//   k_fdwt_fine    the first kf levels of the forward transform W for every layer, on tiles of
//                  level-kf quads with their halo staged in LDS; fused epilogues (alpha D z and the
//                  PCG dot products, or the right-hand side's warm-restart residual update).
//   k_fdwt_coarse  the remaining levels, one workgroup per layer, LDS resident; same epilogues; its
//                  last workgroup forms the Alg. 2 scalars on the device.
//   k_update       fused p, q, c, r update of Alg. 2.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace fewha {

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------------------------
// Geometry helpers
// ---------------------------------------------------------------------------------------------
struct Cell {
    int k0;      // lower grid index
    double t;    // fractional position in [0, 1]
};

__device__ __forceinline__ Cell cell_of(double u, int n) {
    int k = (int)floor(u);
    if (k > n - 2) k = n - 2;
    return {k, u - (double)k};
}

// Grid coordinate on layer L of node index j of a sensor along one axis (h = theta h_l there).
__device__ __forceinline__ double ray_coord(const DevProj &pr, const DevWfs &W, const DevLayer &L, int j, double h) {
    double X = pr.sig * (W.x0 + (double)j * W.d) + h;
    return X / L.spacing + L.half;
}

__device__ __forceinline__ bool subap_active(const DevWfs &W, int i, int j) {
    double xc = ((double)j + 0.5) * W.d + W.x0, yc = ((double)i + 0.5) * W.d + W.x0;
    double r2 = xc * xc + yc * yc;
    return r2 <= W.r_out2 && r2 >= W.r_in2;
}

// phi_g(i, j) = sum_l bilinear(u_l at the ray point)  (P of Sec. 2.1), via the cell tables.
template <typename T>
__device__ __forceinline__ T project_node(const T *__restrict__ u, const Bufs<T> &B, int g, int nl, int i, int j) {
    T acc = 0;
    const Ent<T> *xt = B.xtab + (long)g * nl * B.maxnv;
    const Ent<T> *yt = B.ytab + (long)g * nl * B.maxnv;
    for (int l = 0; l < nl; ++l) {
        const Ent<T> ex = xt[l * B.maxnv + j], ey = yt[l * B.maxnv + i];
        const int n = B.lay[l].n;
        const T *U = u + B.lay[l].c_off + (long)ey.k0 * n + ex.k0;
        acc += (ey.w0 * ex.w0) * U[0] + (ey.w0 * ex.w1) * U[1] + (ey.w1 * ex.w0) * U[n] + (ey.w1 * ex.w1) * U[n + 1];
    }
    return acc;
}

// ---------------------------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block in fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Publish this block's partials at slot `slot` of each of `nrows` rows (row pitch `pitch`);
// return true in the one block of the grid that finishes last, when every earlier write of
// this and of previous kernels on the stream is visible.  The counter returns to zero.
__device__ __forceinline__ bool publish_last(double *partials, int pitch, int nrows, int slot, const double *vals,
                                             unsigned *counter) {
    __shared__ bool last;
    if (threadIdx.x == 0) {
        for (int k = 0; k < nrows; ++k)
            __hip_atomic_store(partials + (size_t)k * pitch + slot, vals[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        unsigned prev = atomicAdd(counter, 1u);
        last = (prev == gridDim.x - 1);
        if (last) {
            __threadfence();
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    return last;
}

// Sum slots [0, count) of one partial row in fixed order, cooperatively by one block.
__device__ __forceinline__ double gather_partials(const double *partials, int pitch, int row, int count, double *sh) {
    double v = 0.0;
    for (int b = threadIdx.x; b < count; b += blockDim.x)
        v += __hip_atomic_load(partials + (size_t)row * pitch + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum(v, sh);
}

// Alg. 2 scalars from the reduced (rho, mu) of pass k (thread 0 of the last block only).
__device__ void pcg_scalars(Scalars *sc, double R, double Mu, int k, double *resnorm) {
    sc->rho = R;
    sc->mu = Mu;
    if (sc->stopped) return;
    if (!isfinite(R) || !isfinite(Mu)) {
        sc->status = FEWHA_ERR_NONFINITE;
        sc->stopped = 1;
        return;
    }
    if (resnorm) resnorm[k] = sqrt(R);
    if (R == 0.0) {
        sc->stopped = 1;
        return;
    }
    double beta = 0.0, den = Mu;
    if (k > 0) {
        beta = R / sc->rho_old;
        den = Mu - R * beta / sc->alpha_old;
    }
    if (!(den > 0.0)) {
        sc->status = FEWHA_ERR_BREAKDOWN;
        sc->stopped = 1;
        return;
    }
    const double alpha = R / den;
    sc->alpha = alpha;
    sc->beta = beta;
    sc->rho_old = R;
    sc->alpha_old = alpha;
}

__device__ __forceinline__ void reset_scalars(Scalars *sc) {
    sc->rho = sc->mu = sc->rho_old = sc->alpha = sc->alpha_old = sc->beta = 0.0;
    sc->stopped = 0;
    sc->status = FEWHA_OK;
}

// Level and orientation of Mallat position (row, col) of an n x n pyramid with J levels.
__device__ __forceinline__ void band_at(int row, int col, int n, int log2n, int J, int &s, int &o) {
    const int v = row > col ? row : col;
    if (v < (n >> J)) {
        s = J;
        o = 0;
    } else {
        const int lv = 31 - __clz(v);
        const int m = 1 << lv;
        s = log2n - lv;
        o = (row < m) ? 1 : ((col < m) ? 2 : 3);
    }
}

// ---------------------------------------------------------------------------------------------
// W^T: multi-level inverse DWT, one launch, cone recomputation per output tile.
// ---------------------------------------------------------------------------------------------
template <typename T, bool SCALE>
__global__ __launch_bounds__(kBlock) void k_idwt(const T *__restrict__ c, T *__restrict__ out,
                                                 const Tile *__restrict__ tiles, const DevLayer *__restrict__ lays,
                                                 int J, const T *__restrict__ jinv, Taps<T> tp) {
    constexpr int TILE = kIdwtTile;
    constexpr int R = TILE / 2 + 2;  // longest coefficient run any level needs
    __shared__ T sA[R * R], sB[R * R], sHL[R * R], sLH[R * R], sHH[R * R];
    __shared__ T sAX[TILE * R], sDX[TILE * R];

    const Tile t = tiles[blockIdx.x];
    const DevLayer L = lays[t.a];
    const int n = L.n, T0 = t.d;
    const T *cl = c + L.c_off;

    // cone bounds per level (unwrapped indices; periodic wrap happens only on loads)
    __shared__ int loY[kMaxJ + 1], loX[kMaxJ + 1], lnY[kMaxJ + 1], lnX[kMaxJ + 1];
    if (threadIdx.x == 0) {
        int ly = t.b, hy = t.b + T0 - 1, lx = t.c, hx = t.c + T0 - 1;
        loY[0] = ly;
        loX[0] = lx;
        lnY[0] = T0;
        lnX[0] = T0;
        for (int s = 1; s <= J; ++s) {
            ly = (ly >> 1) - 2;
            hy >>= 1;
            lx = (lx >> 1) - 2;
            hx >>= 1;
            loY[s] = ly;
            loX[s] = lx;
            lnY[s] = hy - ly + 1;
            lnX[s] = hx - lx + 1;
        }
    }
    __syncthreads();
    auto scale = [&](int s, int o) -> T {
        if constexpr (SCALE) return jinv[(t.a * (J + 1) + s) * 4 + o];
        else return (T)1;
    };

    // coarsest level: LL and the three detail bands of the cone region
    {
        const int m = n >> J, msk = m - 1, ny = lnY[J], nx = lnX[J];
        const T s0 = scale(J, 0), s1 = scale(J, 1), s2 = scale(J, 2), s3 = scale(J, 3);
        for (int idx = threadIdx.x; idx < ny * nx; idx += blockDim.x) {
            int r = idx / nx, q = idx - r * nx;
            int gr = (loY[J] + r) & msk, gc = (loX[J] + q) & msk;
            sA[r * R + q] = cl[(long)gr * n + gc] * s0;
            sHL[r * R + q] = cl[(long)gr * n + m + gc] * s1;
            sLH[r * R + q] = cl[(long)(m + gr) * n + gc] * s2;
            sHH[r * R + q] = cl[(long)(m + gr) * n + m + gc] * s3;
        }
    }
    __syncthreads();

    T *LL = sA, *NX = sB;
    for (int s = J; s >= 1; --s) {
        const int ny = lnY[s - 1], nxk = lnX[s], nx = lnX[s - 1];
        const int oy = loY[s - 1], ky = loY[s], ox = loX[s - 1], kx = loX[s];
        // undo the y analysis: (LL, x-low/y-high) -> x-low rows, (x-high/y-low, HH) -> x-high rows
        for (int idx = threadIdx.x; idx < ny * nxk; idx += blockDim.x) {
            int r = idx / nxk, q = idx - r * nxk;
            int y = oy + r, p = y & 1, kb = (y >> 1) - ky;
            T a = 0, d = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int at = (kb - j) * R + q;
                a += tp.h[p + 2 * j] * LL[at] + tp.g[p + 2 * j] * sLH[at];
                d += tp.h[p + 2 * j] * sHL[at] + tp.g[p + 2 * j] * sHH[at];
            }
            sAX[r * R + q] = a;
            sDX[r * R + q] = d;
        }
        __syncthreads();
        // undo the x analysis
        for (int idx = threadIdx.x; idx < ny * nx; idx += blockDim.x) {
            int r = idx / nx, q = idx - r * nx;
            int x = ox + q, p = x & 1, kb = (x >> 1) - kx;
            T v = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int at = r * R + kb - j;
                v += tp.h[p + 2 * j] * sAX[at] + tp.g[p + 2 * j] * sDX[at];
            }
            if (s > 1) NX[r * R + q] = v;
            else out[L.c_off + (long)(oy + r) * n + ox + q] = v;
        }
        if (s > 1) {
            // detail bands of level s-1 over the region just synthesised
            const int m = n >> (s - 1), msk = m - 1;
            const T s1 = scale(s - 1, 1), s2 = scale(s - 1, 2), s3 = scale(s - 1, 3);
            for (int idx = threadIdx.x; idx < ny * nx; idx += blockDim.x) {
                int r = idx / nx, q = idx - r * nx;
                int gr = (oy + r) & msk, gc = (ox + q) & msk;
                sHL[r * R + q] = cl[(long)gr * n + m + gc] * s1;
                sLH[r * R + q] = cl[(long)(m + gr) * n + gc] * s2;
                sHH[r * R + q] = cl[(long)(m + gr) * n + m + gc] * s3;
            }
            T *tmp = LL;
            LL = NX;
            NX = tmp;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Node-tile kernels (Kernel-2 stage): P, Gamma, C_eta^-1, Gamma^T.
// ---------------------------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_nodes(const T *__restrict__ in, T *__restrict__ v, Bufs<T> B, int nl) {
    constexpr int NT = kNodeTile, NP = NT + 2, NS = NT + 1;
    __shared__ T sPhi[NP * NP];
    __shared__ T sSx[NS * NS], sSy[NS * NS];
    const Tile t = B.node_tiles[blockIdx.x];
    const DevWfs W = B.wfs[t.a];
    const int ns = W.n_sub, nv = W.nv, i0 = t.b, j0 = t.c;

    if constexpr (MODE == kModeM) {
        for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
            int a = idx / NP, b = idx - a * NP, i = i0 - 1 + a, j = j0 - 1 + b;
            T val = 0;
            if (i >= 0 && i <= ns && j >= 0 && j <= ns) val = project_node(in, B, t.a, nl, i, j);
            sPhi[idx] = val;
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < NS * NS; idx += blockDim.x) {
        int a = idx / NS, b = idx - a * NS, i = i0 - 1 + a, j = j0 - 1 + b;
        T sx = 0, sy = 0;
        if (i >= 0 && i < ns && j >= 0 && j < ns && subap_active(W, i, j)) {
            const T w = (MODE == kModeAdj) ? (T)1 : (T)W.inv_var;
            if constexpr (MODE == kModeM) {
                const T p00 = sPhi[a * NP + b], p01 = sPhi[a * NP + b + 1];
                const T p10 = sPhi[(a + 1) * NP + b], p11 = sPhi[(a + 1) * NP + b + 1];
                sx = w * ((T)0.5 * ((p01 - p00) + (p11 - p10)));
                sy = w * ((T)0.5 * ((p10 - p00) + (p11 - p01)));
            } else {
                sx = w * in[W.s_off + (long)i * ns + j];
                sy = w * in[W.s_off + (long)ns * ns + (long)i * ns + j];
            }
        }
        sSx[idx] = sx;
        sSy[idx] = sy;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NT * NT; idx += blockDim.x) {
        int a = idx / NT, b = idx - a * NT, i = i0 + a, j = j0 + b;
        if (i > ns || j > ns) continue;
        // node (i, j) is a corner of subapertures (i, j), (i, j-1), (i-1, j), (i-1, j-1)
        const int s11 = (a + 1) * NS + (b + 1), s10 = (a + 1) * NS + b, s01 = a * NS + (b + 1), s00 = a * NS + b;
        T val = (T)0.5 * ((-sSx[s11] - sSy[s11]) + (sSx[s10] - sSy[s10]) + (-sSx[s01] + sSy[s01]) + (sSx[s00] + sSy[s00]));
        v[W.v_off + (long)i * nv + j] = val;
    }
}

// s = mask Gamma P u on subaperture tiles.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_slopes(const T *__restrict__ u, T *__restrict__ s, Bufs<T> B, int nl) {
    constexpr int NT = kNodeTile, NP = NT + 1;
    __shared__ T sPhi[NP * NP];
    const Tile t = B.sub_tiles[blockIdx.x];
    const DevWfs W = B.wfs[t.a];
    const int ns = W.n_sub, i0 = t.b, j0 = t.c;
    for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
        int a = idx / NP, b = idx - a * NP, i = i0 + a, j = j0 + b;
        T val = 0;
        if (i <= ns && j <= ns) val = project_node(u, B, t.a, nl, i, j);
        sPhi[idx] = val;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NT * NT; idx += blockDim.x) {
        int a = idx / NT, b = idx - a * NT, i = i0 + a, j = j0 + b;
        if (i >= ns || j >= ns) continue;
        T sx = 0, sy = 0;
        if (subap_active(W, i, j)) {
            const T p00 = sPhi[a * NP + b], p01 = sPhi[a * NP + b + 1];
            const T p10 = sPhi[(a + 1) * NP + b], p11 = sPhi[(a + 1) * NP + b + 1];
            sx = (T)0.5 * ((p01 - p00) + (p11 - p10));
            sy = (T)0.5 * ((p10 - p00) + (p11 - p01));
        }
        s[W.s_off + (long)i * ns + j] = sx;
        s[W.s_off + (long)ns * ns + (long)i * ns + j] = sy;
    }
}

// ---------------------------------------------------------------------------------------------
// P^T as a gather over layer-node tiles, through the transpose ranges of the cell tables.
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pt(const T *__restrict__ v, T *__restrict__ x, Bufs<T> B, int nl,
                                               int nw) {
    constexpr int NT = kNodeTile;
    const Tile t = B.lay_tiles[blockIdx.x];
    const DevLayer L = B.lay[t.a];
    const int k = t.b + (int)(threadIdx.x / NT), q = t.c + (int)(threadIdx.x % NT);
    if (k >= L.n || q >= L.n) return;
    T acc = 0;
    for (int g = 0; g < nw; ++g) {
        const Range rx = B.xrng[(long)g * B.sum_n + L.r_off + q];
        const Range ry = B.yrng[(long)g * B.sum_n + L.r_off + k];
        if (rx.lo > rx.hi || ry.lo > ry.hi) continue;
        const Ent<T> *xt = B.xtab + ((long)g * nl + t.a) * B.maxnv;
        const Ent<T> *yt = B.ytab + ((long)g * nl + t.a) * B.maxnv;
        const DevWfs W = B.wfs[g];
        const T *vg = v + W.v_off;
        for (int i = ry.lo; i <= ry.hi; ++i) {
            const Ent<T> ey = yt[i];
            const T wy = (ey.k0 == k) ? ey.w0 : ey.w1;
            const T *row = vg + (long)i * W.nv;
            for (int j = rx.lo; j <= rx.hi; ++j) {
                const Ent<T> ex = xt[j];
                const T wx = (ex.k0 == q) ? ex.w0 : ex.w1;
                acc += (wy * wx) * row[j];
            }
        }
    }
    x[L.c_off + (long)k * L.n + q] = acc;
}

// ---------------------------------------------------------------------------------------------
// Forward transform W with fused epilogues.
// ---------------------------------------------------------------------------------------------
struct EpiArgs {
    const void *cin;   // kEpiPrior: c of y = W x + alpha D c
    void *out;         // destination coefficient vector (y, or b for kEpiRhs)
    void *c;           // kEpiRhs + cold: caller's c, zeroed
    int cold;          // kEpiRhs
    int k;             // kEpiPcg: pass index
    double *resnorm;   // kEpiPcg
    int nfine;         // partial slots used by the tiled kernel
};

// Deliver one coefficient of W x to its destination; accumulate the PCG dot partials.
template <typename T, int EPI>
__device__ __forceinline__ void epilogue(const Bufs<T> &B, const EpiArgs &E, long i, int l, int s, int o, int J, T w,
                                         double &rho, double &mu) {
    T *out = static_cast<T *>(E.out);
    if constexpr (EPI == kEpiPlain) {
        out[i] = w;
    } else if constexpr (EPI == kEpiPrior) {
        out[i] = w + B.ad[l * (J + 1) + s] * static_cast<const T *>(E.cin)[i];
    } else if constexpr (EPI == kEpiPcg) {
        const T ri = B.r[i];
        const T z = ri * B.jinv[(l * (J + 1) + s) * 4 + o];
        const T yi = w + B.ad[l * (J + 1) + s] * z;
        out[i] = yi;
        rho += (double)ri * (double)z;
        mu += (double)yi * (double)z;
    } else {  // kEpiRhs: b = W x; r = (b - b_prev) + r (cold: r = b, c = 0); b_prev = b
        out[i] = w;
        if (E.cold) {
            B.r[i] = w;
            static_cast<T *>(E.c)[i] = 0;
        } else {
            B.r[i] = (w - B.b_prev[i]) + B.r[i];
        }
        B.b_prev[i] = w;
    }
}

// Region geometry of the tiled forward DWT: a tile of TQ x TQ level-KF approximation
// coefficients needs LL_{s} on a run of len(s) = TQ 2^(KF-s) + 4 (2^(KF-s) - 1) indices.
template <int KF, int TQ>
struct FineGeom {
    static constexpr int len(int s) { return TQ * (1 << (KF - s)) + 4 * ((1 << (KF - s)) - 1); }
};

template <typename T, int KF, int TQ, int EPI>
__global__ __launch_bounds__(kBlock) void k_fdwt_fine(const T *__restrict__ x, T *__restrict__ ll_out, Bufs<T> B,
                                                      int J, EpiArgs E, Taps<T> tp, int last) {
    using G = FineGeom<KF, TQ>;
    constexpr int L0 = G::len(0), L1 = G::len(1);
    __shared__ T sA[L0 * L0];
    __shared__ T sB[(KF >= 2 ? L1 * L1 : 1)];
    __shared__ double sh[kBlock / 64];
    if constexpr (EPI == kEpiRhs) {
        if (blockIdx.x == 0 && threadIdx.x == 0) reset_scalars(B.sc);
    }

    const Tile t = B.fine_tiles[blockIdx.x];
    const DevLayer L = B.lay[t.a];
    const int n = L.n, tq = t.d, shift = KF;
    // run lengths and origins for this tile (tq <= TQ; small layers use smaller tiles)
    int len[KF + 1];
#pragma unroll
    for (int s = 0; s <= KF; ++s) len[s] = tq * (1 << (KF - s)) + 4 * ((1 << (KF - s)) - 1);
    const int oy = t.b << shift, ox = t.c << shift, nmask = n - 1;

    // stage the input region (periodic wrap) in LDS
    for (int idx = threadIdx.x; idx < len[0] * len[0]; idx += blockDim.x) {
        const int r = idx / len[0], q = idx - r * len[0];
        sA[r * L0 + q] = x[L.c_off + (long)((oy + r) & nmask) * n + ((ox + q) & nmask)];
    }
    __syncthreads();

    double rho = 0.0, mu = 0.0;
#pragma unroll
    for (int s = 1; s <= KF; ++s) {
        const T *src = (s & 1) ? sA : sB;
        T *dst = (s & 1) ? sB : sA;
        const int sp = (s & 1) ? L0 : L1, dp = (s & 1) ? L1 : L0;
        const int ln = len[s], own = tq << (KF - s), m = n >> s;  // output run, owned run, band size
        const int by = t.b << (KF - s), bx = t.c << (KF - s);      // owned origin at level s
        for (int idx = threadIdx.x; idx < ln * ln; idx += blockDim.x) {
            const int r = idx / ln, q = idx - r * ln;
            T ll = 0, lh = 0, hl = 0, hh = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                const T *row = src + (2 * r + a) * sp + 2 * q;
                T ax = 0, dx = 0;
#pragma unroll
                for (int b = 0; b < 6; ++b) {
                    ax += tp.h[b] * row[b];
                    dx += tp.g[b] * row[b];
                }
                ll += tp.h[a] * ax;
                lh += tp.g[a] * ax;
                hl += tp.h[a] * dx;
                hh += tp.g[a] * dx;
            }
            if (s < KF) dst[r * dp + q] = ll;
            if (r < own && q < own) {
                const int gr = by + r, gc = bx + q;
                const long base = L.c_off;
                epilogue<T, EPI>(B, E, base + (long)gr * n + m + gc, t.a, s, 1, J, hl, rho, mu);
                epilogue<T, EPI>(B, E, base + (long)(m + gr) * n + gc, t.a, s, 2, J, lh, rho, mu);
                epilogue<T, EPI>(B, E, base + (long)(m + gr) * n + m + gc, t.a, s, 3, J, hh, rho, mu);
                if (s == KF) {
                    if (KF == J) epilogue<T, EPI>(B, E, base + (long)gr * n + gc, t.a, s, 0, J, ll, rho, mu);
                    else ll_out[(L.c_off >> (2 * KF)) + (long)gr * m + gc] = ll;
                }
            }
        }
        __syncthreads();
    }
    if constexpr (EPI == kEpiPcg) {
        double vals[2];
        vals[0] = block_sum(rho, sh);
        vals[1] = block_sum(mu, sh);
        const int pitch = kPartialPitch;
        const bool am_last = publish_last(B.partials, pitch, 2, blockIdx.x, vals, &B.sc->counter);
        if (!last || !am_last) return;
        const double R = gather_partials(B.partials, pitch, 0, gridDim.x, sh);
        const double Mu = gather_partials(B.partials, pitch, 1, gridDim.x, sh);
        if (threadIdx.x == 0) pcg_scalars(B.sc, R, Mu, E.k, E.resnorm);
    }
}

// Levels KF+1..J of one layer per workgroup; the level-KF approximation comes from ll_in.
template <typename T, int EPI>
__global__ __launch_bounds__(kBlock) void k_fdwt_coarse(const T *__restrict__ ll_in, Bufs<T> B, int J, int KF,
                                                        EpiArgs E, Taps<T> tp) {
    extern __shared__ char smem_raw[];
    T *sA = reinterpret_cast<T *>(smem_raw);
    __shared__ double sh[kBlock / 64];
    const int l = blockIdx.x;
    const DevLayer L = B.lay[l];
    const int n = L.n, m0 = n >> KF;
    T *sB = sA + m0 * m0;
    for (int idx = threadIdx.x; idx < m0 * m0; idx += blockDim.x) sA[idx] = ll_in[(L.c_off >> (2 * KF)) + idx];
    __syncthreads();
    double rho = 0.0, mu = 0.0;
    T *src = sA, *dst = sB;
    for (int s = KF + 1; s <= J; ++s) {
        const int mi = n >> (s - 1), h = mi >> 1, msk = mi - 1;
        for (int idx = threadIdx.x; idx < h * h; idx += blockDim.x) {
            const int r = idx / h, q = idx - r * h;
            int cols[6];
#pragma unroll
            for (int b = 0; b < 6; ++b) cols[b] = (2 * q + b) & msk;
            T ll = 0, lh = 0, hl = 0, hh = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                const T *row = src + ((2 * r + a) & msk) * mi;
                T ax = 0, dx = 0;
#pragma unroll
                for (int b = 0; b < 6; ++b) {
                    const T xv = row[cols[b]];
                    ax += tp.h[b] * xv;
                    dx += tp.g[b] * xv;
                }
                ll += tp.h[a] * ax;
                lh += tp.g[a] * ax;
                hl += tp.h[a] * dx;
                hh += tp.g[a] * dx;
            }
            const long base = L.c_off;
            epilogue<T, EPI>(B, E, base + (long)r * n + h + q, l, s, 1, J, hl, rho, mu);
            epilogue<T, EPI>(B, E, base + (long)(h + r) * n + q, l, s, 2, J, lh, rho, mu);
            epilogue<T, EPI>(B, E, base + (long)(h + r) * n + h + q, l, s, 3, J, hh, rho, mu);
            if (s == J) epilogue<T, EPI>(B, E, base + (long)r * n + q, l, s, 0, J, ll, rho, mu);
            else dst[r * h + q] = ll;
        }
        __syncthreads();
        // the next level reads what was just written; the old input becomes the next output
        T *tmp = src;
        src = dst;
        dst = tmp;
    }
    if constexpr (EPI == kEpiPcg) {
        double vals[2];
        vals[0] = block_sum(rho, sh);
        vals[1] = block_sum(mu, sh);
        const int pitch = kPartialPitch;
        if (!publish_last(B.partials, pitch, 2, E.nfine + blockIdx.x, vals, &B.sc->counter)) return;
        const double R = gather_partials(B.partials, pitch, 0, E.nfine + gridDim.x, sh);
        const double Mu = gather_partials(B.partials, pitch, 1, E.nfine + gridDim.x, sh);
        if (threadIdx.x == 0) pcg_scalars(B.sc, R, Mu, E.k, E.resnorm);
    }
}

// ---------------------------------------------------------------------------------------------
// Element-wise PCG update on coefficient tiles (layer known per tile, band from the index).
// ---------------------------------------------------------------------------------------------
// p = z + beta p; q = y + beta q; c += alpha p; r -= alpha q   (first pass: p = z, q = y)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(T *__restrict__ c, Bufs<T> B, int J, int k) {
    if (B.sc->stopped) return;
    const T alpha = (T)B.sc->alpha, beta = (T)B.sc->beta;
    const Tile t = B.coef_tiles[blockIdx.x];
    const DevLayer L = B.lay[t.a];
#pragma unroll
    for (int e = 0; e < kCoefTile / kBlock; ++e) {
        const int loc = t.b + e * kBlock + (int)threadIdx.x;
        if (loc >= t.b + t.c) break;
        const long i = L.c_off + loc;
        int s, o;
        band_at(loc >> L.log2n, loc & (L.n - 1), L.n, L.log2n, J, s, o);
        const T ri = B.r[i];
        const T z = ri * B.jinv[(t.a * (J + 1) + s) * 4 + o];
        const T p = (k == 0) ? z : z + beta * B.p[i];
        const T q = (k == 0) ? B.y[i] : B.y[i] + beta * B.q[i];
        B.p[i] = p;
        B.q[i] = q;
        c[i] += alpha * p;
        B.r[i] = ri - alpha * q;
    }
}

// Weighted squared norm sum_k C_eta^-1_k s_k^2 (preconditioner probes); result -> sc->rho.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_wnorm(const T *__restrict__ s, Bufs<T> B, int nw) {
    __shared__ double sh[kBlock / 64];
    double acc = 0.0;
    for (int g = 0; g < nw; ++g) {
        const DevWfs W = B.wfs[g];
        const long n2 = (long)W.n_sub * W.n_sub;
        for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
            int r = (int)(i / W.n_sub), q = (int)(i - (long)r * W.n_sub);
            if (!subap_active(W, r, q)) continue;
            const double sx = (double)s[W.s_off + i], sy = (double)s[W.s_off + n2 + i];
            acc += W.inv_var * (sx * sx + sy * sy);
        }
    }
    double v = block_sum(acc, sh);
    if (!publish_last(B.partials, kPartialPitch, 1, blockIdx.x, &v, &B.sc->counter)) return;
    const double tot = gather_partials(B.partials, kPartialPitch, 0, gridDim.x, sh);
    if (threadIdx.x == 0) B.sc->rho = tot;
}

// Fitting (bilinear on-axis sampling of the layers at the actuators of their DM) + gain.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fit(const T *__restrict__ u, const T *__restrict__ a_prev, T *__restrict__ a,
                                                Bufs<T> B, int nl, int nd, long n_act, double gain) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_act) return;
    int m = 0;
    while (m + 1 < nd && B.dm[m + 1].a_off <= i) ++m;
    const DevDm Dm = B.dm[m];
    const long loc = i - Dm.a_off;
    const int ai = (int)(loc / Dm.n_act), aj = (int)(loc - (long)ai * Dm.n_act);
    const double X = ((double)aj - Dm.centre) * Dm.pitch, Y = ((double)ai - Dm.centre) * Dm.pitch;
    T acc = 0;
    for (int l = 0; l < nl; ++l) {
        const DevLayer L = B.lay[l];
        if (L.dm != m) continue;
        Cell cx = cell_of(X / L.spacing + L.half, L.n), cy = cell_of(Y / L.spacing + L.half, L.n);
        T wx1 = (T)cx.t, wx0 = (T)(1.0 - cx.t), wy1 = (T)cy.t, wy0 = (T)(1.0 - cy.t);
        const T *U = u + L.c_off + (long)cy.k0 * L.n + cx.k0;
        acc += (wy0 * wx0) * U[0] + (wy0 * wx1) * U[1] + (wy1 * wx0) * U[L.n] + (wy1 * wx1) * U[L.n + 1];
    }
    const T prev = a_prev ? a_prev[i] : (T)0;
    a[i] = (T)(1.0 - gain) * prev + (T)gain * acc;
}

// Cell tables: entry (g, l, j) of each axis from the ray geometry (setup, once per bind).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_build_tabs(Ent<T> *xtab, Ent<T> *ytab, const DevWfs *__restrict__ wfs,
                                                       const DevProj *__restrict__ proj,
                                                       const DevLayer *__restrict__ lays, int nw, int nl, int maxnv) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nw * nl * maxnv) return;
    const int j = (int)(idx % maxnv), gl = (int)(idx / maxnv), l = gl % nl, g = gl / nl;
    const DevWfs W = wfs[g];
    Ent<T> ex{0, 0, (T)0, (T)0}, ey{0, 0, (T)0, (T)0};
    if (j < W.nv) {
        const DevProj pr = proj[(long)g * nl + l];
        const DevLayer L = lays[l];
        const Cell cx = cell_of(ray_coord(pr, W, L, j, pr.hx), L.n);
        const Cell cy = cell_of(ray_coord(pr, W, L, j, pr.hy), L.n);
        ex = Ent<T>{cx.k0, 0, (T)(1.0 - cx.t), (T)cx.t};
        ey = Ent<T>{cy.k0, 0, (T)(1.0 - cy.t), (T)cy.t};
    }
    xtab[idx] = ex;
    ytab[idx] = ey;
}

// Transpose ranges: for grid line q of layer l, the sensor nodes j with cell k0_j in {q-1, q}
// (k0_j is non-decreasing in j, so they are contiguous).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_build_ranges(Range *xrng, Range *yrng, const Ent<T> *__restrict__ xtab,
                                                         const Ent<T> *__restrict__ ytab,
                                                         const DevWfs *__restrict__ wfs,
                                                         const DevLayer *__restrict__ lays, int nw, int nl, int maxnv,
                                                         int sum_n) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nw * sum_n) return;
    const int g = (int)(idx / sum_n), line = (int)(idx % sum_n);
    int l = 0;
    while (l + 1 < nl && lays[l + 1].r_off <= line) ++l;
    const int q = line - lays[l].r_off, nv = wfs[g].nv;
    for (int axis = 0; axis < 2; ++axis) {
        const Ent<T> *tab = (axis == 0 ? xtab : ytab) + ((long)g * nl + l) * maxnv;
        int lo = nv, hi = -1;
        for (int j = 0; j < nv; ++j) {
            const int k0 = tab[j].k0;
            if (k0 == q || k0 + 1 == q) {
                lo = j < lo ? j : lo;
                hi = j;
            }
        }
        Range r{lo, hi};
        if (hi < 0) r = Range{1, 0};
        (axis == 0 ? xrng : yrng)[idx] = r;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *__restrict__ x, long n, T val) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = val;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(T *__restrict__ dst, const T *__restrict__ src, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) dst[i] = src[i];
}

__global__ void k_init_scalars(Scalars *sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        reset_scalars(sc);
        sc->counter = 0u;
    }
}

int grid_for(long n) {
    long g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    return (int)g;
}

int check() { return hipGetLastError() == hipSuccess ? FEWHA_OK : FEWHA_ERR_HIP; }

template <typename T, int EPI>
int launch_fdwt(const Plan &P, const Bufs<T> &B, hipStream_t st, const T *x, const EpiArgs &E0) {
    const Taps<T> tp = make_taps<T>();
    EpiArgs E = E0;
    const int nfine = (int)P.fine_tiles.size();
    E.nfine = nfine;
    const int last = (P.kf == P.J) ? 1 : 0;
    switch (P.kf) {
        case 1: k_fdwt_fine<T, 1, 16, EPI><<<nfine, kBlock, 0, st>>>(x, B.tmpA, B, P.J, E, tp, last); break;
        case 2: k_fdwt_fine<T, 2, 8, EPI><<<nfine, kBlock, 0, st>>>(x, B.tmpA, B, P.J, E, tp, last); break;
        default: k_fdwt_fine<T, 3, 4, EPI><<<nfine, kBlock, 0, st>>>(x, B.tmpA, B, P.J, E, tp, last); break;
    }
    if (int e = check()) return e;
    if (P.kf < P.J) {
        k_fdwt_coarse<T, EPI><<<P.nl, kBlock, P.coarse_lds, st>>>(B.tmpA, B, P.J, P.kf, E, tp);
        if (int e = check()) return e;
    }
    return FEWHA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
template <typename T>
Taps<T> make_taps() {
    const double q = std::sqrt(10.0), p = std::sqrt(5.0 + 2.0 * std::sqrt(10.0)), s = 16.0 * std::sqrt(2.0);
    const double h[6] = {(1 + q + p) / s,         (5 + q + 3 * p) / s, (10 - 2 * q + 2 * p) / s,
                         (10 - 2 * q - 2 * p) / s, (5 + q - 3 * p) / s, (1 + q - p) / s};
    Taps<T> t;
    for (int n = 0; n < 6; ++n) {
        t.h[n] = (T)h[n];
        t.g[n] = (T)(((n & 1) ? -1.0 : 1.0) * h[5 - n]);
    }
    return t;
}

template <typename T>
int Ops<T>::idwt(const T *c, T *out, bool scale) const {
    const int tiles = (int)P.idwt_tiles.size();
    if (scale)
        k_idwt<T, true><<<tiles, kBlock, 0, st>>>(c, out, B.idwt_tiles, B.lay, P.J, B.jinv, make_taps<T>());
    else
        k_idwt<T, false><<<tiles, kBlock, 0, st>>>(c, out, B.idwt_tiles, B.lay, P.J, B.jinv, make_taps<T>());
    return check();
}

template <typename T>
int Ops<T>::fdwt(const T *x, T *out) const {
    EpiArgs E{};
    E.out = out;
    return launch_fdwt<T, kEpiPlain>(P, B, st, x, E);
}

template <typename T>
int Ops<T>::fdwt_prior(const T *x, const T *cin, T *out) const {
    EpiArgs E{};
    E.out = out;
    E.cin = cin;
    return launch_fdwt<T, kEpiPrior>(P, B, st, x, E);
}

template <typename T>
int Ops<T>::fdwt_pcg(const T *x, int k, double *resnorm) const {
    EpiArgs E{};
    E.out = B.y;
    E.k = k;
    E.resnorm = resnorm;
    return launch_fdwt<T, kEpiPcg>(P, B, st, x, E);
}

template <typename T>
int Ops<T>::fdwt_rhs(const T *x, T *c, bool cold) const {
    EpiArgs E{};
    E.out = B.b;
    E.c = c;
    E.cold = cold ? 1 : 0;
    return launch_fdwt<T, kEpiRhs>(P, B, st, x, E);
}

template <typename T>
int Ops<T>::nodes(const T *in, T *v, int mode) const {
    const int tiles = (int)P.node_tiles.size();
    if (mode == kModeM) k_nodes<T, kModeM><<<tiles, kBlock, 0, st>>>(in, v, B, P.nl);
    else if (mode == kModeRhs) k_nodes<T, kModeRhs><<<tiles, kBlock, 0, st>>>(in, v, B, P.nl);
    else k_nodes<T, kModeAdj><<<tiles, kBlock, 0, st>>>(in, v, B, P.nl);
    return check();
}

template <typename T>
int Ops<T>::slopes(const T *u, T *s) const {
    k_slopes<T><<<(int)P.sub_tiles.size(), kBlock, 0, st>>>(u, s, B, P.nl);
    return check();
}

template <typename T>
int Ops<T>::pt(const T *v, T *x) const {
    k_pt<T><<<(int)P.lay_tiles.size(), kBlock, 0, st>>>(v, x, B, P.nl, P.nw);
    return check();
}

template <typename T>
int Ops<T>::update(T *c, int k) const {
    k_update<T><<<(int)P.coef_tiles.size(), kBlock, 0, st>>>(c, B, P.J, k);
    return check();
}

template <typename T>
int Ops<T>::wnorm(const T *s) const {
    long mx = 0;
    for (auto &w : P.dwfs) mx = mx > (long)w.n_sub * w.n_sub ? mx : (long)w.n_sub * w.n_sub;
    int g = grid_for(mx);
    if (g > P.n_partials) g = P.n_partials;
    k_wnorm<T><<<g, kBlock, 0, st>>>(s, B, P.nw);
    return check();
}

template <typename T>
int Ops<T>::fit(const T *u, const T *a_prev, T *a, double gain) const {
    k_fit<T><<<grid_for((long)P.n_act), kBlock, 0, st>>>(u, a_prev, a, B, P.nl, P.nd, (long)P.n_act, gain);
    return check();
}

template <typename T>
int Ops<T>::build_tables() const {
    const long ne = (long)P.nw * P.nl * P.maxnv;
    k_build_tabs<T><<<(int)((ne + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        const_cast<Ent<T> *>(B.xtab), const_cast<Ent<T> *>(B.ytab), B.wfs, B.proj, B.lay, P.nw, P.nl, P.maxnv);
    if (int e = check()) return e;
    const long nr = (long)P.nw * P.sum_n;
    k_build_ranges<T><<<(int)((nr + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        const_cast<Range *>(B.xrng), const_cast<Range *>(B.yrng), B.xtab, B.ytab, B.wfs, B.lay, P.nw, P.nl, P.maxnv,
        P.sum_n);
    return check();
}

template <typename T>
int Ops<T>::fill(T *x, long n, T val) const {
    k_fill<T><<<grid_for(n), kBlock, 0, st>>>(x, n, val);
    return check();
}

template <typename T>
int Ops<T>::copy(T *dst, const T *src, long n) const {
    k_copy<T><<<grid_for(n), kBlock, 0, st>>>(dst, src, n);
    return check();
}

template <typename T>
int Ops<T>::init_scalars() const {
    k_init_scalars<<<1, 64, 0, st>>>(B.sc);
    return check();
}

template struct Ops<float>;
template struct Ops<double>;

}  // namespace fewha
