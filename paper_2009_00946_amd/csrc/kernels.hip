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
// W^T: multi-level inverse DWT in one launch, with the PCG update fused in front of it.
//
// Each workgroup owns a square output tile and rebuilds, from the coarsest level down, only the
// cone of coefficients that tile depends on.  The whole cone (every level, every band) is
// fetched from global memory in one batch of independent loads into LDS, so the J levels of
// synthesis then run from LDS.  In the update mode the loads bring r_{k-1}, y_{k-1}, q_{k-2},
// the Alg. 2 update is evaluated for every cone coefficient, the coefficients this tile owns are
// written back (p, q, c and the new residual), and the transform runs on z = J^-1 r_k.
// Ownership: at level s a tile owns the indices [y0 >> s, (y0 + T0) >> s) when T0 >= 2^s, else
// index y0 >> s if y0 is a multiple of 2^s (likewise in x), a partition of every band.
// ---------------------------------------------------------------------------------------------

constexpr int kInvSegMax = 3072;  // cone coefficients of a 32 x 32 tile over up to 12 levels

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_inv(Bufs<T> B, int J, InvArgs A, Taps<T> tp) {
    constexpr int TILE = kIdwtTile;
    constexpr int R = TILE / 2 + 2;
    constexpr int MAXI = (kInvSegMax + kBlock - 1) / kBlock;
    __shared__ T sSeg[kInvSegMax];
    __shared__ T sL0[R * R], sL1[R * R];
    __shared__ T sAX[TILE * R], sDX[TILE * R];
    __shared__ int shLoY[kMaxJ + 1], shLoX[kMaxJ + 1], shLnY[kMaxJ + 1], shLnX[kMaxJ + 1], shSeg[kMaxJ + 2];
    __shared__ T sJinv[(kMaxJ + 1) * 4];

    const Tile t = B.idwt_tiles[blockIdx.x];
    const int l = t.a, y0 = t.b, x0 = t.c, T0 = t.d, n = t.f;
    const long coff = t.e;
    // Cone bounds per level, computed by every lane in registers (uniform values): the item
    // decode below then needs no LDS round trips.
    int loY[kMaxJ + 1], loX[kMaxJ + 1], lnY[kMaxJ + 1], lnX[kMaxJ + 1], seg[kMaxJ + 2];
    {
        int ly = y0, hy = y0 + T0 - 1, lx = x0, hx = x0 + T0 - 1, off = 0;
        loY[0] = ly;
        loX[0] = lx;
        lnY[0] = T0;
        lnX[0] = T0;
        seg[0] = 0;
#pragma unroll
        for (int s = 1; s <= kMaxJ; ++s) {
            ly = (ly >> 1) - 2;
            hy >>= 1;
            lx = (lx >> 1) - 2;
            hx >>= 1;
            loY[s] = ly;
            loX[s] = lx;
            lnY[s] = hy - ly + 1;
            lnX[s] = hx - lx + 1;
            seg[s] = off;
            if (s <= J) off += 3 * lnY[s] * lnX[s];
        }
        seg[kMaxJ + 1] = off;  // the coarsest LL starts here
    }
    int lnYJ = 0, lnXJ = 0, loYJ = 0, loXJ = 0;
#pragma unroll
    for (int s = 1; s <= kMaxJ; ++s)
        if (s == J) {
            lnYJ = lnY[s];
            lnXJ = lnX[s];
            loYJ = loY[s];
            loXJ = loX[s];
        }
    const int llOff = seg[kMaxJ + 1], total = llOff + lnYJ * lnXJ;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s <= kMaxJ; ++s) {
            shLoY[s] = loY[s];
            shLoX[s] = loX[s];
            shLnY[s] = lnY[s];
            shLnX[s] = lnX[s];
            shSeg[s] = seg[s];
        }
        shSeg[kMaxJ + 1] = llOff;
    }
    if (MODE != kInvPlain && threadIdx.x < (J + 1) * 4) sJinv[threadIdx.x] = B.jinv[l * (J + 1) * 4 + threadIdx.x];

    double alpha = 0.0, beta = 0.0;
    int stopped = 0;
    if constexpr (MODE == kInvUpdate) {
        alpha = B.sc->alpha;
        beta = B.sc->beta;
        stopped = B.sc->stopped;
    }
    const T *src = static_cast<const T *>(A.src);
    __syncthreads();
    // ---- one batch of independent loads: the whole cone (plus owned-only operands) ----
    for (int base = 0; base < total; base += MAXI * kBlock) {
        long gi[MAXI];
        int li[MAXI], bnd[MAXI];
        bool own[MAXI];
        T rv[MAXI], yv[MAXI], qv[MAXI], pv[MAXI], cv[MAXI];
#pragma unroll
        for (int c = 0; c < MAXI; ++c) {
            const int k = base + c * kBlock + (int)threadIdx.x;
            gi[c] = -1;
            own[c] = false;
            if (k >= total) continue;
            // segment of item k: a detail band of level s, or the coarsest LL
            int s = J, o = 0, ly = loYJ, lx = loXJ, nxs = lnXJ, rem = k - llOff;
#pragma unroll
            for (int ss = 1; ss <= kMaxJ; ++ss) {
                const int sz = lnY[ss] * lnX[ss];
                if (ss <= J && k >= seg[ss] && k < seg[ss] + 3 * sz) {
                    s = ss;
                    ly = loY[ss];
                    lx = loX[ss];
                    nxs = lnX[ss];
                    rem = k - seg[ss];
                    o = 1 + rem / sz;
                    rem -= (o - 1) * sz;
                }
            }
            const int r = rem / nxs, q = rem - r * nxs;
            const int m = n >> s, msk = m - 1;
            const int uy = ly + r, ux = lx + q;
            const int gr = uy & msk, gc = ux & msk;
            const int row = gr + ((o == 2 || o == 3) ? m : 0), col = gc + ((o == 1 || o == 3) ? m : 0);
            gi[c] = coff + (long)row * n + col;
            li[c] = k;
            bnd[c] = s * 4 + o;
            if constexpr (MODE == kInvUpdate) {
                const int ts = T0 >> s, msk2 = (1 << s) - 1;
                const bool oy = ts >= 1 ? (uy >= (y0 >> s) && uy < (y0 >> s) + ts) : ((y0 & msk2) == 0 && uy == (y0 >> s));
                const bool ox = ts >= 1 ? (ux >= (x0 >> s) && ux < (x0 >> s) + ts) : ((x0 & msk2) == 0 && ux == (x0 >> s));
                own[c] = oy && ox;
            }
            rv[c] = src[gi[c]];
            if constexpr (MODE == kInvUpdate) {
                yv[c] = static_cast<const T *>(A.yv)[gi[c]];
                qv[c] = A.first_pass ? (T)0 : static_cast<const T *>(A.qold)[gi[c]];
                if (own[c]) {
                    pv[c] = A.first_pass ? (T)0 : B.p[gi[c]];
                    cv[c] = static_cast<T *>(A.c)[gi[c]];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < MAXI; ++c) {
            if (gi[c] < 0) continue;
            T val = rv[c];
            if constexpr (MODE == kInvFirst) {
                val = rv[c] * sJinv[bnd[c]];
            } else if constexpr (MODE == kInvUpdate) {
                const T ji = sJinv[bnd[c]];
                T rn = rv[c];
                if (!stopped) {
                    const T zo = rv[c] * ji;
                    const T qn = A.first_pass ? yv[c] : yv[c] + (T)beta * qv[c];
                    rn = rv[c] - (T)alpha * qn;
                    if (own[c]) {
                        const T pn = A.first_pass ? zo : zo + (T)beta * pv[c];
                        B.p[gi[c]] = pn;
                        static_cast<T *>(A.qnew)[gi[c]] = qn;
                        static_cast<T *>(A.c)[gi[c]] = cv[c] + (T)alpha * pn;
                    }
                }
                if (own[c]) static_cast<T *>(A.rnew)[gi[c]] = rn;
                val = rn * ji;
            }
            sSeg[li[c]] = val;
        }
    }
    __syncthreads();

    // ---- synthesis from the coarsest level, all in LDS ----
    const T *LL = sSeg + llOff;
    int llp = lnXJ;
    T *NX = sL0;
    T *outp = static_cast<T *>(A.out);
    for (int s = J; s >= 1; --s) {
        const int ny = shLnY[s - 1], nxk = shLnX[s], nx = shLnX[s - 1];
        const int oy = shLoY[s - 1], ky = shLoY[s], ox = shLoX[s - 1], kx = shLoX[s];
        const int bsz = shLnY[s] * shLnX[s], bp = shLnX[s];
        const T *HL = sSeg + shSeg[s], *LH = HL + bsz, *HH = LH + bsz;
        // undo the y analysis: (LL, x-low/y-high) -> x-low rows, (x-high/y-low, HH) -> x-high rows
        for (int idx = threadIdx.x; idx < ny * nxk; idx += blockDim.x) {
            const int r = idx / nxk, q = idx - r * nxk;
            const int y = oy + r, p = y & 1, kb = (y >> 1) - ky;
            T a = 0, d = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int rr = kb - j;
                a += tp.h[p + 2 * j] * LL[rr * llp + q] + tp.g[p + 2 * j] * LH[rr * bp + q];
                d += tp.h[p + 2 * j] * HL[rr * bp + q] + tp.g[p + 2 * j] * HH[rr * bp + q];
            }
            sAX[r * R + q] = a;
            sDX[r * R + q] = d;
        }
        __syncthreads();
        // undo the x analysis
        for (int idx = threadIdx.x; idx < ny * nx; idx += blockDim.x) {
            const int r = idx / nx, q = idx - r * nx;
            const int x = ox + q, p = x & 1, kb = (x >> 1) - kx;
            T v = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int at = r * R + kb - j;
                v += tp.h[p + 2 * j] * sAX[at] + tp.g[p + 2 * j] * sDX[at];
            }
            if (s > 1) NX[r * R + q] = v;
            else outp[coff + (long)(oy + r) * n + ox + q] = v;
        }
        __syncthreads();
        LL = NX;
        llp = R;
        NX = (NX == sL0) ? sL1 : sL0;
    }
}

// Final Alg. 2 update of a solve (elementwise; the residual ends in the state buffer B.r).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_last(T *__restrict__ c, Bufs<T> B, int J, const T *__restrict__ rin,
                                                        const T *__restrict__ qold, T *__restrict__ qnew, int first) {
    const Tile t = B.coef_tiles[blockIdx.x];
    const double alpha = B.sc->alpha, beta = B.sc->beta;
    const int stopped = B.sc->stopped;
#pragma unroll
    for (int e = 0; e < kCoefTile / kBlock; ++e) {
        const int loc = t.b + e * kBlock + (int)threadIdx.x;
        if (loc >= t.b + t.c) break;
        const long i = t.e + loc;
        const T ri = rin[i];
        if (stopped) {
            B.r[i] = ri;
            continue;
        }
        int s, o;
        band_at(loc >> t.g, loc & (t.f - 1), t.f, t.g, J, s, o);
        const T z = ri * B.jinv[(t.a * (J + 1) + s) * 4 + o];
        const T p = first ? z : z + (T)beta * B.p[i];
        const T q = first ? B.y[i] : B.y[i] + (T)beta * qold[i];
        B.p[i] = p;
        qnew[i] = q;
        c[i] += (T)alpha * p;
        B.r[i] = ri - (T)alpha * q;
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

// P + Gamma + C_eta^-1 + Gamma^T on one node tile (the paper's Kernel-2 stage, y-part of M).
// phi is needed on the tile plus a one-node halo.  Layers are processed in chunks: the cell
// table entries of the chunk's rows and columns are staged in LDS, then every (node, layer)
// bilinear gather of the chunk is issued as one batch of independent loads; the per-layer
// contributions are summed in layer order (deterministic), then slopes, weights and Gamma^T
// run from LDS.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_nodes_m(const T *__restrict__ u, T *__restrict__ v, Bufs<T> B, int nl) {
    constexpr int NT = kNodeTile, NP = NT + 2, NS = NT + 1, NN = NP * NP;
    constexpr int LMAX = 12;
    constexpr int MAXI = (NN * LMAX + kBlock - 1) / kBlock;
    __shared__ Ent<T> sX[LMAX * NP], sY[LMAX * NP];
    __shared__ T sPart[LMAX * NN];
    __shared__ T sPhi[NN];
    __shared__ T sSx[NS * NS], sSy[NS * NS];
    __shared__ long sOff[LMAX];
    __shared__ int sN[LMAX];
    const Tile t = B.node_tiles[blockIdx.x];
    const int g = t.a, i0 = t.b, j0 = t.c;
    const DevWfs W = B.wfs[g];
    const int ns = W.n_sub, nv = W.nv;
    for (int idx = threadIdx.x; idx < NN; idx += blockDim.x) sPhi[idx] = 0;
    for (int l0 = 0; l0 < nl; l0 += LMAX) {
        const int nc = (nl - l0) < LMAX ? (nl - l0) : LMAX;
        for (int idx = threadIdx.x; idx < 2 * nc * NP; idx += blockDim.x) {
            const int axis = idx / (nc * NP), rem = idx - axis * nc * NP, l = rem / NP, b = rem - l * NP;
            int node = (axis ? i0 : j0) - 1 + b;
            node = node < 0 ? 0 : (node > ns ? ns : node);
            const long at = ((long)g * nl + l0 + l) * B.maxnv + node;
            if (axis) sY[l * NP + b] = B.ytab[at];
            else sX[l * NP + b] = B.xtab[at];
        }
        if (threadIdx.x < nc) {
            sOff[threadIdx.x] = B.lay[l0 + threadIdx.x].c_off;
            sN[threadIdx.x] = B.lay[l0 + threadIdx.x].n;
        }
        __syncthreads();
        T val[MAXI];
#pragma unroll
        for (int c = 0; c < MAXI; ++c) {
            const int k = c * kBlock + (int)threadIdx.x;
            val[c] = 0;
            if (k < nc * NN) {
                const int l = k / NN, nd = k - l * NN, a = nd / NP, b = nd - a * NP;
                const int i = i0 - 1 + a, j = j0 - 1 + b;
                if (i >= 0 && i <= ns && j >= 0 && j <= ns) {
                    const Ent<T> ex = sX[l * NP + b], ey = sY[l * NP + a];
                    const int n = sN[l];
                    const T *U = u + sOff[l] + (long)ey.k0 * n + ex.k0;
                    val[c] = (ey.w0 * ex.w0) * U[0] + (ey.w0 * ex.w1) * U[1] + (ey.w1 * ex.w0) * U[n] +
                             (ey.w1 * ex.w1) * U[n + 1];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < MAXI; ++c) {
            const int k = c * kBlock + (int)threadIdx.x;
            if (k < nc * NN) sPart[k] = val[c];
        }
        __syncthreads();
        for (int nd = threadIdx.x; nd < NN; nd += blockDim.x) {
            T acc = sPhi[nd];
            for (int l = 0; l < nc; ++l) acc += sPart[l * NN + nd];
            sPhi[nd] = acc;
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < NS * NS; idx += blockDim.x) {
        const int a = idx / NS, b = idx - a * NS, i = i0 - 1 + a, j = j0 - 1 + b;
        T sx = 0, sy = 0;
        if (i >= 0 && i < ns && j >= 0 && j < ns && subap_active(W, i, j)) {
            const T w = (T)W.inv_var;
            const T p00 = sPhi[a * NP + b], p01 = sPhi[a * NP + b + 1];
            const T p10 = sPhi[(a + 1) * NP + b], p11 = sPhi[(a + 1) * NP + b + 1];
            sx = w * ((T)0.5 * ((p01 - p00) + (p11 - p10)));
            sy = w * ((T)0.5 * ((p10 - p00) + (p11 - p01)));
        }
        sSx[idx] = sx;
        sSy[idx] = sy;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NT * NT; idx += blockDim.x) {
        const int a = idx / NT, b = idx - a * NT, i = i0 + a, j = j0 + b;
        if (i > ns || j > ns) continue;
        const int s11 = (a + 1) * NS + (b + 1), s10 = (a + 1) * NS + b, s01 = a * NS + (b + 1), s00 = a * NS + b;
        const T val = (T)0.5 * ((-sSx[s11] - sSy[s11]) + (sSx[s10] - sSy[s10]) + (-sSx[s01] + sSy[s01]) +
                                (sSx[s00] + sSy[s00]));
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
// P^T on a tile of layer nodes, as a gather through the transpose ranges of the cell tables.
// For each sensor the node ranges of the tile's rows and columns are staged in LDS, then the
// sub-block of v_g they span and its table entries arrive in one batch of independent loads;
// each lane sums its node's contributions (sensor, then row, then column order) from LDS.  A
// sensor whose sub-block does not fit the LDS budget is gathered straight from global memory.
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pt(const T *__restrict__ v, T *__restrict__ x, Bufs<T> B, int nl,
                                               int nw) {
    constexpr int NT = kNodeTile, GMAX = kBlock / NT, VMAX = sizeof(T) == 4 ? 4096 : 2048, EMAX = 512, MAXI = 16;
    static_assert(GMAX == 16, "16 lanes per sensor");
    __shared__ Range sRy[GMAX * NT], sRx[GMAX * NT];
    __shared__ T sV[VMAX];
    __shared__ Ent<T> sEy[EMAX], sEx[EMAX];
    __shared__ int sGeo[GMAX][4];  // i0, ni, j0, nj of each sensor's sub-block (ni = 0: empty)
    const Tile t = B.lay_tiles[blockIdx.x];
    const int l = t.a, k0 = t.b, q0 = t.c, n = t.f, roff = t.h;
    const int k = k0 + (int)(threadIdx.x / NT), q = q0 + (int)(threadIdx.x % NT);
    const bool valid = k < n && q < n;
    const int lane = threadIdx.x & (NT - 1), grp = threadIdx.x / NT;
    T acc = 0;
    for (int gb = 0; gb < nw; gb += GMAX) {
        const int gc = (nw - gb) < GMAX ? (nw - gb) : GMAX;
        // 16 lanes per sensor: each loads the range of one tile row and one tile column, then the
        // group reduces them to the sub-block of sensor nodes the whole tile needs
        {
            Range ry{1, 0}, rx{1, 0};
            if (grp < gc) {
                const long base = (long)(gb + grp) * B.sum_n + roff;
                if (k0 + lane < n) ry = B.yrng[base + k0 + lane];
                if (q0 + lane < n) rx = B.xrng[base + q0 + lane];
            }
            sRy[grp * NT + lane] = ry;
            sRx[grp * NT + lane] = rx;
            int i0 = ry.lo <= ry.hi ? ry.lo : (1 << 30), i1 = ry.lo <= ry.hi ? ry.hi : -1;
            int j0 = rx.lo <= rx.hi ? rx.lo : (1 << 30), j1 = rx.lo <= rx.hi ? rx.hi : -1;
#pragma unroll
            for (int m = 1; m < NT; m <<= 1) {
                i0 = min(i0, __shfl_xor(i0, m, NT));
                i1 = max(i1, __shfl_xor(i1, m, NT));
                j0 = min(j0, __shfl_xor(j0, m, NT));
                j1 = max(j1, __shfl_xor(j1, m, NT));
            }
            if (lane == 0) {
                const bool ne = i1 >= i0 && j1 >= j0;
                sGeo[grp][0] = i0;
                sGeo[grp][1] = ne ? i1 - i0 + 1 : 0;
                sGeo[grp][2] = j0;
                sGeo[grp][3] = ne ? j1 - j0 + 1 : 0;
            }
        }
        __syncthreads();
        // staging plan (uniform, in registers): sensors in order while the LDS budget lasts
        int I0[GMAX], NI[GMAX], J0[GMAX], NJ[GMAX], VO[GMAX], EYO[GMAX], EXO[GMAX], CUM[GMAX + 1];
        {
            int vo = 0, eyo = 0, exo = 0, cum = 0;
#pragma unroll
            for (int g = 0; g < GMAX; ++g) {
                I0[g] = sGeo[g][0];
                J0[g] = sGeo[g][2];
                const int ni = g < gc ? sGeo[g][1] : 0, nj = g < gc ? sGeo[g][3] : 0;
                const bool ok = ni > 0 && vo + ni * nj <= VMAX && eyo + ni <= EMAX && exo + nj <= EMAX;
                NI[g] = ok ? ni : (ni > 0 ? -1 : 0);  // -1: not staged, gather from global memory
                NJ[g] = ok ? nj : 0;
                VO[g] = vo;
                EYO[g] = eyo;
                EXO[g] = exo;
                CUM[g] = cum;
                if (ok) {
                    vo += ni * nj;
                    eyo += ni;
                    exo += nj;
                    cum += ni * nj + ni + nj;
                }
            }
            CUM[GMAX] = cum;
        }
        const int total = CUM[GMAX];
        for (int base = 0; base < total; base += MAXI * kBlock) {
            T vv[MAXI], w0[MAXI], w1[MAXI];
            int k0e[MAXI], dst[MAXI], kind[MAXI];
#pragma unroll
            for (int c = 0; c < MAXI; ++c) {
                const int kk = base + c * kBlock + (int)threadIdx.x;
                kind[c] = -1;
                if (kk >= total) continue;
                int g = 0;
#pragma unroll
                for (int gg = 1; gg < GMAX; ++gg)
                    if (kk >= CUM[gg]) g = gg;
                int i0 = 0, j0 = 0, ni = 0, nj = 0, vo = 0, eyo = 0, exo = 0, cm = 0;
#pragma unroll
                for (int gg = 0; gg < GMAX; ++gg)
                    if (gg == g) {
                        i0 = I0[gg];
                        j0 = J0[gg];
                        ni = NI[gg];
                        nj = NJ[gg];
                        vo = VO[gg];
                        eyo = EYO[gg];
                        exo = EXO[gg];
                        cm = CUM[gg];
                    }
                int rem = kk - cm;
                const int sg = gb + g;
                const long tb = ((long)sg * nl + l) * B.maxnv;
                if (rem < ni * nj) {
                    const int a = rem / nj, b = rem - a * nj;
                    const DevWfs &W = B.wfs[sg];
                    vv[c] = v[W.v_off + (long)(i0 + a) * W.nv + j0 + b];
                    dst[c] = vo + rem;
                    kind[c] = 0;
                } else {
                    rem -= ni * nj;
                    const bool isy = rem < ni;
                    if (!isy) rem -= ni;
                    const Ent<T> e = isy ? B.ytab[tb + i0 + rem] : B.xtab[tb + j0 + rem];
                    k0e[c] = e.k0;
                    w0[c] = e.w0;
                    w1[c] = e.w1;
                    dst[c] = (isy ? eyo : exo) + rem;
                    kind[c] = isy ? 1 : 2;
                }
            }
#pragma unroll
            for (int c = 0; c < MAXI; ++c) {
                if (kind[c] == 0) sV[dst[c]] = vv[c];
                else if (kind[c] > 0) {
                    Ent<T> &e = (kind[c] == 1) ? sEy[dst[c]] : sEx[dst[c]];
                    e.k0 = k0e[c];
                    e.w0 = w0[c];
                    e.w1 = w1[c];
                }
            }
        }
        __syncthreads();
        if (valid) {
#pragma unroll
            for (int g = 0; g < GMAX; ++g) {
                const Range ry = sRy[g * NT + (k - k0)], rx = sRx[g * NT + (q - q0)];
                if (g >= gc || ry.lo > ry.hi || rx.lo > rx.hi) continue;
                if (NI[g] > 0) {
                    const T *V = sV + VO[g];
                    for (int i = ry.lo; i <= ry.hi; ++i) {
                        const Ent<T> ey = sEy[EYO[g] + i - I0[g]];
                        const T wy = (ey.k0 == k) ? ey.w0 : ey.w1;
                        for (int j = rx.lo; j <= rx.hi; ++j) {
                            const Ent<T> ex = sEx[EXO[g] + j - J0[g]];
                            const T wx = (ex.k0 == q) ? ex.w0 : ex.w1;
                            acc += (wy * wx) * V[(i - I0[g]) * NJ[g] + (j - J0[g])];
                        }
                    }
                } else {  // did not fit the LDS budget: straight from global memory
                    const int sg = gb + g;
                    const DevWfs W = B.wfs[sg];
                    const Ent<T> *xt = B.xtab + ((long)sg * nl + l) * B.maxnv;
                    const Ent<T> *yt = B.ytab + ((long)sg * nl + l) * B.maxnv;
                    for (int i = ry.lo; i <= ry.hi; ++i) {
                        const Ent<T> ey = yt[i];
                        const T wy = (ey.k0 == k) ? ey.w0 : ey.w1;
                        for (int j = rx.lo; j <= rx.hi; ++j) {
                            const Ent<T> ex = xt[j];
                            const T wx = (ex.k0 == q) ? ex.w0 : ex.w1;
                            acc += (wy * wx) * v[W.v_off + (long)i * W.nv + j];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (valid) x[(long)t.e + (long)k * n + q] = acc;
}

// ---------------------------------------------------------------------------------------------
// Forward transform W in one launch, with fused epilogues.
//
// Fine part: a workgroup owns a TQ x TQ tile of level-KF approximation coefficients; it stages
// the input region with its halo (periodic wrap) and the epilogue operands of every coefficient
// it owns in one batch of independent loads, then runs levels 1..KF from LDS.  Coarse part: the
// last tile of a layer to finish (per-layer counter) runs levels KF+1..J of that layer in LDS.
// The last layer to finish combines the FP64 partial sums of every workgroup, in a fixed order,
// into the Alg. 2 scalars.
// ---------------------------------------------------------------------------------------------

// Region geometry of the fine part: a tile of TQ x TQ level-KF approximation coefficients needs
// LL_s on a run of len(s) = TQ 2^(KF-s) + 4 (2^(KF-s) - 1) indices (s = 0 is the input).
template <int KF, int TQ>
struct FineGeom {
    static constexpr int len(int s) { return TQ * (1 << (KF - s)) + 4 * ((1 << (KF - s)) - 1); }
};

// Deliver one coefficient w of W x (operands e0, e1 prefetched); accumulate PCG dot partials.
template <typename T, int EPI>
__device__ __forceinline__ void deliver(const Bufs<T> &B, const FwdArgs &E, long i, T w, T ad, T ji, T e0, T e1,
                                        double &rho, double &mu) {
    if constexpr (EPI == kEpiPlain) {
        static_cast<T *>(E.out)[i] = w;
    } else if constexpr (EPI == kEpiPrior) {
        static_cast<T *>(E.out)[i] = w + ad * e0;
    } else if constexpr (EPI == kEpiPcg) {
        const T z = e0 * ji;
        const T yi = w + ad * z;
        static_cast<T *>(E.out)[i] = yi;
        rho += (double)e0 * (double)z;
        mu += (double)yi * (double)z;
    } else {  // b = W x:  r = (b - b_prev) + r  (cold: r = b, c = 0);  b_prev = b
        if (E.cold) {
            B.r[i] = w;
            static_cast<T *>(E.c)[i] = 0;
        } else {
            B.r[i] = (w - e0) + e1;
        }
        B.b_prev[i] = w;
    }
}

template <typename T, int EPI>
__device__ __forceinline__ void prefetch(const Bufs<T> &B, const FwdArgs &E, long i, T &e0, T &e1) {
    if constexpr (EPI == kEpiPrior) e0 = static_cast<const T *>(E.cin)[i];
    else if constexpr (EPI == kEpiPcg) e0 = static_cast<const T *>(E.rk)[i];
    else if constexpr (EPI == kEpiRhs) {
        e0 = B.b_prev[i];
        e1 = B.r[i];
    }
}

// Global index of coefficient (r, q) of band o (0 LL, 1 x-high, 2 y-high, 3 HH) at level s.
__device__ __forceinline__ long band_index(long coff, int n, int s, int o, int r, int q) {
    const int m = n >> s;
    return coff + (long)(r + ((o == 2 || o == 3) ? m : 0)) * n + q + ((o == 1 || o == 3) ? m : 0);
}

template <typename T, int KF, int TQ, int EPI>
__global__ __launch_bounds__(kBlock) void k_fwd(const T *__restrict__ x, Bufs<T> B, int J, int nl, FwdArgs E,
                                                Taps<T> tp) {
    using G = FineGeom<KF, TQ>;
    constexpr int L0 = G::len(0), L1 = G::len(1), EMAX = 1024;
    constexpr int NE = (EPI == kEpiRhs) ? 2 : ((EPI == kEpiPlain) ? 0 : 1);
    constexpr int FINE = L0 * L0 + (KF >= 2 ? L1 * L1 : 0) + NE * EMAX;
    constexpr int COARSE = 64 * 64 + 32 * 32;
    constexpr int SMEM = FINE > COARSE ? FINE : COARSE;
    constexpr int MAXI = 8;
    __shared__ T sm[SMEM];
    __shared__ T sAd[kMaxJ + 1], sJi[(kMaxJ + 1) * 4];
    __shared__ double sh[kBlock / 64];
    __shared__ int sLast;
    T *sA = sm, *sB = sm + L0 * L0, *sE0 = sB + (KF >= 2 ? L1 * L1 : 0), *sE1 = sE0 + EMAX;

    if constexpr (EPI == kEpiRhs) {
        if (blockIdx.x == 0 && threadIdx.x == 0) reset_scalars(B.sc);
    }
    const Tile t = B.fine_tiles[blockIdx.x];
    const int l = t.a, qy = t.b, qx = t.c, tq = t.d, n = t.f, ntiles = t.h;
    const long coff = t.e;
    if (threadIdx.x <= J) sAd[threadIdx.x] = (EPI == kEpiPrior || EPI == kEpiPcg) ? B.ad[l * (J + 1) + threadIdx.x] : (T)0;
    if (EPI == kEpiPcg && threadIdx.x < (J + 1) * 4) sJi[threadIdx.x] = B.jinv[l * (J + 1) * 4 + threadIdx.x];

    int len[KF + 1], own[KF + 1], eoff[KF + 2];
    eoff[1] = 0;
#pragma unroll
    for (int s = 0; s <= KF; ++s) {
        len[s] = tq * (1 << (KF - s)) + 4 * ((1 << (KF - s)) - 1);
        own[s] = tq << (KF - s);
        if (s >= 1) eoff[s + 1] = eoff[s] + 3 * own[s] * own[s];
    }
    const int ne = eoff[KF + 1] + (KF == J ? own[KF] * own[KF] : 0);
    const int oy = qy << KF, ox = qx << KF, nmask = n - 1;

    // ---- one batch of loads: input region + epilogue operands of the owned coefficients ----
    {
        const int nreg = len[0] * len[0], tot = nreg + (NE ? ne : 0);
        for (int base = 0; base < tot; base += MAXI * kBlock) {
            T v0[MAXI], v1[MAXI];
            int d[MAXI];
#pragma unroll
            for (int c = 0; c < MAXI; ++c) {
                const int k = base + c * kBlock + (int)threadIdx.x;
                d[c] = -1;
                if (k >= tot) continue;
                if (k < nreg) {
                    const int r = k / len[0], q = k - r * len[0];
                    v0[c] = x[coff + (long)((oy + r) & nmask) * n + ((ox + q) & nmask)];
                    d[c] = r * L0 + q;
                } else {
                    const int e = k - nreg;
                    int s = 1;
                    while (s < KF && e >= eoff[s + 1]) ++s;
                    int o, r, q;
                    if (e >= eoff[KF + 1]) {  // LL at level KF == J
                        s = KF;
                        o = 0;
                        const int rem = e - eoff[KF + 1];
                        r = rem / own[KF];
                        q = rem - r * own[KF];
                    } else {
                        const int rem = e - eoff[s], b2 = own[s] * own[s];
                        o = 1 + rem / b2;
                        const int rr = rem - (o - 1) * b2;
                        r = rr / own[s];
                        q = rr - r * own[s];
                    }
                    const long gi = band_index(coff, n, s, o, (qy << (KF - s)) + r, (qx << (KF - s)) + q);
                    T a0 = 0, a1 = 0;
                    prefetch<T, EPI>(B, E, gi, a0, a1);
                    v0[c] = a0;
                    v1[c] = a1;
                    d[c] = SMEM + e;  // marks an epilogue slot
                }
            }
#pragma unroll
            for (int c = 0; c < MAXI; ++c) {
                if (d[c] < 0) continue;
                if (d[c] < SMEM) sA[d[c]] = v0[c];
                else {
                    sE0[d[c] - SMEM] = v0[c];
                    if (NE == 2) sE1[d[c] - SMEM] = v1[c];
                }
            }
        }
    }
    __syncthreads();

    double rho = 0.0, mu = 0.0;
#pragma unroll
    for (int s = 1; s <= KF; ++s) {
        const T *src = (s & 1) ? sA : sB;
        T *dst = (s & 1) ? sB : sA;
        const int sp = (s & 1) ? L0 : L1, dp = (s & 1) ? L1 : L0;
        const int ln = len[s], ow = own[s];
        const int by = qy << (KF - s), bx = qx << (KF - s);
        const T ad = sAd[s];
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
            if (r < ow && q < ow) {
                const int e = eoff[s] + r * ow + q, b2 = ow * ow;
                const T w[3] = {hl, lh, hh};
#pragma unroll
                for (int o = 1; o <= 3; ++o) {
                    const int ei = e + (o - 1) * b2;
                    const T e0 = NE ? sE0[ei] : (T)0, e1 = NE == 2 ? sE1[ei] : (T)0;
                    deliver<T, EPI>(B, E, band_index(coff, n, s, o, by + r, bx + q), w[o - 1], ad,
                                    EPI == kEpiPcg ? sJi[s * 4 + o] : (T)0, e0, e1, rho, mu);
                }
                if (s == KF) {
                    if (KF == J) {
                        const int ei = eoff[KF + 1] + r * ow + q;
                        const T e0 = NE ? sE0[ei] : (T)0, e1 = NE == 2 ? sE1[ei] : (T)0;
                        deliver<T, EPI>(B, E, band_index(coff, n, s, 0, by + r, bx + q), ll, ad,
                                        EPI == kEpiPcg ? sJi[s * 4] : (T)0, e0, e1, rho, mu);
                    } else {
                        B.tmpA[(coff >> (2 * KF)) + (long)(by + r) * (n >> KF) + bx + q] = ll;
                    }
                }
            }
        }
        __syncthreads();
    }

    double vals[2];
    if constexpr (EPI == kEpiPcg) {
        vals[0] = block_sum(rho, sh);
        vals[1] = block_sum(mu, sh);
    }
    const int nfine = gridDim.x;
    if (KF == J) {
        if constexpr (EPI == kEpiPcg) {
            if (!publish_last(B.partials, kPartialPitch, 2, blockIdx.x, vals, &B.sc->counter)) return;
            const double R = gather_partials(B.partials, kPartialPitch, 0, nfine, sh);
            const double Mu = gather_partials(B.partials, kPartialPitch, 1, nfine, sh);
            if (threadIdx.x == 0) pcg_scalars(B.sc, R, Mu, E.k, E.resnorm);
        }
        return;
    }
    // ---- hand the layer's remaining levels to its last tile ----
    if (threadIdx.x == 0) {
        if constexpr (EPI == kEpiPcg) {
            __hip_atomic_store(B.partials + blockIdx.x, vals[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(B.partials + kPartialPitch + blockIdx.x, vals[1], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        const unsigned prev = atomicAdd(B.lcount + l, 1u);
        sLast = (prev == (unsigned)(ntiles - 1));
        if (sLast) __hip_atomic_store(B.lcount + l, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!sLast) return;
    __threadfence();

    const int m0 = n >> KF;
    T *cs = sm, *cd = sm + m0 * m0;
    for (int idx = threadIdx.x; idx < m0 * m0; idx += blockDim.x) cs[idx] = B.tmpA[(coff >> (2 * KF)) + idx];
    __syncthreads();
    rho = 0.0;
    mu = 0.0;
    for (int s = KF + 1; s <= J; ++s) {
        const int mi = n >> (s - 1), h = mi >> 1, msk = mi - 1, nq = h * h;
        const T ad = sAd[s];
        for (int base = 0; base < nq; base += 4 * kBlock) {
            T e0[4][4], e1[4][4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int qi = base + c * kBlock + (int)threadIdx.x;
                if (qi >= nq || NE == 0) continue;
                const int r = qi / h, q = qi - r * h;
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    if (o == 0 && s != J) continue;
                    prefetch<T, EPI>(B, E, band_index(coff, n, s, o, r, q), e0[c][o], e1[c][o]);
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int qi = base + c * kBlock + (int)threadIdx.x;
                if (qi >= nq) continue;
                const int r = qi / h, q = qi - r * h;
                int cols[6];
#pragma unroll
                for (int b = 0; b < 6; ++b) cols[b] = (2 * q + b) & msk;
                T ll = 0, lh = 0, hl = 0, hh = 0;
#pragma unroll
                for (int a = 0; a < 6; ++a) {
                    const T *row = cs + ((2 * r + a) & msk) * mi;
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
                const T w[4] = {ll, hl, lh, hh};
#pragma unroll
                for (int o = 1; o <= 3; ++o)
                    deliver<T, EPI>(B, E, band_index(coff, n, s, o, r, q), w[o], ad,
                                    EPI == kEpiPcg ? sJi[s * 4 + o] : (T)0, NE ? e0[c][o] : (T)0,
                                    NE == 2 ? e1[c][o] : (T)0, rho, mu);
                if (s == J)
                    deliver<T, EPI>(B, E, band_index(coff, n, s, 0, r, q), ll, ad, EPI == kEpiPcg ? sJi[s * 4] : (T)0,
                                    NE ? e0[c][0] : (T)0, NE == 2 ? e1[c][0] : (T)0, rho, mu);
                else
                    cd[r * h + q] = ll;
            }
        }
        __syncthreads();
        T *tmp = cs;
        cs = cd;
        cd = tmp;
    }
    if constexpr (EPI == kEpiPcg) {
        vals[0] = block_sum(rho, sh);
        vals[1] = block_sum(mu, sh);
        if (threadIdx.x == 0) {
            __hip_atomic_store(B.partials + nfine + l, vals[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(B.partials + kPartialPitch + nfine + l, vals[1], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            const unsigned prev = atomicAdd(&B.sc->counter, 1u);
            sLast = (prev == (unsigned)(nl - 1));
            if (sLast) {
                __threadfence();
                __hip_atomic_store(&B.sc->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
        if (!sLast) return;
        const double R = gather_partials(B.partials, kPartialPitch, 0, nfine + nl, sh);
        const double Mu = gather_partials(B.partials, kPartialPitch, 1, nfine + nl, sh);
        if (threadIdx.x == 0) pcg_scalars(B.sc, R, Mu, E.k, E.resnorm);
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
int Ops<T>::idwt(const T *c, T *out) const {
    InvArgs A{};
    A.src = c;
    A.out = out;
    k_inv<T, kInvPlain><<<(int)P.idwt_tiles.size(), kBlock, 0, st>>>(B, P.J, A, make_taps<T>());
    return check();
}

template <typename T>
int Ops<T>::idwt_first(const T *r, T *out) const {
    InvArgs A{};
    A.src = r;
    A.out = out;
    k_inv<T, kInvFirst><<<(int)P.idwt_tiles.size(), kBlock, 0, st>>>(B, P.J, A, make_taps<T>());
    return check();
}

template <typename T>
int Ops<T>::idwt_update(const T *r_old, const T *q_old, T *q_new, T *r_new, T *c, bool first_pass, T *out) const {
    InvArgs A{};
    A.src = r_old;
    A.out = out;
    A.yv = B.y;
    A.qold = first_pass ? B.y : q_old;  // never read on the first pass
    A.qnew = q_new;
    A.rnew = r_new;
    A.c = c;
    A.first_pass = first_pass ? 1 : 0;
    k_inv<T, kInvUpdate><<<(int)P.idwt_tiles.size(), kBlock, 0, st>>>(B, P.J, A, make_taps<T>());
    return check();
}

template <typename T>
template <int EPI>
int Ops<T>::fwd(const T *x, const FwdArgs &E) const {
    const int nf = (int)P.fine_tiles.size();
    const Taps<T> tp = make_taps<T>();
    switch (P.kf) {
        case 1: k_fwd<T, 1, 16, EPI><<<nf, kBlock, 0, st>>>(x, B, P.J, P.nl, E, tp); break;
        case 2: k_fwd<T, 2, 8, EPI><<<nf, kBlock, 0, st>>>(x, B, P.J, P.nl, E, tp); break;
        default: k_fwd<T, 3, 4, EPI><<<nf, kBlock, 0, st>>>(x, B, P.J, P.nl, E, tp); break;
    }
    return check();
}

template <typename T>
int Ops<T>::fdwt(const T *x, T *out) const {
    FwdArgs E{};
    E.out = out;
    return fwd<kEpiPlain>(x, E);
}

template <typename T>
int Ops<T>::fdwt_prior(const T *x, const T *cin, T *out) const {
    FwdArgs E{};
    E.out = out;
    E.cin = cin;
    return fwd<kEpiPrior>(x, E);
}

template <typename T>
int Ops<T>::fdwt_pcg(const T *x, const T *rk, int k, double *resnorm) const {
    FwdArgs E{};
    E.out = B.y;
    E.rk = rk;
    E.k = k;
    E.resnorm = resnorm;
    return fwd<kEpiPcg>(x, E);
}

template <typename T>
int Ops<T>::fdwt_rhs(const T *x, T *c, bool cold) const {
    FwdArgs E{};
    E.c = c;
    E.cold = cold ? 1 : 0;
    return fwd<kEpiRhs>(x, E);
}

template <typename T>
int Ops<T>::nodes(const T *in, T *v, int mode) const {
    const int tiles = (int)P.node_tiles.size();
    if (mode == kModeM) k_nodes_m<T><<<tiles, kBlock, 0, st>>>(in, v, B, P.nl);
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
int Ops<T>::update_last(T *c, const T *r_in, const T *q_old, T *q_new, bool first_pass) const {
    k_update_last<T><<<(int)P.coef_tiles.size(), kBlock, 0, st>>>(c, B, P.J, r_in, first_pass ? B.y : q_old, q_new,
                                                                    first_pass ? 1 : 0);
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
