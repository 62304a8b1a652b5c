// HIP kernels of the FEWHA hot path for gfx950 (CDNA4, wave64).
//
// Every stage is bandwidth/latency bound (no dense contraction anywhere), so the kernels are
// gather-only stencils: each output element is written by exactly one lane and results are
// bitwise reproducible run to run.  Device-scope atomics on a shared address serialise on this
// chip (tens of ns each), so the per-frame path uses none: reductions leave one FP64 partial
// per workgroup and the next kernel, which needs the Alg. 2 scalars anyway, sums them itself
// (every workgroup redundantly, in a fixed order, so all agree bit for bit).
//
//   k_inv          W^T (= W^-1) of every layer, all J levels in one launch: each workgroup owns
//                  a square output tile and rebuilds, from the coarsest level down, only the cone
//                  of coefficients that tile depends on, loaded in one batch into LDS.  Modes:
//                  plain c | z = J^-1 r | the Alg. 2 update of the previous pass fused in front.
//   k_nodes_m      per WFS node tile: P (bilinear ray gather from all layers through per-axis
//                  cell tables, LGS cone included), Gamma, C_eta^-1 and Gamma^T through LDS
//                  (the paper's Kernel-2 stage).  k_nodes: Gamma^T C s / Gamma^T mask s.
//   k_slopes       mask Gamma P u on subaperture tiles (forward operator A).
//   k_pt_tab       P^T as a gather per layer node through the transpose tables (the sensor nodes
//                  and weights that touch each layer grid line, the very entries P uses): the
//                  exact transpose of P without atomics.  k_pt_scan: same result by scanning
//                  the cell tables, for geometries whose transpose rows exceed the table width.
//   k_fwd_fine     the first kf levels of W for every layer, on tiles of level-kf quads with
//                  their halo in LDS; epilogues: alpha D z and the PCG dot-product partials, or
//                  the right-hand side's warm-restart residual update, or alpha D c.
//   k_fwd_coarse   the remaining levels, one workgroup per layer, LDS resident; same epilogues.
//   k_update_last  the last Alg. 2 update of a solve.
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
// Reductions and the Alg. 2 scalars
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

__device__ __forceinline__ void reset_scalars(Scalars *sc) {
    sc->rho = sc->mu = sc->rho_old = sc->alpha = sc->alpha_old = sc->beta = 0.0;
    sc->stopped = 0;
    sc->status = FEWHA_OK;
}

// One step of the Alg. 2 scalar recurrence for pass k from the reduced (rho, mu) and the state
// after pass k-1:  beta = rho / rho_old, alpha = rho / (mu - rho beta / alpha_old)  (first pass:
// beta = 0, alpha = rho / mu).  rho = 0 stops (exact solution); non-finite sums or a
// non-positive denominator stop with a status.  Returns the state after pass k.
__device__ Scalars alg2_step(const Scalars &prev, double R, double Mu, int k) {
    Scalars nx = prev;
    nx.rho = R;
    nx.mu = Mu;
    nx.alpha = 0.0;
    nx.beta = 0.0;
    if (prev.stopped) return nx;
    if (!isfinite(R) || !isfinite(Mu)) {
        nx.status = FEWHA_ERR_NONFINITE;
        nx.stopped = 1;
        return nx;
    }
    if (R == 0.0) {
        nx.stopped = 1;
        return nx;
    }
    double beta = 0.0, den = Mu;
    if (k > 0) {
        beta = R / prev.rho_old;
        den = Mu - R * beta / prev.alpha_old;
    }
    if (!(den > 0.0)) {
        nx.status = FEWHA_ERR_BREAKDOWN;
        nx.stopped = 1;
        return nx;
    }
    nx.alpha = R / den;
    nx.beta = beta;
    nx.rho_old = R;
    nx.alpha_old = nx.alpha;
    return nx;
}

// Every workgroup of a consumer kernel: sum the partials of pass k in fixed order, step the
// scalar recurrence from sc[(k-1)&1], and (workgroup 0) publish the new state to sc[k&1] and
// sqrt(rho) to resnorm[k].  Returns (alpha, beta, stopped) to all lanes.
struct StepOut {
    double alpha, beta;
    int stopped;
};

__device__ StepOut consume_pass(const double *__restrict__ partials, int nparts, Scalars *sc, int k, double *resnorm) {
    __shared__ double sh[16];
    __shared__ StepOut so;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        a += partials[i];
        b += partials[kPartialPitch + i];
    }
    const double R = block_sum(a, sh);
    const double Mu = block_sum(b, sh);
    if (threadIdx.x == 0) {
        const Scalars prev = sc[(k - 1) & 1];
        const Scalars nx = alg2_step(prev, R, Mu, k);
        so = StepOut{nx.alpha, nx.beta, nx.stopped};
        if (blockIdx.x == 0) {
            sc[k & 1] = nx;
            if (resnorm && !prev.stopped && isfinite(R)) resnorm[k] = sqrt(R);
        }
    }
    __syncthreads();
    return so;
}

// ---------------------------------------------------------------------------------------------
// W^T: multi-level inverse DWT in one launch, with the PCG update fused in front of it.
//
// The whole cone of a tile (every level, every band) is fetched in one batch of independent
// loads into LDS, then the J levels of synthesis run from LDS.  In the update mode the loads
// bring r_{k-1}, y_{k-1}, q_{k-2}; the Alg. 2 update of pass k-1 is evaluated for every cone
// coefficient, the coefficients this tile owns are written back (p, q, c and the new residual),
// and the transform runs on z = J^-1 r_k.  Ownership: at level s a tile owns the indices
// [y0 >> s, (y0 + T0) >> s) when T0 >= 2^s, else index y0 >> s if y0 is a multiple of 2^s
// (likewise in x), which partitions every band.
// ---------------------------------------------------------------------------------------------
constexpr int kInvBlock = 512;
constexpr int kInvSegMax = 4096;  // cone of a 32 x 32 tile, rows padded to power-of-two pitches

// ceil(log2(v)) for 1 <= v <= 2^30
__device__ __forceinline__ int clog2(int v) { return v <= 1 ? 0 : 32 - __clz(v - 1); }

template <typename T, int MODE>
__global__ __launch_bounds__(kInvBlock) void k_inv(Bufs<T> B, int J, InvArgs A, Taps<T> tp) {
    constexpr int TILE = kIdwtTile;
    constexpr int MAXI = kInvSegMax / kInvBlock;
    __shared__ T sSeg[kInvSegMax];
    __shared__ T sL0[(TILE / 2 + 2) * TILE], sL1[(TILE / 2 + 2) * TILE];  // level-1 rows x pitch 32
    __shared__ T sAX[TILE * TILE], sDX[TILE * TILE];
    __shared__ int shLoY[kMaxJ + 1], shLoX[kMaxJ + 1], shLnY[kMaxJ + 1], shLnX[kMaxJ + 1], shLp[kMaxJ + 1];
    __shared__ int shSeg[kMaxJ + 2];
    __shared__ T sJinv[(kMaxJ + 1) * 4];

    const Tile t = B.idwt_tiles[blockIdx.x];
    const int l = t.a, y0 = t.b, x0 = t.c, T0 = t.d, n = t.f;
    const long coff = t.e;
    // Cone bounds per level, computed by every lane in registers (uniform values).  Each band
    // region is stored with rows padded to a power-of-two pitch, so decoding an item needs only
    // compares and shifts.
    int loY[kMaxJ + 1], loX[kMaxJ + 1], lnY[kMaxJ + 1], lnX[kMaxJ + 1], lp[kMaxJ + 1], seg[kMaxJ + 2];
    {
        int ly = y0, hy = y0 + T0 - 1, lx = x0, hx = x0 + T0 - 1, off = 0;
        loY[0] = ly;
        loX[0] = lx;
        lnY[0] = T0;
        lnX[0] = T0;
        lp[0] = clog2(T0);
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
            lp[s] = clog2(lnX[s]);
            seg[s] = off;
            if (s <= J) off += 3 * (lnY[s] << lp[s]);
        }
        seg[kMaxJ + 1] = off;  // the coarsest LL starts here
    }
    int lnYJ = 0, lpJ = 0;
#pragma unroll
    for (int s = 1; s <= kMaxJ; ++s)
        if (s == J) {
            lnYJ = lnY[s];
            lpJ = lp[s];
        }
    const int llOff = seg[kMaxJ + 1], total = llOff + (lnYJ << lpJ);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s <= kMaxJ; ++s) {
            shLoY[s] = loY[s];
            shLoX[s] = loX[s];
            shLnY[s] = lnY[s];
            shLnX[s] = lnX[s];
            shLp[s] = lp[s];
            shSeg[s] = seg[s];
        }
        shSeg[kMaxJ + 1] = llOff;
    }
    if (MODE != kInvPlain && threadIdx.x < (J + 1) * 4) sJinv[threadIdx.x] = B.jinv[l * (J + 1) * 4 + threadIdx.x];

    double alpha = 0.0, beta = 0.0;
    int stopped = 0;
    if constexpr (MODE == kInvUpdate) {
        const StepOut so = consume_pass(B.partials, A.nparts, B.sc, A.kprev, A.resnorm);
        alpha = so.alpha;
        beta = so.beta;
        stopped = so.stopped;
    }
    const T *__restrict__ src = static_cast<const T *>(A.src);
    const T *__restrict__ yin = static_cast<const T *>(A.yv);
    const T *__restrict__ qin = static_cast<const T *>(A.qold);
    T *__restrict__ pio = B.p;
    T *__restrict__ cio = static_cast<T *>(A.c);
    __syncthreads();
    // ---- one batch of independent loads: the whole cone (plus owned-only operands) ----
    for (int base = 0; base < total; base += MAXI * kInvBlock) {
        long gi[MAXI];
        int bnd[MAXI];
        bool own[MAXI];
        T rv[MAXI], yv[MAXI], qv[MAXI], pv[MAXI], cv[MAXI];
#pragma unroll
        for (int c = 0; c < MAXI; ++c) {
            const int k = base + c * kInvBlock + (int)threadIdx.x;
            gi[c] = -1;
            own[c] = false;
            if (k >= total) continue;
            // level (compare chain over uniform offsets), band, row, column (shifts)
            int s = J, o = 0, ly = 0, lx = 0, nxs = 1, lps = 0, rem = k - llOff;
#pragma unroll
            for (int ss = 1; ss <= kMaxJ; ++ss) {
                if (ss <= J && k >= seg[ss] && k < seg[ss + 1 <= kMaxJ ? ss + 1 : kMaxJ + 1]) s = ss;
            }
#pragma unroll
            for (int ss = 1; ss <= kMaxJ; ++ss)
                if (ss == s) {
                    ly = loY[ss];
                    lx = loX[ss];
                    nxs = lnX[ss];
                    lps = lp[ss];
                }
            if (k < llOff) {
                int lny = 0, sg = 0;
#pragma unroll
                for (int ss = 1; ss <= kMaxJ; ++ss)
                    if (ss == s) {
                        lny = lnY[ss];
                        sg = seg[ss];
                    }
                const int bsz = lny << lps, kk = k - sg;
                o = 1 + (kk >= bsz) + (kk >= 2 * bsz);
                rem = kk - (o - 1) * bsz;
            }
            const int r = rem >> lps, q = rem & ((1 << lps) - 1);
            if (q >= nxs) continue;  // row padding
            const int m = n >> s, msk = m - 1;
            const int uy = ly + r, ux = lx + q;
            const int gr = uy & msk, gc = ux & msk;
            const int row = gr + ((o == 2 || o == 3) ? m : 0), col = gc + ((o == 1 || o == 3) ? m : 0);
            gi[c] = coff + (long)row * n + col;
            bnd[c] = s * 4 + o;
            if constexpr (MODE == kInvUpdate) {
                const int ts = T0 >> s, msk2 = (1 << s) - 1;
                const bool oy = ts >= 1 ? (uy >= (y0 >> s) && uy < (y0 >> s) + ts) : ((y0 & msk2) == 0 && uy == (y0 >> s));
                const bool ox = ts >= 1 ? (ux >= (x0 >> s) && ux < (x0 >> s) + ts) : ((x0 & msk2) == 0 && ux == (x0 >> s));
                own[c] = oy && ox;
            }
            rv[c] = src[gi[c]];
            if constexpr (MODE == kInvUpdate) {
                yv[c] = yin[gi[c]];
                qv[c] = A.first_pass ? (T)0 : qin[gi[c]];
                if (own[c]) {
                    pv[c] = A.first_pass ? (T)0 : pio[gi[c]];
                    cv[c] = cio[gi[c]];
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
                        pio[gi[c]] = pn;
                        static_cast<T *>(A.qnew)[gi[c]] = qn;
                        cio[gi[c]] = cv[c] + (T)alpha * pn;
                    }
                }
                if (own[c]) static_cast<T *>(A.rnew)[gi[c]] = rn;
                val = rn * ji;
            }
            sSeg[base + c * kInvBlock + (int)threadIdx.x] = val;
        }
    }
    __syncthreads();

    // ---- synthesis from the coarsest level, all in LDS (power-of-two row pitches) ----
    const T *LL = sSeg + llOff;
    int llp = lpJ;
    T *NX = sL0;
    T *__restrict__ outp = static_cast<T *>(A.out);
    for (int s = J; s >= 1; --s) {
        const int ny = shLnY[s - 1], nxk = shLnX[s], nx = shLnX[s - 1];
        const int oy = shLoY[s - 1], ky = shLoY[s], ox = shLoX[s - 1], kx = shLoX[s];
        const int bp = shLp[s], op = shLp[s - 1];
        const int bsz = shLnY[s] << bp;
        const T *HL = sSeg + shSeg[s], *LH = HL + bsz, *HH = LH + bsz;
        // undo the y analysis: (LL, x-low/y-high) -> x-low rows, (x-high/y-low, HH) -> x-high rows
        for (int idx = threadIdx.x; idx < (ny << bp); idx += blockDim.x) {
            const int r = idx >> bp, q = idx & ((1 << bp) - 1);
            if (q >= nxk) continue;
            const int y = oy + r, p = y & 1, kb = (y >> 1) - ky;
            T a = 0, d = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int rr = kb - j;
                a += tp.h[p + 2 * j] * LL[(rr << llp) + q] + tp.g[p + 2 * j] * LH[(rr << bp) + q];
                d += tp.h[p + 2 * j] * HL[(rr << bp) + q] + tp.g[p + 2 * j] * HH[(rr << bp) + q];
            }
            sAX[idx] = a;
            sDX[idx] = d;
        }
        __syncthreads();
        // undo the x analysis
        for (int idx = threadIdx.x; idx < (ny << op); idx += blockDim.x) {
            const int r = idx >> op, q = idx & ((1 << op) - 1);
            if (q >= nx) continue;
            const int x = ox + q, p = x & 1, kb = (x >> 1) - kx;
            T v = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int at = (r << bp) + kb - j;
                v += tp.h[p + 2 * j] * sAX[at] + tp.g[p + 2 * j] * sDX[at];
            }
            if (s > 1) NX[idx] = v;
            else outp[coff + (long)(oy + r) * n + ox + q] = v;
        }
        __syncthreads();
        LL = NX;
        llp = op;
        NX = (NX == sL0) ? sL1 : sL0;
    }
}

// Last Alg. 2 update of a solve (elementwise); the residual lands in the state buffer B.r.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_last(T *__restrict__ c, Bufs<T> B, int J, const T *__restrict__ rin,
                                                        const T *__restrict__ qold, T *__restrict__ qnew, int first,
                                                        int nparts, int kprev, double *resnorm) {
    constexpr int E = kCoefTile / kBlock;
    __shared__ T sJ[(kMaxJ + 1) * 4];
    const Tile t = B.coef_tiles[blockIdx.x];
    if (threadIdx.x < (J + 1) * 4) sJ[threadIdx.x] = B.jinv[t.a * (J + 1) * 4 + threadIdx.x];
    const StepOut so = consume_pass(B.partials, nparts, B.sc, kprev, resnorm);
    T *__restrict__ pp = B.p;
    T *__restrict__ rr = B.r;
    const T *__restrict__ yy = B.y;
    T rv[E], pv[E], yv[E], qv[E], cv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int loc = t.b + e * kBlock + (int)threadIdx.x;
        if (loc >= t.b + t.c) continue;
        const long i = t.e + loc;
        rv[e] = rin[i];
        yv[e] = yy[i];
        cv[e] = c[i];
        pv[e] = first ? (T)0 : pp[i];
        qv[e] = first ? (T)0 : qold[i];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int loc = t.b + e * kBlock + (int)threadIdx.x;
        if (loc >= t.b + t.c) continue;
        const long i = t.e + loc;
        if (so.stopped) {
            rr[i] = rv[e];
            continue;
        }
        int s, o;
        band_at(loc >> t.g, loc & (t.f - 1), t.f, t.g, J, s, o);
        const T z = rv[e] * sJ[s * 4 + o];
        const T p = first ? z : z + (T)so.beta * pv[e];
        const T q = first ? yv[e] : yv[e] + (T)so.beta * qv[e];
        pp[i] = p;
        qnew[i] = q;
        c[i] = cv[e] + (T)so.alpha * p;
        rr[i] = rv[e] - (T)so.alpha * q;
    }
}

// ---------------------------------------------------------------------------------------------
// Node-tile kernels (Kernel-2 stage): P, Gamma, C_eta^-1, Gamma^T.
// ---------------------------------------------------------------------------------------------
constexpr int kNodeBlock = 512;

// y-part of M on one node tile: phi on the tile plus a one-node halo (one node per lane), then
// weighted Fried slopes and Gamma^T from LDS.  The cell-table entries of the tile's rows and
// columns are staged in LDS per chunk of layers; each lane then issues the bilinear loads of
// eight layers at a time before accumulating them in layer order.
template <typename T>
__global__ __launch_bounds__(kNodeBlock) void k_nodes_m(const T *__restrict__ u, T *__restrict__ v, Bufs<T> B,
                                                        int nl) {
    constexpr int NT = kNodeTile, NP = NT + 2, NS = NT + 1, LMAX = 16, LCH = 8;
    __shared__ int sXk[LMAX * NP], sYk[LMAX * NP];
    __shared__ T sXw0[LMAX * NP], sXw1[LMAX * NP], sYw0[LMAX * NP], sYw1[LMAX * NP];
    __shared__ long sOff[LMAX];
    __shared__ int sN[LMAX];
    __shared__ T sPhi[NP * NP];
    __shared__ T sSx[NS * NS], sSy[NS * NS];
    const Tile t = B.node_tiles[blockIdx.x];
    const DevWfs W = B.wfs[t.a];
    const int g = t.a, ns = W.n_sub, nv = W.nv, i0 = t.b, j0 = t.c;
    const int a = (int)threadIdx.x / NP, b = (int)threadIdx.x - a * NP, i = i0 - 1 + a, j = j0 - 1 + b;
    const bool node = threadIdx.x < NP * NP && i >= 0 && i <= ns && j >= 0 && j <= ns;
    const Ent<T> *__restrict__ xt = B.xtab + (long)g * nl * B.maxnv;
    const Ent<T> *__restrict__ yt = B.ytab + (long)g * nl * B.maxnv;
    T phi = 0;
    for (int l0 = 0; l0 < nl; l0 += LMAX) {
        const int nc = (nl - l0) < LMAX ? (nl - l0) : LMAX;
        for (int idx = threadIdx.x; idx < 2 * nc * NP; idx += blockDim.x) {
            const int axis = idx / (nc * NP), rem = idx - axis * nc * NP, l = rem / NP, bb = rem - l * NP;
            int nd = (axis ? i0 : j0) - 1 + bb;
            nd = nd < 0 ? 0 : (nd > ns ? ns : nd);
            const Ent<T> e = (axis ? yt : xt)[(long)(l0 + l) * B.maxnv + nd];
            if (axis) {
                sYk[rem] = e.k0;
                sYw0[rem] = e.w0;
                sYw1[rem] = e.w1;
            } else {
                sXk[rem] = e.k0;
                sXw0[rem] = e.w0;
                sXw1[rem] = e.w1;
            }
        }
        if (threadIdx.x < nc) {
            sOff[threadIdx.x] = B.lay[l0 + threadIdx.x].c_off;
            sN[threadIdx.x] = B.lay[l0 + threadIdx.x].n;
        }
        __syncthreads();
        if (node) {
            for (int lc = 0; lc < nc; lc += LCH) {
                T uv[LCH][4], wy0[LCH], wy1[LCH], wx0[LCH], wx1[LCH];
#pragma unroll
                for (int c = 0; c < LCH; ++c) {
                    const int l = lc + c;
                    const bool ok = l < nc;
                    const int xs = ok ? l * NP + b : 0, ys = ok ? l * NP + a : 0;
                    const int n = ok ? sN[l] : 0;
                    wx0[c] = ok ? sXw0[xs] : (T)0;
                    wx1[c] = ok ? sXw1[xs] : (T)0;
                    wy0[c] = ok ? sYw0[ys] : (T)0;
                    wy1[c] = ok ? sYw1[ys] : (T)0;
                    const T *U = u + (ok ? sOff[l] + (long)sYk[ys] * n + sXk[xs] : 0);
                    uv[c][0] = U[0];
                    uv[c][1] = ok ? U[1] : (T)0;
                    uv[c][2] = ok ? U[n] : (T)0;
                    uv[c][3] = ok ? U[n + 1] : (T)0;
                }
#pragma unroll
                for (int c = 0; c < LCH; ++c)
                    phi += (wy0[c] * wx0[c]) * uv[c][0] + (wy0[c] * wx1[c]) * uv[c][1] + (wy1[c] * wx0[c]) * uv[c][2] +
                           (wy1[c] * wx1[c]) * uv[c][3];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < NP * NP) sPhi[threadIdx.x] = node ? phi : (T)0;
    __syncthreads();
    if (threadIdx.x < NS * NS) {
        const int aa = threadIdx.x / NS, bb = threadIdx.x - aa * NS, ii = i0 - 1 + aa, jj = j0 - 1 + bb;
        T sx = 0, sy = 0;
        if (ii >= 0 && ii < ns && jj >= 0 && jj < ns && subap_active(W, ii, jj)) {
            const T w = (T)W.inv_var;
            const T p00 = sPhi[aa * NP + bb], p01 = sPhi[aa * NP + bb + 1];
            const T p10 = sPhi[(aa + 1) * NP + bb], p11 = sPhi[(aa + 1) * NP + bb + 1];
            sx = w * ((T)0.5 * ((p01 - p00) + (p11 - p10)));
            sy = w * ((T)0.5 * ((p10 - p00) + (p11 - p01)));
        }
        sSx[threadIdx.x] = sx;
        sSy[threadIdx.x] = sy;
    }
    __syncthreads();
    if (threadIdx.x < NT * NT) {
        const int aa = threadIdx.x / NT, bb = threadIdx.x - aa * NT, ii = i0 + aa, jj = j0 + bb;
        if (ii <= ns && jj <= ns) {
            // node (i, j) is a corner of subapertures (i, j), (i, j-1), (i-1, j), (i-1, j-1)
            const int s11 = (aa + 1) * NS + (bb + 1), s10 = (aa + 1) * NS + bb, s01 = aa * NS + (bb + 1), s00 = aa * NS + bb;
            v[W.v_off + (long)ii * nv + jj] = (T)0.5 * ((-sSx[s11] - sSy[s11]) + (sSx[s10] - sSy[s10]) +
                                                        (-sSx[s01] + sSy[s01]) + (sSx[s00] + sSy[s00]));
        }
    }
}

// Gamma^T C s (MODE kModeRhs) or Gamma^T mask s (kModeAdj) on one node tile.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_nodes(const T *__restrict__ in, T *__restrict__ v, Bufs<T> B) {
    constexpr int NT = kNodeTile, NS = NT + 1;
    __shared__ T sSx[NS * NS], sSy[NS * NS];
    const Tile t = B.node_tiles[blockIdx.x];
    const DevWfs W = B.wfs[t.a];
    const int ns = W.n_sub, nv = W.nv, i0 = t.b, j0 = t.c;
    for (int idx = threadIdx.x; idx < NS * NS; idx += blockDim.x) {
        const int a = idx / NS, b = idx - a * NS, i = i0 - 1 + a, j = j0 - 1 + b;
        T sx = 0, sy = 0;
        if (i >= 0 && i < ns && j >= 0 && j < ns && subap_active(W, i, j)) {
            const T w = (MODE == kModeAdj) ? (T)1 : (T)W.inv_var;
            sx = w * in[W.s_off + (long)i * ns + j];
            sy = w * in[W.s_off + (long)ns * ns + (long)i * ns + j];
        }
        sSx[idx] = sx;
        sSy[idx] = sy;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NT * NT; idx += blockDim.x) {
        const int a = idx / NT, b = idx - a * NT, i = i0 + a, j = j0 + b;
        if (i > ns || j > ns) continue;
        const int s11 = (a + 1) * NS + (b + 1), s10 = (a + 1) * NS + b, s01 = a * NS + (b + 1), s00 = a * NS + b;
        v[W.v_off + (long)i * nv + j] = (T)0.5 * ((-sSx[s11] - sSy[s11]) + (sSx[s10] - sSy[s10]) +
                                                  (-sSx[s01] + sSy[s01]) + (sSx[s00] + sSy[s00]));
    }
}

// s = mask Gamma P u on subaperture tiles.
template <typename T>
__global__ __launch_bounds__(kNodeBlock) void k_slopes(const T *__restrict__ u, T *__restrict__ s, Bufs<T> B, int nl) {
    constexpr int NT = kNodeTile, NP = NT + 1;
    __shared__ T sPhi[NP * NP];
    const Tile t = B.sub_tiles[blockIdx.x];
    const DevWfs W = B.wfs[t.a];
    const int ns = W.n_sub, i0 = t.b, j0 = t.c;
    if (threadIdx.x < NP * NP) {
        const int a = threadIdx.x / NP, b = threadIdx.x - a * NP, i = i0 + a, j = j0 + b;
        T val = 0;
        if (i <= ns && j <= ns) val = project_node(u, B, t.a, nl, i, j);
        sPhi[threadIdx.x] = val;
    }
    __syncthreads();
    if (threadIdx.x < NT * NT) {
        const int a = threadIdx.x / NT, b = threadIdx.x - a * NT, i = i0 + a, j = j0 + b;
        if (i < ns && j < ns) {
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
}

// ---------------------------------------------------------------------------------------------
// P^T
// ---------------------------------------------------------------------------------------------
// Through the transpose tables: for each sensor, the tile rows' and columns' (node, weight)
// lists are staged in LDS (structure of arrays, entry-major, so the 16 lanes of a tile row read
// consecutive words); each lane then gathers the v values of its node's non-zero pairs, two
// sensors' loads in flight at a time.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pt_tab(const T *__restrict__ v, T *__restrict__ x, Bufs<T> B, int nl,
                                                   int nw) {
    constexpr int NT = kNodeTile, RW = kRtabWidth, GMAX = 16, GCH = 2;
    constexpr int NSTAGE = 2 * GMAX * NT * RW, MAXI = NSTAGE / kBlock;
    static_assert(NT == 16 && RW == 4 && kBlock == 256, "index arithmetic below assumes these sizes");
    __shared__ int sIdx[NSTAGE];  // [axis][g][entry][line]
    __shared__ T sW[NSTAGE];
    __shared__ long sVoff[GMAX];
    __shared__ int sNv[GMAX];
    const Tile t = B.lay_tiles[blockIdx.x];
    const int k0 = t.b, q0 = t.c, n = t.f, roff = t.h;
    const int rk = (int)(threadIdx.x >> 4), rq = (int)(threadIdx.x & 15);
    const bool valid = k0 + rk < n && q0 + rq < n;
    const RtabEnt<T> *__restrict__ xrt = B.xrtab;
    const RtabEnt<T> *__restrict__ yrt = B.yrtab;
    T acc = 0;
    for (int gb = 0; gb < nw; gb += GMAX) {
        const int gc = (nw - gb) < GMAX ? (nw - gb) : GMAX;
        {
            int id[MAXI];
            T w[MAXI];
#pragma unroll
            for (int c = 0; c < MAXI; ++c) {
                // staged slot e = (((axis * 16 + g) * 4 + entry) * 16 + line); loads are read in
                // (line, entry) order for coalescing
                const int e = c * kBlock + (int)threadIdx.x;
                const int axis = e >> 10, g = (e >> 6) & 15, line = (e >> 2) & 15, entry = e & 3;
                const int gl = (axis ? k0 : q0) + line;
                RtabEnt<T> en{0, (T)0};
                if (g < gc && gl < n) en = (axis ? yrt : xrt)[((long)(gb + g) * B.sum_n + roff + gl) * RW + entry];
                id[c] = en.idx;
                w[c] = en.w;
            }
#pragma unroll
            for (int c = 0; c < MAXI; ++c) {
                const int e = c * kBlock + (int)threadIdx.x;
                const int axis = e >> 10, g = (e >> 6) & 15, line = (e >> 2) & 15, entry = e & 3;
                const int slot = (((axis * GMAX + g) * RW + entry) * NT) + line;
                sIdx[slot] = id[c];
                sW[slot] = w[c];
            }
        }
        if (threadIdx.x < gc) {
            sVoff[threadIdx.x] = B.wfs[gb + threadIdx.x].v_off;
            sNv[threadIdx.x] = B.wfs[gb + threadIdx.x].nv;
        }
        __syncthreads();
        if (valid) {
            for (int g0 = 0; g0 < gc; g0 += GCH) {
                T val[GCH][RW][RW], wy[GCH][RW], wx[GCH][RW];
#pragma unroll
                for (int gg = 0; gg < GCH; ++gg) {
                    const int g = g0 + gg;
                    int iy[RW], ix[RW];
#pragma unroll
                    for (int a = 0; a < RW; ++a) {
                        const int sy = ((GMAX + g) * RW + a) * NT + rk, sx = (g * RW + a) * NT + rq;
                        iy[a] = g < gc ? sIdx[sy] : 0;
                        wy[gg][a] = g < gc ? sW[sy] : (T)0;
                        ix[a] = g < gc ? sIdx[sx] : 0;
                        wx[gg][a] = g < gc ? sW[sx] : (T)0;
                    }
                    const T *vg = v + (g < gc ? sVoff[g] : 0);
                    const int nv = g < gc ? sNv[g] : 0;
#pragma unroll
                    for (int a = 0; a < RW; ++a)
#pragma unroll
                        for (int b = 0; b < RW; ++b)
                            val[gg][a][b] = (wy[gg][a] != (T)0 && wx[gg][b] != (T)0) ? vg[(long)iy[a] * nv + ix[b]] : (T)0;
                }
#pragma unroll
                for (int gg = 0; gg < GCH; ++gg)
#pragma unroll
                    for (int a = 0; a < RW; ++a)
#pragma unroll
                        for (int b = 0; b < RW; ++b) acc += (wy[gg][a] * wx[gg][b]) * val[gg][a][b];
            }
        }
        __syncthreads();
    }
    if (valid) x[(long)t.e + (long)(k0 + rk) * n + q0 + rq] = acc;
}

// By scanning the cell tables over each layer node's contiguous node ranges (any geometry).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pt_scan(const T *__restrict__ v, T *__restrict__ x, Bufs<T> B, int nl,
                                                    int nw) {
    constexpr int NT = kNodeTile;
    const Tile t = B.lay_tiles[blockIdx.x];
    const int l = t.a, k = t.b + (int)(threadIdx.x / NT), q = t.c + (int)(threadIdx.x % NT), n = t.f;
    if (k >= n || q >= n) return;
    T acc = 0;
    for (int g = 0; g < nw; ++g) {
        const Range rx = B.xrng[(long)g * B.sum_n + t.h + q];
        const Range ry = B.yrng[(long)g * B.sum_n + t.h + k];
        if (rx.lo > rx.hi || ry.lo > ry.hi) continue;
        const Ent<T> *xt = B.xtab + ((long)g * nl + l) * B.maxnv;
        const Ent<T> *yt = B.ytab + ((long)g * nl + l) * B.maxnv;
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
    x[(long)t.e + (long)k * n + q] = acc;
}

// ---------------------------------------------------------------------------------------------
// Forward transform W with fused epilogues.
// ---------------------------------------------------------------------------------------------
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

// Region geometry of the fine part: a tile of TQ x TQ level-KF approximation coefficients needs
// LL_s on a run of len(s) = TQ 2^(KF-s) + 4 (2^(KF-s) - 1) indices (s = 0 is the input).
template <int KF, int TQ>
struct FineGeom {
    static constexpr int len(int s) { return TQ * (1 << (KF - s)) + 4 * ((1 << (KF - s)) - 1); }
};

// Levels 1..KF on a tile of TQ x TQ level-KF approximation coefficients: the input region with
// its halo (periodic wrap) and the epilogue operands of every owned coefficient arrive in one
// batch of independent loads, then the levels run from LDS.
constexpr int kFwdBlock = 512;

template <typename T, int KF, int TQ, int EPI>
__global__ __launch_bounds__(kFwdBlock) void k_fwd_fine(const T *__restrict__ x, Bufs<T> B, int J, FwdArgs E,
                                                     Taps<T> tp) {
    using G = FineGeom<KF, TQ>;
    constexpr int L0 = G::len(0), L1 = G::len(1), EMAX = 1024;
    constexpr int NE = (EPI == kEpiRhs) ? 2 : ((EPI == kEpiPlain) ? 0 : 1);
    constexpr int MAXI = 6;
    __shared__ T sA[L0 * L0];
    __shared__ T sB[KF >= 2 ? L1 * L1 : 1];
    __shared__ T sE0[NE >= 1 ? EMAX : 1], sE1[NE >= 2 ? EMAX : 1];
    __shared__ T sAd[kMaxJ + 1], sJi[(kMaxJ + 1) * 4];
    __shared__ double sh[kFwdBlock / 64];

    if constexpr (EPI == kEpiRhs) {
        if (blockIdx.x == 0 && threadIdx.x == 0) reset_scalars(B.sc + 1);  // state "before pass 0"
    }
    const Tile t = B.fine_tiles[blockIdx.x];
    const int l = t.a, qy = t.b, qx = t.c, tq = t.d, n = t.f;
    const long coff = t.e;
    if ((EPI == kEpiPrior || EPI == kEpiPcg) && threadIdx.x <= J) sAd[threadIdx.x] = B.ad[l * (J + 1) + threadIdx.x];
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
    {
        const int nreg = len[0] * len[0], tot = nreg + (NE ? ne : 0);
        for (int base = 0; base < tot; base += MAXI * kFwdBlock) {
            T v0[MAXI], v1[MAXI];
            int d[MAXI];
#pragma unroll
            for (int c = 0; c < MAXI; ++c) {
                const int k = base + c * kFwdBlock + (int)threadIdx.x;
                d[c] = -1;
                if (k >= tot) continue;
                if (k < nreg) {
                    const int r = k / len[0], q = k - r * len[0];
                    v0[c] = x[coff + (long)((oy + r) & nmask) * n + ((ox + q) & nmask)];
                    d[c] = r * L0 + q;
                } else {
                    const int e = k - nreg;
                    int s = 1;
#pragma unroll
                    for (int ss = 2; ss <= KF; ++ss)
                        if (e >= eoff[ss]) s = ss;
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
                    T a0 = 0, a1 = 0;
                    prefetch<T, EPI>(B, E, band_index(coff, n, s, o, (qy << (KF - s)) + r, (qx << (KF - s)) + q), a0,
                                     a1);
                    v0[c] = a0;
                    v1[c] = a1;
                    d[c] = L0 * L0 + e;
                }
            }
#pragma unroll
            for (int c = 0; c < MAXI; ++c) {
                if (d[c] < 0) continue;
                if (d[c] < L0 * L0) sA[d[c]] = v0[c];
                else {
                    if constexpr (NE >= 1) sE0[d[c] - L0 * L0] = v0[c];
                    if constexpr (NE >= 2) sE1[d[c] - L0 * L0] = v1[c];
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
        const T ad = (EPI == kEpiPrior || EPI == kEpiPcg) ? sAd[s] : (T)0;
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
                    T e0 = 0, e1 = 0;
                    if constexpr (NE >= 1) e0 = sE0[ei];
                    if constexpr (NE >= 2) e1 = sE1[ei];
                    deliver<T, EPI>(B, E, band_index(coff, n, s, o, by + r, bx + q), w[o - 1], ad,
                                    EPI == kEpiPcg ? sJi[s * 4 + o] : (T)0, e0, e1, rho, mu);
                }
                if (s == KF) {
                    if (KF == J) {
                        const int ei = eoff[KF + 1] + r * ow + q;
                        T e0 = 0, e1 = 0;
                        if constexpr (NE >= 1) e0 = sE0[ei];
                        if constexpr (NE >= 2) e1 = sE1[ei];
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
    if constexpr (EPI == kEpiPcg) {
        const double a = block_sum(rho, sh), b = block_sum(mu, sh);
        if (threadIdx.x == 0) {
            B.partials[blockIdx.x] = a;
            B.partials[kPartialPitch + blockIdx.x] = b;
        }
    }
}

// Levels KF+1..J of one layer per workgroup: the level-KF approximation (from tmpA) and the
// epilogue operands of the layer's top-left m0 x m0 block (exactly the coefficients of these
// levels) arrive in one batch of loads, then the levels run from LDS (dynamic shared memory:
// (1 + 1/4 + NE) m0^2 values).
template <typename T, int EPI>
__global__ __launch_bounds__(512) void k_fwd_coarse(Bufs<T> B, int J, int KF, FwdArgs E, Taps<T> tp, int nfine) {
    extern __shared__ char smem_raw[];
    constexpr int NE = (EPI == kEpiRhs) ? 2 : ((EPI == kEpiPlain) ? 0 : 1);
    __shared__ T sAd[kMaxJ + 1], sJi[(kMaxJ + 1) * 4];
    __shared__ double sh[512 / 64];
    const int l = blockIdx.x;
    const DevLayer L = B.lay[l];
    const int n = L.n, m0 = n >> KF;
    const long coff = L.c_off;
    T *cs = reinterpret_cast<T *>(smem_raw), *cd = cs + m0 * m0, *e0s = cd + (m0 * m0) / 4 + 1, *e1s = e0s + m0 * m0;
    if ((EPI == kEpiPrior || EPI == kEpiPcg) && threadIdx.x <= J) sAd[threadIdx.x] = B.ad[l * (J + 1) + threadIdx.x];
    if (EPI == kEpiPcg && threadIdx.x < (J + 1) * 4) sJi[threadIdx.x] = B.jinv[l * (J + 1) * 4 + threadIdx.x];
    const int lm = L.log2n - KF;
    const T *__restrict__ llin = B.tmpA + (coff >> (2 * KF));
    for (int base = 0; base < m0 * m0; base += 8 * 512) {
        T cv[8], a0v[8], a1v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int idx = base + c * 512 + (int)threadIdx.x;
            a0v[c] = 0;
            a1v[c] = 0;
            if (idx >= m0 * m0) continue;
            prefetch<T, EPI>(B, E, coff + (long)(idx >> lm) * n + (idx & (m0 - 1)), a0v[c], a1v[c]);
            cv[c] = llin[idx];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int idx = base + c * 512 + (int)threadIdx.x;
            if (idx >= m0 * m0) continue;
            cs[idx] = cv[c];
            if constexpr (NE >= 1) e0s[idx] = a0v[c];
            if constexpr (NE >= 2) e1s[idx] = a1v[c];
        }
    }
    __syncthreads();
    double rho = 0.0, mu = 0.0;
    for (int s = KF + 1; s <= J; ++s) {
        const int mi = n >> (s - 1), h = mi >> 1, msk = mi - 1, nq = h * h, lh = L.log2n - s;
        const T ad = (EPI == kEpiPrior || EPI == kEpiPcg) ? sAd[s] : (T)0;
        for (int qi = threadIdx.x; qi < nq; qi += blockDim.x) {
            const int r = qi >> lh, q = qi & (h - 1);
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
            for (int o = 0; o <= 3; ++o) {
                if (o == 0 && s != J) continue;
                const int lr = r + ((o == 2 || o == 3) ? h : 0), lc = q + ((o == 1 || o == 3) ? h : 0);
                const int li = (lr << lm) + lc;
                T e0 = 0, e1 = 0;
                if constexpr (NE >= 1) e0 = e0s[li];
                if constexpr (NE >= 2) e1 = e1s[li];
                deliver<T, EPI>(B, E, coff + (long)lr * n + lc, w[o], ad, EPI == kEpiPcg ? sJi[s * 4 + o] : (T)0, e0,
                                e1, rho, mu);
            }
            if (s != J) cd[r * h + q] = ll;
        }
        __syncthreads();
        T *tmp = cs;
        cs = cd;
        cd = tmp;
    }
    if constexpr (EPI == kEpiPcg) {
        const double a = block_sum(rho, sh), b = block_sum(mu, sh);
        if (threadIdx.x == 0) {
            B.partials[nfine + l] = a;
            B.partials[kPartialPitch + nfine + l] = b;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Setup and small kernels
// ---------------------------------------------------------------------------------------------
// Weighted squared norm sum_k C_eta^-1_k s_k^2 (preconditioner probes): one partial per block.
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
    const double v = block_sum(acc, sh);
    if (threadIdx.x == 0) B.partials[blockIdx.x] = v;
}

// Sum of n partials in fixed order -> sc[2].rho (single workgroup).
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double *__restrict__ partials, int n, Scalars *sc) {
    __shared__ double sh[kBlock / 64];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += partials[i];
    const double t = block_sum(a, sh);
    if (threadIdx.x == 0) sc[2].rho = t;
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

// Transpose of the cell tables: for grid line q of layer l, the sensor nodes j whose cell
// touches it (k0_j in {q-1, q}; contiguous since k0_j is non-decreasing in j) as a range, and as
// a zero-padded list of (j, weight) pairs of width kRtabWidth; lines with more pairs than that
// set over[g] (the plan then uses the scanning transpose).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_build_ranges(Range *xrng, Range *yrng, RtabEnt<T> *xrt, RtabEnt<T> *yrt,
                                                         const Ent<T> *__restrict__ xtab,
                                                         const Ent<T> *__restrict__ ytab,
                                                         const DevWfs *__restrict__ wfs,
                                                         const DevLayer *__restrict__ lays, int nw, int nl, int maxnv,
                                                         int sum_n, int *over) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nw * sum_n) return;
    const int g = (int)(idx / sum_n), line = (int)(idx % sum_n);
    int l = 0;
    while (l + 1 < nl && lays[l + 1].r_off <= line) ++l;
    const int q = line - lays[l].r_off, nv = wfs[g].nv;
    for (int axis = 0; axis < 2; ++axis) {
        const Ent<T> *tab = (axis == 0 ? xtab : ytab) + ((long)g * nl + l) * maxnv;
        RtabEnt<T> *rt = (axis == 0 ? xrt : yrt) + idx * kRtabWidth;
        int lo = nv, hi = -1, cnt = 0;
        for (int j = 0; j < nv; ++j) {
            const Ent<T> e = tab[j];
            if (e.k0 == q || e.k0 + 1 == q) {
                lo = j < lo ? j : lo;
                hi = j;
                if (cnt < kRtabWidth) rt[cnt] = RtabEnt<T>{j, e.k0 == q ? e.w0 : e.w1};
                ++cnt;
            }
        }
        for (int c = cnt; c < kRtabWidth; ++c) rt[c] = RtabEnt<T>{0, (T)0};
        if (cnt > kRtabWidth) over[g] = 1;  // idempotent flag, no read-modify-write needed
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
    if (threadIdx.x < 3 && blockIdx.x == 0) {
        reset_scalars(sc + threadIdx.x);
        sc[threadIdx.x].counter = 0u;
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
int Ops<T>::nparts() const {
    return (int)P.fine_tiles.size() + (P.kf < P.J ? P.nl : 0);
}

template <typename T>
int Ops<T>::idwt(const T *c, T *out) const {
    InvArgs A{};
    A.src = c;
    A.out = out;
    k_inv<T, kInvPlain><<<(int)P.idwt_tiles.size(), kInvBlock, 0, st>>>(B, P.J, A, make_taps<T>());
    return check();
}

template <typename T>
int Ops<T>::idwt_first(const T *r, T *out) const {
    InvArgs A{};
    A.src = r;
    A.out = out;
    k_inv<T, kInvFirst><<<(int)P.idwt_tiles.size(), kInvBlock, 0, st>>>(B, P.J, A, make_taps<T>());
    return check();
}

template <typename T>
int Ops<T>::idwt_update(const T *r_old, const T *q_old, T *q_new, T *r_new, T *c, int kprev, double *resnorm,
                        T *out) const {
    InvArgs A{};
    A.src = r_old;
    A.out = out;
    A.yv = B.y;
    A.qold = kprev == 0 ? B.y : q_old;  // never read after the first pass
    A.qnew = q_new;
    A.rnew = r_new;
    A.c = c;
    A.first_pass = kprev == 0 ? 1 : 0;
    A.kprev = kprev;
    A.nparts = nparts();
    A.resnorm = resnorm;
    k_inv<T, kInvUpdate><<<(int)P.idwt_tiles.size(), kInvBlock, 0, st>>>(B, P.J, A, make_taps<T>());
    return check();
}

template <typename T>
template <int EPI>
size_t Ops<T>::coarse_lds() const {
    constexpr int NE = (EPI == kEpiRhs) ? 2 : ((EPI == kEpiPlain) ? 0 : 1);
    size_t m0 = 0;
    for (auto &L : P.lay) m0 = (size_t)(L.n >> P.kf) > m0 ? (size_t)(L.n >> P.kf) : m0;
    return (m0 * m0 + m0 * m0 / 4 + 1 + NE * m0 * m0) * sizeof(T);
}

template <typename T>
template <int EPI>
int Ops<T>::fwd(const T *x, const FwdArgs &E) const {
    const int nf = (int)P.fine_tiles.size();
    const Taps<T> tp = make_taps<T>();
    switch (P.kf) {
        case 1: k_fwd_fine<T, 1, 16, EPI><<<nf, kFwdBlock, 0, st>>>(x, B, P.J, E, tp); break;
        case 2: k_fwd_fine<T, 2, 8, EPI><<<nf, kFwdBlock, 0, st>>>(x, B, P.J, E, tp); break;
        default: k_fwd_fine<T, 3, 4, EPI><<<nf, kFwdBlock, 0, st>>>(x, B, P.J, E, tp); break;
    }
    if (int e = check()) return e;
    if (P.kf < P.J) {
        k_fwd_coarse<T, EPI><<<P.nl, 512, coarse_lds<EPI>(), st>>>(B, P.J, P.kf, E, tp, nf);
        if (int e = check()) return e;
    }
    return FEWHA_OK;
}

template <typename T>
int Ops<T>::prepare() const {
    // the per-layer coarse transform may need more than the default 64 KiB of dynamic LDS
    const void *fns[4] = {(const void *)k_fwd_coarse<T, kEpiPlain>, (const void *)k_fwd_coarse<T, kEpiPrior>,
                          (const void *)k_fwd_coarse<T, kEpiPcg>, (const void *)k_fwd_coarse<T, kEpiRhs>};
    const size_t need[4] = {coarse_lds<kEpiPlain>(), coarse_lds<kEpiPrior>(), coarse_lds<kEpiPcg>(),
                            coarse_lds<kEpiRhs>()};
    for (int i = 0; i < 4; ++i)
        if (need[i] > 48 * 1024 &&
            hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)need[i]) != hipSuccess)
            return FEWHA_ERR_UNSUPPORTED;
    return FEWHA_OK;
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
int Ops<T>::fdwt_pcg(const T *x, const T *rk) const {
    FwdArgs E{};
    E.out = B.y;
    E.rk = rk;
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
    if (mode == kModeM) k_nodes_m<T><<<tiles, kNodeBlock, 0, st>>>(in, v, B, P.nl);
    else if (mode == kModeRhs) k_nodes<T, kModeRhs><<<tiles, kBlock, 0, st>>>(in, v, B);
    else k_nodes<T, kModeAdj><<<tiles, kBlock, 0, st>>>(in, v, B);
    return check();
}

template <typename T>
int Ops<T>::slopes(const T *u, T *s) const {
    k_slopes<T><<<(int)P.sub_tiles.size(), kNodeBlock, 0, st>>>(u, s, B, P.nl);
    return check();
}

template <typename T>
int Ops<T>::pt(const T *v, T *x) const {
    if (P.rtab_ok) k_pt_tab<T><<<(int)P.lay_tiles.size(), kBlock, 0, st>>>(v, x, B, P.nl, P.nw);
    else k_pt_scan<T><<<(int)P.lay_tiles.size(), kBlock, 0, st>>>(v, x, B, P.nl, P.nw);
    return check();
}

template <typename T>
int Ops<T>::update_last(T *c, const T *r_in, const T *q_old, T *q_new, int kprev, double *resnorm) const {
    k_update_last<T><<<(int)P.coef_tiles.size(), kBlock, 0, st>>>(c, B, P.J, r_in, kprev == 0 ? B.y : q_old, q_new,
                                                                    kprev == 0 ? 1 : 0, nparts(), kprev, resnorm);
    return check();
}

template <typename T>
int Ops<T>::wnorm(const T *s) const {
    long mx = 0;
    for (auto &w : P.dwfs) mx = mx > (long)w.n_sub * w.n_sub ? mx : (long)w.n_sub * w.n_sub;
    int g = grid_for(mx);
    if (g > kPartialPitch) g = kPartialPitch;
    k_wnorm<T><<<g, kBlock, 0, st>>>(s, B, P.nw);
    if (int e = check()) return e;
    k_sum_partials<<<1, kBlock, 0, st>>>(B.partials, g, B.sc);
    return check();
}

template <typename T>
int Ops<T>::fit(const T *u, const T *a_prev, T *a, double gain) const {
    k_fit<T><<<grid_for((long)P.n_act), kBlock, 0, st>>>(u, a_prev, a, B, P.nl, P.nd, (long)P.n_act, gain);
    return check();
}

template <typename T>
int Ops<T>::build_tables(int *over) const {
    const long ne = (long)P.nw * P.nl * P.maxnv;
    k_build_tabs<T><<<(int)((ne + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        const_cast<Ent<T> *>(B.xtab), const_cast<Ent<T> *>(B.ytab), B.wfs, B.proj, B.lay, P.nw, P.nl, P.maxnv);
    if (int e = check()) return e;
    const long nr = (long)P.nw * P.sum_n;
    k_build_ranges<T><<<(int)((nr + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        const_cast<Range *>(B.xrng), const_cast<Range *>(B.yrng), const_cast<RtabEnt<T> *>(B.xrtab),
        const_cast<RtabEnt<T> *>(B.yrtab), B.xtab, B.ytab, B.wfs, B.lay, P.nw, P.nl, P.maxnv, P.sum_n, over);
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
