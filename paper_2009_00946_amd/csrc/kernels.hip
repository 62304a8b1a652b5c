// HIP kernels of the FEWHA hot path for gfx950 (CDNA4, wave64).
//
// Every stage is bandwidth/latency bound (no dense contraction anywhere), so the kernels are
// gather-only stencils: each output element is written by exactly one lane, nothing uses
// atomics except the last-block-done counter of the reductions, and results are bitwise
// reproducible run to run.
//
//   k_idwt       W^T (= W^-1) of every layer, all J levels in one launch: each workgroup owns a
//                square output tile and rebuilds, level by level from the coarsest, only the
//                cone of approximation coefficients that tile depends on (LDS resident);
//                optionally scales coefficients by the Jacobi preconditioner on load (z = J^-1 r).
//   k_nodes      per WFS node tile: P (bilinear ray gather from all layers, LGS cone), Gamma,
//                C_eta^-1 and Gamma^T fused through LDS (the Kernel-2 stage of the paper), or
//                Gamma^T C s / Gamma^T mask s for right-hand sides and adjoints.
//   k_slopes     mask Gamma P u on subaperture tiles (forward operator A).
//   k_pt         P^T as a gather per layer node: recomputes, with the same code as the forward,
//                the cell and weights of every candidate WFS node and keeps the ones that touch
//                this node, so P^T is the exact transpose of the implemented P without atomics.
//   k_fdwt_level one level of the forward periodic db3 transform for all layers.
//   k_dots       alpha D z epilogue of M z plus the two PCG reductions (r, z), (Mz, z) in FP64;
//                the last block to finish forms the Alg. 2 scalars on the device.
//   k_update     fused p, q, c, r update of Alg. 2.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace fewha {

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------------------------
// Geometry helpers shared by the forward projection and its transpose (identical arithmetic).
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

// Grid coordinate on layer l of node index j of WFS g along one axis (h = theta h_l of that axis).
__device__ __forceinline__ double ray_coord(const DevProj &pr, const DevWfs &W, const DevLayer &L, int j, double h) {
    double X = pr.sig * (W.x0 + (double)j * W.d) + h;
    return X / L.spacing + L.half;
}

__device__ __forceinline__ bool subap_active(const DevWfs &W, int i, int j) {
    double xc = ((double)j + 0.5) * W.d + W.x0, yc = ((double)i + 0.5) * W.d + W.x0;
    double r2 = xc * xc + yc * yc;
    return r2 <= W.r_out2 && r2 >= W.r_in2;
}

// phi_g(i, j) = sum_l bilinear(u_l at the ray point)  (P of Sec. 2.1)
template <typename T>
__device__ __forceinline__ T project_node(const T *__restrict__ u, const DevWfs &W, const DevProj *__restrict__ proj,
                                          const DevLayer *__restrict__ lays, int nl, int i, int j) {
    T acc = 0;
    for (int l = 0; l < nl; ++l) {
        const DevProj pr = proj[l];
        const DevLayer L = lays[l];
        Cell cx = cell_of(ray_coord(pr, W, L, j, pr.hx), L.n);
        Cell cy = cell_of(ray_coord(pr, W, L, i, pr.hy), L.n);
        T wx1 = (T)cx.t, wx0 = (T)(1.0 - cx.t), wy1 = (T)cy.t, wy0 = (T)(1.0 - cy.t);
        const T *U = u + L.c_off + (long)cy.k0 * L.n + cx.k0;
        acc += (wy0 * wx0) * U[0] + (wy0 * wx1) * U[1] + (wy1 * wx0) * U[L.n] + (wy1 * wx1) * U[L.n + 1];
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

// Publish this block's partials; return true in the one block that finishes last (all
// partials are then visible to it).  The counter returns to zero for the next use.
__device__ __forceinline__ bool publish_last(double *partials, int nparts, const double *vals, unsigned *counter) {
    __shared__ bool last;
    if (threadIdx.x == 0) {
        for (int k = 0; k < nparts; ++k)
            __hip_atomic_store(partials + (size_t)k * gridDim.x + blockIdx.x, vals[k], __ATOMIC_RELAXED,
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

// Sum one partial row in fixed (block index) order, cooperatively by the last block.
__device__ __forceinline__ double gather_partials(const double *partials, int row, double *sh) {
    double v = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
        v += __hip_atomic_load(partials + (size_t)row * gridDim.x + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum(v, sh);
}

// Layer, level and orientation of coefficient index i.
struct Band {
    int l, s, o;
    long off;
};

__device__ __forceinline__ Band band_of(long i, const DevLayer *__restrict__ lays, int nl, int J) {
    int lo = 0, hi = nl - 1;
    while (lo < hi) {  // last layer with c_off <= i
        int mid = (lo + hi + 1) >> 1;
        if (lays[mid].c_off <= i) lo = mid;
        else hi = mid - 1;
    }
    const DevLayer L = lays[lo];
    long loc = i - L.c_off;
    int row = (int)(loc >> L.log2n), col = (int)(loc & (L.n - 1));
    int v = row > col ? row : col;
    Band b;
    b.l = lo;
    b.off = L.c_off;
    if (v < (L.n >> J)) {
        b.s = J;
        b.o = 0;
    } else {
        int lv = 31 - __clz(v);
        int m = 1 << lv;
        b.s = L.log2n - lv;
        b.o = (row < m) ? 1 : ((col < m) ? 2 : 3);
    }
    return b;
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
        const DevProj *proj = B.proj + (long)t.a * nl;
        for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
            int a = idx / NP, b = idx - a * NP, i = i0 - 1 + a, j = j0 - 1 + b;
            T val = 0;
            if (i >= 0 && i <= ns && j >= 0 && j <= ns) val = project_node(in, W, proj, B.lay, nl, i, j);
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
    const DevProj *proj = B.proj + (long)t.a * nl;
    for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
        int a = idx / NP, b = idx - a * NP, i = i0 + a, j = j0 + b;
        T val = 0;
        if (i <= ns && j <= ns) val = project_node(u, W, proj, B.lay, nl, i, j);
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
// P^T as a gather over layer-node tiles.
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pt(const T *__restrict__ v, T *__restrict__ x, Bufs<T> B, int nl,
                                               int nw) {
    constexpr int NT = kNodeTile, MAXC = 24;
    const Tile t = B.lay_tiles[blockIdx.x];
    const DevLayer L = B.lay[t.a];
    const int k = t.b + (int)(threadIdx.x / NT), q = t.c + (int)(threadIdx.x % NT);
    if (k >= L.n || q >= L.n) return;
    T acc = 0;
    for (int g = 0; g < nw; ++g) {
        const DevWfs W = B.wfs[g];
        const DevProj pr = B.proj[(long)g * nl + t.a];
        const int ns = W.n_sub;
        // candidate nodes: those whose affine coordinate is within one cell (+1 node of slack)
        int jlo = (int)floor((q - 1 - pr.bx) / pr.slope) - 1, jhi = (int)ceil((q + 1 - pr.bx) / pr.slope) + 1;
        int ilo = (int)floor((k - 1 - pr.by) / pr.slope) - 1, ihi = (int)ceil((k + 1 - pr.by) / pr.slope) + 1;
        jlo = jlo < 0 ? 0 : jlo;
        ilo = ilo < 0 ? 0 : ilo;
        jhi = jhi > ns ? ns : jhi;
        ihi = ihi > ns ? ns : ihi;
        if (jlo > jhi || ilo > ihi) continue;
        int jn[MAXC];
        T jw[MAXC];
        int cnt = 0;
        for (int j = jlo; j <= jhi && cnt < MAXC; ++j) {
            Cell cx = cell_of(ray_coord(pr, W, L, j, pr.hx), L.n);
            if (cx.k0 == q) {
                jn[cnt] = j;
                jw[cnt++] = (T)(1.0 - cx.t);
            } else if (cx.k0 + 1 == q) {
                jn[cnt] = j;
                jw[cnt++] = (T)cx.t;
            }
        }
        if (cnt == 0) continue;
        const T *vg = v + W.v_off;
        for (int i = ilo; i <= ihi; ++i) {
            Cell cy = cell_of(ray_coord(pr, W, L, i, pr.hy), L.n);
            T wy;
            if (cy.k0 == k) wy = (T)(1.0 - cy.t);
            else if (cy.k0 + 1 == k) wy = (T)cy.t;
            else continue;
            for (int c = 0; c < cnt; ++c) acc += (wy * jw[c]) * vg[(long)i * W.nv + jn[c]];
        }
    }
    x[L.c_off + (long)k * L.n + q] = acc;
}

// ---------------------------------------------------------------------------------------------
// W: one level of the forward transform for every layer (thread per output quad).
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fdwt_level(const T *__restrict__ src, T *__restrict__ dst,
                                                       T *__restrict__ ll_out, const DevLayer *__restrict__ lays,
                                                       int nl, int lev, int J, long nquads, Taps<T> tp) {
    long qi = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= nquads) return;
    const int sh = 2 * (lev + 1);
    int lo = 0, hi = nl - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((lays[mid].c_off >> sh) <= qi) lo = mid;
        else hi = mid - 1;
    }
    const DevLayer L = lays[lo];
    const int n = L.n, m = n >> lev, h2 = m >> 1, msk = m - 1;
    const long loc = qi - (L.c_off >> sh);
    const int kr = (int)(loc / h2), kc = (int)(loc - (long)kr * h2);
    const T *S;
    int pitch;
    if (lev == 0) {
        S = src + L.c_off;
        pitch = n;
    } else {
        S = src + (L.c_off >> (2 * lev));
        pitch = m;
    }
    int cols[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) cols[b] = (2 * kc + b) & msk;
    T ll = 0, lh = 0, hl = 0, hh = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        const T *row = S + (long)((2 * kr + a) & msk) * pitch;
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
    T *D = dst + L.c_off;
    D[(long)kr * n + h2 + kc] = hl;
    D[(long)(h2 + kr) * n + kc] = lh;
    D[(long)(h2 + kr) * n + h2 + kc] = hh;
    if (lev == J - 1) D[(long)kr * n + kc] = ll;
    else ll_out[(L.c_off >> sh) + (long)kr * h2 + kc] = ll;
}

// ---------------------------------------------------------------------------------------------
// PCG pieces (Alg. 2)
// ---------------------------------------------------------------------------------------------

// y += alpha D z with z = J^-1 r; partial (r, z), (y, z); the last block forms the scalars.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dots(T *__restrict__ y, const T *__restrict__ r, Bufs<T> B, int nl, int J,
                                                 long N, int k, double *resnorm) {
    __shared__ double sh[kBlock / 64];
    double rho = 0.0, mu = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
        Band b = band_of(i, B.lay, nl, J);
        const T z = r[i] * B.jinv[(b.l * (J + 1) + b.s) * 4 + b.o];
        const T yi = y[i] + B.ad[b.l * (J + 1) + b.s] * z;
        y[i] = yi;
        rho += (double)r[i] * (double)z;
        mu += (double)yi * (double)z;
    }
    double vals[2];
    vals[0] = block_sum(rho, sh);
    vals[1] = block_sum(mu, sh);
    if (!publish_last(B.partials, 2, vals, &B.sc->counter)) return;
    const double R = gather_partials(B.partials, 0, sh);
    const double Mu = gather_partials(B.partials, 1, sh);
    if (threadIdx.x != 0) return;
    Scalars *sc = B.sc;
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

// p = z + beta p; q = y + beta q; c += alpha p; r -= alpha q   (first pass: p = z, q = y)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(T *__restrict__ c, Bufs<T> B, int nl, int J, long N, int k) {
    if (B.sc->stopped) return;
    const T alpha = (T)B.sc->alpha, beta = (T)B.sc->beta;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
        Band b = band_of(i, B.lay, nl, J);
        const T ri = B.r[i];
        const T z = ri * B.jinv[(b.l * (J + 1) + b.s) * 4 + b.o];
        const T p = (k == 0) ? z : z + beta * B.p[i];
        const T q = (k == 0) ? B.y[i] : B.y[i] + beta * B.q[i];
        B.p[i] = p;
        B.q[i] = q;
        c[i] += alpha * p;
        B.r[i] = ri - alpha * q;
    }
}

// y += alpha D c  (tail of apply_M)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_prior(T *__restrict__ y, const T *__restrict__ c, Bufs<T> B, int nl,
                                                      int J, long N) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
        Band b = band_of(i, B.lay, nl, J);
        y[i] += B.ad[b.l * (J + 1) + b.s] * c[i];
    }
}

// Residual update of Alg. 1 and reset of the PCG scalars.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual(T *__restrict__ c, Bufs<T> B, long N, int cold) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Scalars *sc = B.sc;
        sc->rho = sc->mu = sc->rho_old = sc->alpha = sc->alpha_old = sc->beta = 0.0;
        sc->stopped = 0;
        sc->status = FEWHA_OK;
    }
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
        const T b = B.b[i];
        if (cold) {
            c[i] = 0;
            B.r[i] = b;
        } else {
            B.r[i] = (b - B.b_prev[i]) + B.r[i];
        }
        B.b_prev[i] = b;
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
    if (!publish_last(B.partials, 1, &v, &B.sc->counter)) return;
    const double tot = gather_partials(B.partials, 0, sh);
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
        sc->rho = sc->mu = sc->rho_old = sc->alpha = sc->alpha_old = sc->beta = 0.0;
        sc->stopped = 0;
        sc->status = FEWHA_OK;
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
    const Taps<T> tp = make_taps<T>();
    const T *src = x;
    for (int lev = 0; lev < P.J; ++lev) {
        T *ll = (lev & 1) ? B.tmpB : B.tmpA;
        const long nq = (long)(P.n_coef >> (2 * (lev + 1)));
        k_fdwt_level<T><<<(int)((nq + kBlock - 1) / kBlock), kBlock, 0, st>>>(src, out, ll, B.lay, P.nl, lev, P.J, nq,
                                                                              tp);
        if (int e = check()) return e;
        src = ll;
    }
    return FEWHA_OK;
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
int Ops<T>::add_prior(T *y, const T *c) const {
    k_add_prior<T><<<grid_for((long)P.n_coef), kBlock, 0, st>>>(y, c, B, P.nl, P.J, (long)P.n_coef);
    return check();
}

template <typename T>
int Ops<T>::residual(T *c, bool cold) const {
    k_residual<T><<<grid_for((long)P.n_coef), kBlock, 0, st>>>(c, B, (long)P.n_coef, cold ? 1 : 0);
    return check();
}

template <typename T>
int Ops<T>::dots(int k, double *resnorm) const {
    int g = grid_for((long)P.n_coef);
    if (g > P.n_partials) g = P.n_partials;
    k_dots<T><<<g, kBlock, 0, st>>>(B.y, B.r, B, P.nl, P.J, (long)P.n_coef, k, resnorm);
    return check();
}

template <typename T>
int Ops<T>::update(T *c, int k) const {
    k_update<T><<<grid_for((long)P.n_coef), kBlock, 0, st>>>(c, B, P.nl, P.J, (long)P.n_coef, k);
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
