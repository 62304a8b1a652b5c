// HIP kernels of the FEWHA hot path for gfx950 (CDNA4, wave64).
//
// The frame is a chain of small dependent launches over an L2-resident working set, so every
// kernel is built to need one round of independent global loads: a workgroup finds its tile
// from a table passed as a kernel argument (no tile records in memory), issues all of its loads
// at once, and then works from LDS and registers.  Every output element is written by exactly
// one lane and every sum runs in a fixed order, so results are bitwise reproducible.  There are
// no atomics: reductions leave one FP64 partial per workgroup, summed in fixed order by the
// kernels that need the result.
//
// One PCG pass of Alg. 2 (Jacobi-preconditioned, one reduction point) is five launches:
//   k_wt<pcg>    z = J^-1 r and u = W^T z on 32 x 32 output tiles (all J levels per tile from a
//                cone of coefficients)
//   k_proj<M>    per 16 x 16 node tile of each guide star: phi = P u (bilinear rays, cone effect),
//                Gamma, C_eta^-1, Gamma^T -> v; partial of sum C (Gamma P u)^2
//   k_pt         x = P^T v on 16 x 16 layer tiles, from staged node rectangles and the transpose
//                tables (the same matrix entries as P); one extra workgroup steps the scalars
//   k_fwd/k_coarse<pcg>  y = W x + alpha D z on the fine levels (tiles) and the coarse levels
//                (one workgroup per layer), then the pass's update in place, with the partials of
//                rho = (r, z) and (z, alpha D z) of the new residual for the next pass.
// The denominator mu = (M z, z) is formed from the partials as (C Gamma P W^T z, Gamma P W^T z)
// + (z, alpha D z): W is orthonormal and every adjoint here is the exact transpose of its
// forward operator, so this equals (y, z) without waiting for y, and the update of a pass can
// run in the same launch that produces y.
//
// With the fold (k_wt<fold>) a pass's coarse levels run at the start of the next pass's inverse
// DWT, so a pass is four launches; the last pass's coarse levels run in the tail workgroups of an
// inverse-DWT launch (k_wt<tail>: beside the fit's W^T c in a whole frame), its step of c in the
// fine transform.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace fewha {

namespace {

constexpr int kB = 256;       // workgroup size of the tile kernels
constexpr int kCB = 1024;     // workgroup size of the per-layer coarse forward DWT
constexpr size_t kCoarseLdsMax = 150 * 1024;  // dynamic LDS of the coarse forward DWT (at most)

// ---------------------------------------------------------------------------------------------
// Kernel-argument tables and small helpers
// ---------------------------------------------------------------------------------------------
struct InvVar {               // sigma^-2 per guide star
    double v[kMaxWfs];
};

struct WfsOff {               // node grid offset and row pitch per guide star
    int v_off[kMaxWfs];
    int vp[kMaxWfs];
};

struct PupilArgs {            // subaperture (i, j) of guide star g is active iff its centre is in
    double D;                 // the annulus r_in^2 <= r^2 <= r_out^2 (d = D / n_sub, x0 = -D/2)
    double r_out2, r_in2;
};

// The tile of this workgroup and its segment's entries.  Every lane of the wave reads one
// segment's entries in a single round of loads (entries past the last segment start at INT_MAX);
// a ballot then picks the last segment starting at or before this workgroup and its entries are
// broadcast from that lane.  All 64 lanes of the wave must be active.
struct TileId {
    int seg, loc;
    int off, n, lt, aux, rw, pitch, id;
};

// Workgroups are dealt to the chip's 8 XCDs round-robin (workgroup b runs on XCD b mod 8), and
// every XCD has its own L2.  Tile kernels renumber their ntiles workgroups: with chunk K = 0 each
// XCD receives one contiguous run of tiles (neighbouring tiles share halos and table lines, which
// then meet in one L2); with K > 0 the tile list is cut into chunks of K consecutive tiles dealt to
// the XCDs in turn, so that every XCD gets a share of every layer (tiles of different layers
// differ in cost) and the segments listed first are dispatched first, while a chunk's tiles still
// share an L2.  Tiles past the last whole round of 8 chunks keep their own number.
__device__ __forceinline__ int xcd_tile(int K, int ntiles, int b) {
    if (K == 0) {
        const int q = ntiles >> 3, rem = ntiles & 7, x = b & 7;
        return x * q + min(x, rem) + (b >> 3);
    }
    const int full = ntiles / (8 * K) * (8 * K);
    if (b >= full) return b;
    const int i = b >> 3;
    return ((i / K) * 8 + (b & 7)) * K + (i % K);
}

__device__ __forceinline__ int xcd_tile(int K, int ntiles) { return xcd_tile(K, ntiles, (int)blockIdx.x); }

__device__ __forceinline__ TileId find_tile(const SegTab &S, int b) {
    if (S.ilv) {  // interleaved equal segments: tile b / nseg of segment b % nseg
        const int s0 = b % S.nseg;
        b = S.start[s0] + b / S.nseg;
    }
    const int lane = threadIdx.x & 63;
    const int st = S.start[lane], of = S.off[lane], nn = S.n[lane], l2 = S.lt[lane], ax = S.aux[lane];
    const int rw = S.rw[lane], pi = S.pitch[lane], ix = S.id[lane];
    const unsigned long long m = __ballot(b >= st);
    const int s = 63 - __clzll(m);
    TileId t;
    t.seg = s;
    t.loc = b - __builtin_amdgcn_readlane(st, s);
    t.off = __builtin_amdgcn_readlane(of, s);
    t.n = __builtin_amdgcn_readlane(nn, s);
    t.lt = __builtin_amdgcn_readlane(l2, s);
    t.aux = __builtin_amdgcn_readlane(ax, s);
    t.rw = __builtin_amdgcn_readlane(rw, s);
    t.pitch = __builtin_amdgcn_readlane(pi, s);
    t.id = __builtin_amdgcn_readlane(ix, s);
    return t;
}

// Frame blockIdx.y of a batch: its per-frame vectors, partial sums and scalar slots.
template <typename T>
__device__ __forceinline__ Bufs<T> at_frame(Bufs<T> B) {
    const long f = blockIdx.y, c = f * B.fs_c;
    B.b_prev += c;
    B.r += c;
    B.p += c;
    B.q += c;
    B.u += c;
    B.x += c;
    B.v += f * B.fs_v;
    B.ll += f * B.fs_ll;
    B.partials += f * 3 * kPartialPitch;
    B.sc += f * kScalarSlots;
    return B;
}

// The caller's coefficient vectors of frame blockIdx.y (frame-major, fs_c apart).
template <typename T>
__device__ __forceinline__ FwdArgs frame_args(FwdArgs E, long fs_c) {
    const long c = blockIdx.y * fs_c;
    if (E.out) E.out = static_cast<T *>(E.out) + c;
    if (E.cin) E.cin = static_cast<const T *>(E.cin) + c;
    if (E.c) E.c = static_cast<T *>(E.c) + c;
    if (E.r_in) E.r_in = static_cast<const T *>(E.r_in) + c;
    if (E.q_in) E.q_in = static_cast<const T *>(E.q_in) + c;
    if (E.b_in) E.b_in = static_cast<const T *>(E.b_in) + c;
    if (E.cc) E.cc = static_cast<T *>(E.cc) + c;
    if (E.cc_r) E.cc_r = static_cast<const T *>(E.cc_r) + c;
    return E;
}

__device__ __forceinline__ bool subap_active(const PupilArgs &pa, int ns, int i, int j) {
    const double d = pa.D / ns, x0 = -0.5 * pa.D;
    const double xc = ((double)j + 0.5) * d + x0, yc = ((double)i + 0.5) * d + x0;
    const double r2 = xc * xc + yc * yc;
    return r2 <= pa.r_out2 && r2 >= pa.r_in2;
}

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

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block in fixed order; the result is returned to every lane.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Two sums over the block at once, each in the fixed order of block_sum (so bitwise equal to two
// block_sum calls): the shuffles of both interleave and one barrier pair serves both.  sh holds
// 2 * (blockDim.x / 64) values.
__device__ __forceinline__ void block_sum2(double &a, double &b, double *sh) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
    if (lane == 0) {
        sh[wid] = a;
        sh[nw + wid] = b;
    }
    __syncthreads();
    double s = 0.0, t = 0.0;
    for (int w = 0; w < nw; ++w) {
        s += sh[w];
        t += sh[nw + w];
    }
    __syncthreads();
    a = s;
    b = t;
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

struct StepOut {
    double alpha, beta;
    int stopped;
};

// The scalar step of pass k, done once by one extra workgroup of the P^T launch (whose inputs
// are complete by then: the partials of (r, z) and (z, alpha D z) left by the forward transforms
// that wrote r, and those of C (Gamma P u)^2 left by the projection): reduce the partials in
// fixed order, step the recurrence from sc[(k-1)&1], store (alpha, beta, stopped) in sc[3] for the
// forward transform that applies the update and, if `publish`, the new state in sc[k&1] and
// sqrt(rho) in resnorm[k].
__device__ void scalar_step(const double *__restrict__ part, int nwt, int nproj, Scalars *sc, int k,
                            double *resnorm, int publish) {
    __shared__ double sh[2 * (kB / 64)];
    double R = 0.0, Mu = 0.0;
    for (int i = threadIdx.x; i < nwt; i += blockDim.x) {
        R += part[i];
        Mu += part[kPartialPitch + i];
    }
    for (int i = threadIdx.x; i < nproj; i += blockDim.x) Mu += part[2 * kPartialPitch + i];
    block_sum2(R, Mu, sh);
    if (threadIdx.x == 0) {
        const Scalars prev = sc[(k - 1) & 1];
        const Scalars nx = alg2_step(prev, R, Mu, k);
        Scalars st = nx;
        st.stopped = nx.stopped;
        sc[3] = st;
        if (publish) {
            sc[k & 1] = nx;
            if (resnorm && !prev.stopped && isfinite(R)) resnorm[k] = sqrt(R);
        }
    }
}

// (alpha, beta, stopped) of the current pass, as left in sc[3] by the P^T launch.
__device__ __forceinline__ StepOut read_step(const Scalars *sc) {
    const Scalars st = sc[3];
    return StepOut{st.alpha, st.beta, st.stopped};
}

// float-reciprocal quotient of small non-negative integers (a < 2^20, b <= 2^10): exact
__device__ __forceinline__ int small_div(int a, float rb) { return (int)(((float)a + 0.5f) * rb); }

// ---------------------------------------------------------------------------------------------
// W^T: the inverse DWT of every layer, all J levels in one launch.
//
// A workgroup owns a T0 x T0 output tile (T0 = min(32, n)).  In level-s index space the tile
// depends on the region [lo_s, hi_s] per axis, lo_s = ((lo_{s-1} >> 1) - 2) rounded down to even,
// hi_s = hi_{s-1} >> 1 (periodic, so indices wrap modulo n >> s).  The whole cone (three detail
// bands per level and the coarsest LL) arrives in one batch of loads, then the J synthesis
// levels run in LDS: along y (pairs of output rows share their three taps), then along x.
// In PCG mode the cone holds z = J^-1 r and the workgroup reduces (r, z) and (z, alpha D z) over
// the coefficients it owns (at level s: indices [y0 >> s, (y0 + T0) >> s), or y0 >> s alone when
// T0 < 2^s and y0 is a multiple of 2^s), which partition every band.
// ---------------------------------------------------------------------------------------------
constexpr int kWtLL = 18 * 32;   // LL_{s-1} region of a level s >= 2 (rows x the level's pitch)
constexpr int kWtX = 32 * 32;    // y-synthesis output: (rows of level s-1) x (pitch of level s)
constexpr int kWB = 256;         // workgroup of one inverse-DWT tile
constexpr int kWtSlots = 9 + 3 + (kMaxJ - 2);

// Cone layout: level 1 in nine passes of 8 rows x 32 lanes, level 2 in three passes of 16 rows x
// 16 lanes, each coarser level in one pass of 32 rows x 8 lanes.  Pass p of level s is LDS slot
// wt_slot0(s) + p (kWB values, in lane order), so level s is a row-major block of pitch
// 2^wt_lanes_log2(s) whose rows are band * LY_s + r (bands x-high, y-high, HH, and LL at s = J).
__host__ __device__ constexpr int wt_passes(int s) { return s == 1 ? 9 : (s == 2 ? 3 : 1); }
__host__ __device__ constexpr int wt_lanes_log2(int s) { return s == 1 ? 5 : (s == 2 ? 4 : 3); }
__host__ __device__ constexpr int wt_slot0(int s) { return s == 1 ? 0 : (s == 2 ? 9 : 12 + (s - 3)); }
// Slots of a J-level cone, the launch's dynamic LDS: through level J's (a level-2 pass of 16-byte
// copies spans four slots, so J <= 2 keeps 13), at most kWtSlots.
__host__ __device__ constexpr int wt_slots(int J) { return J <= 2 ? 13 : J + 10; }
static_assert(wt_slots(kMaxJ) == kWtSlots, "the cone of the deepest transform");

// Asynchronous copy of one 4-byte value per active lane from global memory into LDS at
// wave_base[lane] (lane = threadIdx.x & 63) without registers; complete at s_waitcnt vmcnt(0).
// wave_base must be the same for every lane of the wave.
__device__ __forceinline__ void g2lds(const float *gp, float *wave_base) {
    __builtin_amdgcn_global_load_lds(gp, (__attribute__((address_space(3))) void *)wave_base, 4, 0, 0);
}

// The same with 16 bytes (four floats) per lane, to wave_base + 16 lane bytes.
__device__ __forceinline__ void g2lds16(const float *gp, float *wave_base) {
    __builtin_amdgcn_global_load_lds(gp, (__attribute__((address_space(3))) void *)wave_base, 16, 0, 0);
}

__device__ __forceinline__ void lds_fence() {
    __builtin_amdgcn_s_waitcnt(0);  // every outstanding load, including those into LDS
    __syncthreads();
}

// kWtFold: kWtPcg after the folded coarse update (see FoldArgs).  kWtTail: kWtPlain tiles after
// F.ntail workgroups that run the last pass's coarse levels (coarse_tail).
enum { kWtPlain = 0, kWtPcg = 1, kWtFold = 2, kWtTail = 3 };

// Coarse block of a layer that the fold handles: levels 3..J of layers up to 256 x 256 (level-2
// block at most 64 x 64); a tile owns at most kFoldOwn of its coefficients.
constexpr int kFoldM0 = 64;

// The updates of Alg. 1 (residual line) and Alg. 2 (vector lines) at one coarse coefficient, with
// every product and sum rounded on its own: each tile of a layer recomputes them at the
// coefficients of its cone, and must reproduce bit for bit what the coefficient's owner stores.
struct FoldNew {
    float p, q, c, r;
};

__device__ __forceinline__ float fold_rhs(float w, float b_prev, float r_prev, int cold) {
#pragma clang fp contract(off)
    return cold ? w : (w - b_prev) + r_prev;
}

__device__ __forceinline__ FoldNew fold_pcg(float w, float r, float c, float p, float q, float ji, float ad, float al,
                                            float be, bool first) {
#pragma clang fp contract(off)
    const float z = r * ji, az = ad * z, y = w + az;
    FoldNew o;
    if (first) {
        o.p = z;
        o.q = y;
    } else {
        const float bp = be * p, bq = be * q;
        o.p = z + bp;
        o.q = y + bq;
    }
    const float ap = al * o.p, aq = al * o.q;
    o.c = c + ap;
    o.r = r - aq;
    return o;
}

// Level s >= 1 and orientation (0 LL, 1 x-high, 2 y-high, 3 HH) of Mallat position (row, col) of
// an n = 2^log2n layer with J levels.
__device__ __forceinline__ void band_of(int log2n, int J, int row, int col, int &s, int &o) {
    const int mx = row > col ? row : col;
    s = mx == 0 ? J : log2n - (31 - __clz(mx));
    if (s > J) s = J;
    const int m = 1 << (log2n - s);
    o = (col >= m ? 1 : 0) + (row >= m ? 2 : 0);
}

// One level of the forward DWT, in place on the MI x MI approximation at the top-left of sB (row
// pitch P): afterwards that corner holds the next approximation (top-left MI/2 x MI/2) and the
// level's three bands in Mallat position (x-high top-right, y-high bottom-left, HH bottom-right).
// Separable and periodic: the x pass takes every row to its low and high halves, output j the
// sum over b of tap[b] x[(2j + b) mod MI]; the y pass does the same down every column.  Products
// are accumulated in tap order, so the result is one fixed function of the block.  Each pass
// computes into registers, then (after a barrier) writes in place.  x pass: lane j of a row
// group reads its six inputs as three aligned pairs (a row group's lanes cover contiguous words);
// y pass: a lane owns a column and K consecutive outputs, sharing 2K + 4 input rows.
template <int MI, int P>
__device__ __forceinline__ void dwt_level_inplace(float *sB, const Taps<float> &tp) {
    constexpr int H = MI / 2, N = MI * H;  // output pairs of one pass
    constexpr int K = N > kWB ? N / kWB : 1, NT = N / K;
    static_assert(N % K == 0 && H % K == 0 && NT <= kWB, "pass layout");
    const int tid = threadIdx.x;
    const bool act = tid < NT;
    float lo[K], hi[K];
    {
        const int j = tid % H, r0 = tid / H;
        if (act) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float *row = sB + (r0 + k * (NT / H)) * P;
                float x[6];
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    const float2 v = *reinterpret_cast<const float2 *>(row + ((2 * j + 2 * u) & (MI - 1)));
                    x[2 * u] = v.x;
                    x[2 * u + 1] = v.y;
                }
                float l = 0, g = 0;
#pragma unroll
                for (int b = 0; b < 6; ++b) {
                    l += tp.h[b] * x[b];
                    g += tp.g[b] * x[b];
                }
                lo[k] = l;
                hi[k] = g;
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                float *row = sB + (r0 + k * (NT / H)) * P;
                row[j] = lo[k];
                row[j + H] = hi[k];
            }
        }
        __syncthreads();
    }
    {
        const int c = tid % MI, i0 = K * (tid / MI);
        if (act) {
            float x[2 * K + 4];
#pragma unroll
            for (int a = 0; a < 2 * K + 4; ++a) x[a] = sB[((2 * i0 + a) & (MI - 1)) * P + c];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                float l = 0, g = 0;
#pragma unroll
                for (int a = 0; a < 6; ++a) {
                    l += tp.h[a] * x[2 * k + a];
                    g += tp.g[a] * x[2 * k + a];
                }
                lo[k] = l;
                hi[k] = g;
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                sB[(i0 + k) * P + c] = lo[k];
                sB[(i0 + k + H) * P + c] = hi[k];
            }
        }
        __syncthreads();
    }
}

// The same for an input of at most 16 x 16 (2^lmi rows, row pitch P), one output pair per lane.
__device__ __forceinline__ void dwt_level_small(float *sB, int lmi, int P, const Taps<float> &tp) {
    const int MI = 1 << lmi, H = MI >> 1, tid = threadIdx.x;
    const bool act = tid < MI * H;
    float lo = 0, hi = 0;
    {
        const int j = tid & (H - 1), r = tid >> (lmi - 1);
        if (act) {
            const float *row = sB + r * P;
            float x[6];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const float2 v = *reinterpret_cast<const float2 *>(row + ((2 * j + 2 * u) & (MI - 1)));
                x[2 * u] = v.x;
                x[2 * u + 1] = v.y;
            }
#pragma unroll
            for (int b = 0; b < 6; ++b) {
                lo += tp.h[b] * x[b];
                hi += tp.g[b] * x[b];
            }
        }
        __syncthreads();
        if (act) {
            sB[r * P + j] = lo;
            sB[r * P + j + H] = hi;
        }
        __syncthreads();
    }
    {
        const int c = tid & (MI - 1), i = tid >> lmi;
        lo = 0;
        hi = 0;
        if (act) {
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                const float x = sB[((2 * i + a) & (MI - 1)) * P + c];
                lo += tp.h[a] * x;
                hi += tp.g[a] * x;
            }
        }
        __syncthreads();
        if (act) {
            sB[i * P + c] = lo;
            sB[(i + H) * P + c] = hi;
        }
        __syncthreads();
    }
}

// Levels kf+1..kf+nlev of W x, in place on the level-kf approximation sB (m0 x m0, pitch m0, at
// most kFoldM0): afterwards sB holds the Mallat layout of those levels, the coarsest LL at (0, 0).
// The 64- and 32-row levels have compile-time shapes (several output pairs per lane); every
// smaller level runs the one runtime-shaped routine.
__device__ __forceinline__ void coarse_analysis(float *sB, int m0, int nlev, const Taps<float> &tp) {
    static_assert(kFoldM0 == 64, "compile-time levels for 64 and 32 rows");
    int lmi = 31 - __clz(m0);
    if (m0 == 64 && nlev > 0) {
        dwt_level_inplace<64, 64>(sB, tp);
        --nlev;
        --lmi;
        if (nlev > 0) {
            dwt_level_inplace<32, 64>(sB, tp);
            --nlev;
            --lmi;
        }
    } else if (m0 == 32 && nlev > 0) {
        dwt_level_inplace<32, 32>(sB, tp);
        --nlev;
        --lmi;
    }
    for (; nlev > 0 && lmi >= 1; --nlev, --lmi) dwt_level_small(sB, lmi, m0, tp);  // uniform trip count
}

// The last pass's coarse levels kf+1..J of the forward transform, for a solve whose earlier coarse
// levels were folded (the fine transform of that pass stepped c there already, c + alpha p needing
// no W x): workgroup t of the layer's F.parts recomputes W x of the layer's coarse block from the
// level-kf approximation and, at its own part of the block, applies Alg. 2's p, q and r lines (in
// the fold's arithmetic) and copies the right-hand side's coarse coefficients to b_prev.
template <typename T>
__device__ void coarse_tail(const SegTab &S, Bufs<T> B, const FoldArgs &F, const Taps<T> &tp, int J, int t, T *sL,
                            T *sJi, T *sAd) {
    static_assert(sizeof(T) == 4, "the fold's arithmetic is FP32");
    if (t >= S.nseg * F.parts) return;                  // padding workgroups
    const int l = t / F.parts, part = t - l * F.parts;  // segment l of the inverse DWT's table is layer l
    const int tid = threadIdx.x, n = S.n[l], kf = F.kf, m0 = n >> kf, lm = __ffs(m0) - 1, mm = m0 * m0;
    const int per = mm / F.parts;                       // at most 4 kWB (checked by the host)
    const long coff = S.off[l];
    B = at_frame(B);
    const long fc = blockIdx.y * B.fs_c;
    const float *rin = static_cast<const float *>(F.rin) + fc;
    const float *qin = F.qin ? static_cast<const float *>(F.qin) + fc : nullptr;
    const float *bin = F.bsh ? static_cast<const float *>(F.bsh) + fc : nullptr;
    // one round of loads: the approximation block, the tables, the step and this part's operands
    const float *llin = reinterpret_cast<const float *>(B.ll + (coff >> (2 * kf)));
#pragma unroll
    for (int c = 0; c < kFoldM0 * kFoldM0 / (4 * kWB); ++c) {
        const int k4 = tid + c * kWB;
        if (4 * k4 < mm) g2lds16(llin + 4 * k4, reinterpret_cast<float *>(sL) + 4 * (c * kWB + (tid & ~63)));
    }
    const T jl = B.jinv[l * (J + 1) * 4 + min(tid, (J + 1) * 4 - 1)];
    const T adv = B.ad[l * (J + 1) + min(tid, J)];
    float o_r[4] = {}, o_q[4] = {}, o_p[4] = {}, o_b[4] = {};
    long gi[4] = {};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = tid + i * kWB;
        if (e < per) {
            const int idx = part * per + e, row = idx >> lm, col = idx & (m0 - 1);
            gi[i] = coff + (long)row * n + col;
            o_r[i] = rin[gi[i]];
            if (qin) o_q[i] = qin[gi[i]];
            if (F.e >= 1) o_p[i] = B.p[gi[i]];
            if (bin) o_b[i] = bin[gi[i]];
        }
    }
    const StepOut so = read_step(B.sc);
    if (tid < (J + 1) * 4) sJi[tid] = jl;
    if (tid <= J) sAd[tid] = adv;
    lds_fence();
    coarse_analysis(sL, m0, J - kf, tp);
    const float al = (float)so.alpha, be = (float)so.beta;
    const int log2n = __ffs(n) - 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = tid + i * kWB;
        if (e < per) {
            const int idx = part * per + e, row = idx >> lm, col = idx & (m0 - 1);
            int sl, ol;
            band_of(log2n, J, row, col, sl, ol);
            if (!so.stopped) {
                const FoldNew u = fold_pcg(sL[row * m0 + col], o_r[i], 0.0f, o_p[i], o_q[i], sJi[sl * 4 + ol], sAd[sl],
                                           al, be, F.e == 0);
                B.p[gi[i]] = u.p;
                B.q[gi[i]] = u.q;
                B.r[gi[i]] = u.r;
            }
            if (bin) B.b_prev[gi[i]] = o_b[i];
        }
    }
}

template <typename T, int MODE, int JM>
__global__ __launch_bounds__(kWB) void k_wt(SegTab S, const T *__restrict__ src, T *__restrict__ out, Bufs<T> B,
                                           Taps<T> tp, int J, FoldArgs F) {
    constexpr bool FOLD = MODE == kWtFold && sizeof(T) == 4, TAIL = MODE == kWtTail && sizeof(T) == 4;
    constexpr bool PC = MODE == kWtPcg || MODE == kWtFold;
    static_assert(JM >= 3 && JM <= kMaxJ, "level bound of the unrolled loops and cone registers");
    // the cone: wt_slots(J) slots of kWB values, the launch's dynamic LDS
    extern __shared__ __attribute__((aligned(16))) char wt_cone[];
    T *const sCone = reinterpret_cast<T *>(wt_cone);
    // synthesis regions: two LL buffers and the y-synthesis outputs.  Before the synthesis the
    // fold keeps there the second operand (q or b_prev) at the cone's coarse positions.
    __shared__ __attribute__((aligned(16))) T sSyn[2 * kWtLL + 2 * kWtX];
    static_assert((JM - 2) * kWB <= 2 * kWtLL + 2 * kWtX, "cone operands fit the synthesis regions");
    T (*const sLL)[kWtLL] = reinterpret_cast<T (*)[kWtLL]>(sSyn);
    T *const sXl = sSyn + 2 * kWtLL, *const sXh = sXl + kWtX;
    T *const sCone2 = sSyn;
    __shared__ T sJi[(JM + 1) * 4];
    // fold: the level-2 approximation (transformed in place into the coarse coefficients of W x)
    // and alpha D per level
    __shared__ __attribute__((aligned(16))) T sLLb[FOLD || TAIL ? kFoldM0 * kFoldM0 : 1];
    __shared__ T sAd[FOLD || TAIL ? JM + 1 : 1];
    __shared__ double sRed[2][FOLD ? kFoldOwn : 1];

    if constexpr (TAIL) {
        if ((int)blockIdx.x < F.ntail) {
            coarse_tail<T>(S, B, F, tp, J, (int)blockIdx.x, sLLb, sJi, sAd);
            return;
        }
    }
    const int ntail = TAIL ? F.ntail : 0;  // tiles follow the tail workgroups (a multiple of 8 of them)
    src += blockIdx.y * B.fs_c;
    out += blockIdx.y * B.fs_c;
    const int tid = threadIdx.x;
    const int tile = xcd_tile(S.chunk, (int)gridDim.x - ntail, (int)blockIdx.x - ntail);
    const TileId id = find_tile(S, tile);
    const int l = id.id, n = id.n, lt = id.lt;
    const int T0 = n < kWtTile ? n : kWtTile;
    const int y0 = (id.loc >> lt) * T0, x0 = (id.loc & ((1 << lt) - 1)) * T0;
    const long coff = id.off;

    // cone bounds (uniform; compile-time indexed, so they stay in scalar registers)
    int loY[JM + 1], loX[JM + 1], LY[JM + 1], LX[JM + 1];
    {
        int ly = y0, hy = y0 + T0 - 1, lx = x0, hx = x0 + T0 - 1;
        loY[0] = ly;
        loX[0] = lx;
        LY[0] = T0;
        LX[0] = T0;
#pragma unroll
        for (int s = 1; s <= JM; ++s) {
            ly = ((ly >> 1) - 2) & ~1;
            hy >>= 1;
            lx = ((lx >> 1) - 2) & (s == 1 ? ~3 : ~1);  // level 1 starts on a multiple of 4 (16-byte copies)
            hx >>= 1;
            loY[s] = ly;
            loX[s] = lx;
            LY[s] = hy - ly + 1;
            LX[s] = hx - lx + 1;
        }
    }
    // preconditioner of the layer's bands (PCG), loaded with the cone
    T jl = 1;
    if (PC) jl = B.jinv[l * (J + 1) * 4 + min(tid, (J + 1) * 4 - 1)];

    // fold: frame f's workspace and caller vectors; the tile's share of the layer's coarse block
    // (an sub x sub block of the m0 x m0 level-2 block, one coefficient per lane of wave 0); its
    // operands, the level-2 approximation and alpha D, all in the same round of loads as the cone
    const int kf = FOLD ? F.kf : 0, m0 = n >> kf, sub = T0 >> kf, nown = sub * sub;
    const bool own = FOLD && tid < nown;
    long gown = 0;
    T o_r = 0, o_q = 0, o_c = 0, o_p = 0, o_b = 0, adv = 0;
    const T *rin = nullptr, *qin = nullptr;
    StepOut fso{0.0, 0.0, 0};  // the step (alpha, beta, stopped) of the update the fold applies
    if constexpr (FOLD) {
        B = at_frame(B);
        const long fc = blockIdx.y * B.fs_c;
        rin = static_cast<const T *>(F.rin) + fc;
        qin = F.e >= 1 ? static_cast<const T *>(F.qin) + fc : nullptr;
        F.c = static_cast<T *>(F.c) + fc;
        F.rout = static_cast<T *>(F.rout) + fc;
        if (F.e >= 0) F.qout = static_cast<T *>(F.qout) + fc;
        else F.bsh = static_cast<T *>(F.bsh) + fc;
        const int ty = id.loc >> lt, tx = id.loc & ((1 << lt) - 1);
        const int t = own ? tid : 0, orow = ty * sub + t / sub, ocol = tx * sub + t % sub;
        gown = coff + (long)orow * n + ocol;
        o_r = rin[gown];
        if (F.e < 0) {
            o_b = B.b_prev[gown];
        } else {
            o_c = static_cast<const T *>(F.c)[gown];
            if (F.e >= 1) {
                o_q = qin[gown];
                o_p = B.p[gown];
            }
        }
        adv = B.ad[l * (J + 1) + min(tid, J)];
        if (F.e >= 0) fso = read_step(B.sc);
        const float *llin = reinterpret_cast<const float *>(B.ll + (coff >> (2 * kf)));
        const int mm = m0 * m0;
#pragma unroll
        for (int c = 0; c < kFoldM0 * kFoldM0 / (4 * kWB); ++c) {
            const int k4 = tid + c * kWB;
            if (4 * k4 < mm) g2lds16(llin + 4 * k4, reinterpret_cast<float *>(sLLb) + 4 * (c * kWB + (tid & ~63)));
        }
    }

    // ---- one batch of independent loads: the whole cone, straight into LDS ----
    // Levels 1 and 2 (most of the cone) arrive in 16-byte copies when the source is 16-byte
    // aligned and the level's column start is a multiple of 4: lane i of a 4-slot pass copies the
    // four values 4i..4i+3 of the same row-major slot block (pitch 2^lp), so the layout is that of
    // the 4-byte copies.  Rows past the cone's bands are not copied, so a pass never writes into
    // the next level's slots.
    const bool src16 = sizeof(T) == 4 && (reinterpret_cast<uintptr_t>(src) & 15) == 0;
#pragma unroll
    for (int s = 1; s <= JM; ++s) {
        if (s <= J) {
            const int lp = wt_lanes_log2(s), ly = LY[s], lx = LX[s], m = n >> s, mk = m - 1;
            if (s <= 2 && src16 && m >= 4 && (loX[s] & 3) == 0) {
                const int lq = lp - 2;  // 4-value chunks per row, log2
#pragma unroll
                for (int p4 = 0; p4 < (wt_passes(s) + 3) / 4; ++p4) {
                    const int rowi = (tid >> lq) + p4 * (kWB >> lq), q = 4 * (tid & ((1 << lq) - 1));
                    const int bi = (rowi >= ly) + (rowi >= 2 * ly) + (rowi >= 3 * ly);
                    const int r = rowi - bi * ly, o = bi == 3 ? 0 : bi + 1;
                    const int gr = ((loY[s] + r) & mk) + (o >= 2 ? m : 0);
                    const int gc = ((loX[s] + q) & mk) + ((o & 1) ? m : 0);
                    if (q < lx && rowi < (s == J ? 4 : 3) * ly)
                        g2lds16(reinterpret_cast<const float *>(src + coff + (long)gr * n + gc),
                                reinterpret_cast<float *>(sCone + (wt_slot0(s) + 4 * p4) * kWB + 4 * (tid & ~63)));
                }
                continue;
            }
            const bool coarse = FOLD && s > kf;  // fold: r before the update, and q or b_prev beside it
            const T *base = coarse ? rin : src;
            const T *base2 = coarse ? (F.e < 0 ? B.b_prev : qin) : nullptr;
#pragma unroll
            for (int p = 0; p < wt_passes(s); ++p) {
                const int rowi = (tid >> lp) + p * (kWB >> lp), q = tid & ((1 << lp) - 1);
                const int bi = (rowi >= ly) + (rowi >= 2 * ly) + (rowi >= 3 * ly);
                const int r = rowi - bi * ly, o = bi == 3 ? 0 : bi + 1;
                const int gr = ((loY[s] + r) & mk) + (o >= 2 ? m : 0);
                const int gc = ((loX[s] + q) & mk) + ((o & 1) ? m : 0);
                if (q < lx && rowi < (s == J ? 4 : 3) * ly) {
                    const T *gp = base + coff + (long)gr * n + gc;
                    T *dst = sCone + (wt_slot0(s) + p) * kWB;
                    if constexpr (sizeof(T) == 4) g2lds(gp, dst + (tid & ~63));
                    else dst[tid] = *gp;
                    if constexpr (FOLD) {
                        if (coarse && base2)
                            g2lds(base2 + coff + (long)gr * n + gc, sCone2 + (s - 3) * kWB + (tid & ~63));
                    }
                }
            }
        }
    }
    if (PC && tid < (J + 1) * 4) sJi[tid] = jl;
    if (FOLD && tid <= J) sAd[tid] = adv;
    lds_fence();
    if constexpr (FOLD) {
        coarse_analysis(sLLb, m0, J - kf, tp);
        const StepOut so = fso;
        const float al = (float)so.alpha, be = (float)so.beta;
        const int log2n = __ffs(n) - 1;
        // the tile's own coefficients: stored, with their partial sums of (r, z) and (z, alpha D z)
        double rho = 0.0, dz = 0.0;
        if (own) {
            const int t = tid, orow = (id.loc >> lt) * sub + t / sub, ocol = (id.loc & ((1 << lt) - 1)) * sub + t % sub;
            int sl, ol;
            band_of(log2n, J, orow, ocol, sl, ol);
            const float w = sLLb[orow * m0 + ocol], ji = sJi[sl * 4 + ol], ad = sAd[sl];
            float rn;
            if (F.e < 0) {
                rn = fold_rhs(w, o_b, o_r, F.cold);
                static_cast<T *>(F.bsh)[gown] = w;
                if (F.cold) static_cast<T *>(F.c)[gown] = 0;
            } else if (!so.stopped) {
                const FoldNew u = fold_pcg(w, o_r, o_c, o_p, o_q, ji, ad, al, be, F.e == 0);
                B.p[gown] = u.p;
                static_cast<T *>(F.c)[gown] = u.c;
                static_cast<T *>(F.qout)[gown] = u.q;
                rn = u.r;
            } else {
                static_cast<T *>(F.qout)[gown] = o_q;
                rn = o_r;
            }
            static_cast<T *>(F.rout)[gown] = rn;
            const T zn = rn * ji;
            rho = (double)rn * (double)zn;
            dz = (double)ad * (double)zn * (double)zn;
        }
        if (tid < kFoldOwn) {  // summed below, kFoldOwn / kFoldParts per partial pair
            sRed[0][tid] = rho;
            sRed[1][tid] = dz;
        }
        // the cone's coarse coefficients: r after the update, recomputed exactly as its owner does
#pragma unroll
        for (int s = 3; s <= JM; ++s) {  // compile-time level index: the cone bounds stay in registers
            if (s <= J && s > kf) {
                constexpr int lp = 3;
                const int ly = LY[s], lx = LX[s], m = n >> s, mk = m - 1;
                const int rowi = tid >> lp, q = tid & ((1 << lp) - 1);
                const int bi = (rowi >= ly) + (rowi >= 2 * ly) + (rowi >= 3 * ly);
                const int r = rowi - bi * ly, o = bi == 3 ? 0 : bi + 1;
                if (q < lx && rowi < (s == J ? 4 : 3) * ly) {
                    const int gr = ((loY[s] + r) & mk) + (o >= 2 ? m : 0);
                    const int gc = ((loX[s] + q) & mk) + ((o & 1) ? m : 0);
                    T *slot = sCone + wt_slot0(s) * kWB + tid;
                    const float w = sLLb[gr * m0 + gc], r0 = *slot, x2 = sCone2[(s - 3) * kWB + tid];
                    float rn;
                    if (F.e < 0) rn = fold_rhs(w, x2, r0, F.cold);
                    else if (so.stopped) rn = r0;
                    else rn = fold_pcg(w, r0, 0.0f, 0.0f, F.e >= 1 ? x2 : 0.0f, sJi[s * 4 + o], sAd[s], al, be, F.e == 0).r;
                    *slot = rn;
                }
            }
        }
        __syncthreads();
        if (tid < kFoldParts) {  // fixed-order sums of the owned coefficients' contributions
            constexpr int per = kFoldOwn / kFoldParts;
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int i = 0; i < per; ++i) {
                a += sRed[0][tid * per + i];
                b += sRed[1][tid * per + i];
            }
            B.partials[F.nfine + tile * kFoldParts + tid] = a;
            B.partials[kPartialPitch + F.nfine + tile * kFoldParts + tid] = b;
        }
    }

    // ---- synthesis, coarsest level first, all in LDS.  Levels are unrolled so that every
    // region pitch is the compile-time power of two of its level (LL_s below J and the y-pass
    // outputs use the level's pitch too).  In PCG mode the cone holds r: the band scales J^-1
    // are applied as the values are read (the synthesized LL below J is z-space already). ----
    int cur = 0;
#pragma unroll
    for (int s = JM; s >= 1; --s) {
        if (s <= J) {
            const int lp = wt_lanes_log2(s), PB = 1 << lp;
            const int lpo = s > 1 ? wt_lanes_log2(s - 1) : 5, PO = 1 << lpo;  // level 0: tiles <= 32 wide
            const int LYs = LY[s], LXs = LX[s], LYo = LY[s - 1], LXo = LX[s - 1];
            const int dY = (loY[s - 1] >> 1) - loY[s], dX = (loX[s - 1] >> 1) - loX[s];
            const T *B1 = sCone + wt_slot0(s) * kWB, *B2 = B1 + LYs * PB, *B3 = B2 + LYs * PB;
            const T *LLs = s == J ? B3 + LYs * PB : sLL[cur];
            const T jL = (PC && s == J) ? sJi[s * 4] : (T)1;
            const T j1 = PC ? sJi[s * 4 + 1] : (T)1, j2 = PC ? sJi[s * 4 + 2] : (T)1, j3 = PC ? sJi[s * 4 + 3] : (T)1;
            if (s >= 3) {
                // small coarse regions: both directions at once, one output per item (no barrier
                // between the y and x passes): the y synthesis of the three input columns the
                // output needs, in registers, then the x synthesis
                T *dst = sLL[cur ^ 1];
                for (int it = tid; it < (LYo << lpo); it += kWB) {
                    const int y = it >> lpo, xq = it & (PO - 1);
                    if (xq < LXo) {
                        const int py = y & 1, px = xq & 1, ky = (y >> 1) + dY, kx = (xq >> 1) + dX;
                        T cL[3], c1[3], c2[3], c3[3];
#pragma unroll
                        for (int jy = 0; jy < 3; ++jy) {
                            const T hy = py ? tp.h[2 * jy + 1] : tp.h[2 * jy], gy = py ? tp.g[2 * jy + 1] : tp.g[2 * jy];
                            cL[jy] = hy * jL;
                            c1[jy] = hy * j1;
                            c2[jy] = gy * j2;
                            c3[jy] = gy * j3;
                        }
                        T acc = 0;
#pragma unroll
                        for (int jx = 0; jx < 3; ++jx) {
                            T xl = 0, xh = 0;  // x-low and x-high rows of column kx - jx
#pragma unroll
                            for (int jy = 0; jy < 3; ++jy) {
                                const int o = (ky - jy) * PB + kx - jx;
                                xl += cL[jy] * LLs[o] + c2[jy] * B2[o];
                                xh += c1[jy] * B1[o] + c3[jy] * B3[o];
                            }
                            const T hx = px ? tp.h[2 * jx + 1] : tp.h[2 * jx], gx = px ? tp.g[2 * jx + 1] : tp.g[2 * jx];
                            acc += hx * xl + gx * xh;
                        }
                        dst[y * PO + xq] = acc;
                    }
                }
                __syncthreads();
                cur ^= 1;
                continue;
            }
            const int npair = (LYo + 1) >> 1;
            // y: (LL, x-low/y-high) -> x-low rows; (x-high/y-low, HH) -> x-high rows; two rows per item
            for (int it = tid; it < (npair << lp); it += kWB) {
                const int a = it >> lp, c = it & (PB - 1);
                if (c < LXs) {
                    const int at = (a + dY) * PB + c;
                    T xl0 = 0, xl1 = 0, xh0 = 0, xh1 = 0;
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const int o = at - j * PB;
                        const T ll = jL * LLs[o], b1 = j1 * B1[o], b2 = j2 * B2[o], b3 = j3 * B3[o];
                        xl0 += tp.h[2 * j] * ll + tp.g[2 * j] * b2;
                        xl1 += tp.h[2 * j + 1] * ll + tp.g[2 * j + 1] * b2;
                        xh0 += tp.h[2 * j] * b1 + tp.g[2 * j] * b3;
                        xh1 += tp.h[2 * j + 1] * b1 + tp.g[2 * j + 1] * b3;
                    }
                    sXl[(2 * a) * PB + c] = xl0;
                    sXl[(2 * a + 1) * PB + c] = xl1;
                    sXh[(2 * a) * PB + c] = xh0;
                    sXh[(2 * a + 1) * PB + c] = xh1;
                }
            }
            __syncthreads();
            // x: two output columns per item
            T *dst = sLL[cur ^ 1];
            const int lq = lpo - 1, PQ = 1 << lq;  // output pairs per row, padded
            for (int it = tid; it < (LYo << lq); it += kWB) {
                const int y = it >> lq, bq = it & (PQ - 1);
                if (2 * bq < LXo) {
                    const int at = y * PB + bq + dX;
                    T o0 = 0, o1 = 0;
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const T xl = sXl[at - j], xh = sXh[at - j];
                        o0 += tp.h[2 * j] * xl + tp.g[2 * j] * xh;
                        o1 += tp.h[2 * j + 1] * xl + tp.g[2 * j + 1] * xh;
                    }
                    if (s > 1) {
                        dst[y * PO + 2 * bq] = o0;
                        if (2 * bq + 1 < LXo) dst[y * PO + 2 * bq + 1] = o1;
                    } else {
                        T *orow = out + coff + (long)(y0 + y) * n + x0 + 2 * bq;
                        orow[0] = o0;
                        orow[1] = o1;
                    }
                }
            }
            __syncthreads();
            cur ^= 1;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Node tiles of a guide star: 16 x 16 nodes computed (a one-node halo), the inner 14 x 14
// delivered; the 15 x 15 subapertures between them carry the slopes.
// ---------------------------------------------------------------------------------------------
constexpr int kPR = kProjTile + 2;   // computed region edge (16)
constexpr int kPS = kProjTile + 1;   // subaperture block edge (15)
constexpr int kProjLch = 12;         // layers whose bilinear loads are in flight together
constexpr int kProjEntFast = 2;     // entry slots of a lane whose loads are in flight together (16 layers)

// kProjM: v = Gamma^T C Gamma P u with the partial sum C (Gamma P u)^2 (Kernel 2 of the paper);
// kProjA: s = mask Gamma P u; kProjCA: s = C mask Gamma P u; kProjPol: s = mask (add + Gamma P u)
// with the DMs' actuator grids and cell tables in place of the layers'.  phi = P u comes from the bilinear cell tables of the region's 16
// rows and columns on every layer, staged in LDS; each lane then gathers its node's four
// neighbours on kProjLch layers at a time and sums the layers in order.
template <typename T, int MODE>
__global__ __launch_bounds__(kB) void k_proj(SegTab S, LayTab LT, InvVar IV, PupilArgs pa, const T *__restrict__ u,
                                             T *__restrict__ out, const T *__restrict__ add, Bufs<T> B, int nl) {
    // the cell entries [axis][layer][line] (cell, weights), the launch's dynamic LDS for its nl
    // layers (proj_lds)
    extern __shared__ __attribute__((aligned(16))) char proj_ent[];
    int *const sK = reinterpret_cast<int *>(proj_ent);
    T *const sW0 = reinterpret_cast<T *>(proj_ent + sizeof(T) * 2 * nl * kPR);  // after sK, T-aligned
    T *const sW1 = sW0 + 2 * nl * kPR;
    __shared__ T sPhi[kPR * kPR];
    __shared__ T sSx[kPS * kPS], sSy[kPS * kPS];

    B = at_frame(B);
    u += blockIdx.y * (MODE == kProjPol ? B.fs_a : B.fs_c);
    out += blockIdx.y * (MODE == kProjM ? B.fs_v : B.fs_s);
    if (MODE == kProjPol) add += blockIdx.y * B.fs_s;
    const int tid = threadIdx.x;
    const int tile = xcd_tile(S.chunk, gridDim.x);
    const TileId id = find_tile(S, tile);
    const int g = id.id, ns = id.n, tpr = id.lt;
    const int ti = id.loc / tpr, tj = id.loc - ti * tpr;
    const int i0 = ti * kProjTile, j0 = tj * kProjTile;
    const Ent<T> *__restrict__ xt = (MODE == kProjPol ? B.xdm : B.xtab) + (long)g * nl * B.maxnv;
    const Ent<T> *__restrict__ yt = (MODE == kProjPol ? B.ydm : B.ytab) + (long)g * nl * B.maxnv;

    // cell entries of the region's rows and columns on every layer: e = (l * 2 + axis) * 16 + idx,
    // stored at [(axis * nl + l) * kPR + idx]; the first kProjEntFast slots of a lane load together
    // (lanes past the last entry load nothing, so whole waves drop out), the rest (over 16 layers)
    // one after another
    {
        const int ne = 2 * nl * kPR;
        auto entry = [&](int e) {
            const int l = e >> 5, axis = (e >> 4) & 1, idx = e & 15;
            int nd = (axis ? i0 : j0) - 1 + idx;
            nd = nd < 0 ? 0 : (nd > ns ? ns : nd);
            return (axis ? yt : xt)[(long)l * B.maxnv + nd];
        };
        auto store = [&](int e, const Ent<T> &en) {
            const int l = e >> 5, axis = (e >> 4) & 1, idx = e & 15, at = (axis * nl + l) * kPR + idx;
            sK[at] = en.k0;
            sW0[at] = en.w0;
            sW1[at] = en.w1;
        };
        Ent<T> en[kProjEntFast];
#pragma unroll
        for (int c = 0; c < kProjEntFast; ++c) en[c] = tid + c * kB < ne ? entry(tid + c * kB) : Ent<T>{};
#pragma unroll
        for (int c = 0; c < kProjEntFast; ++c)
            if (tid + c * kB < ne) store(tid + c * kB, en[c]);
        for (int e = tid + kProjEntFast * kB; e < ne; e += kB) store(e, entry(e));
    }
    __syncthreads();

    const int a = tid >> 4, b = tid & 15, i = i0 - 1 + a, j = j0 - 1 + b;
    const bool node = i >= 0 && i <= ns && j >= 0 && j <= ns;
    const int lay_off = LT.off[tid & 63], lay_n = LT.n[tid & 63];  // lane l holds layer l
    T phi = 0;
    for (int l0 = 0; l0 < nl; l0 += kProjLch) {
        T uv[kProjLch][4];
#pragma unroll
        for (int c = 0; c < kProjLch; ++c) {
            const int l = min(l0 + c, nl - 1);
            if (l0 + c < nl) {
                const int n = __builtin_amdgcn_readlane(lay_n, l);
                const T *U = u + __builtin_amdgcn_readlane(lay_off, l) + (long)sK[(nl + l) * kPR + a] * n + sK[l * kPR + b];
                uv[c][0] = U[0];
                uv[c][1] = U[1];
                uv[c][2] = U[n];
                uv[c][3] = U[n + 1];
            } else {
                uv[c][0] = uv[c][1] = uv[c][2] = uv[c][3] = (T)0;
            }
        }
        // slots past the last layer (a branch uniform over the workgroup) load nothing and hold
        // zeros; every slot reads its weights at the clamped layer, so that the weight reads of
        // all slots issue together
#pragma unroll
        for (int c = 0; c < kProjLch; ++c) {
            const int l = min(l0 + c, nl - 1);
            const T wy0 = sW0[(nl + l) * kPR + a], wy1 = sW1[(nl + l) * kPR + a], wx0 = sW0[l * kPR + b],
                    wx1 = sW1[l * kPR + b];
            phi += (wy0 * wx0) * uv[c][0] + (wy0 * wx1) * uv[c][1] + (wy1 * wx0) * uv[c][2] +
                   (wy1 * wx1) * uv[c][3];  // (garbage on rows outside the grid: sPhi drops it)
        }
    }
    sPhi[tid] = node ? phi : (T)0;
    __syncthreads();

    double e2 = 0.0;
    if (tid < kPS * kPS) {
        const int aa = tid / kPS, bb = tid - aa * kPS, ii = i0 - 1 + aa, jj = j0 - 1 + bb;
        T sx = 0, sy = 0;
        const bool act = ii >= 0 && ii < ns && jj >= 0 && jj < ns && subap_active(pa, ns, ii, jj);
        if (act) {
            const T p00 = sPhi[aa * kPR + bb], p01 = sPhi[aa * kPR + bb + 1];
            const T p10 = sPhi[(aa + 1) * kPR + bb], p11 = sPhi[(aa + 1) * kPR + bb + 1];
            sx = (T)0.5 * ((p01 - p00) + (p11 - p10));
            sy = (T)0.5 * ((p10 - p00) + (p11 - p01));
        }
        const bool own = aa >= 1 && bb >= 1 && ii < ns && jj < ns;
        if (MODE == kProjPol) {
            if (own) {
                const long ix = id.aux + (long)ii * ns + jj, iy = ix + (long)ns * ns;
                out[ix] = act ? add[ix] + sx : (T)0;
                out[iy] = act ? add[iy] + sy : (T)0;
            }
        } else if (MODE != kProjM) {
            const T wgt = MODE == kProjCA ? (T)IV.v[g] : (T)1;
            if (own) {
                out[id.aux + (long)ii * ns + jj] = wgt * sx;
                out[id.aux + (long)ns * ns + (long)ii * ns + jj] = wgt * sy;
            }
        } else {
            const double iv = IV.v[g];
            if (own && act) e2 = iv * ((double)sx * (double)sx + (double)sy * (double)sy);
            sSx[tid] = (T)iv * sx;
            sSy[tid] = (T)iv * sy;
        }
    }
    if (MODE != kProjM) return;
    __syncthreads();
    if (tid < kProjTile * kProjTile) {
        const int aa = tid / kProjTile, bb = tid - aa * kProjTile, ii = i0 + aa, jj = j0 + bb;
        if (ii <= ns && jj <= ns) {
            // node (i, j) is a corner of subapertures (i, j), (i, j-1), (i-1, j), (i-1, j-1)
            const int s11 = (aa + 1) * kPS + (bb + 1), s10 = (aa + 1) * kPS + bb, s01 = aa * kPS + (bb + 1),
                      s00 = aa * kPS + bb;
            out[id.off + (long)ii * id.pitch + jj] =
                (T)0.5 * ((-sSx[s11] - sSy[s11]) + (sSx[s10] - sSy[s10]) + (-sSx[s01] + sSy[s01]) + (sSx[s00] + sSy[s00]));
        }
    }
    // one partial per wave, no block reduction: slots tile * (kB / 64) + wave (by tile, so that the
    // sums' order does not depend on the workgroup order)
    static_assert(kB / 64 == kProjWaves, "one projection partial slot per wave");
    e2 = wave_sum(e2);
    if ((tid & 63) == 0) B.partials[2 * kPartialPitch + tile * kProjWaves + (tid >> 6)] = e2;
}

// Gamma^T C s (kGtRhs) or Gamma^T mask s (kGtAdj) on the node tiles of k_proj.
template <typename T, int MODE>
__global__ __launch_bounds__(kB) void k_gt(SegTab S, InvVar IV, PupilArgs pa, const T *__restrict__ in,
                                           T *__restrict__ v, long fs_s, long fs_v) {
    __shared__ T sSx[kPS * kPS], sSy[kPS * kPS];
    in += blockIdx.y * fs_s;
    v += blockIdx.y * fs_v;
    const int tid = threadIdx.x;
    const TileId id = find_tile(S, xcd_tile(S.chunk, gridDim.x));
    const int g = id.id, ns = id.n, tpr = id.lt;
    const int ti = id.loc / tpr, tj = id.loc - ti * tpr;
    const int i0 = ti * kProjTile, j0 = tj * kProjTile;
    {
        const int t = tid < kPS * kPS ? tid : 0;
        const int aa = t / kPS, bb = t - aa * kPS, ii = i0 - 1 + aa, jj = j0 - 1 + bb;
        const bool in_grid = ii >= 0 && ii < ns && jj >= 0 && jj < ns;
        const long at = id.aux + (in_grid ? (long)ii * ns + jj : 0L);  // every lane loads
        const T vx = in[at], vy = in[at + (long)ns * ns];
        if (tid < kPS * kPS) {
            const bool act = in_grid && subap_active(pa, ns, ii, jj);
            const T w = (MODE == kGtAdj) ? (T)1 : (T)IV.v[g];
            sSx[tid] = act ? w * vx : (T)0;
            sSy[tid] = act ? w * vy : (T)0;
        }
    }
    __syncthreads();
    if (tid < kProjTile * kProjTile) {
        const int aa = tid / kProjTile, bb = tid - aa * kProjTile, ii = i0 + aa, jj = j0 + bb;
        if (ii <= ns && jj <= ns) {
            const int s11 = (aa + 1) * kPS + (bb + 1), s10 = (aa + 1) * kPS + bb, s01 = aa * kPS + (bb + 1),
                      s00 = aa * kPS + bb;
            v[id.off + (long)ii * id.pitch + jj] =
                (T)0.5 * ((-sSx[s11] - sSy[s11]) + (sSx[s10] - sSy[s10]) + (-sSx[s01] + sSy[s01]) + (sSx[s00] + sSy[s00]));
        }
    }
}

// ---------------------------------------------------------------------------------------------
// P^T
// ---------------------------------------------------------------------------------------------
// Staged gather on a 16 x 16 layer tile.  The transpose-table lines of the tile's rows and
// columns (rw (node, weight) pairs each, per guide star, rw the layer's largest pair count, at
// most kRtabWidth) and each guide star's record (the node rows / columns those pairs name and the
// largest pair count over the tile's rows / columns, precomputed at bind time) come first.  Each
// guide star's node rectangle is then staged in LDS, widened to 16-byte column chunks (node grid
// rows are 16-byte aligned), one guide star after the other with one 16-byte copy per lane and
// chunk, and each lane sums
//   x(k, q) = sum_g sum_{(i, wy) in row k} wy sum_{(j, wx) in column q} wx v_g(i, j)
// from LDS, with loop bounds uniform over the tile (missing pairs carry weight 0).  The pairs are
// the very matrix entries P uses, so P^T is P's exact transpose.

// The sum of one lane over the guide stars with R pairs per line (R the layer's pair width, so
// that the loops unroll): every R x R pair product of a guide star is summed without per-pair
// conditions, so that its LDS reads issue together.  The entries carry staged offsets (a row
// entry the offset of its node row in the stage, a column entry its column within the row), so
// that a product reads sV at the sum of the two; pairs past a line's count are padding (weight 0,
// offset of the rectangle's first row / column), adding exact zeros.  Only a guide star with no
// rectangle on this tile is skipped.
template <typename T, int R, int RS>
__device__ __forceinline__ T pt_sum(const RtabEnt<T> *sPairs, const T *sV, int nw, int a, int b, int pitch) {
    // the pairs of line idx, entry e, axis, guide star g at [((g * 2 + axis) * RS + e) * 16 + idx]
    // (RS >= R entries stored per line; the first R are summed)
    const RtabEnt<T>(*sP)[2][RS][kPtTile] = reinterpret_cast<const RtabEnt<T>(*)[2][RS][kPtTile]>(sPairs);
    T acc = 0;
    for (int g = 0; g < nw; ++g) {
        if (__builtin_amdgcn_readlane(pitch, g) == 0) continue;
        int jx[R];
        T wx[R];
#pragma unroll
        for (int e = 0; e < R; ++e) {
            const RtabEnt<T> p = sP[g][0][e][b];
            jx[e] = p.idx;
            wx[e] = p.w;
        }
#pragma unroll
        for (int ea = 0; ea < R; ++ea) {
            const RtabEnt<T> p = sP[g][1][ea][a];
            const T *Vr = sV + p.idx;
            T t = 0;
#pragma unroll
            for (int eb = 0; eb < R; ++eb) t += wx[eb] * Vr[jx[eb]];
            acc += p.w * t;
        }
    }
    return acc;
}

// R: the plan's widest pair count (the launch's template argument): every layer's lines are read
// with R entries, the ones past a line's count being the tables' padding (index -1, weight 0).
template <typename T, int R>
__global__ __launch_bounds__(kB) void k_pt(SegTab S, WfsOff WO, const T *__restrict__ v, T *__restrict__ x, Bufs<T> B,
                                           int nw, PassArgs PA) {
    constexpr int NT = kPtTile, RW = kRtabWidth, CH = 16 / sizeof(T);  // values per 16-byte chunk
    static_assert(NT == 16 && 2 * kPtMaxWfs * NT == 2 * kB, "line decode below assumes these sizes");
    static_assert(R >= 1 && R <= RW, "pair width");
    // dynamic LDS: the tile's (node, weight) pairs [g][axis][entry][line], then the staged node
    // rectangles
    extern __shared__ char smem_raw[];
    RtabEnt<T> *sP = reinterpret_cast<RtabEnt<T> *>(smem_raw);
    T *sV = reinterpret_cast<T *>(smem_raw + sizeof(RtabEnt<T>) * 2 * R * NT * nw);

    B = at_frame(B);
    v += blockIdx.y * B.fs_v;
    x += blockIdx.y * B.fs_c;
    if (PA.k >= 0 && blockIdx.x == gridDim.x - 1) {  // the pass's scalar step (extra workgroup)
        scalar_step(B.partials, PA.nwt, PA.nproj, B.sc, PA.k, PA.resnorm ? PA.resnorm + blockIdx.y * PA.rstride : nullptr,
                    PA.publish);
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int vt = xcd_tile(S.chunk, PA.k >= 0 ? (int)gridDim.x - 1 : (int)gridDim.x);

    // lane g of every wave holds guide star g's record: node rows iA..iB, first staged column c0
    // (16-byte aligned), last column jB, pair counts, node grid offset / pitch, and the LDS
    // offset / pitch of its staged rectangle.  The records are indexed by the tile number alone,
    // so they (and the copies they drive) go out before the segment lookup, whose round trip
    // then overlaps theirs.
    const int tg = min(lane, nw - 1);
    const int4 rec = B.rects[(long)vt * nw + tg];
    const int gv = WO.v_off[tg], gp = WO.vp[tg];
    const int iA = rec.x & 0xffff, iB = rec.x >> 16, c0 = (rec.y & 0xffff) & ~(CH - 1), jB = rec.y >> 16;
    const int pitch = lane < nw && iA <= iB ? ((jB - c0) / CH + 1) * CH : 0;
    const int sz = pitch ? (iB - iA + 1) * pitch : 0;
    int incl = sz;  // inclusive prefix sum over the lanes
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const int sbase = incl - sz;

    // node rectangles: wave w copies those of guide stars w, w + kB / 64, ... (the copies of all
    // of them in flight); item it of guide star g (row it / chunks, 16-byte chunk it % chunks of
    // the row) lands at sV + sbase_g + it CH
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int g = wave; g < nw; g += kB / 64) {
        const int pg = __builtin_amdgcn_readlane(pitch, g);
        if (pg == 0) continue;
        const int ra = __builtin_amdgcn_readlane(iA, g), rb = __builtin_amdgcn_readlane(iB, g);
        const int cg = __builtin_amdgcn_readlane(c0, g), bg = __builtin_amdgcn_readlane(sbase, g);
        const int vg = __builtin_amdgcn_readlane(gv, g), vpg = __builtin_amdgcn_readlane(gp, g);
        const int chunks = pg / CH, items = (rb - ra + 1) * chunks;
        const float rch = 1.0f / (float)chunks;
        for (int i0 = 0; i0 < items; i0 += 64) {
            const int it = i0 + lane;
            if (it < items) {
                const int r = small_div(it, rch), c4 = it - r * chunks;
                const T *src = v + vg + (long)(ra + r) * vpg + cg + c4 * CH;
                if constexpr (sizeof(T) == 4) {
                    g2lds16(src, sV + bg + i0 * CH);
                } else {
#pragma unroll
                    for (int e = 0; e < CH; ++e) sV[bg + it * CH + e] = src[e];
                }
            }
        }
    }

    const TileId id = find_tile(S, vt);
    const int n = id.n, lt = id.lt;
    const int T0 = n < NT ? n : NT;
    const int k0 = (id.loc >> lt) * T0, q0 = (id.loc & ((1 << lt) - 1)) * T0;
    const int roff = id.aux, rw = id.rw;  // this layer's pair count per line (at most R)

    // the first R pairs of the transpose-table lines e = (g * 2 + axis) * 16 + idx; lanes of guide
    // stars the plan does not have load nothing (32 lanes share g, so whole waves drop out), and
    // a clamped index stands in for a line the tile does not have
    RtabEnt<T> pe[2][R];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int e = tid + c * kB, g = e >> 5, axis = (e >> 4) & 1, idx = min(e & 15, T0 - 1);
        if (g < nw) {
            const RtabEnt<T> *rt = (axis ? B.yrtab : B.xrtab) + ((long)g * B.sum_n + roff + (axis ? k0 : q0) + idx) * RW;
#pragma unroll
            for (int a = 0; a < R; ++a) pe[c][a] = rt[a];
        } else {
#pragma unroll
            for (int a = 0; a < R; ++a) pe[c][a] = RtabEnt<T>{0, T(0)};
        }
    }
    // written with their staged offsets: a row entry sbase + (max(i, iA) - iA) pitch, a column
    // entry max(j, c0) - c0, from guide star g's record (lane g of this wave)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int e = tid + c * kB, g = e >> 5, axis = (e >> 4) & 1, idx = e & 15;
        const int ga = __shfl(iA, g, 64), gc = __shfl(c0, g, 64), gpt = __shfl(pitch, g, 64), gsb = __shfl(sbase, g, 64);
        if (g < nw && idx < T0) {
#pragma unroll
            for (int a = 0; a < R; ++a) {
                RtabEnt<T> p = pe[c][a];
                p.idx = axis ? gsb + (max(p.idx, ga) - ga) * gpt : max(p.idx, gc) - gc;
                sP[((g * 2 + axis) * R + a) * NT + idx] = p;
            }
        }
    }
    lds_fence();

    const int a = tid >> 4, b = tid & 15;
    if (a < T0 && b < T0) {
        T acc;
        if (R >= 2 && rw == 1) acc = pt_sum<T, 1, R>(sP, sV, nw, a, b, pitch);  // uniform over the workgroup
        else if (R >= 3 && rw == 2) acc = pt_sum<T, (R >= 3 ? 2 : R), R>(sP, sV, nw, a, b, pitch);
        else if (R >= 4 && rw == 3) acc = pt_sum<T, (R >= 4 ? 3 : R), R>(sP, sV, nw, a, b, pitch);
        else acc = pt_sum<T, R, R>(sP, sV, nw, a, b, pitch);
        x[id.off + (long)(k0 + a) * n + q0 + b] = acc;
    }
}

// By scanning the cell tables over each layer node's contiguous node ranges (any geometry).
template <typename T>
__global__ __launch_bounds__(kB) void k_pt_scan(SegTab S, const T *__restrict__ v, T *__restrict__ x, Bufs<T> B,
                                                int nl, int nw, PassArgs PA) {
    constexpr int NT = kPtTile;
    B = at_frame(B);
    v += blockIdx.y * B.fs_v;
    x += blockIdx.y * B.fs_c;
    if (PA.k >= 0 && blockIdx.x == gridDim.x - 1) {  // the pass's scalar step (extra workgroup)
        scalar_step(B.partials, PA.nwt, PA.nproj, B.sc, PA.k, PA.resnorm ? PA.resnorm + blockIdx.y * PA.rstride : nullptr,
                    PA.publish);
        return;
    }
    const int vt = xcd_tile(S.chunk, PA.k >= 0 ? (int)gridDim.x - 1 : (int)gridDim.x);
    const TileId id = find_tile(S, vt);
    const int l = id.id, n = id.n, lt = id.lt;
    const int T0 = n < NT ? n : NT;
    const int a = threadIdx.x >> 4, b = threadIdx.x & 15;
    if (a >= T0 || b >= T0) return;
    const int k = (id.loc >> lt) * T0 + a, q = (id.loc & ((1 << lt) - 1)) * T0 + b;
    T acc = 0;
    for (int g = 0; g < nw; ++g) {
        const Range rx = B.xrng[(long)g * B.sum_n + id.aux + q];
        const Range ry = B.yrng[(long)g * B.sum_n + id.aux + k];
        if (rx.lo > rx.hi || ry.lo > ry.hi) continue;
        const Ent<T> *xt = B.xtab + ((long)g * nl + l) * B.maxnv;
        const Ent<T> *yt = B.ytab + ((long)g * nl + l) * B.maxnv;
        const DevWfs W = B.wfs[g];
        const T *vg = v + W.v_off;
        for (int i = ry.lo; i <= ry.hi; ++i) {
            const Ent<T> ey = yt[i];
            const T wy = (ey.k0 == k) ? ey.w0 : ey.w1;
            const T *row = vg + (long)i * W.vp;
            for (int j = rx.lo; j <= rx.hi; ++j) {
                const Ent<T> ex = xt[j];
                const T wx = (ex.k0 == q) ? ex.w0 : ex.w1;
                acc += (wy * wx) * row[j];
            }
        }
    }
    x[id.off + (long)k * n + q] = acc;
}

// ---------------------------------------------------------------------------------------------
// Forward transform W with fused epilogues.
// ---------------------------------------------------------------------------------------------
// Global index of coefficient (r, q) of band o (0 LL, 1 x-high/y-low, 2 x-low/y-high, 3 HH) at
// level s.
__device__ __forceinline__ long band_index(long coff, int n, int s, int o, int r, int q) {
    const int m = n >> s;
    return coff + (long)(r + (o >= 2 ? m : 0)) * n + q + ((o & 1) ? m : 0);
}

// One 2D analysis step on the 6 x 6 input patch at (2r, 2q): rows along x, then columns along y.
template <typename T>
__device__ __forceinline__ void analyse(const T *src, int pitch, int r, int q, const Taps<T> &tp, T &ll, T &hl,
                                        T &lh, T &hh) {
    ll = hl = lh = hh = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        const T *row = src + (2 * r + a) * pitch + 2 * q;
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
}

template <int EPI>
struct EpiOps {
    static constexpr int n = EPI == kEpiPcg ? 4 : (EPI == kEpiRhs ? 2 : (EPI == kEpiPrior ? 1 : 0));
};

// Operands of coefficient i: prior c | pcg r, c, p, q | rhs b_prev, r.
template <typename T, int EPI>
__device__ __forceinline__ void epi_load(const Bufs<T> &B, const FwdArgs &E, long i, T *op) {
    if constexpr (EPI == kEpiPrior) {
        op[0] = static_cast<const T *>(E.cin)[i];
    } else if constexpr (EPI == kEpiPcg) {
        op[0] = E.r_in ? static_cast<const T *>(E.r_in)[i] : B.r[i];
        op[1] = E.c ? static_cast<const T *>(E.c)[i] : (T)0;
        op[2] = E.k > 0 ? B.p[i] : (T)0;
        op[3] = E.k > 0 ? (E.q_in ? static_cast<const T *>(E.q_in)[i] : B.q[i]) : (T)0;
    } else if constexpr (EPI == kEpiRhs) {
        op[0] = E.cold ? (T)0 : B.b_prev[i];
        op[1] = E.cold ? (T)0 : B.r[i];
    }
}

// Deliver coefficient i of W x (value w) through the epilogue.  pcg and rhs also accumulate the
// next pass's (r, z) and (z, alpha D z) over the residual they write (z = J^-1 r).
template <typename T, int EPI>
__device__ __forceinline__ void epi_store(const Bufs<T> &B, const FwdArgs &E, long i, T w, const T *op, T ji, T ad,
                                          const StepOut &so, double &rho, double &dz) {
    if constexpr (EPI == kEpiPlain) {
        static_cast<T *>(E.out)[i] = w;
    } else if constexpr (EPI == kEpiPrior) {
        static_cast<T *>(E.out)[i] = w + ad * op[0];
        if (E.rzero) B.r[i] = 0;
    } else if constexpr (EPI == kEpiPcg) {
        T rn = op[0];
        if (!so.stopped) {
            const T r = op[0], z = r * ji, y = w + ad * z;
            const T al = (T)so.alpha, be = (T)so.beta;
            const T p = E.k > 0 ? z + be * op[2] : z;
            const T q = E.k > 0 ? y + be * op[3] : y;
            B.p[i] = p;
            B.q[i] = q;
            if (E.c) static_cast<T *>(E.c)[i] = op[1] + al * p;
            rn = r - al * q;
            B.r[i] = rn;
        }
        if (E.b_in) B.b_prev[i] = static_cast<const T *>(E.b_in)[i];
        const T zn = rn * ji;
        rho += (double)rn * (double)zn;
        dz += (double)ad * (double)zn * (double)zn;
    } else {  // b = W x:  r = (b - b_prev) + r  (cold: r = b, c = 0);  b_prev = b
        T rn;
        if (E.cold) {
            rn = w;
            static_cast<T *>(E.c)[i] = 0;
        } else {
            rn = (w - op[0]) + op[1];
        }
        B.r[i] = rn;
        B.b_prev[i] = w;
        const T zn = rn * ji;
        rho += (double)rn * (double)zn;
        dz += (double)ad * (double)zn * (double)zn;
    }
}

// Level region of the fine part: a tile of TQ x TQ level-KF quads needs LL_s on a run of
// len(s) = TQ 2^(KF-s) + 4 (2^(KF-s) - 1) indices (s = 0 is x) and owns TQ 2^(KF-s) of them.
template <int KF, int TQ>
struct FineGeom {
    static constexpr int len(int s) { return TQ * (1 << (KF - s)) + 4 * ((1 << (KF - s)) - 1); }
    static constexpr int own(int s) { return TQ << (KF - s); }
};

// Levels 1..KF on a tile of TQ x TQ level-KF quads.  The input region with its periodic halo
// (straight into LDS), the epilogue operands of the coefficients each lane will deliver, and
// (pcg) the pass's scalar step arrive in one round of loads; the levels then run from LDS.  Lane
// roles: lanes [0, O1^2) own the level-1 quads, the next H1 lanes compute the level-1 halo quads
// (LL only, for level 2), and the O2^2 lanes from fwd_l2<KF, TQ>() own the level-2 quads.
template <int KF, int TQ>
struct FwdLanes {
    static constexpr int O1 = TQ << (KF - 1), L1 = TQ * (1 << (KF - 1)) + 4 * ((1 << (KF - 1)) - 1);
    static constexpr int H1 = KF >= 2 ? L1 * L1 - O1 * O1 : 0;
    static constexpr int O2 = KF >= 2 ? TQ : 1;
    static constexpr int l2 = ((O1 * O1 + H1 + 63) / 64) * 64;  // first level-2 lane (wave aligned)
    static constexpr int block = ((KF >= 2 ? l2 + O2 * O2 : O1 * O1) + 255) / 256 * 256;
};

template <typename T, int KF, int TQ, int EPI>
__global__ __launch_bounds__((FwdLanes<KF, TQ>::block)) void k_fwd(SegTab S, const T *__restrict__ x, Bufs<T> B, FwdArgs E,
                                                                    Taps<T> tp, int J) {
    using G = FineGeom<KF, TQ>;
    using R = FwdLanes<KF, TQ>;
    constexpr int FB = R::block, L0 = G::len(0), L1 = G::len(1), NX = (L0 * L0 + FB - 1) / FB;
    constexpr int O1 = R::O1, O2 = R::O2, H1 = R::H1, L2 = R::l2;
    constexpr int NOP = EpiOps<EPI>::n, HW = L1 > O1 ? L1 - O1 : 1;
    __shared__ T sA[L0 * L0];
    __shared__ T sB[KF >= 2 ? L1 * L1 : 1];

    B = at_frame(B);
    E = frame_args<T>(E, B.fs_c);
    x += blockIdx.y * B.fs_c;
    const int tid = threadIdx.x;
    if constexpr (EPI == kEpiRhs) {
        if (blockIdx.x == 0 && tid == 0) reset_scalars(B.sc + 1);  // the state "before pass 0"
    }
    const int tile = xcd_tile(S.chunk, gridDim.x);
    const TileId id = find_tile(S, tile);
    const int l = id.id, n = id.n, lt = id.lt, nm = n - 1;
    const int qy = (id.loc >> lt) * TQ, qx = (id.loc & ((1 << lt) - 1)) * TQ;
    const long coff = id.off;
    const int oy = qy << KF, ox = qx << KF;

    // x region with its periodic halo, straight into LDS (row-major, pitch L0)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
        const int k = tid + c * FB;
        if (k < L0 * L0) {
            const int r = k / L0, q = k - r * L0;
            const T *gp = x + coff + (long)((oy + r) & nm) * n + ((ox + q) & nm);
            if constexpr (sizeof(T) == 4) g2lds(gp, sA + c * FB + (tid & ~63));
            else sA[k] = *gp;
        }
    }
    // the quad this lane delivers: level 1 (owner), level 2 (owner), or none (quad 0 of level 1
    // stands in so that every lane issues the same loads)
    const bool own1 = tid < O1 * O1, own2 = KF >= 2 && tid >= L2 && tid < L2 + O2 * O2;
    const int s_own = own2 ? 2 : 1;
    const int t1 = own1 ? tid : 0, t2 = own2 ? tid - L2 : 0;
    const int rq = own2 ? t2 / O2 : t1 / O1, cq = own2 ? t2 - (t2 / O2) * O2 : t1 - (t1 / O1) * O1;
    const int by = (qy << (KF - s_own)) + rq, bx = (qx << (KF - s_own)) + cq;
    T op[4][NOP > 0 ? NOP : 1];
    if (NOP > 0) {
#pragma unroll
        for (int o = 0; o < 4; ++o)
            if (o > 0 || KF == J) epi_load<T, EPI>(B, E, band_index(coff, n, s_own, o, by, bx), op[o]);
    }
    // prior weight and Jacobi factors of the lane's level, in the same round of loads
    T ad = 0, ji[4] = {0, 0, 0, 0};
    if (EPI != kEpiPlain) ad = B.ad[l * (J + 1) + s_own];
    if (EPI == kEpiPcg || EPI == kEpiRhs) {
#pragma unroll
        for (int o = 0; o < 4; ++o) ji[o] = B.jinv[(l * (J + 1) + s_own) * 4 + o];
    }
    // last pass (cc set): this tile's share of the layer's coarse block of c, the level-KF
    // positions of its TQ x TQ quads, stepped here (c + alpha p, p = z + beta p_old, z = J^-1 r
    // needs no W x), so that the coarse levels' launch leaves c alone
    T cr = 0, cp = 0, cv = 0, cj = 0;
    long ci = 0;
    bool cown = false;
    if constexpr (EPI == kEpiPcg) {
        cown = KF < J && E.cc != nullptr && tid < TQ * TQ;
        if (cown) {
            const int ry = qy + tid / TQ, rx = qx + tid % TQ;
            int sl, ol;
            band_of(__ffs(n) - 1, J, ry, rx, sl, ol);
            ci = coff + (long)ry * n + rx;
            cr = E.cc_r ? static_cast<const T *>(E.cc_r)[ci] : B.r[ci];
            cp = E.k > 0 ? B.p[ci] : (T)0;
            cv = static_cast<const T *>(E.cc)[ci];
            cj = B.jinv[(l * (J + 1) + sl) * 4 + ol];
        }
    }
    StepOut so{0.0, 0.0, 0};
    if constexpr (EPI == kEpiPcg) so = read_step(B.sc);
    lds_fence();

    if constexpr (EPI == kEpiPcg) {
        if (cown && !so.stopped) {
            const T z = cr * cj, al = (T)so.alpha, be = (T)so.beta;
            const T p = E.k > 0 ? z + be * cp : z;
            static_cast<T *>(E.cc)[ci] = cv + al * p;
        }
    }
    double rho = 0.0, dz = 0.0;  // (r, z), (z, alpha D z) of the residual written (pcg, rhs)
#pragma unroll
    for (int s = 1; s <= KF; ++s) {
        const T *src = s == 1 ? sA : sB;
        const int sp = s == 1 ? L0 : L1;
        const bool mine = s == 1 ? own1 : own2;
        if (mine) {
            T w[4];
            analyse(src, sp, rq, cq, tp, w[0], w[1], w[2], w[3]);
#pragma unroll
            for (int o = 1; o < 4; ++o) epi_store<T, EPI>(B, E, band_index(coff, n, s, o, by, bx), w[o], op[o], ji[o], ad, so, rho, dz);
            if (s < KF) {
                sB[rq * L1 + cq] = w[0];
            } else if (KF == J) {
                epi_store<T, EPI>(B, E, band_index(coff, n, s, 0, by, bx), w[0], op[0], ji[0], ad, so, rho, dz);
            } else {
                B.ll[(coff >> (2 * KF)) + (long)by * (n >> KF) + bx] = w[0];
            }
        }
        if (s < KF && tid >= O1 * O1 && tid < O1 * O1 + H1) {  // halo quads of level 1: LL only
            const int h = tid - O1 * O1, rs = O1 * HW;
            int hr, hc;
            if (h < rs) {
                hr = h / HW;
                hc = O1 + h - hr * HW;
            } else {
                hr = O1 + (h - rs) / L1;
                hc = (h - rs) - (hr - O1) * L1;
            }
            T w[4];
            analyse(src, sp, hr, hc, tp, w[0], w[1], w[2], w[3]);
            sB[hr * L1 + hc] = w[0];
        }
        if (s < KF) __syncthreads();
    }
    if constexpr (EPI == kEpiPcg || EPI == kEpiRhs) {
        // one partial pair per wave, no block reduction: slots tile * (FB / 64) + wave (by tile)
        rho = wave_sum(rho);
        dz = wave_sum(dz);
        if ((tid & 63) == 0) {
            const int slot = tile * (FB / 64) + (tid >> 6);
            B.partials[slot] = rho;
            B.partials[kPartialPitch + slot] = dz;
        }
    }
}

// Levels KF+1..J of one layer per workgroup, from the level-KF approximation left by k_fwd
// (periodic, so indices wrap).  Every coefficient of these levels lies in the layer's top-left
// m0 x m0 block (m0 = n >> KF).  With `pre`, that block of every epilogue operand is staged in
// LDS together with the approximation, in one round of loads; otherwise each level requests its
// operands before its analysis.  Dynamic LDS: m0^2 + (m0/2)^2 (+ NOP m0^2 with `pre`) values.
// With `gin` (a block too large for LDS) level KF+1 reads the approximation from global memory
// and the LDS holds only the smaller levels: (m0/4)^2 + (m0/2)^2 values.
// Operand modes of the coarse levels (compile time, so that the staged mode's level loop holds no
// global-memory waits): operands staged in LDS | loaded per level | loaded per level, with level
// KF+1 reading the approximation from global memory.
enum { kCoarseStaged = 0, kCoarseDirect = 1, kCoarseGlobalIn = 2 };

template <typename T, int EPI, int CM>
__global__ __launch_bounds__(kCB) void k_coarse(LayTab LT, Bufs<T> B, FwdArgs E, Taps<T> tp, int J, int KF, int nfine) {
    constexpr bool pre = CM == kCoarseStaged && EpiOps<EPI>::n > 0, gin = CM == kCoarseGlobalIn;
    extern __shared__ char smem_raw[];
    constexpr int NOP = EpiOps<EPI>::n, NL = 16;
    B = at_frame(B);
    E = frame_args<T>(E, B.fs_c);
    const int tid = threadIdx.x, l = blockIdx.x, n = LT.n[l], m0 = n >> KF, mm = m0 * m0;
    const long coff = LT.off[l];
    T *cs = reinterpret_cast<T *>(smem_raw), *cd = cs + (gin ? mm / 16 : mm), *opl = cd + mm / 4;
    const T *__restrict__ llin = B.ll + (coff >> (2 * KF));
    // prior weight and Jacobi factor values for the LDS table below, requested first (every lane,
    // clamped) so that waiting for them does not wait for the block copies issued after them
    const T adv = EPI != kEpiPlain ? B.ad[l * (J + 1) + min(tid, J)] : (T)0;
    const T jiv = (EPI == kEpiPcg || EPI == kEpiRhs) ? B.jinv[l * (J + 1) * 4 + min(tid, 4 * (J + 1) - 1)] : (T)0;
    if constexpr (!gin) {
        if constexpr (sizeof(T) == 4) {
            // 16-byte copies: lane chunk k4 holds values 4 k4 .. 4 k4 + 3 (the block is contiguous
            // in the workspace, 16-byte aligned)
#pragma unroll
            for (int c = 0; c < NL / 4; ++c) {
                const int k4 = tid + c * kCB;
                if (4 * c * kCB < mm && 4 * k4 < mm) g2lds16(llin + 4 * k4, cs + 4 * (c * kCB + (tid & ~63)));
            }
        } else {
#pragma unroll
            for (int c = 0; c < NL; ++c) {
                const int k = tid + c * kCB;
                if (c * kCB < mm && k < mm) cs[k] = llin[k];
            }
        }
    }
    if constexpr (pre) {
        // operand j of block element (r, c) -> opl[j * mm + r * m0 + c]
        const T *srcs[4] = {nullptr, nullptr, nullptr, nullptr};
        int nsrc = 0;
        if constexpr (EPI == kEpiPrior) {
            srcs[0] = static_cast<const T *>(E.cin);
            nsrc = 1;
        } else if constexpr (EPI == kEpiPcg) {
            srcs[0] = E.r_in ? static_cast<const T *>(E.r_in) : B.r;
            srcs[1] = static_cast<const T *>(E.c);
            srcs[2] = B.p;
            srcs[3] = E.q_in ? static_cast<const T *>(E.q_in) : B.q;
            nsrc = E.k > 0 ? 4 : 2;
        } else if constexpr (EPI == kEpiRhs) {
            srcs[0] = B.b_prev;
            srcs[1] = B.r;
            nsrc = E.cold ? 0 : 2;
        }
        const int lm = __ffs(m0) - 1;
#pragma unroll
        for (int j = 0; j < (NOP > 0 ? NOP : 1); ++j) {
            if (j < nsrc && srcs[j]) {  // (c is null when the fine transform stepped it)
                if (sizeof(T) == 4 && m0 >= 4 && (reinterpret_cast<uintptr_t>(srcs[j]) & 15) == 0) {
                    // a 16-byte aligned operand (the workspace's always; the caller's when its
                    // vector is): 16-byte copies of four values of one row (rows of m0 >= 4 values
                    // at offsets that are multiples of 4)
#pragma unroll
                    for (int c = 0; c < NL / 4; ++c) {
                        const int k = 4 * (tid + c * kCB);
                        if (4 * c * kCB < mm && k < mm)
                            g2lds16(reinterpret_cast<const float *>(srcs[j] + coff + (long)(k >> lm) * n + (k & (m0 - 1))),
                                    reinterpret_cast<float *>(opl + j * mm + 4 * (c * kCB + (tid & ~63))));
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < NL; ++c) {
                        const int k = tid + c * kCB;
                        if (c * kCB < mm && k < mm) {
                            const T *gp = srcs[j] + coff + (long)(k >> lm) * n + (k & (m0 - 1));
                            if constexpr (sizeof(T) == 4) g2lds(gp, opl + j * mm + c * kCB + (tid & ~63));
                            else opl[j * mm + k] = *gp;
                        }
                    }
                }
            }
        }
    }
    // prior weights and Jacobi factors of the layer's levels: [s] = alpha D, [kMaxJ + 1 + 4 s + o] = J^-1
    __shared__ T sW[5 * (kMaxJ + 1)];
    if (EPI != kEpiPlain && tid <= J) sW[tid] = adv;
    if ((EPI == kEpiPcg || EPI == kEpiRhs) && tid < 4 * (J + 1)) sW[kMaxJ + 1 + tid] = jiv;
    StepOut so{0.0, 0.0, 0};
    if constexpr (EPI == kEpiPcg) so = read_step(B.sc);
    lds_fence();
    double rho = 0.0, dz = 0.0;  // (r, z), (z, alpha D z) of the residual written (pcg, rhs)
    for (int s = KF + 1; s <= J; ++s) {
        const int mi = n >> (s - 1), h = mi >> 1, msk = mi - 1, nq = h * h;
        T ad = 0, ji[4] = {0, 0, 0, 0};
        if (EPI != kEpiPlain) ad = sW[s];
        if (EPI == kEpiPcg || EPI == kEpiRhs) {
#pragma unroll
            for (int o = 0; o < 4; ++o) ji[o] = sW[kMaxJ + 1 + 4 * s + o];
        }
        if (sizeof(T) == 4 && 4 * nq <= kCB) {
            // a small level: four lanes per quad, lane o = tid & 3 computes band o alone with the
            // same two filter passes (so the same coefficient value) and delivers it; one lane's
            // work per level is then a quarter of a quad's (FP32 only: in FP64 the band's filters
            // push this kernel into register spills)
            const int qi = tid >> 2, o = tid & 3;
            if (4 * nq > (tid & ~63)) {  // the wave holds quads
                const bool act = qi < nq, deliver = o > 0 || s == J;
                const int r = act ? qi / h : 0, q = act ? qi - r * h : 0;
                const int br = r + (o >= 2 ? h : 0), bc = q + ((o & 1) ? h : 0);
                T op1[NOP > 0 ? NOP : 1];
                if (NOP > 0) {
                    if constexpr (pre) {
#pragma unroll
                        for (int j = 0; j < (NOP > 0 ? NOP : 1); ++j) op1[j] = opl[j * mm + br * m0 + bc];
                        if (EPI == kEpiPcg && E.k == 0) op1[2] = op1[3] = (T)0;
                        if (EPI == kEpiRhs && E.cold) op1[0] = op1[1] = (T)0;
                    } else {
                        epi_load<T, EPI>(B, E, coff + (long)br * n + bc, op1);
                    }
                }
                if (act) {
                    T fy[6], fx[6];  // the band's filters along y (rows) and x (columns)
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        fy[k] = o >= 2 ? tp.g[k] : tp.h[k];
                        fx[k] = (o & 1) ? tp.g[k] : tp.h[k];
                    }
                    T w = 0;
                    auto band = [&](const T *src) {
#pragma unroll
                        for (int a = 0; a < 6; ++a) {
                            const T *row = src + ((2 * r + a) & msk) * mi;
                            T acc = 0;
#pragma unroll
                            for (int b = 0; b < 6; ++b) acc += fx[b] * row[(2 * q + b) & msk];
                            w += fy[a] * acc;
                        }
                    };
                    if constexpr (gin) {
                        if (s == KF + 1) band(llin);
                        else band(cs);
                    } else {
                        band(cs);
                    }
                    const T jio = o == 0 ? ji[0] : (o == 1 ? ji[1] : (o == 2 ? ji[2] : ji[3]));
                    if (deliver) epi_store<T, EPI>(B, E, band_index(coff, n, s, o, r, q), w, op1, jio, ad, so, rho, dz);
                    else cd[r * h + q] = w;
                }
            }
        } else
        for (int q0 = 0; q0 < nq; q0 += kCB) {
            if (q0 + (tid & ~63) >= nq) break;  // no quad of this level left for the wave
            const int qi = q0 + tid;
            const bool act = qi < nq;
            const int r = act ? qi / h : 0, q = act ? qi - r * h : 0;
            T op[4][NOP > 0 ? NOP : 1];
            if (NOP > 0) {
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    if (o > 0 || s == J) {
                        const int br = r + (o >= 2 ? h : 0), bc = q + ((o & 1) ? h : 0);
                        if constexpr (pre) {
#pragma unroll
                            for (int j = 0; j < (NOP > 0 ? NOP : 1); ++j) op[o][j] = opl[j * mm + br * m0 + bc];
                            if (EPI == kEpiPcg && E.k == 0) op[o][2] = op[o][3] = (T)0;
                            if (EPI == kEpiRhs && E.cold) op[o][0] = op[o][1] = (T)0;
                        } else {  // every lane loads (quad 0 stands in for lanes without one)
                            epi_load<T, EPI>(B, E, coff + (long)br * n + bc, op[o]);
                        }
                    }
                }
            }
            if (act) {
                T w[4] = {0, 0, 0, 0};
                auto analyse_wrap = [&](const T *src) {
#pragma unroll
                    for (int a = 0; a < 6; ++a) {
                        const T *row = src + ((2 * r + a) & msk) * mi;
                        T ax = 0, dx = 0;
#pragma unroll
                        for (int b = 0; b < 6; ++b) {
                            const T xv = row[(2 * q + b) & msk];
                            ax += tp.h[b] * xv;
                            dx += tp.g[b] * xv;
                        }
                        w[0] += tp.h[a] * ax;
                        w[2] += tp.g[a] * ax;
                        w[1] += tp.h[a] * dx;
                        w[3] += tp.g[a] * dx;
                    }
                };
                if constexpr (gin) {
                    if (s == KF + 1) analyse_wrap(llin);
                    else analyse_wrap(cs);
                } else {
                    analyse_wrap(cs);
                }
#pragma unroll
                for (int o = 1; o < 4; ++o) epi_store<T, EPI>(B, E, band_index(coff, n, s, o, r, q), w[o], op[o], ji[o], ad, so, rho, dz);
                if (s == J) epi_store<T, EPI>(B, E, band_index(coff, n, s, 0, r, q), w[0], op[0], ji[0], ad, so, rho, dz);
                else cd[r * h + q] = w[0];
            }
        }
        __syncthreads();
        T *t = cs;
        cs = cd;
        cd = t;
    }
    if constexpr (EPI == kEpiPcg || EPI == kEpiRhs) {
        // one partial pair per wave, no block reduction: slots after the fine tiles' partials,
        // kCoarseWaves per layer (every wave writes its own, also when it delivered nothing)
        static_assert(kCB / 64 == kCoarseWaves, "one partial slot per wave of the coarse workgroup");
        rho = wave_sum(rho);
        dz = wave_sum(dz);
        if ((tid & 63) == 0) {
            const int slot = nfine + l * kCoarseWaves + (tid >> 6);
            B.partials[slot] = rho;
            B.partials[kPartialPitch + slot] = dz;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Setup and small kernels
// ---------------------------------------------------------------------------------------------
// Weighted squared norm sum_k C_eta^-1_k s_k^2 (preconditioner probes): one partial per block.
template <typename T>
__global__ __launch_bounds__(kB) void k_wnorm(const T *__restrict__ s, Bufs<T> B, int nw, PupilArgs pa) {
    __shared__ double sh[kB / 64];
    double acc = 0.0;
    for (int g = 0; g < nw; ++g) {
        const DevWfs W = B.wfs[g];
        const long n2 = (long)W.n_sub * W.n_sub;
        for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
            int r = (int)(i / W.n_sub), q = (int)(i - (long)r * W.n_sub);
            if (!subap_active(pa, W.n_sub, r, q)) continue;
            const double sx = (double)s[W.s_off + i], sy = (double)s[W.s_off + n2 + i];
            acc += W.inv_var * (sx * sx + sy * sy);
        }
    }
    const double v = block_sum(acc, sh);
    if (threadIdx.x == 0) B.partials[blockIdx.x] = v;
}

// Sum of n partials in fixed order -> sc[2].rho (single workgroup).
__global__ __launch_bounds__(kB) void k_sum_partials(const double *__restrict__ partials, int n, Scalars *sc) {
    __shared__ double sh[kB / 64];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += partials[i];
    const double t = block_sum(a, sh);
    if (threadIdx.x == 0) sc[2].rho = t;
}

// Fitting (bilinear on-axis sampling of the layers at the actuators of their DM) + gain.
template <typename T>
__global__ __launch_bounds__(kB) void k_fit(const T *__restrict__ u, const T *__restrict__ a_prev, T *__restrict__ a,
                                            const T *__restrict__ a_m1, Bufs<T> B, int nl, int nd, long n_act,
                                            double gain) {
    u += blockIdx.y * B.fs_c;
    if (a_prev) a_prev += blockIdx.y * B.fs_a;
    if (a_m1) a_m1 += blockIdx.y * B.fs_a;
    a += blockIdx.y * B.fs_a;
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
    if (a_m1) a[i] = prev + (T)gain * (acc - a_m1[i]);  // closed loop: a0 + gain (F W^T c - a^(-1))
    else a[i] = (T)(1.0 - gain) * prev + (T)gain * acc;
}

// Cell tables: entry (g, l, j) of each axis from the ray geometry (setup, once per bind).
// Per layer l (one workgroup each): out[l] = sum over the layer's coefficients of x alpha D y in
// FP64, fixed order.  The level of coefficient (r, q) of an n x n Mallat pyramid is J inside the
// top-left (n >> J)^2 block, else log2 n - floor(log2 max(r, q)).
struct LayScale {             // a factor per layer
    double s[kMaxLayers];
};

template <typename T>
__global__ __launch_bounds__(kB) void k_prior_dot(LayTab LT, LayScale sc, const T *__restrict__ x, const T *__restrict__ y,
                                                  const T *__restrict__ ad, int J, double *out) {
    __shared__ double sh[kB / 64];
    const int l = blockIdx.x, n = LT.n[l], ln = 31 - __clz(n);
    const long off = LT.off[l];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n * n; i += kB) {
        const int r = i >> ln, q = i & (n - 1), t = r > q ? r : q;
        const int s = t < (n >> J) ? J : ln - (31 - __clz(t));
        acc += (double)x[off + i] * (double)ad[l * (J + 1) + s] * (double)y[off + i];
    }
    const double v = block_sum(acc, sh);
    if (threadIdx.x == 0) out[l] = v * sc.s[l];
}

// ---------------------------------------------------------------------------------------------
// Least-squares DM fitting over the probe directions (more layers than DMs).  Points: probe
// direction t of the 5 x 5 grid (theta in {-60, -30, 0, 30, 60} arcsec per axis) and node (i, j)
// of the first sensor's grid inside the pupil annulus; natural-star rays meet altitude h at
// (x_j + theta_x h, y_i + theta_y h).  Layers and DMs are the hat (piecewise bilinear) surfaces
// over their grids, zero beyond them.  With H the DM surfaces at the points and y0 the layers
// there, the fit takes n_cg CG steps on (H^T H + eps I) a = H^T y0 from a = 0.
// ---------------------------------------------------------------------------------------------
struct FitGeom {
    double D, d;                 // pupil diameter, node spacing
    const unsigned char *in;     // nv x nv: 1 for nodes inside the pupil annulus
    int nv;                      // nodes per side
    double hl[kMaxLayers];       // layer altitudes
    double hm[kMaxDms];          // DM altitudes
};

__device__ __forceinline__ void probe_dir(int t, double &tx, double &ty) {
    const double as = 3.14159265358979323846 / (180.0 * 3600.0);
    tx = (-60.0 + 30.0 * (t % 5)) * as;
    ty = (-60.0 + 30.0 * (t / 5)) * as;
}

// The cell k0 in [0, n-2] and the hat weights of its lines k0, k0+1 at coordinate u of a grid
// with lines 0..n-1: lines beyond the grid carry weight 0 (a cell straddling an edge keeps its
// inside line only).
__device__ __forceinline__ void hat_cell(double u, int n, int &k0, double &w0, double &w1) {
    const int k = (int)floor(u);
    const double t = u - k;
    if (k >= 0 && k <= n - 2) {
        k0 = k;
        w0 = 1.0 - t;
        w1 = t;
    } else if (k == -1) {
        k0 = 0;
        w0 = t;
        w1 = 0.0;
    } else if (k == n - 1) {
        k0 = n - 2;
        w0 = 0.0;
        w1 = 1.0 - t;
    } else {
        k0 = 0;
        w0 = w1 = 0.0;
    }
}

// y[t][i][j] = the layers (LAYERS) or the DMs (!LAYERS) summed along the ray of point (t, i, j).
template <typename T, bool LAYERS>
__global__ __launch_bounds__(kB) void k_fit_points(const T *__restrict__ src, T *__restrict__ y, Bufs<T> B, FitGeom G,
                                                   int ngrid, int npts) {
    const int id = blockIdx.x * kB + threadIdx.x;
    if (id >= npts) return;
    const int t = id / (G.nv * G.nv), rem = id - t * G.nv * G.nv, i = rem / G.nv, j = rem - i * G.nv;
    const double x = -0.5 * G.D + j * G.d, yy = -0.5 * G.D + i * G.d;
    T acc = 0;
    if (G.in[rem]) {
        double tx, ty;
        probe_dir(t, tx, ty);
        for (int q = 0; q < ngrid; ++q) {
            double u, v;
            int n;
            long off;
            if (LAYERS) {
                const DevLayer L = B.lay[q];
                u = (x + tx * G.hl[q]) / L.spacing + L.half;
                v = (yy + ty * G.hl[q]) / L.spacing + L.half;
                n = L.n;
                off = L.c_off;
            } else {
                const DevDm Dm = B.dm[q];
                u = (x + tx * G.hm[q]) / Dm.pitch + Dm.centre;
                v = (yy + ty * G.hm[q]) / Dm.pitch + Dm.centre;
                n = Dm.n_act;
                off = Dm.a_off;
            }
            int kx, ky;
            double wx0, wx1, wy0, wy1;
            hat_cell(u, n, kx, wx0, wx1);
            hat_cell(v, n, ky, wy0, wy1);
            const T *U = src + off + (long)ky * n + kx;
            acc += (T)(wy0 * wx0) * U[0] + (T)(wy0 * wx1) * U[1] + (T)(wy1 * wx0) * U[n] + (T)(wy1 * wx1) * U[n + 1];
        }
    }
    y[id] = acc;
}

// out = H^T y (+ eps p): actuator (m, ai, aj) collects, for every direction, the points whose
// node lies within one pitch of it.
template <typename T>
__global__ __launch_bounds__(kB) void k_fit_adjoint(const T *__restrict__ y, const T *__restrict__ p, T *__restrict__ out,
                                                    Bufs<T> B, FitGeom G, int nd, long n_act, double eps) {
    const long id = (long)blockIdx.x * kB + threadIdx.x;
    if (id >= n_act) return;
    int m = 0;
    while (m + 1 < nd && B.dm[m + 1].a_off <= id) ++m;
    const DevDm Dm = B.dm[m];
    const long loc = id - Dm.a_off;
    const int ai = (int)(loc / Dm.n_act), aj = (int)(loc - (long)ai * Dm.n_act);
    const double h = G.hm[m], ca = (aj - Dm.centre) * Dm.pitch, ra = (ai - Dm.centre) * Dm.pitch;
    double acc = 0.0;
    for (int t = 0; t < kProbes; ++t) {
        double tx, ty;
        probe_dir(t, tx, ty);
        // nodes with |x_j + tx h - ca| < pitch (x_j = -D/2 + j d)
        const int j0 = max(0, (int)ceil((ca - Dm.pitch - tx * h + 0.5 * G.D) / G.d));
        const int j1 = min(G.nv - 1, (int)floor((ca + Dm.pitch - tx * h + 0.5 * G.D) / G.d));
        const int i0 = max(0, (int)ceil((ra - Dm.pitch - ty * h + 0.5 * G.D) / G.d));
        const int i1 = min(G.nv - 1, (int)floor((ra + Dm.pitch - ty * h + 0.5 * G.D) / G.d));
        for (int i = i0; i <= i1; ++i) {
            const double wy = 1.0 - fabs((-0.5 * G.D + i * G.d + ty * h - ra) / Dm.pitch);
            if (wy <= 0.0) continue;
            for (int j = j0; j <= j1; ++j) {
                const double wx = 1.0 - fabs((-0.5 * G.D + j * G.d + tx * h - ca) / Dm.pitch);
                if (wx > 0.0) acc += wx * wy * (double)y[((long)t * G.nv + i) * G.nv + j];
            }
        }
    }
    out[id] = (T)(acc + (p ? eps * (double)p[id] : 0.0));
}

// One workgroup runs the vector part of CG on the actuators.  init: x = 0, r = p = b (in r),
// rr = (r, r).  step: alpha = rr / (p, q), x += alpha p, r -= alpha q, rr' = (r, r),
// p = r + (rr' / rr) p.  Sums in FP64 in a fixed order; rr = 0 leaves everything unchanged.
template <typename T>
__global__ __launch_bounds__(1024) void k_fit_cg(T *__restrict__ x, T *__restrict__ r, T *__restrict__ p,
                                                 const T *__restrict__ q, double *rr, long n, int init) {
    __shared__ double sh[16];
    const int tid = threadIdx.x;
    if (init) {
        double s = 0.0;
        for (long i = tid; i < n; i += 1024) {
            const T ri = r[i];
            x[i] = 0;
            p[i] = ri;
            s += (double)ri * (double)ri;
        }
        const double t = block_sum(s, sh);
        if (tid == 0) rr[0] = t;
        return;
    }
    const double rr0 = rr[0];
    if (!(rr0 > 0.0)) return;
    double s = 0.0;
    for (long i = tid; i < n; i += 1024) s += (double)p[i] * (double)q[i];
    const double pq = block_sum(s, sh);
    if (!(pq > 0.0)) return;
    const double al = rr0 / pq;
    s = 0.0;
    for (long i = tid; i < n; i += 1024) {
        x[i] += (T)al * p[i];
        const T ri = r[i] - (T)al * q[i];
        r[i] = ri;
        s += (double)ri * (double)ri;
    }
    const double rn = block_sum(s, sh);
    const T be = (T)(rn / rr0);
    for (long i = tid; i < n; i += 1024) p[i] = r[i] + be * p[i];
    if (tid == 0) rr[0] = rn;
}

// a = (1 - gain) a_prev + gain x (a_prev may be null).
template <typename T>
__global__ __launch_bounds__(kB) void k_fit_gain(const T *__restrict__ x, const T *__restrict__ a_prev, T *__restrict__ a,
                                                 long n, double gain) {
    const long i = (long)blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const T prev = a_prev ? a_prev[i] : (T)0;
    a[i] = (T)(1.0 - gain) * prev + (T)gain * x[i];
}

template <typename T>
__global__ __launch_bounds__(kB) void k_build_tabs(Ent<T> *xtab, Ent<T> *ytab, const DevWfs *__restrict__ wfs,
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
// a list of (j, weight) pairs of width kRtabWidth padded with index -1; lines with more pairs than
// that set over[g] (the plan then uses the scanning transpose).
template <typename T>
__global__ __launch_bounds__(kB) void k_build_ranges(Range *xrng, Range *yrng, RtabEnt<T> *xrt, RtabEnt<T> *yrt,
                                                     const Ent<T> *__restrict__ xtab, const Ent<T> *__restrict__ ytab,
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
        for (int c = cnt; c < kRtabWidth; ++c) rt[c] = RtabEnt<T>{-1, (T)0};
        if (cnt > kRtabWidth) over[g] = 1;  // idempotent flag, no read-modify-write needed
        Range r{lo, hi};
        if (hi < 0) r = Range{1, 0};
        (axis == 0 ? xrng : yrng)[idx] = r;
    }
}

// Record of every (P^T tile, guide star): the node rows / columns that the transpose pairs of
// the tile's rows / columns name, packed as (lo | hi << 16) (empty: lo > hi), and the largest pair
// count over the tile's rows and over its columns.  One workgroup per tile.
__global__ __launch_bounds__(kMaxWfs) void k_build_rects(SegTab S, const Range *__restrict__ xrng,
                                                         const Range *__restrict__ yrng, int4 *rects, int nw, int sum_n) {
    const int g = threadIdx.x;
    const TileId id = find_tile(S, (int)blockIdx.x);  // the whole wave: lane s reads segment s
    if (g >= nw) return;
    const int n = id.n, lt = id.lt;
    const int T0 = n < kPtTile ? n : kPtTile;
    const int k0 = (id.loc >> lt) * T0, q0 = (id.loc & ((1 << lt) - 1)) * T0;
    int iA = 1 << 30, iB = -1, jA = 1 << 30, jB = -1, cy = 0, cx = 0;
    for (int t = 0; t < T0; ++t) {
        const Range ry = yrng[(long)g * sum_n + id.aux + k0 + t];
        const Range rx = xrng[(long)g * sum_n + id.aux + q0 + t];
        if (ry.lo <= ry.hi) {
            iA = ry.lo < iA ? ry.lo : iA;
            iB = ry.hi > iB ? ry.hi : iB;
            cy = ry.hi - ry.lo + 1 > cy ? ry.hi - ry.lo + 1 : cy;
        }
        if (rx.lo <= rx.hi) {
            jA = rx.lo < jA ? rx.lo : jA;
            jB = rx.hi > jB ? rx.hi : jB;
            cx = rx.hi - rx.lo + 1 > cx ? rx.hi - rx.lo + 1 : cx;
        }
    }
    if (iA > iB || jA > jB) {
        iA = jA = 1;
        iB = jB = 0;
        cy = cx = 0;
    }
    rects[(long)blockIdx.x * nw + g] = make_int4(iA | (iB << 16), jA | (jB << 16), cy, cx);
}

template <typename T>
__global__ __launch_bounds__(kB) void k_fill(T *__restrict__ x, long n, T val) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = val;
}

template <typename T>
__global__ __launch_bounds__(kB) void k_copy(T *__restrict__ dst, const T *__restrict__ src, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) dst[i] = src[i];
}

__global__ void k_init_scalars(Scalars *sc) {
    sc += blockIdx.y * kScalarSlots;
    if (threadIdx.x < kScalarSlots && blockIdx.x == 0) reset_scalars(sc + threadIdx.x);
}

int grid_for(long n) {
    long g = (n + kB - 1) / kB;
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    return (int)g;
}

int launch_status(const char *file, int line) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FEWHA_OK : hip_failure(e, "kernel launch", file, line);
}
#define check() launch_status(__FILE__, __LINE__)

InvVar inv_var_tab(const Plan &P) {
    InvVar t{};
    for (int g = 0; g < P.nw; ++g) t.v[g] = P.dwfs[g].inv_var;
    return t;
}

WfsOff wfs_off_tab(const Plan &P) {
    WfsOff t{};
    for (int g = 0; g < P.nw; ++g) {
        t.v_off[g] = (int)P.dwfs[g].v_off;
        t.vp[g] = P.dwfs[g].vp;
    }
    return t;
}

PupilArgs pupil(const Plan &P) {
    const double ro = P.D / 2, ri = P.obstruction * P.D / 2;
    return PupilArgs{P.D, ro * ro, ri * ri};
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
// Level bound of the inverse-DWT launches of plans with at most this many levels (their unrolled
// level loops and cone registers stop there; deeper plans take kMaxJ).
constexpr int kWtJSmall = 6;

// Dynamic LDS of an inverse-DWT launch: the cone of the plan's J levels.
inline size_t wt_lds(const Plan &P) { return (size_t)wt_slots(P.J) * kWB * P.elem; }

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
int Ops<T>::wt(const T *c, T *out) const {
    if (P.J <= kWtJSmall) k_wt<T, kWtPlain, kWtJSmall><<<dim3(P.n_wt, nb), kWB, wt_lds(P), st>>>(P.seg_wt, c, out, B, make_taps<T>(), P.J, FoldArgs{});
    else k_wt<T, kWtPlain, kMaxJ><<<dim3(P.n_wt, nb), kWB, wt_lds(P), st>>>(P.seg_wt, c, out, B, make_taps<T>(), P.J, FoldArgs{});
    return check();
}

template <typename T>
int Ops<T>::wt_pcg(const T *r, T *out) const {
    if (P.J <= kWtJSmall) k_wt<T, kWtPcg, kWtJSmall><<<dim3(P.n_wt, nb), kWB, wt_lds(P), st>>>(P.seg_wt, r, out, B, make_taps<T>(), P.J, FoldArgs{});
    else k_wt<T, kWtPcg, kMaxJ><<<dim3(P.n_wt, nb), kWB, wt_lds(P), st>>>(P.seg_wt, r, out, B, make_taps<T>(), P.J, FoldArgs{});
    return check();
}

template <typename T>
int Ops<T>::wt_fold(const T *r, T *out, const FoldArgs &F) const {
    if (sizeof(T) != 4 || !P.fold) return FEWHA_ERR_UNSUPPORTED;
    FoldArgs G = F;
    G.kf = P.kf;
    G.nfine = P.n_fwd * fwd_waves(P.kf, P.tq);
    if (P.J <= kWtJSmall) k_wt<T, kWtFold, kWtJSmall><<<dim3(P.n_wt, nb), kWB, wt_lds(P), st>>>(P.seg_wt, r, out, B, make_taps<T>(), P.J, G);
    else k_wt<T, kWtFold, kMaxJ><<<dim3(P.n_wt, nb), kWB, wt_lds(P), st>>>(P.seg_wt, r, out, B, make_taps<T>(), P.J, G);
    return check();
}

template <typename T>
int Ops<T>::wt_tail(const T *c, T *out, const FoldArgs &F) const {
    if (sizeof(T) != 4 || !P.fold || (P.lay.empty())) return FEWHA_ERR_UNSUPPORTED;
    FoldArgs G = F;
    G.kf = P.kf;
    G.parts = kTailParts;
    G.ntail = (P.nl * kTailParts + 7) & ~7;  // whole rounds of the eight XCDs
    const dim3 grid(G.ntail + (c ? P.n_wt : 0), nb);
    if (P.J <= kWtJSmall) k_wt<T, kWtTail, kWtJSmall><<<grid, kWB, wt_lds(P), st>>>(P.seg_wt, c, out, B, make_taps<T>(), P.J, G);
    else k_wt<T, kWtTail, kMaxJ><<<grid, kWB, wt_lds(P), st>>>(P.seg_wt, c, out, B, make_taps<T>(), P.J, G);
    return check();
}

// Dynamic LDS of a projection launch over nl layers (or DMs): its cell entries.
template <typename T>
inline size_t proj_lds(int nl) { return (size_t)2 * nl * kPR * (sizeof(T) + 2 * sizeof(T)); }

template <typename T>
int Ops<T>::proj(const T *u, T *out, int mode) const {
    if (mode == kProjM)
        k_proj<T, kProjM><<<dim3(P.n_proj, nb), kB, proj_lds<T>(P.nl), st>>>(P.seg_proj, P.laytab, inv_var_tab(P), pupil(P), u, out, nullptr, B,
                                                                          P.nl);
    else if (mode == kProjCA)
        k_proj<T, kProjCA><<<dim3(P.n_proj, nb), kB, proj_lds<T>(P.nl), st>>>(P.seg_proj, P.laytab, inv_var_tab(P), pupil(P), u, out, nullptr, B,
                                                                          P.nl);
    else
        k_proj<T, kProjA><<<dim3(P.n_proj, nb), kB, proj_lds<T>(P.nl), st>>>(P.seg_proj, P.laytab, inv_var_tab(P), pupil(P), u, out, nullptr, B,
                                                                          P.nl);
    return check();
}

template <typename T>
int Ops<T>::pol(const T *a_m1, const T *s, T *s_pol) const {
    k_proj<T, kProjPol><<<dim3(P.n_proj, nb), kB, proj_lds<T>(P.nd), st>>>(P.seg_proj, P.dmtab, inv_var_tab(P), pupil(P),
                                                                           a_m1, s_pol, s, B, P.nd);
    return check();
}

template <typename T>
int Ops<T>::gt(const T *s, T *v, int mode) const {
    const dim3 grid(P.n_proj, nb);
    if (mode == kGtRhs) k_gt<T, kGtRhs><<<grid, kB, 0, st>>>(P.seg_proj, inv_var_tab(P), pupil(P), s, v, B.fs_s, B.fs_v);
    else k_gt<T, kGtAdj><<<grid, kB, 0, st>>>(P.seg_proj, inv_var_tab(P), pupil(P), s, v, B.fs_s, B.fs_v);
    return check();
}

template <typename T>
int Ops<T>::pt(const T *v, T *x, const PassArgs &PA) const {
    const dim3 grid(P.n_pt + (PA.k >= 0 ? 1 : 0), nb);
    if (!P.rtab_ok) {
        k_pt_scan<T><<<grid, kB, 0, st>>>(P.seg_pt, v, x, B, P.nl, P.nw, PA);
        return check();
    }
    switch (P.pt_rw) {  // the plan's widest pair count
        case 1: k_pt<T, 1><<<grid, kB, P.pt_lds, st>>>(P.seg_pt, wfs_off_tab(P), v, x, B, P.nw, PA); break;
        case 2: k_pt<T, 2><<<grid, kB, P.pt_lds, st>>>(P.seg_pt, wfs_off_tab(P), v, x, B, P.nw, PA); break;
        case 3: k_pt<T, 3><<<grid, kB, P.pt_lds, st>>>(P.seg_pt, wfs_off_tab(P), v, x, B, P.nw, PA); break;
        default: k_pt<T, kRtabWidth><<<grid, kB, P.pt_lds, st>>>(P.seg_pt, wfs_off_tab(P), v, x, B, P.nw, PA); break;
    }
    return check();
}

int fwd_waves(int kf, int tq) {
#define FEWHA_FWD_WAVES(KF, TQ) return FwdLanes<KF, TQ>::block / 64
    if (kf == 1) {
        switch (tq) {
            case 1: FEWHA_FWD_WAVES(1, 1);
            case 2: FEWHA_FWD_WAVES(1, 2);
            case 4: FEWHA_FWD_WAVES(1, 4);
            default: FEWHA_FWD_WAVES(1, 8);
        }
    }
    switch (tq) {
        case 1: FEWHA_FWD_WAVES(2, 1);
        case 2: FEWHA_FWD_WAVES(2, 2);
        case 4: FEWHA_FWD_WAVES(2, 4);
        default: FEWHA_FWD_WAVES(2, 8);
    }
#undef FEWHA_FWD_WAVES
}

template <typename T, int EPI>
static int fwd_launch(const Plan &P, const Bufs<T> &B, hipStream_t st, int nb, const T *x, const FwdArgs &E,
                      bool fine, bool coarse) {
    const Taps<T> tp = make_taps<T>();
    const int nf = P.n_fwd;
    const int nfs = nf * fwd_waves(P.kf, P.tq);  // the fine tiles' partial slots (one per wave)
    FwdArgs Ef = E;  // the shadows of a folded solve concern the coarse levels only
    Ef.r_in = Ef.q_in = Ef.b_in = nullptr;
#define FEWHA_FWD(KF, TQ) k_fwd<T, KF, TQ, EPI><<<dim3(nf, nb), (FwdLanes<KF, TQ>::block), 0, st>>>(P.seg_fwd, x, B, Ef, tp, P.J)
    if (!fine) {
    } else if (P.kf == 1) {
        switch (P.tq) {
            case 1: FEWHA_FWD(1, 1); break;
            case 2: FEWHA_FWD(1, 2); break;
            case 4: FEWHA_FWD(1, 4); break;
            default: FEWHA_FWD(1, 8); break;
        }
    } else {
        switch (P.tq) {
            case 1: FEWHA_FWD(2, 1); break;
            case 2: FEWHA_FWD(2, 2); break;
            case 4: FEWHA_FWD(2, 4); break;
            default: FEWHA_FWD(2, 8); break;
        }
    }
#undef FEWHA_FWD
    if (int e = check()) return e;
    if (P.kf < P.J && coarse) {
        FwdArgs Ec = E;  // c's coarse share, if any, is the fine transform's
        if (E.cc) Ec.c = nullptr;
        Ec.cc = nullptr;
        Ec.cc_r = nullptr;
        size_t m = 0;
        for (auto &L : P.lay) m = (size_t)(L.n >> P.kf) > m ? (size_t)(L.n >> P.kf) : m;
        size_t base = (m * m + m * m / 4) * sizeof(T);
        const size_t opb = (size_t)EpiOps<EPI>::n * m * m * sizeof(T);
        const int gin = base > kCoarseLdsMax ? 1 : 0;
        if (gin) base = (m * m / 16 + m * m / 4) * sizeof(T);
        if (base > kCoarseLdsMax) return FEWHA_ERR_UNSUPPORTED;
        const int pre = !gin && EpiOps<EPI>::n > 0 && base + opb <= kCoarseLdsMax ? 1 : 0;
        const dim3 grid(P.nl, nb);
        const size_t lds = base + (pre ? opb : 0);
        if (pre) k_coarse<T, EPI, kCoarseStaged><<<grid, kCB, lds, st>>>(P.laytab, B, Ec, tp, P.J, P.kf, nfs);
        else if (gin) k_coarse<T, EPI, kCoarseGlobalIn><<<grid, kCB, lds, st>>>(P.laytab, B, Ec, tp, P.J, P.kf, nfs);
        else k_coarse<T, EPI, kCoarseDirect><<<grid, kCB, lds, st>>>(P.laytab, B, Ec, tp, P.J, P.kf, nfs);
        if (int e = check()) return e;
    }
    return FEWHA_OK;
}

template <typename T>
int Ops<T>::fwd(const T *x, const FwdArgs &E, int epi, bool coarse, bool fine) const {
    switch (epi) {
        case kEpiPlain: return fwd_launch<T, kEpiPlain>(P, B, st, nb, x, E, fine, coarse);
        case kEpiPrior: return fwd_launch<T, kEpiPrior>(P, B, st, nb, x, E, fine, coarse);
        case kEpiPcg: return fwd_launch<T, kEpiPcg>(P, B, st, nb, x, E, fine, coarse);
        default: return fwd_launch<T, kEpiRhs>(P, B, st, nb, x, E, fine, coarse);
    }
}

template <typename T>
int Ops<T>::prepare() const {
    // the per-layer coarse transform may need more than the default 64 KiB of dynamic LDS
#define FEWHA_COARSE3(EPI) (const void *)k_coarse<T, EPI, kCoarseStaged>, (const void *)k_coarse<T, EPI, kCoarseDirect>, \
                           (const void *)k_coarse<T, EPI, kCoarseGlobalIn>
    const void *fns[12] = {FEWHA_COARSE3(kEpiPlain), FEWHA_COARSE3(kEpiPrior), FEWHA_COARSE3(kEpiPcg),
                           FEWHA_COARSE3(kEpiRhs)};
#undef FEWHA_COARSE3
    for (int i = 0; i < 12; ++i)
        if (hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCoarseLdsMax) != hipSuccess)
            return FEWHA_ERR_UNSUPPORTED;
    // staged P^T: the tile's transpose pairs and node rectangles
    const int pt_max = (int)(kPtMaxWfs * 2 * kRtabWidth * kPtTile * sizeof(RtabEnt<T>) + kPtStage * sizeof(T));
    const void *pts[4] = {(const void *)k_pt<T, 1>, (const void *)k_pt<T, 2>, (const void *)k_pt<T, 3>,
                          (const void *)k_pt<T, kRtabWidth>};
    for (const void *f : pts)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, pt_max) != hipSuccess)
            return FEWHA_ERR_UNSUPPORTED;
    return FEWHA_OK;
}

template <typename T>
int Ops<T>::wnorm(const T *s) const {
    long mx = 0;
    for (auto &w : P.dwfs) mx = mx > (long)w.n_sub * w.n_sub ? mx : (long)w.n_sub * w.n_sub;
    int g = grid_for(mx);
    if (g > kPartialPitch) g = kPartialPitch;
    k_wnorm<T><<<g, kB, 0, st>>>(s, B, P.nw, pupil(P));
    if (int e = check()) return e;
    k_sum_partials<<<1, kB, 0, st>>>(B.partials, g, B.sc);
    return check();
}

template <typename T>
int Ops<T>::fit(const T *u, const T *a_prev, T *a, double gain, const T *a_m1) const {
    k_fit<T><<<dim3(grid_for((long)P.n_act), nb), kB, 0, st>>>(u, a_prev, a, a_m1, B, P.nl, P.nd, (long)P.n_act, gain);
    return check();
}

template <typename T>
int Ops<T>::build_tables(int *over) const {
    const long ne = (long)P.nw * P.nl * P.maxnv;
    k_build_tabs<T><<<(int)((ne + kB - 1) / kB), kB, 0, st>>>(const_cast<Ent<T> *>(B.xtab), const_cast<Ent<T> *>(B.ytab),
                                                              B.wfs, B.proj, B.lay, P.nw, P.nl, P.maxnv);
    if (int e = check()) return e;
    const long nr = (long)P.nw * P.sum_n;
    k_build_ranges<T><<<(int)((nr + kB - 1) / kB), kB, 0, st>>>(
        const_cast<Range *>(B.xrng), const_cast<Range *>(B.yrng), const_cast<RtabEnt<T> *>(B.xrtab),
        const_cast<RtabEnt<T> *>(B.yrtab), B.xtab, B.ytab, B.wfs, B.lay, P.nw, P.nl, P.maxnv, P.sum_n, over);
    if (int e = check()) return e;
    k_build_rects<<<P.n_pt, kMaxWfs, 0, st>>>(P.seg_pt, B.xrng, B.yrng, const_cast<int4 *>(B.rects), P.nw, P.sum_n);
    return check();
}

template <typename T>
int Ops<T>::prior_dot(const T *x, const T *y, double *out, bool per_gamma) const {
    LayScale sc{};
    for (int l = 0; l < P.nl; ++l) sc.s[l] = per_gamma ? 1.0 / P.lay[l].cn2_weight : 1.0;
    k_prior_dot<T><<<P.nl, kB, 0, st>>>(P.laytab, sc, x, y, B.ad, P.J, out);
    return check();
}

FitGeom fit_geom(const Plan &P) {
    FitGeom G{};
    G.D = P.D;
    G.d = P.D / P.wfs[0].n_sub;
    G.in = reinterpret_cast<const unsigned char *>(P.ws + P.o_fmask);
    G.nv = P.wfs[0].n_sub + 1;
    for (int l = 0; l < P.nl; ++l) G.hl[l] = P.lay[l].height;
    for (int m = 0; m < P.nd; ++m) G.hm[m] = P.dm[m].height;
    return G;
}

template <typename T>
int Ops<T>::fit_ls(const T *u, const T *a_prev, T *a, double gain, int n_cg, double eps) const {
    const FitGeom G = fit_geom(P);
    const int np = (int)P.n_fit;
    const long na = (long)P.n_act;
    char *w = P.ws;
    T *y = reinterpret_cast<T *>(w + P.o_fy), *x = reinterpret_cast<T *>(w + P.o_fx);
    T *r = reinterpret_cast<T *>(w + P.o_fr), *p = reinterpret_cast<T *>(w + P.o_fp);
    T *q = reinterpret_cast<T *>(w + P.o_fq);
    double *rr = reinterpret_cast<double *>(w + P.o_frr);
    const int gp = (np + kB - 1) / kB, ga = (int)((na + kB - 1) / kB);
    k_fit_points<T, true><<<gp, kB, 0, st>>>(u, y, B, G, P.nl, np);
    k_fit_adjoint<T><<<ga, kB, 0, st>>>(y, nullptr, r, B, G, P.nd, na, 0.0);
    k_fit_cg<T><<<1, 1024, 0, st>>>(x, r, p, q, rr, na, 1);
    for (int it = 0; it < n_cg; ++it) {
        k_fit_points<T, false><<<gp, kB, 0, st>>>(p, y, B, G, P.nd, np);
        k_fit_adjoint<T><<<ga, kB, 0, st>>>(y, p, q, B, G, P.nd, na, eps);
        k_fit_cg<T><<<1, 1024, 0, st>>>(x, r, p, q, rr, na, 0);
    }
    k_fit_gain<T><<<ga, kB, 0, st>>>(x, a_prev, a, na, gain);
    return check();
}

template <typename T>
int Ops<T>::fill(T *x, long n, T val) const {
    k_fill<T><<<grid_for(n), kB, 0, st>>>(x, n, val);
    return check();
}

template <typename T>
int Ops<T>::copy(T *dst, const T *src, long n) const {
    k_copy<T><<<grid_for(n), kB, 0, st>>>(dst, src, n);
    return check();
}

template <typename T>
int Ops<T>::init_scalars() const {
    k_init_scalars<<<dim3(1, nb), 64, 0, st>>>(B.sc);
    return check();
}

template struct Ops<float>;
template struct Ops<double>;

}  // namespace fewha
