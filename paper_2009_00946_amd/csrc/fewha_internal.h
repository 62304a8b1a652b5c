// Internal declarations of the FEWHA MI355X library: host plan, device geometry records and
// the launchers of the HIP kernels.  Not part of the public ABI (include/fewha.h).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/fewha.h"

namespace fewha {

constexpr int kMaxLayers = 64;
constexpr int kMaxWfs = 64;
constexpr int kMaxDms = 16;
constexpr int kMaxJ = 12;
constexpr int kMaxGrid = 4096;    // sensor subapertures per side
constexpr int kMaxLayerGrid = 512; // layer nodes per side

// Output tile edge of the inverse DWT (layers smaller than this form one tile of n x n).
constexpr int kWtTile = 32;
// Node tile of the projection kernels: 16 x 16 nodes computed, the inner 14 x 14 delivered.
constexpr int kProjTile = 14;
// Layer-node tile edge of the transpose projection P^T.
constexpr int kPtTile = 16;
// Level-kf quads per tile edge of the fine forward DWT (at most).
constexpr int kFwdQuads = 8;
// LDS values available to the P^T tile for its staged node rectangles (all guide stars).
constexpr int kPtStage = 6144;
// Guide stars whose transpose tables the P^T tile stages at once (more: the scanning P^T).
constexpr int kPtMaxWfs = 16;
// Slots per row of the FP64 partial-sum buffer (one per workgroup of a reduction).
constexpr int kPartialPitch = 65536;
// Least-squares DM fitting: the 5 x 5 quality evaluation grid of probe directions.
constexpr int kProbes = 25;
// Scalar records per frame: two pass-parity slots, the right-hand-side record, the current pass.
constexpr int kScalarSlots = 4;
// Frames of one batched launch (grid y).
constexpr int kMaxBatch = 1024;
// Segments (layers or guide stars) of one launch's tile table.
constexpr int kMaxSeg = 64;

// Tile decode table of one launch, passed by value as a kernel argument so that a workgroup
// finds its tile without touching memory written by earlier kernels.  Segment i (a layer or a
// guide star) owns workgroups [start[i], start[i+1]).
struct SegTab {
    int nseg;
    int chunk;            // tiles per XCD chunk of the workgroup order (0: one contiguous run per XCD)
    int ilv;              // 1: segments of equal tile counts interleaved, tile b being tile b / nseg of
                          // segment b % nseg (sensor tiles over one pupil region run side by side)
    int start[kMaxSeg + 1];
    int off[kMaxSeg];     // element offset of the segment's array (layer c_off / sensor v_off)
    int aux[kMaxSeg];     // layers: first grid line in the per-axis line tables; sensors: s_off
    int n[kMaxSeg];       // layer n, or sensor n_sub
    int lt[kMaxSeg];      // layers: log2 of tiles per row; sensors: tiles per row
    int rw[kMaxSeg];      // P^T (layer segments): transpose pairs per grid line, 1..kRtabWidth
    int pitch[kMaxSeg];   // sensors: row pitch of the node grid (n_sub + 1 rounded up to 4)
    int id[kMaxSeg];      // the segment's layer or guide-star index (segments may be reordered)
};

// Per-layer offsets and sizes, as a kernel argument (the projection reads every layer).
struct LayTab {
    int off[kMaxLayers];
    int n[kMaxLayers];
};

// Per guide star, as the kernels read it.
struct DevWfs {
    double d;        // subaperture size D / n_sub
    double x0;       // -D / 2: coordinate of node 0
    double inv_var;  // sigma^-2
    double r_out2;   // (D/2)^2: active iff r^2 <= r_out2 and r^2 >= r_in2
    double r_in2;    // (obstruction D/2)^2
    long s_off;      // offset of the s^x plane in the slope vector
    long v_off;      // offset of the (n_sub+1) x vp node grid in the node vector
    int n_sub;
    int nv;          // n_sub + 1
    int vp;          // node grid row pitch: nv rounded up to a multiple of 4 (16-byte rows)
};

// Per layer.
struct DevLayer {
    long c_off;      // offset in coefficient / layer vectors
    double spacing;  // delta
    double half;     // n / 2 (grid coordinate of the origin)
    int n;
    int log2n;
    int dm;          // fitting DM index
    int r_off;       // offset of this layer's n grid lines in the per-axis range tables
};

// One node of a sensor grid seen on one layer along one axis: bilinear cell k0 and the
// weights (1 - t, t) of grid lines k0 and k0 + 1.  Built once per plan on the device by the
// same arithmetic for every consumer, so P and P^T use identical matrix entries.
template <typename T>
struct Ent {
    int k0;
    int pad;
    T w0, w1;
};

// One (sensor node, weight) pair of a transpose-table row: the nodes of a sensor grid line whose
// bilinear cells touch a given layer grid line, zero-padded to kRtabWidth pairs.
constexpr int kRtabWidth = 4;
template <typename T>
struct RtabEnt {
    int idx;
    T w;
};

// Per (guide star, layer): ray geometry of Sec. 2.1.  Node (i, j) lands at grid coordinates
// u = (sig (x0 + j d) + hx) / spacing + n/2, v = (sig (x0 + i d) + hy) / spacing + n/2;
// slope / intercept give the same map in affine form, used only to bound candidate searches.
struct DevProj {
    double sig;      // cone factor 1 - h/H (LGS) or 1 (NGS)
    double hx, hy;   // theta_x h, theta_y h
    double slope;    // sig d / spacing
    double bx, by;   // u(j=0), v(i=0)
};

struct DevDm {
    long a_off;
    double pitch;
    double centre;   // (n_act - 1) / 2
    int n_act;
    int pad;
};

// Inclusive range [lo, hi] of sensor node indices (empty when lo > hi).
struct Range {
    int lo, hi;
};

// PCG scalars of Alg. 2 in FP64, kept on the device so no pass needs a host round trip.  The
// workspace holds four: the states after even and odd passes (the scalar step of pass k reads
// slot (k-1)&1 and writes slot k&1), one for setup-time reductions, and the (alpha, beta,
// stopped) of the current pass for the kernels that apply its update.
struct Scalars {
    double rho, mu, rho_old, alpha, alpha_old, beta;
    int stopped;     // zero residual, breakdown or non-finite: later passes are no-ops
    int status;      // FEWHA_OK, FEWHA_ERR_BREAKDOWN or FEWHA_ERR_NONFINITE
};

// Device pointers into the bound workspace, typed per precision.
template <typename T>
struct Bufs {
    const DevWfs *wfs;
    const DevLayer *lay;
    const DevProj *proj;
    const DevDm *dm;
    const Ent<T> *xtab, *ytab;        // [nw][nl][maxnv]
    const Range *xrng, *yrng;         // [nw][sum_n]: sensor nodes touching each layer grid line
    const RtabEnt<T> *xrtab, *yrtab;  // [nw][sum_n][kRtabWidth]: the same as (node, weight) lists
    const int4 *rects;                // [P^T tile][nw]: node rows / columns a tile's lines touch
    const Ent<T> *xdm, *ydm;          // [nw][nd][maxnv]: DM actuator cells of every sensor node (closed loop)
    int maxnv, sum_n;                 // table pitch, total grid lines
    const T *jinv;                    // [nl][J+1][4] inverse preconditioner per band
    const T *ad;                      // [nl][J+1] alpha D per level
    T *b_prev, *r, *p, *q, *u, *x, *v, *ll, *probe_c, *probe_s;
    T *rsh[2], *qsh[2], *bsh;         // folded coarse updates: r, q by epilogue parity, b (N_c each)
    int *over;                        // per-sensor flags: a transpose row exceeded kRtabWidth (setup)
    double *partials;                 // [3][kPartialPitch]: (r, z) and (z, alpha D z) per wave of the
                                      // forward-DWT workgroups, sum C (Gamma P u)^2 per projection tile
    Scalars *sc;                      // [kScalarSlots]
    // a batch of frames of the same geometry: frame f's vectors, partial sums and scalar slots sit
    // f strides after frame 0's (in elements): coefficients, node grids, slopes, actuators,
    // level-kf approximations
    long fs_c, fs_v, fs_s, fs_a, fs_ll;
};

struct Plan {
    std::vector<fewha_wfs> wfs;
    std::vector<fewha_layer> lay;
    std::vector<fewha_dm> dm;
    double D = 0, obstruction = 0, alpha_reg = 0;
    int J = 0, nl = 0, nw = 0, nd = 0, prec = 0;
    size_t elem = 4;
    size_t n_coef = 0, n_slopes = 0, n_nodes = 0, n_act = 0;

    std::vector<DevWfs> dwfs;
    std::vector<DevLayer> dlay;
    std::vector<DevProj> dproj;
    std::vector<DevDm> ddm;
    // tile tables of the launches (kernel arguments)
    SegTab seg_wt{}, seg_pt{}, seg_fwd{}, seg_proj{};
    LayTab laytab{};
    LayTab dmtab{};       // per DM: actuator offset and actuators per side
    size_t n_fit = 0;     // least-squares fitting points: probe directions x first sensor's nodes
    int n_wt = 0, n_pt = 0, n_fwd = 0, n_proj = 0;  // workgroups of each launch
    int maxnv = 0, sum_n = 0;
    int kf = 1;           // forward-DWT levels done on tiles; the rest per layer in one workgroup
    int tq = 8;           // level-kf quads per tile edge of the fine forward DWT
    bool fold = false;    // coarse forward levels of all but the last pass folded into the next W^T
    bool rtab_ok = true;  // the staged transpose gather applies (else the scanning P^T)
    int last_slot = 1;    // scalar slot holding the state after the last enqueued solve
    int max_batch = 1;    // frames the workspace holds state for (same geometry, one launch per stage)
    size_t coarse_lds = 0;
    size_t pt_lds = 0;    // dynamic LDS of the staged P^T (node rectangles of every guide star)
    int pt_rw = kRtabWidth;  // the widest transpose pair count of any layer (the pairs' LDS stride)
    std::vector<double> ad;     // alpha D per (layer, level)
    std::vector<double> jtab;   // alpha D + tau per (layer, level, orientation), after bind

    // workspace layout (byte offsets)
    size_t o_wfs = 0, o_lay = 0, o_proj = 0, o_dm = 0;
    size_t o_xtab = 0, o_ytab = 0, o_xrng = 0, o_yrng = 0, o_xrtab = 0, o_yrtab = 0, o_rects = 0;
    size_t o_xdm = 0, o_ydm = 0;
    size_t o_fy = 0, o_fx = 0, o_fr = 0, o_fp = 0, o_fq = 0, o_frr = 0;  // least-squares DM fitting
    size_t o_fmask = 0;   // least-squares fitting: 1 for the first sensor's nodes inside the pupil
    size_t o_jinv = 0, o_ad = 0, o_bprev = 0, o_r = 0, o_p = 0, o_q = 0, o_u = 0, o_x = 0, o_v = 0;
    size_t o_rsh[2] = {0, 0}, o_qsh[2] = {0, 0}, o_bsh = 0;
    size_t o_ll = 0, o_stage = 0, o_probe_c = 0, o_probe_s = 0, o_partials = 0, o_scalars = 0, o_over = 0;
    size_t ws_bytes = 0;

    char *ws = nullptr;
    bool bound = false;
    int device = -1;
};

// plan.cpp (host only)
int plan_create(const fewha_config *cfg, Plan **out);
// A failed HIP call or launch: with FEWHA_DEBUG set in the environment, names it on stderr
// (call, source location, HIP's error string); returns FEWHA_ERR_HIP.
int hip_failure(hipError_t e, const char *what, const char *file, int line);

// Waves of a projection workgroup: each leaves its own partial of sum C (Gamma P u)^2.
constexpr int kProjWaves = 4;

// Waves of a coarse forward-DWT workgroup: each leaves its own pair of residual partials.
constexpr int kCoarseWaves = 16;
// Workgroups per layer that run the last pass's coarse levels of a folded solve (each recomputes W x
// of the layer's coarse block and updates a quarter of it: at most 4 coefficients per lane).
constexpr int kTailParts = 4;
// Coarse coefficients an inverse-DWT tile owns in a folded update, and the partial pairs it
// leaves for them.
constexpr int kFoldOwn = 64;
constexpr int kFoldParts = 8;

// Residual partial pairs a pass leaves for the next scalar step: one per wave of every fine
// forward-DWT tile and of every layer's coarse workgroup.
// Waves of a fine forward-DWT workgroup for the plan's (kf, tq) (each leaves its own pair).
int fwd_waves(int kf, int tq);
// With the fold, the coarse part comes from the inverse-DWT tiles instead: one pair per tile.
inline int residual_partials(const Plan &P) {
    return P.n_fwd * fwd_waves(P.kf, P.tq) + (P.kf < P.J ? (P.fold ? P.n_wt * kFoldParts : P.nl * kCoarseWaves) : 0);
}
// The fold applies (FP32; two fine levels; the level-2 block of every layer within 64 x 64).
bool fold_possible(const Plan &P);

// Values per frame of the level-kf approximation region (at most n_coef / 4 plus one), rounded up
// to a multiple of 4 so that every frame's blocks start 16-byte aligned.
inline size_t ll_stride(size_t n_coef) { return (n_coef / 4 + 1 + 3) & ~size_t(3); }

void layout_workspace(Plan *P);
// Forward-DWT split and fine-tile table (validated; FEWHA_OK, _INVALID_ARG or _UNSUPPORTED).
int set_fwd_split(Plan *P, int kf, int tq);
int level_band(int n, int J, int row, int col, int *s, int *o);
// Inverse-DWT cone of a tile: level-s region origins / sizes (level-s index space), s = 0..J.
void wt_cone(int y0, int x0, int T0, int J, int *loY, int *loX, int *LY, int *LX);

}  // namespace fewha

struct fewha_plan {
    fewha::Plan p;
};
