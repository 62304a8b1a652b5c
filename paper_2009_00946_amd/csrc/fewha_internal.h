// Internal declarations of the FEWHA MI355X library: host plan, device geometry records and
// the launchers of the HIP kernels.  Not part of the public ABI (include/fewha.h).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/fewha.h"

namespace fewha {

constexpr int kMaxLayers = 64;
constexpr int kMaxWfs = 64;
constexpr int kMaxDms = 16;
constexpr int kMaxJ = 12;
constexpr int kMaxGrid = 4096;    // sensor subapertures per side
constexpr int kMaxLayerGrid = 512; // layer nodes per side

// Inverse-DWT output tile edge (nodes); layers smaller than this form a single tile.
constexpr int kIdwtTile = 32;
// Node / subaperture / layer-node tile edge of the projection kernels.
constexpr int kNodeTile = 16;
// Coefficients per workgroup of the element-wise PCG kernels (4 per lane, 256 lanes).
constexpr int kCoefTile = 1024;
// Slots per row of the FP64 partial-sum buffer (one per workgroup of a reduction chain).
constexpr int kPartialPitch = 4096;

// Per guide star, as the kernels read it.
struct DevWfs {
    double d;        // subaperture size D / n_sub
    double x0;       // -D / 2: coordinate of node 0
    double inv_var;  // sigma^-2
    double r_out2;   // (D/2)^2: active iff r^2 <= r_out2 and r^2 >= r_in2
    double r_in2;    // (obstruction D/2)^2
    long s_off;      // offset of the s^x plane in the slope vector
    long v_off;      // offset of the (n_sub+1)^2 node grid in the node vector
    int n_sub;
    int nv;          // n_sub + 1
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

// Work-item record of a tiled kernel: a = layer or sensor, b, c = tile origin, d = tile size,
// e = coefficient offset of the layer, f = its grid size n, g = log2 n, h = tiles of that layer.
struct Tile {
    int a, b, c, d, e, f, g, h;
};

// Inclusive range [lo, hi] of sensor node indices (empty when lo > hi).
struct Range {
    int lo, hi;
};

// PCG scalars of Alg. 2 in FP64, kept on the device so no pass needs a host round trip.  The
// workspace holds three: the states after even and odd passes (written by workgroup 0 of the
// kernel that consumes a pass's reduction while the others still read the previous state) and
// one for setup-time reductions.
struct Scalars {
    double rho, mu, rho_old, alpha, alpha_old, beta;
    int stopped;     // zero residual, breakdown or non-finite: later passes are no-ops
    int status;      // FEWHA_OK, FEWHA_ERR_BREAKDOWN or FEWHA_ERR_NONFINITE
    unsigned counter;  // last-block-done counter of the reduction (returns to 0 after each use)
    int pad;
};

// Device pointers into the bound workspace, typed per precision.
template <typename T>
struct Bufs {
    const DevWfs *wfs;
    const DevLayer *lay;
    const DevProj *proj;
    const DevDm *dm;
    const Tile *idwt_tiles, *node_tiles, *sub_tiles, *lay_tiles, *fine_tiles, *coef_tiles;
    const Ent<T> *xtab, *ytab;  // [nw][nl][maxnv]
    const Range *xrng, *yrng;   // [nw][sum_n]: sensor nodes touching each layer grid line
    const RtabEnt<T> *xrtab, *yrtab;  // [nw][sum_n][kRtabWidth]: the same as (node, weight) lists
    int maxnv, sum_n, kf;       // table pitch, total grid lines, levels done by the tiled forward DWT
    const T *jinv;   // [nl][J+1][4] inverse preconditioner per band
    const T *ad;     // [nl][J+1] alpha D per level
    T *b_prev, *r, *p, *q, *y, *u, *x, *v, *tmpA, *tmpB, *b, *probe_c, *probe_s;
    T *r2, *q2;           // second residual / search-direction image buffers (PCG ping-pong)
    int *over;            // per-sensor flags: a transpose row exceeded kRtabWidth (setup only)
    double *partials;
    Scalars *sc;
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
    std::vector<Tile> idwt_tiles, node_tiles, sub_tiles, lay_tiles, fine_tiles, coef_tiles;
    int maxnv = 0, sum_n = 0;
    int kf = 1;        // forward-DWT levels done by the tiled kernel; the rest per layer in one workgroup
    bool rtab_ok = true;  // every transpose row fits kRtabWidth pairs (else the scanning P^T)
    int last_slot = 1;    // scalar slot holding the state after the last enqueued solve
    int tq = 8;        // level-kf quads per tile edge of the tiled forward DWT
    size_t coarse_lds = 0;
    std::vector<double> ad;     // alpha D per (layer, level)
    std::vector<double> jtab;   // alpha D + tau per (layer, level, orientation), after bind

    // workspace layout (byte offsets)
    size_t o_wfs = 0, o_lay = 0, o_proj = 0, o_dm = 0, o_idwt = 0, o_node = 0, o_sub = 0, o_laytile = 0;
    size_t o_fine = 0, o_coef = 0, o_xtab = 0, o_ytab = 0, o_xrng = 0, o_yrng = 0;
    size_t o_jinv = 0, o_ad = 0, o_bprev = 0, o_r = 0, o_p = 0, o_q = 0, o_y = 0, o_u = 0, o_x = 0, o_v = 0;
    size_t o_tmpA = 0, o_tmpB = 0, o_b = 0, o_probe_c = 0, o_probe_s = 0, o_partials = 0, o_scalars = 0;
    size_t o_r2 = 0, o_q2 = 0, o_lcount = 0, o_xrtab = 0, o_yrtab = 0;
    size_t ws_bytes = 0;
    int n_partials = 0;

    char *ws = nullptr;
    bool bound = false;
    int device = -1;
};

// plan.cpp (host only)
int plan_create(const fewha_config *cfg, Plan **out);
int level_band(int n, int J, int row, int col, int *s, int *o);

}  // namespace fewha

struct fewha_plan {
    fewha::Plan p;
};
