// Host side of the FEWHA plan: configuration checks, ray geometry, vector layouts, tile tables
// and the workspace map.  Touches no GPU, so configuration validation is testable anywhere.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "fewha_internal.h"

namespace fewha {

namespace {

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int ilog2(int n) {
    int k = 0;
    while ((1 << k) < n) ++k;
    return k;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Grid coordinate of a metric position on a layer (node k at (k - n/2) spacing).
double grid_coord(const fewha_layer &l, double X) { return X / l.spacing + l.n / 2; }

bool inside(double u, int n) { return u >= 0.0 && u <= double(n - 1); }

}  // namespace

// Level s (1 finest .. J) and orientation o (0 LL, 1 x-high/y-low, 2 x-low/y-high, 3 HH) of
// Mallat position (row, col) in an n x n pyramid of J levels.
int level_band(int n, int J, int row, int col, int *s, int *o) {
    int v = row > col ? row : col;
    int mJ = n >> J;
    if (v < mJ) {
        *s = J;
        *o = 0;
        return 0;
    }
    int lv = 0;
    while ((2 << lv) <= v) ++lv;  // 2^lv <= v < 2^(lv+1): band size m = 2^lv
    int m = 1 << lv;
    *s = ilog2(n) - lv;
    *o = (row < m) ? 1 : ((col < m) ? 2 : 3);
    return 0;
}

void wt_cone(int y0, int x0, int T0, int J, int *loY, int *loX, int *LY, int *LX) {
    int ly = y0, hy = y0 + T0 - 1, lx = x0, hx = x0 + T0 - 1;
    loY[0] = ly;
    loX[0] = lx;
    LY[0] = LX[0] = T0;
    for (int s = 1; s <= J; ++s) {
        ly = ((ly >> 1) - 2) & ~1;
        hy >>= 1;
        lx = ((lx >> 1) - 2) & ~1;
        hx >>= 1;
        loY[s] = ly;
        loX[s] = lx;
        LY[s] = hy - ly + 1;
        LX[s] = hx - lx + 1;
    }
}

// Byte offsets of every workspace region (tables once; per-frame state max_batch times).
void layout_workspace(Plan *P) {
    size_t o = 0;
    const size_t MB = size_t(P->max_batch);  // frames with their own vectors, partials and scalars
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t E = P->elem, N = P->n_coef;
    P->o_wfs = take(sizeof(DevWfs) * P->nw);
    P->o_lay = take(sizeof(DevLayer) * P->nl);
    P->o_proj = take(sizeof(DevProj) * P->nw * P->nl);
    P->o_dm = take(sizeof(DevDm) * P->nd);
    const size_t ent = P->prec == FEWHA_FP64 ? 24 : 16;
    P->o_xtab = take(ent * P->nw * P->nl * P->maxnv);
    P->o_ytab = take(ent * P->nw * P->nl * P->maxnv);
    P->o_xrng = take(sizeof(Range) * P->nw * P->sum_n);
    P->o_yrng = take(sizeof(Range) * P->nw * P->sum_n);
    P->o_xrtab = take((P->prec == FEWHA_FP64 ? 16 : 8) * size_t(kRtabWidth) * P->nw * P->sum_n);
    P->o_yrtab = take((P->prec == FEWHA_FP64 ? 16 : 8) * size_t(kRtabWidth) * P->nw * P->sum_n);
    P->o_rects = take(16 * size_t(P->n_pt) * P->nw);
    P->o_xdm = take(ent * P->nw * P->nd * P->maxnv);
    P->o_ydm = take(ent * P->nw * P->nd * P->maxnv);
    P->n_fit = size_t(kProbes) * (P->wfs[0].n_sub + 1) * (P->wfs[0].n_sub + 1);
    P->o_fy = take(E * P->n_fit);
    P->o_fx = take(E * P->n_act);
    P->o_fr = take(E * P->n_act);
    P->o_fp = take(E * P->n_act);
    P->o_fq = take(E * P->n_act);
    P->o_frr = take(sizeof(double) * 2);
    P->o_fmask = take(size_t(P->wfs[0].n_sub + 1) * (P->wfs[0].n_sub + 1));
    P->o_jinv = take(E * P->nl * (P->J + 1) * 4);
    P->o_ad = take(E * P->nl * (P->J + 1));
    P->o_bprev = take(E * N * MB);
    P->o_r = take(E * N * MB);
    P->o_p = take(E * N * MB);
    P->o_q = take(E * N * MB);
    P->o_u = take(E * N * MB);
    P->o_x = take(E * N * MB);
    P->o_v = take(E * P->n_nodes * MB);
    P->o_ll = take(E * ll_stride(N) * MB);
    // folded coarse updates (used at the coarse coefficients only)
    for (int i = 0; i < 2; ++i) {
        P->o_rsh[i] = take(E * N * MB);
        P->o_qsh[i] = take(E * N * MB);
    }
    P->o_bsh = take(E * N * MB);
    P->o_probe_c = take(E * N);
    P->o_stage = take(4 * E * N * MB);  // stage timing: scratch r, p, q, c of every frame
    P->o_probe_s = take(E * P->n_slopes);
    P->o_over = take(sizeof(int) * P->nw);
    P->o_partials = take(sizeof(double) * 3 * kPartialPitch * MB);
    P->o_scalars = take(kScalarSlots * sizeof(Scalars) * MB);
    P->ws_bytes = o;
}

// Forward-DWT split (Eq. (fewha)'s W): levels 1..kf on tiles of tq x tq level-kf quads over the
// whole GPU, levels kf+1..J per layer in one workgroup whose LDS holds the level-kf approximation.
// Rebuilds the fine tiles' segment table; the workspace layout does not depend on the split.
bool fold_possible(const Plan &P) {
    int max_n = 0;
    for (auto &L : P.lay) max_n = L.n > max_n ? L.n : max_n;
    return P.prec == FEWHA_FP32 && P.kf == 2 && P.J > 2 && (max_n >> 2) <= 64 &&
           P.n_fwd * fwd_waves(P.kf, P.tq) + P.n_wt * kFoldParts <= kPartialPitch;
}

int set_fwd_split(Plan *P, int kf, int tq) {
    int max_n = 0, min_n = 1 << 30;
    for (auto &L : P->lay) {
        max_n = L.n > max_n ? L.n : max_n;
        min_n = L.n < min_n ? L.n : min_n;
    }
    if (kf < 1 || kf > 2 || kf > P->J || (tq != 1 && tq != 2 && tq != 4 && tq != 8) || tq > (min_n >> kf))
        return FEWHA_ERR_INVALID_ARG;
    // the level-kf block and its first coarse level in LDS; a block too large for that is read from
    // global memory by the first coarse level, leaving two smaller levels in LDS
    const size_t m = size_t(max_n >> kf);
    size_t lds = kf < P->J ? (m * m + (m / 2) * (m / 2)) * P->elem : 0;
    if (lds > 150 * 1024) lds = ((m / 4) * (m / 4) + (m / 2) * (m / 2)) * P->elem;
    if (lds > 150 * 1024 || m * m > size_t(16) * 1024) return FEWHA_ERR_UNSUPPORTED;
    SegTab S{};
    S.nseg = P->nl;
    S.chunk = P->seg_fwd.chunk;
    for (int i = 0; i <= kMaxSeg; ++i) S.start[i] = 0x7fffffff;  // past the last segment: no match
    int n_fwd = 0;
    for (int l = 0; l < P->nl; ++l) {
        const int n = P->lay[l].n, nq = (n >> kf) / tq;
        int lt = 0;
        while ((1 << lt) < nq) ++lt;
        S.start[l] = n_fwd;
        S.off[l] = int(P->dlay[l].c_off);
        S.aux[l] = P->dlay[l].r_off;
        S.n[l] = n;
        S.lt[l] = lt;
        S.id[l] = l;
        n_fwd += nq * nq;
    }
    S.start[P->nl] = n_fwd;
    int nc = P->nl * kCoarseWaves;
    if (P->fold) nc = nc > P->n_wt * kFoldParts ? nc : P->n_wt * kFoldParts;
    const int nres = n_fwd * fwd_waves(kf, tq) + (kf < P->J ? nc : 0);
    if (nres > kPartialPitch) return FEWHA_ERR_UNSUPPORTED;
    P->kf = kf;
    P->tq = tq;
    P->coarse_lds = lds;
    P->seg_fwd = S;
    P->n_fwd = n_fwd;
    return FEWHA_OK;
}

int plan_create(const fewha_config *cfg, Plan **out) {
    if (!cfg || !out) return FEWHA_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->n_wfs < 1 || cfg->n_layers < 1 || cfg->n_dms < 1 || cfg->J < 1 || !cfg->wfs || !cfg->layers ||
        !cfg->dms)
        return FEWHA_ERR_INVALID_ARG;
    if (cfg->n_wfs > kMaxWfs || cfg->n_layers > kMaxLayers || cfg->n_dms > kMaxDms || cfg->J > kMaxJ)
        return FEWHA_ERR_UNSUPPORTED;
    if (!(cfg->D > 0) || !(cfg->obstruction >= 0 && cfg->obstruction < 1) || !(cfg->alpha_reg > 0) ||
        !std::isfinite(cfg->D) || !std::isfinite(cfg->alpha_reg))
        return FEWHA_ERR_INVALID_ARG;
    if (cfg->precision != FEWHA_FP32 && cfg->precision != FEWHA_FP64) return FEWHA_ERR_INVALID_ARG;
    for (int l = 0; l < cfg->n_layers; ++l) {
        const fewha_layer &L = cfg->layers[l];
        if (!pow2(L.n) || L.n < 2 || (L.n >> cfg->J) < 1 || !(L.spacing > 0) || !(L.cn2_weight > 0) ||
            !(L.height >= 0) || !std::isfinite(L.spacing) || !std::isfinite(L.height))
            return FEWHA_ERR_INVALID_ARG;
        if (L.n > kMaxLayerGrid) return FEWHA_ERR_UNSUPPORTED;
    }
    for (int g = 0; g < cfg->n_wfs; ++g) {
        const fewha_wfs &W = cfg->wfs[g];
        if (W.n_sub < 1 || !(W.sigma > 0) || !(W.gs_height >= 0) || !std::isfinite(W.theta_x) ||
            !std::isfinite(W.theta_y) || !std::isfinite(W.gs_height))
            return FEWHA_ERR_INVALID_ARG;
        if (W.n_sub > kMaxGrid) return FEWHA_ERR_UNSUPPORTED;
    }
    for (int m = 0; m < cfg->n_dms; ++m)
        if (cfg->dms[m].n_act < 2 || !(cfg->dms[m].pitch > 0) || !std::isfinite(cfg->dms[m].height))
            return FEWHA_ERR_INVALID_ARG;

    Plan *P = new (std::nothrow) Plan();
    if (!P) return FEWHA_ERR_INVALID_ARG;
    P->wfs.assign(cfg->wfs, cfg->wfs + cfg->n_wfs);
    P->lay.assign(cfg->layers, cfg->layers + cfg->n_layers);
    P->dm.assign(cfg->dms, cfg->dms + cfg->n_dms);
    P->D = cfg->D;
    P->obstruction = cfg->obstruction;
    P->alpha_reg = cfg->alpha_reg;
    P->J = cfg->J;
    P->nl = cfg->n_layers;
    P->nw = cfg->n_wfs;
    P->nd = cfg->n_dms;
    P->prec = cfg->precision;
    P->elem = P->prec == FEWHA_FP64 ? 8 : 4;

    // layers
    for (int l = 0; l < P->nl; ++l) {
        const fewha_layer &L = P->lay[l];
        DevLayer d{};
        d.c_off = long(P->n_coef);
        d.spacing = L.spacing;
        d.half = L.n / 2;
        d.n = L.n;
        d.log2n = ilog2(L.n);
        // fitting: nearest DM in altitude, ties to the lower one
        int best = 0;
        for (int m = 1; m < P->nd; ++m) {
            double dn = std::fabs(L.height - P->dm[m].height), db = std::fabs(L.height - P->dm[best].height);
            if (dn < db || (dn == db && P->dm[m].height < P->dm[best].height)) best = m;
        }
        d.dm = best;
        d.r_off = P->sum_n;
        P->sum_n += L.n;
        P->dlay.push_back(d);
        P->n_coef += size_t(L.n) * L.n;
    }
    // guide stars
    for (int g = 0; g < P->nw; ++g) {
        const fewha_wfs &W = P->wfs[g];
        DevWfs d{};
        d.d = P->D / W.n_sub;
        d.x0 = -P->D / 2;
        d.inv_var = 1.0 / (W.sigma * W.sigma);
        d.r_out2 = (P->D / 2) * (P->D / 2);
        d.r_in2 = (P->obstruction * P->D / 2) * (P->obstruction * P->D / 2);
        d.s_off = long(P->n_slopes);
        d.v_off = long(P->n_nodes);
        d.n_sub = W.n_sub;
        d.nv = W.n_sub + 1;
        d.vp = (d.nv + 3) & ~3;
        if (d.nv > P->maxnv) P->maxnv = d.nv;
        P->dwfs.push_back(d);
        P->n_slopes += 2 * size_t(W.n_sub) * W.n_sub;
        P->n_nodes += size_t(d.nv) * d.vp;
    }
    // DMs
    for (int m = 0; m < P->nd; ++m) {
        DevDm d{};
        d.a_off = long(P->n_act);
        d.pitch = P->dm[m].pitch;
        d.centre = (P->dm[m].n_act - 1) / 2.0;
        d.n_act = P->dm[m].n_act;
        P->ddm.push_back(d);
        P->n_act += size_t(P->dm[m].n_act) * P->dm[m].n_act;
    }
    // ray geometry and the grid checks of Sec. 2.1
    int status = FEWHA_OK;
    for (int g = 0; g < P->nw && status == FEWHA_OK; ++g) {
        const fewha_wfs &W = P->wfs[g];
        const DevWfs &dw = P->dwfs[g];
        for (int l = 0; l < P->nl; ++l) {
            const fewha_layer &L = P->lay[l];
            if (W.gs_height > 0 && !(L.height < W.gs_height)) {
                status = FEWHA_ERR_GEOMETRY;
                break;
            }
            DevProj pr{};
            pr.sig = W.gs_height > 0 ? 1.0 - L.height / W.gs_height : 1.0;
            pr.hx = W.theta_x * L.height;
            pr.hy = W.theta_y * L.height;
            pr.slope = pr.sig * dw.d / L.spacing;
            pr.bx = grid_coord(L, pr.sig * dw.x0 + pr.hx);
            pr.by = grid_coord(L, pr.sig * dw.x0 + pr.hy);
            // the map is affine and increasing in the node index: checking both ends suffices
            double u0 = grid_coord(L, pr.sig * (dw.x0 + 0 * dw.d) + pr.hx);
            double u1 = grid_coord(L, pr.sig * (dw.x0 + W.n_sub * dw.d) + pr.hx);
            double v0 = grid_coord(L, pr.sig * (dw.x0 + 0 * dw.d) + pr.hy);
            double v1 = grid_coord(L, pr.sig * (dw.x0 + W.n_sub * dw.d) + pr.hy);
            if (!inside(u0, L.n) || !inside(u1, L.n) || !inside(v0, L.n) || !inside(v1, L.n)) {
                status = FEWHA_ERR_GEOMETRY;
                break;
            }
            // the transpose gather keeps at most 24 sensor nodes per layer node and axis
            if (pr.slope < 0.1) {
                status = FEWHA_ERR_UNSUPPORTED;
                break;
            }
            P->dproj.push_back(pr);
        }
    }
    for (int l = 0; l < P->nl && status == FEWHA_OK; ++l) {
        const fewha_layer &L = P->lay[l];
        const DevDm &d = P->ddm[P->dlay[l].dm];
        double lo = grid_coord(L, (0 - d.centre) * d.pitch), hi = grid_coord(L, ((d.n_act - 1) - d.centre) * d.pitch);
        if (!inside(lo, L.n) || !inside(hi, L.n)) status = FEWHA_ERR_GEOMETRY;
    }
    if (status != FEWHA_OK) {
        delete P;
        return status;
    }

    // alpha D per (layer, level): prior read as the Kolmogorov scale law
    // gamma^-1 (spacing / d_1)^(-5/3) 2^(-(11/3)(s-1)), d_1 = subaperture size of the first sensor
    P->ad.assign(size_t(P->nl) * (P->J + 1), 0.0);
    for (int l = 0; l < P->nl; ++l)
        for (int s = 1; s <= P->J; ++s)
            P->ad[size_t(l) * (P->J + 1) + s] = P->alpha_reg / P->lay[l].cn2_weight *
                                                std::pow(P->lay[l].spacing / P->dwfs[0].d, -5.0 / 3.0) *
                                                std::pow(2.0, -(11.0 / 3.0) * (s - 1));

    if (P->n_coef >= (size_t(1) << 31) || P->n_nodes >= (size_t(1) << 31) || P->n_slopes >= (size_t(1) << 31)) {
        delete P;
        return FEWHA_ERR_UNSUPPORTED;
    }

    // tile tables (kernel arguments): inverse DWT, P^T and fine forward DWT per layer, projection
    // node tiles per guide star
    auto lg2 = [](int v) {
        int k = 0;
        while ((1 << k) < v) ++k;
        return k;
    };
    P->seg_wt.nseg = P->seg_pt.nseg = P->nl;
    // P^T: chunks of 16 tiles per XCD turn (every XCD gets a share of the heavy, first-listed layers)
    P->seg_pt.chunk = 16;
    for (int i = 0; i <= kMaxSeg; ++i)  // entries past the last segment never match a workgroup
        P->seg_wt.start[i] = P->seg_pt.start[i] = P->seg_fwd.start[i] = P->seg_proj.start[i] = 0x7fffffff;
    // P^T segments (layers) heaviest first: a tile's gather work grows with the sensor nodes per
    // layer cell, so the coarsest grids come first and their tiles are dispatched first
    std::vector<int> pt_order(P->nl);
    for (int l = 0; l < P->nl; ++l) pt_order[l] = l;
    std::stable_sort(pt_order.begin(), pt_order.end(),
                     [&](int a, int b) { return P->lay[a].spacing > P->lay[b].spacing; });
    for (int i = 0; i < P->nl; ++i) {
        const int l = pt_order[i];
        const int n = P->lay[l].n, tp = n < kPtTile ? n : kPtTile;
        SegTab &S = P->seg_pt;
        S.start[i] = P->n_pt;
        S.off[i] = int(P->dlay[l].c_off);
        S.aux[i] = P->dlay[l].r_off;
        S.n[i] = n;
        S.lt[i] = lg2(n / tp);
        S.id[i] = l;
        P->n_pt += (n / tp) * (n / tp);
    }
    for (int l = 0; l < P->nl; ++l) {
        const int n = P->lay[l].n, tw = n < kWtTile ? n : kWtTile;
        SegTab &S = P->seg_wt;
        S.start[l] = P->n_wt;
        S.off[l] = int(P->dlay[l].c_off);
        S.aux[l] = P->dlay[l].r_off;
        S.n[l] = n;
        S.lt[l] = lg2(n / tw);
        S.id[l] = l;
        P->n_wt += (n / tw) * (n / tw);
        // every inverse-DWT cone of this layer must fit the kernel's load slots and LDS
        for (int y0 = 0; y0 < n; y0 += tw)
            for (int x0 = 0; x0 < n; x0 += tw) {
                int loY[kMaxJ + 1], loX[kMaxJ + 1], LY[kMaxJ + 1], LX[kMaxJ + 1];
                wt_cone(y0, x0, tw, P->J, loY, loX, LY, LX);
                bool ok = true;
                for (int s = 1; s <= P->J; ++s) {
                    // load slots of the inverse DWT (lanes per row, rows per level) and the LDS
                    // regions of its synthesis (rows x the level's power-of-two pitch)
                    const int lanes = s == 1 ? 32 : (s == 2 ? 16 : 8), rows = (s == 1 ? 72 : (s == 2 ? 48 : 32));
                    const int lanes_o = s - 1 == 0 ? 32 : (s - 1 == 1 ? 32 : (s - 1 == 2 ? 16 : 8));
                    ok = ok && LX[s] <= lanes && (s == P->J ? 4 : 3) * LY[s] <= rows;
                    ok = ok && LX[s - 1] <= lanes_o;
                    if (s >= 2) ok = ok && LY[s - 1] * lanes_o <= 18 * 32;
                    ok = ok && ((LY[s - 1] + 1) & ~1) * lanes <= 32 * 32;
                }
                if (!ok) {
                    delete P;
                    return FEWHA_ERR_UNSUPPORTED;
                }
            }
    }
    P->seg_wt.start[P->nl] = P->n_wt;
    P->seg_pt.start[P->nl] = P->n_pt;
    {
        // forward DWT split: two levels on tiles of (at most) 8 x 8 level-2 quads
        int min_n = 1 << 30;
        for (auto &L : P->lay) min_n = L.n < min_n ? L.n : min_n;
        const int kf = P->J < 2 ? P->J : 2;
        int tq = kFwdQuads;
        while (tq > (min_n >> kf)) tq >>= 1;
        if (set_fwd_split(P, kf, tq) != FEWHA_OK) {
            delete P;
            return FEWHA_ERR_UNSUPPORTED;
        }
        P->fold = fold_possible(*P);
    }
    P->seg_proj.nseg = P->nw;
    for (int g = 0; g < P->nw; ++g) {
        const int nv = P->wfs[g].n_sub + 1, tpr = (nv + kProjTile - 1) / kProjTile;
        P->seg_proj.start[g] = P->n_proj;
        P->seg_proj.off[g] = int(P->dwfs[g].v_off);
        P->seg_proj.pitch[g] = P->dwfs[g].vp;
        P->seg_proj.aux[g] = int(P->dwfs[g].s_off);
        P->seg_proj.n[g] = P->wfs[g].n_sub;
        P->seg_proj.lt[g] = tpr;
        P->seg_proj.id[g] = g;
        P->n_proj += tpr * tpr;
    }
    P->seg_proj.start[P->nw] = P->n_proj;
    // sensors of one tile count: interleave their tiles, so that the tiles over one pupil region
    // (which read the same layer nodes) run side by side on the same XCD
    P->seg_proj.ilv = 1;
    for (int g = 1; g < P->nw; ++g)
        if (P->seg_proj.start[g + 1] - P->seg_proj.start[g] != P->seg_proj.start[1] - P->seg_proj.start[0])
            P->seg_proj.ilv = 0;
    for (int l = 0; l < P->nl; ++l) {
        P->laytab.off[l] = int(P->dlay[l].c_off);
        P->laytab.n[l] = P->lay[l].n;
    }
    for (int m = 0; m < P->nd; ++m) {
        P->dmtab.off[m] = int(P->ddm[m].a_off);
        P->dmtab.n[m] = P->ddm[m].n_act;
    }
    if (P->n_proj * kProjWaves > kPartialPitch) {
        delete P;
        return FEWHA_ERR_UNSUPPORTED;
    }

    layout_workspace(P);
    *out = P;
    return FEWHA_OK;
}

}  // namespace fewha
