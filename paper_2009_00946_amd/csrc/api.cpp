// C ABI of the FEWHA library (include/fewha.h): argument checks, workspace binding and the
// sequences of kernel launches behind each call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"
#include "trace.h"

using namespace fewha;

namespace {

template <typename T>
Bufs<T> bufs(const Plan &P) {
    Bufs<T> b{};
    char *w = P.ws;
    b.wfs = reinterpret_cast<const DevWfs *>(w + P.o_wfs);
    b.lay = reinterpret_cast<const DevLayer *>(w + P.o_lay);
    b.proj = reinterpret_cast<const DevProj *>(w + P.o_proj);
    b.dm = reinterpret_cast<const DevDm *>(w + P.o_dm);
    b.xtab = reinterpret_cast<const Ent<T> *>(w + P.o_xtab);
    b.ytab = reinterpret_cast<const Ent<T> *>(w + P.o_ytab);
    b.xrng = reinterpret_cast<const Range *>(w + P.o_xrng);
    b.yrng = reinterpret_cast<const Range *>(w + P.o_yrng);
    b.xrtab = reinterpret_cast<const RtabEnt<T> *>(w + P.o_xrtab);
    b.yrtab = reinterpret_cast<const RtabEnt<T> *>(w + P.o_yrtab);
    b.rects = reinterpret_cast<const int4 *>(w + P.o_rects);
    b.xdm = reinterpret_cast<const Ent<T> *>(w + P.o_xdm);
    b.ydm = reinterpret_cast<const Ent<T> *>(w + P.o_ydm);
    b.maxnv = P.maxnv;
    b.sum_n = P.sum_n;
    b.jinv = reinterpret_cast<const T *>(w + P.o_jinv);
    b.ad = reinterpret_cast<const T *>(w + P.o_ad);
    b.b_prev = reinterpret_cast<T *>(w + P.o_bprev);
    b.r = reinterpret_cast<T *>(w + P.o_r);
    b.p = reinterpret_cast<T *>(w + P.o_p);
    b.q = reinterpret_cast<T *>(w + P.o_q);
    b.u = reinterpret_cast<T *>(w + P.o_u);
    b.x = reinterpret_cast<T *>(w + P.o_x);
    b.v = reinterpret_cast<T *>(w + P.o_v);
    b.ll = reinterpret_cast<T *>(w + P.o_ll);
    for (int i = 0; i < 2; ++i) {
        b.rsh[i] = reinterpret_cast<T *>(w + P.o_rsh[i]);
        b.qsh[i] = reinterpret_cast<T *>(w + P.o_qsh[i]);
    }
    b.bsh = reinterpret_cast<T *>(w + P.o_bsh);
    b.probe_c = reinterpret_cast<T *>(w + P.o_probe_c);
    b.probe_s = reinterpret_cast<T *>(w + P.o_probe_s);
    b.over = reinterpret_cast<int *>(w + P.o_over);
    b.partials = reinterpret_cast<double *>(w + P.o_partials);
    b.sc = reinterpret_cast<Scalars *>(w + P.o_scalars);
    b.fs_c = (long)P.n_coef;
    b.fs_v = (long)P.n_nodes;
    b.fs_s = (long)P.n_slopes;
    b.fs_a = (long)P.n_act;
    b.fs_ll = (long)ll_stride(P.n_coef);
    return b;
}

template <typename T>
Ops<T> ops(const Plan &P, void *stream, int nb = 1) {
    Ops<T> o{P, bufs<T>(P), static_cast<hipStream_t>(stream)};
    o.nb = nb;
    return o;
}

#define TRY(x)                          \
    do {                                \
        int _e = (x);                   \
        if (_e != FEWHA_OK) return _e;  \
    } while (0)

#define HIPTRY(x)                                                       \
    do {                                                                \
        const hipError_t _h = (x);                                      \
        if (_h != hipSuccess) return hip_failure(_h, #x, __FILE__, __LINE__); \
    } while (0)

}  // namespace

int fewha::hip_failure(hipError_t e, const char *what, const char *file, int line) {
    if (std::getenv("FEWHA_DEBUG"))
        std::fprintf(stderr, "fewha: %s failed at %s:%d: %s\n", what, file, line, hipGetErrorString(e));
    return FEWHA_ERR_HIP;
}

namespace {

int ready(const fewha_plan *p) {
    if (!p) return FEWHA_ERR_INVALID_ARG;
    if (!p->p.bound) return FEWHA_ERR_WORKSPACE;
    return FEWHA_OK;
}

template <typename T>
int apply_A(const Plan &P, const void *c, void *s, void *stream, int nb = 1) {
    auto o = ops<T>(P, stream, nb);
    TRY(o.wt(static_cast<const T *>(c), o.B.u));
    return o.proj(o.B.u, static_cast<T *>(s), kProjA);
}

template <typename T>
int apply_At(const Plan &P, const void *s, void *c, void *stream, int nb = 1) {
    auto o = ops<T>(P, stream, nb);
    TRY(o.gt(static_cast<const T *>(s), o.B.v, kGtAdj));
    TRY(o.pt(o.B.v, o.B.x, PassArgs{-1, 0, 0, 0, nullptr, 0}));
    FwdArgs E{};
    E.out = c;
    return o.fwd(o.B.x, E, kEpiPlain);
}

template <typename T>
int apply_M(const Plan &P, const void *c, void *y, void *stream, int nb = 1) {
    auto o = ops<T>(P, stream, nb);
    TRY(o.wt(static_cast<const T *>(c), o.B.u));
    TRY(o.proj(o.B.u, o.B.v, kProjM));
    TRY(o.pt(o.B.v, o.B.x, PassArgs{-1, 0, 0, 0, nullptr, 0}));
    FwdArgs E{};
    E.out = y;
    E.cin = c;
    return o.fwd(o.B.x, E, kEpiPrior);
}

// The right-hand side's forward transform (Eq. (fewha)'s b = W x) with the residual update of
// Alg. 1.  With the fold (and at least one pass to fold it into) only the fine levels run here;
// the coarse ones run in the first pass's inverse DWT.
template <typename T>
int rhs_transform(const Plan &P, const Ops<T> &o, void *c, int cold, int n_iter) {
    FwdArgs R{};
    R.c = c;
    R.cold = cold;
    return o.fwd(o.B.x, R, kEpiRhs, !(P.fold && n_iter > 0));
}

// n_iter passes of Alg. 2 from the residual and scalar state a right-hand-side epilogue left.
//
// With the fold, the coarse levels of every forward transform but the last run in the next
// pass's inverse DWT (pass k applies epilogue e = k - 1, the right-hand side's for k = 0).  While
// the passes run, the coarse coefficients of r and q live in shadows by epilogue parity (epilogue
// e writes r, q to shadow (e + 1) & 1 and reads shadow e & 1), because every tile of a layer reads
// them at its cone while their owners write the new values; b's coarse coefficients wait in their
// own shadow.  The last pass reads the shadows and leaves r, q, p, c and b_prev whole (last_fwd).
// The last pass's coarse levels when the caller launches them (see last_fwd).
struct Deferred {
    bool set = false;
    FoldArgs F{};
};

// The last pass's forward transform.  c's share of the coarse levels needs no W x (c + alpha p),
// so the fine launch steps it; the coarse levels then update r, q, p (and b_prev) there and leave
// c alone: for a folded solve in the tail workgroups of an inverse-DWT launch (their arguments go
// to `defer` when the caller launches them beside its own W^T c, else they run here alone),
// otherwise in the coarse forward launch.
template <typename T>
int last_fwd(const Ops<T> &o, FwdArgs E, void *c, bool fold, int k, Deferred *defer) {
    E.cc = c;
    E.cc_r = fold ? o.B.rsh[k & 1] : nullptr;
    TRY(o.fwd(o.B.x, E, kEpiPcg, false, true));
    if (!fold) return o.fwd(o.B.x, E, kEpiPcg, true, false);
    FoldArgs F{};
    F.e = k;
    F.rin = o.B.rsh[k & 1];
    F.qin = k >= 1 ? o.B.qsh[k & 1] : nullptr;
    F.bsh = o.B.bsh;
    if (!defer) return o.wt_tail(nullptr, nullptr, F);
    defer->set = true;
    defer->F = F;
    return FEWHA_OK;
}

template <typename T>
int pcg_passes(const Plan &P, const Ops<T> &o, void *c, int n_iter, double *resnorm, int cold = 0,
               Deferred *defer = nullptr) {
    // partial sums of (r, z) and (z, alpha D z) come from the transforms that write r
    const int nres = residual_partials(P);
    const bool fold = P.fold && n_iter > 0;
    static const char *const kPassName[] = {"PCG pass 0", "PCG pass 1", "PCG pass 2", "PCG pass 3",
                                            "PCG pass 4", "PCG pass 5", "PCG pass 6", "PCG pass 7"};
    for (int k = 0; k < n_iter; ++k) {
        trace::Range tr(k < 8 ? kPassName[k] : "PCG pass");
        if (fold) {
            FoldArgs F{};                        // the previous epilogue's coarse levels, then u
            F.e = k - 1;
            F.cold = cold;
            F.c = c;
            F.rin = k == 0 ? o.B.r : o.B.rsh[(k - 1) & 1];
            F.qin = k >= 2 ? o.B.qsh[(k - 1) & 1] : nullptr;
            F.rout = o.B.rsh[k & 1];
            F.qout = o.B.qsh[k & 1];
            F.bsh = o.B.bsh;
            TRY(o.wt_fold(o.B.r, o.B.u, F));
        } else {
            TRY(o.wt_pcg(o.B.r, o.B.u));         // u = W^T J^-1 r
        }
        TRY(o.proj(o.B.u, o.B.v, kProjM));       // v = Gamma^T C Gamma P u; (C Gamma P u, Gamma P u) partials
        TRY(o.pt(o.B.v, o.B.x, PassArgs{k, nres, P.n_proj * kProjWaves, 1, resnorm, n_iter}));  // x = P^T v; Alg. 2 scalars
        FwdArgs E{};                             // y = W x + alpha D z; the pass update
        E.c = c;
        E.k = k;
        E.publish = 1;
        const bool last = k == n_iter - 1;
        if (fold && last) {                      // coarse levels from the shadows of epilogue k - 1
            E.r_in = o.B.rsh[k & 1];
            E.q_in = k >= 1 ? o.B.qsh[k & 1] : nullptr;
            E.b_in = o.B.bsh;
        }
        if (last && P.kf < P.J) TRY(last_fwd<T>(o, E, c, fold, k, defer));
        else TRY(o.fwd(o.B.x, E, kEpiPcg, !fold || last));
    }
    const_cast<Plan &>(P).last_slot = n_iter > 0 ? ((n_iter - 1) & 1) : 1;
    return FEWHA_OK;
}

template <typename T>
int pcg_solve(const Plan &P, const void *s, void *c, int n_iter, int flags, double *resnorm, void *stream,
              int nb = 1, Deferred *defer = nullptr) {
    auto o = ops<T>(P, stream, nb);
    if (flags == FEWHA_REFRESH) {
        trace::Range tr("residual refresh");
        // b_prev = M c and r_prev = 0 (written beside b_prev by the same epilogue), so that the
        // residual update below gives r = b - M c (Alg. 1's residual line in its left-hand form)
        // instead of carrying the previous frame's residual
        FwdArgs E{};
        E.out = o.B.b_prev;
        E.cin = c;
        E.rzero = 1;
        TRY(o.wt(static_cast<const T *>(c), o.B.u));
        TRY(o.proj(o.B.u, o.B.v, kProjM));
        TRY(o.pt(o.B.v, o.B.x, PassArgs{-1, 0, 0, 0, nullptr, 0}));
        TRY(o.fwd(o.B.x, E, kEpiPrior));
    }
    // right-hand side b = W P^T Gamma^T C s, then the warm-restart residual update
    const int cold = flags == FEWHA_COLD ? 1 : 0;
    {
        trace::Range tr("right-hand side");
        TRY(o.gt(static_cast<const T *>(s), o.B.v, kGtRhs));
        TRY(o.pt(o.B.v, o.B.x, PassArgs{-1, 0, 0, 0, nullptr, 0}));
        TRY(rhs_transform<T>(P, o, c, cold, n_iter));
    }
    return pcg_passes<T>(P, o, c, n_iter, resnorm, cold, defer);
}

// M c = b for a right-hand side given in the coefficient domain, from c = 0: x = W^T b first,
// so that the right-hand-side epilogue's W x reproduces b (W W^T = I, to rounding) and starts the
// residual there.
template <typename T>
int solve_M(const Plan &P, const void *b, void *c, int n_iter, double *resnorm, void *stream) {
    auto o = ops<T>(P, stream);
    TRY(o.wt(static_cast<const T *>(b), o.B.x));
    TRY(rhs_transform<T>(P, o, c, 1, n_iter));
    return pcg_passes<T>(P, o, c, n_iter, resnorm, 1);
}

template <typename T>
int apply_CA(const Plan &P, const void *c, void *s, void *stream) {
    auto o = ops<T>(P, stream);
    TRY(o.wt(static_cast<const T *>(c), o.B.u));
    return o.proj(o.B.u, static_cast<T *>(s), kProjCA);
}

template <typename T>
int prior_dot(const Plan &P, const void *x, const void *y, double *out, void *stream, bool per_gamma = false) {
    auto o = ops<T>(P, stream);
    return o.prior_dot(static_cast<const T *>(x), static_cast<const T *>(y), out, per_gamma);
}

template <typename T>
int fit_dm(const Plan &P, const void *c, const void *a_prev, double gain, void *a, void *stream, int nb = 1) {
    auto o = ops<T>(P, stream, nb);
    TRY(o.wt(static_cast<const T *>(c), o.B.u));
    return o.fit(o.B.u, static_cast<const T *>(a_prev), static_cast<T *>(a), gain);
}

// One reconstruction of Alg. 1: the solve, then the fit of its c.  In a folded solve the last
// pass's coarse levels (which the fit does not read) run as extra workgroups of the fit's W^T c.
template <typename T>
int reconstruct(const fewha_plan *h, const void *s, void *c, int n_iter, int flags, double *resnorm,
                const void *a_prev, double gain, void *a, void *stream, int nb = 1) {
    Deferred d;
    TRY(pcg_solve<T>(h->p, s, c, n_iter, flags, resnorm, stream, nb, &d));
    trace::Range tr("fit");
    if (!d.set) return fit_dm<T>(h->p, c, a_prev, gain, a, stream, nb);
    auto o = ops<T>(h->p, stream, nb);
    TRY(o.wt_tail(static_cast<const T *>(c), o.B.u, d.F));
    return o.fit(o.B.u, static_cast<const T *>(a_prev), static_cast<T *>(a), gain);
}

// Pseudo-open-loop slopes: s_pol = mask (s + Gamma P_DM a^(-1)), the projection kernel run over the
// DMs (their actuator grids as the "layers", their cell tables) with the input slopes added.
template <typename T>
int pol_slopes(const Plan &P, const void *s, const void *a_m1, void *s_pol, void *stream, int nb = 1) {
    auto o = ops<T>(P, stream, nb);
    return o.pol(static_cast<const T *>(a_m1), static_cast<const T *>(s), static_cast<T *>(s_pol));
}

template <typename T>
int fit_closed(const Plan &P, const void *c, const void *a0, const void *a_m1, double gain, void *a, void *stream,
               int nb = 1) {
    auto o = ops<T>(P, stream, nb);
    TRY(o.wt(static_cast<const T *>(c), o.B.u));
    return o.fit(o.B.u, static_cast<const T *>(a0), static_cast<T *>(a), gain, static_cast<const T *>(a_m1));
}

template <typename T>
int stage_launch(const Plan &P, int stage, void *stream, int nb = 1) {
    auto o = ops<T>(P, stream, nb);
    const size_t NS = P.n_coef * size_t(P.max_batch);  // stage scratch: blocks of max_batch frames
    T *scr = reinterpret_cast<T *>(P.ws + P.o_stage);
    switch (stage) {
        case FEWHA_STAGE_WT:
            if (P.fold) {
                // a folded update of pass 1 (the shadows are scratch between solves; p and c are
                // the stage scratch copies), then u = W^T J^-1 r
                FoldArgs F{};
                F.e = 1;
                F.c = scr + 3 * NS;
                F.rin = o.B.rsh[1];
                F.qin = o.B.qsh[1];
                F.rout = o.B.rsh[0];
                F.qout = o.B.qsh[0];
                auto os = o;
                os.B.p = scr + NS;
                return os.wt_fold(o.B.r, o.B.u, F);
            }
            return o.wt_pcg(o.B.r, o.B.u);
        case FEWHA_STAGE_PROJ: return o.proj(o.B.u, o.B.v, kProjM);
        case FEWHA_STAGE_PT:
            return o.pt(o.B.v, o.B.x, PassArgs{1, residual_partials(P), P.n_proj * kProjWaves, 0, nullptr, 0});
        default: {
            // the frame's y = W x + alpha D z with the pass update, applied to scratch copies of
            // r, p, q and c (blocks of max_batch frames each), without publishing scalars; with the
            // fold, the fine levels only (as in every pass but the last)
            o.B.r = scr;
            o.B.p = scr + NS;
            o.B.q = scr + 2 * NS;
            FwdArgs E{};
            E.c = scr + 3 * NS;
            E.k = 1;
            E.publish = 0;
            return o.fwd(o.B.x, E, kEpiPcg, !P.fold);
        }
    }
}

template <typename T>
int bind_tables(Plan &P, hipStream_t st) {
    auto o = ops<T>(P, st);
    char *w = P.ws;
    HIPTRY(hipMemcpy(w + P.o_wfs, P.dwfs.data(), sizeof(DevWfs) * P.dwfs.size(), hipMemcpyHostToDevice));
    HIPTRY(hipMemcpy(w + P.o_lay, P.dlay.data(), sizeof(DevLayer) * P.dlay.size(), hipMemcpyHostToDevice));
    HIPTRY(hipMemcpy(w + P.o_proj, P.dproj.data(), sizeof(DevProj) * P.dproj.size(), hipMemcpyHostToDevice));
    HIPTRY(hipMemcpy(w + P.o_dm, P.ddm.data(), sizeof(DevDm) * P.ddm.size(), hipMemcpyHostToDevice));
    const int nb = P.nl * (P.J + 1);
    std::vector<T> ad(nb);
    for (int k = 0; k < nb; ++k) ad[k] = (T)P.ad[k];
    HIPTRY(hipMemcpy(w + P.o_ad, ad.data(), sizeof(T) * nb, hipMemcpyHostToDevice));
    // DM cells of every sensor node (closed loop): node j of guide star g meets DM m at
    // X = sigma (x0 + j d) + theta h_m; the DM is the piecewise bilinear surface over its actuators,
    // zero beyond the outermost ones, so actuator k carries the weight max(0, 1 - |u - k|) at
    // u = X / pitch + (n_a - 1) / 2 (cells straddling the edge keep their inside actuator only)
    {
        const size_t ne = size_t(P.nw) * P.nd * P.maxnv;
        std::vector<Ent<T>> xd(ne, Ent<T>{0, 0, (T)0, (T)0}), yd(ne, Ent<T>{0, 0, (T)0, (T)0});
        for (int g = 0; g < P.nw; ++g)
            for (int m = 0; m < P.nd; ++m) {
                const DevWfs &W = P.dwfs[g];
                const DevDm &Dm = P.ddm[m];
                const double h = P.dm[m].height, H = P.wfs[g].gs_height;
                const double sig = H > 0 ? 1.0 - h / H : 1.0;
                for (int axis = 0; axis < 2; ++axis) {
                    const double th = axis ? P.wfs[g].theta_y : P.wfs[g].theta_x;
                    for (int j = 0; j < W.nv; ++j) {
                        const double u = (sig * (W.x0 + j * W.d) + th * h) / Dm.pitch + Dm.centre;
                        const int k0 = (int)std::floor(u), na = Dm.n_act;
                        const double t = u - k0;
                        Ent<T> e{0, 0, (T)0, (T)0};
                        if (k0 >= 0 && k0 <= na - 2) e = Ent<T>{k0, 0, (T)(1.0 - t), (T)t};
                        else if (k0 == -1) e = Ent<T>{0, 0, (T)t, (T)0};
                        else if (k0 == na - 1) e = Ent<T>{na - 2, 0, (T)0, (T)(1.0 - t)};
                        (axis ? yd : xd)[(size_t(g) * P.nd + m) * P.maxnv + j] = e;
                    }
                }
            }
        HIPTRY(hipMemcpy(w + P.o_xdm, xd.data(), sizeof(Ent<T>) * ne, hipMemcpyHostToDevice));
        HIPTRY(hipMemcpy(w + P.o_ydm, yd.data(), sizeof(Ent<T>) * ne, hipMemcpyHostToDevice));
    }
    // Least-squares fitting nodes (x_j, y_i) = (-D/2 + j d, -D/2 + i d) of the first sensor's grid
    // inside the closed pupil annulus obstruction D/2 <= r <= D/2; decided here in FP64 once, so
    // that nodes on the rim are kept or dropped by the definition rather than by device rounding
    {
        const int nv = P.wfs[0].n_sub + 1;
        const double d = P.D / P.wfs[0].n_sub;
        std::vector<unsigned char> fm(size_t(nv) * nv);
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < nv; ++j) {
                const double x = -P.D / 2 + j * d, y = -P.D / 2 + i * d, r = std::sqrt(x * x + y * y);
                fm[size_t(i) * nv + j] = r <= P.D / 2 && r >= P.obstruction * P.D / 2;
            }
        HIPTRY(hipMemcpy(w + P.o_fmask, fm.data(), fm.size(), hipMemcpyHostToDevice));
    }
    const long N = (long)P.n_coef;
    TRY(o.prepare());
    HIPTRY(hipMemset(o.B.over, 0, sizeof(int) * P.nw));
    TRY(o.build_tables(o.B.over));
    const long NB = N * P.max_batch;
    TRY(ops<T>(P, st, P.max_batch).init_scalars());
    TRY(o.fill(o.B.b_prev, NB, 0));
    TRY(o.fill(o.B.r, NB, 0));
    TRY(o.fill(o.B.probe_c, N, 0));
    TRY(o.fill(reinterpret_cast<T *>(w + P.o_stage), 4 * N * P.max_batch, 0));
    HIPTRY(hipStreamSynchronize(st));

    // staged P^T: every guide star's node rectangle per tile must fit the LDS stage, every
    // transpose row kRtabWidth pairs; otherwise the scanning P^T
    {
        std::vector<int> over(P.nw, 0);
        HIPTRY(hipMemcpy(over.data(), o.B.over, sizeof(int) * P.nw, hipMemcpyDeviceToHost));
        std::vector<int4> rects(size_t(P.n_pt) * P.nw);
        HIPTRY(hipMemcpy(rects.data(), o.B.rects, sizeof(int4) * rects.size(), hipMemcpyDeviceToHost));
        P.rtab_ok = P.nw <= kPtMaxWfs;
        for (int g = 0; g < P.nw; ++g)
            if (over[g]) P.rtab_ok = false;
        size_t stage = 1;
        const int ch = P.prec == FEWHA_FP64 ? 2 : 4;  // values per 16-byte chunk
        for (int l = 0; l < P.nl; ++l) {
            int rw = 1;  // the layer's pair width: the largest pair count of any of its lines
            for (int t = P.seg_pt.start[l]; t < P.seg_pt.start[l + 1]; ++t) {
                size_t need = 0;
                for (int g = 0; g < P.nw; ++g) {
                    const int4 R = rects[size_t(t) * P.nw + g];  // rows / columns packed lo | hi << 16
                    const int iA = R.x & 0xffff, iB = R.x >> 16, jA = R.y & 0xffff, jB = R.y >> 16;
                    if (iA <= iB) need += size_t(iB - iA + 1) * (((jB - (jA & ~(ch - 1))) / ch + 1) * ch);
                    if (R.z > kRtabWidth || R.w > kRtabWidth) P.rtab_ok = false;
                    rw = R.z > rw ? R.z : rw;
                    rw = R.w > rw ? R.w : rw;
                }
                stage = need > stage ? need : stage;
            }
            P.seg_pt.rw[l] = rw < kRtabWidth ? rw : kRtabWidth;
        }
        if (stage > size_t(kPtStage)) P.rtab_ok = false;
        // the tile's transpose pairs (index, weight) of every guide star, at the widest layer's
        // pair count, then the stage
        P.pt_rw = 1;
        for (int l = 0; l < P.nl; ++l) P.pt_rw = P.seg_pt.rw[l] > P.pt_rw ? P.seg_pt.rw[l] : P.pt_rw;
        P.pt_lds = size_t(P.nw) * 2 * P.pt_rw * kPtTile * (P.prec == FEWHA_FP64 ? 16 : 8) + stage * P.elem;
    }

    // Preconditioner of Sec. 3.4: J = alpha D + tau per (layer, level, orientation), with tau the
    // data-term diagonal ||C^1/2 A e_k||^2 at the band's representative coefficient
    // (block-local position (m/2, m/2)).
    P.jtab.assign(size_t(nb) * 4, 0.0);
    for (int l = 0; l < P.nl; ++l) {
        const int n = P.lay[l].n;
        for (int s = 1; s <= P.J; ++s)
            for (int ori = 0; ori < 4; ++ori) {
                if (ori == 0 && s != P.J) continue;
                const int m = n >> s;
                const int r0 = (ori == 2 || ori == 3) ? m : 0, c0 = (ori == 1 || ori == 3) ? m : 0;
                const long k = P.dlay[l].c_off + (long)(r0 + m / 2) * n + (c0 + m / 2);
                TRY(o.fill(o.B.probe_c + k, 1, (T)1));
                TRY(apply_A<T>(P, o.B.probe_c, o.B.probe_s, st));
                TRY(o.wnorm(o.B.probe_s));
                TRY(o.fill(o.B.probe_c + k, 1, (T)0));
                double tau = 0;
                HIPTRY(hipMemcpyAsync(&tau, &o.B.sc[2].rho, sizeof(double), hipMemcpyDeviceToHost, st));
                HIPTRY(hipStreamSynchronize(st));
                P.jtab[size_t(l * (P.J + 1) + s) * 4 + ori] = P.ad[size_t(l) * (P.J + 1) + s] + tau;
            }
    }
    std::vector<T> jinv(size_t(nb) * 4, (T)0);
    for (size_t k = 0; k < jinv.size(); ++k)
        if (P.jtab[k] > 0) jinv[k] = (T)(1.0 / P.jtab[k]);
    HIPTRY(hipMemcpy(w + P.o_jinv, jinv.data(), sizeof(T) * jinv.size(), hipMemcpyHostToDevice));
    TRY(ops<T>(P, st, P.max_batch).init_scalars());
    HIPTRY(hipStreamSynchronize(st));
    return FEWHA_OK;
}

}  // namespace

extern "C" {

int fewha_plan_create(const fewha_config *cfg, fewha_plan **out) {
    if (!out) return FEWHA_ERR_INVALID_ARG;
    *out = nullptr;
    Plan *P = nullptr;
    int st = plan_create(cfg, &P);
    if (st != FEWHA_OK) return st;
    fewha_plan *h = new (std::nothrow) fewha_plan;
    if (!h) {
        delete P;
        return FEWHA_ERR_INVALID_ARG;
    }
    h->p = std::move(*P);
    delete P;
    *out = h;
    return FEWHA_OK;
}

size_t fewha_workspace_bytes(const fewha_plan *p) { return p ? p->p.ws_bytes : 0; }

int fewha_plan_bind(fewha_plan *p, void *d_workspace, size_t bytes, void *stream) {
    trace::Range trace_call("fewha_plan_bind");
    if (!p || !d_workspace) return FEWHA_ERR_INVALID_ARG;
    Plan &P = p->p;
    if (bytes < P.ws_bytes || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) return FEWHA_ERR_WORKSPACE;
    int dev = -1;
    HIPTRY(hipGetDevice(&dev));
    P.ws = static_cast<char *>(d_workspace);
    P.device = dev;
    P.bound = false;
    int st = P.prec == FEWHA_FP64 ? bind_tables<double>(P, static_cast<hipStream_t>(stream))
                                  : bind_tables<float>(P, static_cast<hipStream_t>(stream));
    if (st != FEWHA_OK) return st;
    P.bound = true;
    return FEWHA_OK;
}

int fewha_plan_destroy(fewha_plan *p) {
    delete p;
    return FEWHA_OK;
}

int fewha_sizes(const fewha_plan *p, size_t *n_coef, size_t *n_slopes, size_t *n_act) {
    if (!p) return FEWHA_ERR_INVALID_ARG;
    if (n_coef) *n_coef = p->p.n_coef;
    if (n_slopes) *n_slopes = p->p.n_slopes;
    if (n_act) *n_act = p->p.n_act;
    return FEWHA_OK;
}

int fewha_apply_A(const fewha_plan *p, const void *d_c, void *d_s, void *stream) {
    trace::Range trace_call("fewha_apply_A");
    TRY(ready(p));
    if (!d_c || !d_s) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? apply_A<double>(p->p, d_c, d_s, stream) : apply_A<float>(p->p, d_c, d_s, stream);
}

int fewha_apply_At(const fewha_plan *p, const void *d_s, void *d_c, void *stream) {
    trace::Range trace_call("fewha_apply_At");
    TRY(ready(p));
    if (!d_c || !d_s) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? apply_At<double>(p->p, d_s, d_c, stream)
                                   : apply_At<float>(p->p, d_s, d_c, stream);
}

int fewha_apply_M(const fewha_plan *p, const void *d_c, void *d_y, void *stream) {
    trace::Range trace_call("fewha_apply_M");
    TRY(ready(p));
    if (!d_c || !d_y || d_c == d_y) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? apply_M<double>(p->p, d_c, d_y, stream) : apply_M<float>(p->p, d_c, d_y, stream);
}

int fewha_dwt_forward(const fewha_plan *p, const void *d_layers, void *d_c, void *stream) {
    trace::Range trace_call("fewha_dwt_forward");
    TRY(ready(p));
    if (!d_layers || !d_c || d_layers == d_c) return FEWHA_ERR_INVALID_ARG;
    if (p->p.prec == FEWHA_FP64) {
        auto o = ops<double>(p->p, stream);
        FwdArgs E{};
        E.out = d_c;
        return o.fwd(static_cast<const double *>(d_layers), E, kEpiPlain);
    }
    auto o = ops<float>(p->p, stream);
    FwdArgs E{};
    E.out = d_c;
    return o.fwd(static_cast<const float *>(d_layers), E, kEpiPlain);
}

int fewha_dwt_inverse(const fewha_plan *p, const void *d_c, void *d_layers, void *stream) {
    trace::Range trace_call("fewha_dwt_inverse");
    TRY(ready(p));
    if (!d_layers || !d_c || d_layers == d_c) return FEWHA_ERR_INVALID_ARG;
    if (p->p.prec == FEWHA_FP64) {
        auto o = ops<double>(p->p, stream);
        return o.wt(static_cast<const double *>(d_c), static_cast<double *>(d_layers));
    }
    auto o = ops<float>(p->p, stream);
    return o.wt(static_cast<const float *>(d_c), static_cast<float *>(d_layers));
}

int fewha_pcg_solve(fewha_plan *p, const void *d_s, void *d_c, int n_iter, int flags, double *d_resnorm,
                    void *stream) {
    trace::Range trace_call("fewha_pcg_solve");
    TRY(ready(p));
    if (!d_s || !d_c || n_iter < 0 || (flags != FEWHA_COLD && flags != FEWHA_WARM && flags != FEWHA_REFRESH)) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? pcg_solve<double>(p->p, d_s, d_c, n_iter, flags, d_resnorm, stream)
                                   : pcg_solve<float>(p->p, d_s, d_c, n_iter, flags, d_resnorm, stream);
}

int fewha_solve_M(fewha_plan *p, const void *d_b, void *d_c, int n_iter, double *d_resnorm, void *stream) {
    trace::Range trace_call("fewha_solve_M");
    TRY(ready(p));
    if (!d_b || !d_c || d_b == d_c || n_iter < 0) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? solve_M<double>(p->p, d_b, d_c, n_iter, d_resnorm, stream)
                                   : solve_M<float>(p->p, d_b, d_c, n_iter, d_resnorm, stream);
}

int fewha_apply_CA(const fewha_plan *p, const void *d_c, void *d_s, void *stream) {
    trace::Range trace_call("fewha_apply_CA");
    TRY(ready(p));
    if (!d_c || !d_s) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? apply_CA<double>(p->p, d_c, d_s, stream) : apply_CA<float>(p->p, d_c, d_s, stream);
}

int fewha_prior_dot(const fewha_plan *p, const void *d_x, const void *d_y, double *d_out, void *stream) {
    trace::Range trace_call("fewha_prior_dot");
    TRY(ready(p));
    if (!d_x || !d_y || !d_out) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? prior_dot<double>(p->p, d_x, d_y, d_out, stream)
                                   : prior_dot<float>(p->p, d_x, d_y, d_out, stream);
}

int fewha_cn2_gradient(const fewha_plan *p, const void *d_lambda, const void *d_c, double *d_out, void *stream) {
    trace::Range trace_call("fewha_cn2_gradient");
    TRY(ready(p));
    if (!d_lambda || !d_c || !d_out) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? prior_dot<double>(p->p, d_lambda, d_c, d_out, stream, true)
                                   : prior_dot<float>(p->p, d_lambda, d_c, d_out, stream, true);
}

int fewha_reconstruct(fewha_plan *p, const void *d_s, void *d_c, int n_iter, int flags, double *d_resnorm,
                      const void *d_a_prev, double gain, void *d_a, void *stream) {
    trace::Range trace_call("fewha_reconstruct");
    TRY(ready(p));
    if (!d_s || !d_c || !d_a || d_a == d_c || d_a == d_s || n_iter < 0 || !std::isfinite(gain) ||
        (flags != FEWHA_COLD && flags != FEWHA_WARM && flags != FEWHA_REFRESH))
        return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64
               ? reconstruct<double>(p, d_s, d_c, n_iter, flags, d_resnorm, d_a_prev, gain, d_a, stream)
               : reconstruct<float>(p, d_s, d_c, n_iter, flags, d_resnorm, d_a_prev, gain, d_a, stream);
}

int fewha_fit_dm(const fewha_plan *p, const void *d_c, const void *d_a_prev, double gain, void *d_a, void *stream) {
    trace::Range trace_call("fewha_fit_dm");
    TRY(ready(p));
    if (!d_c || !d_a || d_a == d_c || !std::isfinite(gain)) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? fit_dm<double>(p->p, d_c, d_a_prev, gain, d_a, stream)
                                   : fit_dm<float>(p->p, d_c, d_a_prev, gain, d_a, stream);
}

int fewha_pol_slopes(const fewha_plan *p, const void *d_s, const void *d_a_m1, void *d_s_pol, void *stream) {
    trace::Range trace_call("fewha_pol_slopes");
    TRY(ready(p));
    if (!d_s || !d_a_m1 || !d_s_pol || d_s_pol == d_a_m1) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? pol_slopes<double>(p->p, d_s, d_a_m1, d_s_pol, stream)
                                   : pol_slopes<float>(p->p, d_s, d_a_m1, d_s_pol, stream);
}

int fewha_fit_dm_closed(const fewha_plan *p, const void *d_c, const void *d_a0, const void *d_a_m1, double gain,
                        void *d_a, void *stream) {
    trace::Range trace_call("fewha_fit_dm_closed");
    TRY(ready(p));
    if (!d_c || !d_a0 || !d_a_m1 || !d_a || d_a == d_c || d_a == d_a_m1 || !std::isfinite(gain))
        return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? fit_closed<double>(p->p, d_c, d_a0, d_a_m1, gain, d_a, stream)
                                   : fit_closed<float>(p->p, d_c, d_a0, d_a_m1, gain, d_a, stream);
}

int fewha_fit_dm_ls(const fewha_plan *p, const void *d_c, const void *d_a_prev, double gain, int n_cg, double eps,
                    void *d_a, void *stream) {
    trace::Range trace_call("fewha_fit_dm_ls");
    TRY(ready(p));
    if (!d_c || !d_a || d_a == d_c || n_cg < 0 || !std::isfinite(gain) || !(eps >= 0) || !std::isfinite(eps))
        return FEWHA_ERR_INVALID_ARG;
    const Plan &P = p->p;
    if (P.prec == FEWHA_FP64) {
        auto o = ops<double>(P, stream);
        TRY(o.wt(static_cast<const double *>(d_c), o.B.u));
        return o.fit_ls(o.B.u, static_cast<const double *>(d_a_prev), static_cast<double *>(d_a), gain, n_cg, eps);
    }
    auto o = ops<float>(P, stream);
    TRY(o.wt(static_cast<const float *>(d_c), o.B.u));
    return o.fit_ls(o.B.u, static_cast<const float *>(d_a_prev), static_cast<float *>(d_a), gain, n_cg, eps);
}

int fewha_plan_set_batch(fewha_plan *p, int max_batch) {
    if (!p || max_batch < 1 || max_batch > kMaxBatch) return FEWHA_ERR_INVALID_ARG;
    p->p.max_batch = max_batch;
    p->p.bound = false;  // the workspace map changed: bind again
    p->p.ws = nullptr;
    layout_workspace(&p->p);
    return FEWHA_OK;
}

static int batch_ok(const fewha_plan *p, int nbatch) {
    TRY(ready(p));
    return nbatch >= 1 && nbatch <= p->p.max_batch ? FEWHA_OK : FEWHA_ERR_INVALID_ARG;
}

int fewha_apply_A_batch(const fewha_plan *p, int nbatch, const void *d_c, void *d_s, void *stream) {
    trace::Range trace_call("fewha_apply_A_batch");
    TRY(batch_ok(p, nbatch));
    if (!d_c || !d_s) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? apply_A<double>(p->p, d_c, d_s, stream, nbatch)
                                   : apply_A<float>(p->p, d_c, d_s, stream, nbatch);
}

int fewha_apply_At_batch(const fewha_plan *p, int nbatch, const void *d_s, void *d_c, void *stream) {
    trace::Range trace_call("fewha_apply_At_batch");
    TRY(batch_ok(p, nbatch));
    if (!d_c || !d_s) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? apply_At<double>(p->p, d_s, d_c, stream, nbatch)
                                   : apply_At<float>(p->p, d_s, d_c, stream, nbatch);
}

int fewha_apply_M_batch(const fewha_plan *p, int nbatch, const void *d_c, void *d_y, void *stream) {
    trace::Range trace_call("fewha_apply_M_batch");
    TRY(batch_ok(p, nbatch));
    if (!d_c || !d_y || d_c == d_y) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? apply_M<double>(p->p, d_c, d_y, stream, nbatch)
                                   : apply_M<float>(p->p, d_c, d_y, stream, nbatch);
}

int fewha_pcg_solve_batch(fewha_plan *p, int nbatch, const void *d_s, void *d_c, int n_iter, int flags,
                          double *d_resnorm, void *stream) {
    trace::Range trace_call("fewha_pcg_solve_batch");
    TRY(batch_ok(p, nbatch));
    if (!d_s || !d_c || n_iter < 0 || (flags != FEWHA_COLD && flags != FEWHA_WARM && flags != FEWHA_REFRESH)) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? pcg_solve<double>(p->p, d_s, d_c, n_iter, flags, d_resnorm, stream, nbatch)
                                   : pcg_solve<float>(p->p, d_s, d_c, n_iter, flags, d_resnorm, stream, nbatch);
}

int fewha_reconstruct_batch(fewha_plan *p, int nbatch, const void *d_s, void *d_c, int n_iter, int flags,
                            double *d_resnorm, const void *d_a_prev, double gain, void *d_a, void *stream) {
    trace::Range trace_call("fewha_reconstruct_batch");
    TRY(batch_ok(p, nbatch));
    if (!d_s || !d_c || !d_a || d_a == d_c || d_a == d_s || n_iter < 0 || !std::isfinite(gain) ||
        (flags != FEWHA_COLD && flags != FEWHA_WARM && flags != FEWHA_REFRESH))
        return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64
               ? reconstruct<double>(p, d_s, d_c, n_iter, flags, d_resnorm, d_a_prev, gain, d_a, stream, nbatch)
               : reconstruct<float>(p, d_s, d_c, n_iter, flags, d_resnorm, d_a_prev, gain, d_a, stream, nbatch);
}

int fewha_fit_dm_batch(const fewha_plan *p, int nbatch, const void *d_c, const void *d_a_prev, double gain,
                       void *d_a, void *stream) {
    trace::Range trace_call("fewha_fit_dm_batch");
    TRY(batch_ok(p, nbatch));
    if (!d_c || !d_a || d_a == d_c || !std::isfinite(gain)) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? fit_dm<double>(p->p, d_c, d_a_prev, gain, d_a, stream, nbatch)
                                   : fit_dm<float>(p->p, d_c, d_a_prev, gain, d_a, stream, nbatch);
}

int fewha_pol_slopes_batch(const fewha_plan *p, int nbatch, const void *d_s, const void *d_a_m1, void *d_s_pol,
                           void *stream) {
    trace::Range trace_call("fewha_pol_slopes_batch");
    TRY(batch_ok(p, nbatch));
    if (!d_s || !d_a_m1 || !d_s_pol || d_s_pol == d_a_m1) return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? pol_slopes<double>(p->p, d_s, d_a_m1, d_s_pol, stream, nbatch)
                                   : pol_slopes<float>(p->p, d_s, d_a_m1, d_s_pol, stream, nbatch);
}

int fewha_fit_dm_closed_batch(const fewha_plan *p, int nbatch, const void *d_c, const void *d_a0, const void *d_a_m1,
                              double gain, void *d_a, void *stream) {
    trace::Range trace_call("fewha_fit_dm_closed_batch");
    TRY(batch_ok(p, nbatch));
    if (!d_c || !d_a0 || !d_a_m1 || !d_a || d_a == d_c || d_a == d_a_m1 || !std::isfinite(gain))
        return FEWHA_ERR_INVALID_ARG;
    return p->p.prec == FEWHA_FP64 ? fit_closed<double>(p->p, d_c, d_a0, d_a_m1, gain, d_a, stream, nbatch)
                                   : fit_closed<float>(p->p, d_c, d_a0, d_a_m1, gain, d_a, stream, nbatch);
}

int fewha_last_status_batch(const fewha_plan *p, int nbatch, int *h_status) {
    TRY(batch_ok(p, nbatch));
    if (!h_status) return FEWHA_ERR_INVALID_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return FEWHA_ERR_HIP;
    std::vector<Scalars> sc(size_t(nbatch) * kScalarSlots);
    if (hipMemcpy(sc.data(), p->p.ws + p->p.o_scalars, sizeof(Scalars) * sc.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return FEWHA_ERR_HIP;
    for (int f = 0; f < nbatch; ++f) h_status[f] = sc[size_t(f) * kScalarSlots + p->p.last_slot].status;
    return FEWHA_OK;
}

int fewha_stage_launch(const fewha_plan *p, int stage, void *stream) {
    TRY(ready(p));
    if (stage < FEWHA_STAGE_WT || stage > FEWHA_STAGE_FWD) return FEWHA_ERR_INVALID_ARG;
    const Plan &P = p->p;
    if (P.prec == FEWHA_FP64) return stage_launch<double>(P, stage, stream);
    return stage_launch<float>(P, stage, stream);
}

int fewha_get_tuning(const fewha_plan *p, fewha_tuning *t) {
    if (!p || !t) return FEWHA_ERR_INVALID_ARG;
    const Plan &P = p->p;
    *t = fewha_tuning{P.kf, P.tq, P.seg_wt.chunk, P.seg_proj.chunk, P.seg_pt.chunk, P.seg_fwd.chunk, P.fold ? 1 : 0};
    return FEWHA_OK;
}

int fewha_set_tuning(fewha_plan *p, const fewha_tuning *t) {
    if (!p || !t) return FEWHA_ERR_INVALID_ARG;
    const int ch[4] = {t->chunk_wt, t->chunk_proj, t->chunk_pt, t->chunk_fwd};
    for (int c : ch)
        if (c < 0 || c > 256) return FEWHA_ERR_INVALID_ARG;
    if (t->fold != 0 && t->fold != 1) return FEWHA_ERR_INVALID_ARG;
    Plan &P = p->p;
    Plan keep = P;
    P.seg_fwd.chunk = t->chunk_fwd;
    P.fold = t->fold == 1;
    int st = set_fwd_split(&P, t->kf, t->tq);
    if (st == FEWHA_OK && P.fold && !fold_possible(P)) st = FEWHA_ERR_UNSUPPORTED;
    if (st != FEWHA_OK) {
        P = keep;
        return st;
    }
    P.seg_wt.chunk = t->chunk_wt;
    P.seg_proj.chunk = t->chunk_proj;
    P.seg_pt.chunk = t->chunk_pt;
    return FEWHA_OK;
}

}  // extern "C"

namespace {

// Device microseconds per launch of one stage over nb frames: `reps` launches captured in a HIP
// graph on stream st, replayed `replays` times between two events.
template <typename T>
int time_stage(const Plan &P, int stage, int nb, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double *us) {
    constexpr int reps = 10, replays = 3;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIPTRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = FEWHA_OK;
    for (int i = 0; i < reps && rc == FEWHA_OK; ++i) rc = stage_launch<T>(P, stage, st, nb);
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (rc != FEWHA_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    HIPTRY(ec);
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(ge, st);  // warm-up replay
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < replays && e == hipSuccess; ++i) e = hipGraphLaunch(ge, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (ge) (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
    HIPTRY(e);
    *us = 1e3 * double(ms) / (reps * replays);
    return FEWHA_OK;
}

template <typename T>
int autotune_on(fewha_plan *h, int nb, hipStream_t st, hipEvent_t e0, hipEvent_t e1, fewha_tuning *best, double *us) {
    Plan &P = h->p;
    const long NB = (long)P.n_coef * nb;
    auto o = ops<T>(P, st, nb);
    // a non-degenerate pass state on every frame: r = 1, then one pass of the stages fills u, v,
    // x, the partial sums and the current step (so that no stage runs a stopped-solve shortcut)
    TRY(o.init_scalars());
    TRY(o.fill(o.B.r, NB, (T)1));
    for (int s = FEWHA_STAGE_WT; s <= FEWHA_STAGE_FWD; ++s) TRY(stage_launch<T>(P, s, st, nb));
    fewha_tuning t{};
    TRY(fewha_get_tuning(h, &t));
    // A candidate replaces the current choice only when it is faster by more than kGain, so that
    // timing noise does not flip the shapes from run to run.
    constexpr double kGain = 0.97;
    // 1. the forward-DWT split (kf, tq), timed on the forward-DWT stage with all its levels,
    // starting from the plan's current split
    const int fold_default = t.fold;
    t.fold = 0;
    TRY(fewha_set_tuning(h, &t));
    double bt = 0;
    TRY(time_stage<T>(P, FEWHA_STAGE_FWD, nb, st, e0, e1, &bt));
    fewha_tuning bs = t;
    for (int kf = 1; kf <= 2; ++kf)
        for (int tq : {1, 2, 4, 8}) {
            fewha_tuning c = t;
            c.kf = kf;
            c.tq = tq;
            if ((kf == t.kf && tq == t.tq) || fewha_set_tuning(h, &c) != FEWHA_OK) continue;
            double u = 0;
            TRY(time_stage<T>(P, FEWHA_STAGE_FWD, nb, st, e0, e1, &u));
            if (u < kGain * bt) {
                bt = u;
                bs = c;
            }
        }
    t = bs;
    TRY(fewha_set_tuning(h, &t));
    // 2. the fold against none, on the inverse and forward DWT stages together (where it applies)
    {
        fewha_tuning c = t;
        c.fold = 1;
        if (fewha_set_tuning(h, &c) == FEWHA_OK) {
            double w1 = 0, f1 = 0, w0 = 0, f0 = 0;
            TRY(time_stage<T>(P, FEWHA_STAGE_WT, nb, st, e0, e1, &w1));
            TRY(time_stage<T>(P, FEWHA_STAGE_FWD, nb, st, e0, e1, &f1));
            TRY(fewha_set_tuning(h, &t));
            TRY(time_stage<T>(P, FEWHA_STAGE_WT, nb, st, e0, e1, &w0));
            TRY(time_stage<T>(P, FEWHA_STAGE_FWD, nb, st, e0, e1, &f0));
            // the plan's default (fold where it applies) unless the other is clearly faster
            const bool on = fold_default ? !(w0 + f0 < kGain * (w1 + f1)) : (w1 + f1 < kGain * (w0 + f0));
            if (on) t = c;
            TRY(fewha_set_tuning(h, &t));
        }
    }
    // 3. each tile kernel's XCD chunk, on its own stage
    int *chunk[4] = {&t.chunk_wt, &t.chunk_proj, &t.chunk_pt, &t.chunk_fwd};
    for (int s = FEWHA_STAGE_WT; s <= FEWHA_STAGE_FWD; ++s) {
        const int k0 = *chunk[s];
        double bu = 0;
        TRY(time_stage<T>(P, s, nb, st, e0, e1, &bu));
        int bk = k0;
        for (int k : {0, 4, 8, 16, 32}) {
            if (k == k0) continue;
            *chunk[s] = k;
            TRY(fewha_set_tuning(h, &t));
            double u = 0;
            TRY(time_stage<T>(P, s, nb, st, e0, e1, &u));
            if (u < kGain * bu) {
                bu = u;
                bk = k;
            }
        }
        *chunk[s] = bk;
        TRY(fewha_set_tuning(h, &t));
        if (us) us[s] = bu;
    }
    // the state fewha_plan_bind leaves: no warm-restart history, fresh scalars
    TRY(o.fill(o.B.b_prev, NB, (T)0));
    TRY(o.fill(o.B.r, NB, (T)0));
    TRY(o.init_scalars());
    HIPTRY(hipStreamSynchronize(st));
    *best = t;
    return FEWHA_OK;
}

}  // namespace

extern "C" {

int fewha_autotune(fewha_plan *p, int nbatch, fewha_tuning *h_best, double *h_us) {
    trace::Range trace_call("fewha_autotune");
    TRY(batch_ok(p, nbatch));
    if (!h_best) return FEWHA_ERR_INVALID_ARG;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPTRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
    int rc = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess ? FEWHA_OK : FEWHA_ERR_HIP;
    fewha_tuning keep{};
    fewha_get_tuning(p, &keep);
    if (rc == FEWHA_OK)
        rc = p->p.prec == FEWHA_FP64 ? autotune_on<double>(p, nbatch, st, e0, e1, h_best, h_us)
                                     : autotune_on<float>(p, nbatch, st, e0, e1, h_best, h_us);
    if (rc != FEWHA_OK) fewha_set_tuning(p, &keep);
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    return rc;
}

int fewha_stage_launch_batch(const fewha_plan *p, int nbatch, int stage, void *stream) {
    TRY(batch_ok(p, nbatch));
    if (stage < FEWHA_STAGE_WT || stage > FEWHA_STAGE_FWD) return FEWHA_ERR_INVALID_ARG;
    const Plan &P = p->p;
    if (P.prec == FEWHA_FP64) return stage_launch<double>(P, stage, stream, nbatch);
    return stage_launch<float>(P, stage, stream, nbatch);
}

int fewha_state_get(const fewha_plan *p, void *d_b_prev, void *d_r_prev, void *stream) {
    trace::Range trace_call("fewha_state_get");
    TRY(ready(p));
    if (!d_b_prev || !d_r_prev) return FEWHA_ERR_INVALID_ARG;
    const long N = (long)p->p.n_coef;
    if (p->p.prec == FEWHA_FP64) {
        auto o = ops<double>(p->p, stream);
        TRY(o.copy(static_cast<double *>(d_b_prev), o.B.b_prev, N));
        return o.copy(static_cast<double *>(d_r_prev), o.B.r, N);
    }
    auto o = ops<float>(p->p, stream);
    TRY(o.copy(static_cast<float *>(d_b_prev), o.B.b_prev, N));
    return o.copy(static_cast<float *>(d_r_prev), o.B.r, N);
}

int fewha_state_set(fewha_plan *p, const void *d_b_prev, const void *d_r_prev, void *stream) {
    trace::Range trace_call("fewha_state_set");
    TRY(ready(p));
    if (!d_b_prev || !d_r_prev) return FEWHA_ERR_INVALID_ARG;
    const long N = (long)p->p.n_coef;
    if (p->p.prec == FEWHA_FP64) {
        auto o = ops<double>(p->p, stream);
        TRY(o.copy(o.B.b_prev, static_cast<const double *>(d_b_prev), N));
        return o.copy(o.B.r, static_cast<const double *>(d_r_prev), N);
    }
    auto o = ops<float>(p->p, stream);
    TRY(o.copy(o.B.b_prev, static_cast<const float *>(d_b_prev), N));
    return o.copy(o.B.r, static_cast<const float *>(d_r_prev), N);
}

int fewha_precond_table(const fewha_plan *p, double *h_jdiag) {
    TRY(ready(p));
    if (!h_jdiag) return FEWHA_ERR_INVALID_ARG;
    std::memcpy(h_jdiag, p->p.jtab.data(), sizeof(double) * p->p.jtab.size());
    return FEWHA_OK;
}

int fewha_last_status(const fewha_plan *p) {
    TRY(ready(p));
    if (hipDeviceSynchronize() != hipSuccess) return FEWHA_ERR_HIP;  // final, on every stream
    int st = 0;
    const Scalars *sc = reinterpret_cast<const Scalars *>(p->p.ws + p->p.o_scalars) + p->p.last_slot;
    if (hipMemcpy(&st, &sc->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return FEWHA_ERR_HIP;
    return st;
}

const char *fewha_strerror(int status) {
    switch (status) {
        case FEWHA_OK: return "ok";
        case FEWHA_ERR_INVALID_ARG: return "invalid argument";
        case FEWHA_ERR_GEOMETRY: return "geometry: a projected point or actuator leaves its layer grid";
        case FEWHA_ERR_UNSUPPORTED: return "configuration outside the implemented limits";
        case FEWHA_ERR_HIP: return "HIP runtime error";
        case FEWHA_ERR_WORKSPACE: return "plan not bound or workspace too small";
        case FEWHA_ERR_BREAKDOWN: return "PCG breakdown (non-positive curvature)";
        case FEWHA_ERR_NONFINITE: return "non-finite value in a PCG reduction";
        default: return "unknown status";
    }
}

}  // extern "C"
