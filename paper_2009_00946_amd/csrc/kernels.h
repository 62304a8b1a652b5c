// Launch interface of the FEWHA kernels (kernels.hip), used by the C ABI layer (api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include "fewha_internal.h"

namespace fewha {

// Operands of the forward transform's epilogues.
struct FwdArgs {
    void *out;          // plain / prior: destination coefficients
    const void *cin;    // prior: c of y = W x + alpha D c
    void *c;            // pcg: iterate c (updated); rhs: caller's c (zeroed on a cold start)
    int cold;           // rhs: cold start
    int rzero;          // prior: also set the plan's r to 0 at every coefficient written
    int k;              // pcg: pass index (0 = first pass: beta = 0, p = z, q = y)
    int publish;        // pcg: workgroup 0 stores the pass's scalar state (0 for stage timing)
    // pcg, coarse levels of a solve whose earlier coarse updates were folded into the inverse DWT:
    // r and q before the update come from these shadows, and b_in (the right-hand side's coarse
    // coefficients) is copied to b_prev (null: the plan's own r, q; no copy)
    const void *r_in, *q_in, *b_in;
    // pcg, last pass: the fine transform's workgroups also step the coarse coefficients of c (each
    // its share of the layer's coarse block; c's update needs no W x), from cc_r, the residual
    // before the update there (null: the plan's r); the coarse levels then run with c null and
    // leave c alone, so that nothing that reads only c waits for them
    void *cc;
    const void *cc_r;
};

// The coarse levels (kf+1..J) of the forward transform that precedes an inverse DWT, folded into
// that inverse DWT: every tile of a layer recomputes them from the level-kf approximation, applies
// the update of epilogue e at the coefficients of its cone and at its own share of the layer's
// coarse block, and leaves the partial sums of its share.
struct FoldArgs {
    int e;              // -1: the right-hand side's (r = (b - b_prev) + r_prev); k >= 0: pass k's update
    int cold;           // e = -1: cold start (r = b, c = 0)
    int kf;             // levels done on the fine tiles
    int nfine;          // partial slots of the fine tiles (the fold's slots follow, one per tile)
    void *c;            // caller's iterate (updated at the owned coefficients)
    const void *rin;    // r before the update: the plan's r for e = -1, else the shadow of e - 1
    const void *qin;    // q before the update (e >= 1)
    void *rout, *qout;  // r, q after the update (shadows of e)
    void *bsh;          // e = -1: b at the coarse coefficients (copied to b_prev at the solve's end)
    // the last pass's coarse levels (kWtTail): workgroups [0, ntail) of the launch, `parts` per
    // layer, update p, q, r (from rin, qin) and copy bsh to b_prev; the tiles follow them
    int ntail, parts;
};

// The PCG pass whose scalar step an x = P^T v launch also performs (k < 0: none).
struct PassArgs {
    int k;              // pass index
    int nwt, nproj;     // partial sums of the residual-writing transforms and of the projection
    int publish;        // store the new scalar state in the slot of pass k and sqrt(rho) in resnorm
    double *resnorm;    // frame f's values start at resnorm + f * rstride
    int rstride;
};

// Daubechies-3 analysis taps h and high-pass partner g_n = (-1)^n h_{5-n}.
template <typename T>
struct Taps {
    T h[6];
    T g[6];
};

template <typename T>
Taps<T> make_taps();

// Node-tile modes: Gamma^T C Gamma P u (with the data-term partial) | mask Gamma P u |
// C mask Gamma P u | mask (s + Gamma P_DM a) (pseudo-open-loop slopes; the DMs as the "layers").
enum { kProjM = 0, kProjA = 1, kProjCA = 2, kProjPol = 3 };
// Gamma^T modes: Gamma^T C s (right-hand side) | Gamma^T mask s (adjoint of A).
enum { kGtRhs = 0, kGtAdj = 1 };

// Epilogues of the forward transform:
//   plain  y = W x
//   prior  y = W x + alpha D c
//   pcg    y = W x + alpha D z (z = J^-1 r), then the Alg. 2 update of the pass in place:
//          p = z + beta p, q = y + beta q, c += alpha p, r -= alpha q
//   rhs    b = W x, then the warm-restart residual update r = (b - b_prev) + r, b_prev = b
enum { kEpiPlain = 0, kEpiPrior = 1, kEpiPcg = 2, kEpiRhs = 3 };

// Enqueues the kernels of one plan on one stream; every call returns FEWHA_OK or FEWHA_ERR_HIP.
template <typename T>
struct Ops {
    const Plan &P;
    Bufs<T> B;
    hipStream_t st;
    int nb = 1;  // frames per launch (grid y); caller vectors are [nb][length], frame-major

    int prepare() const;                                  // per-device kernel attributes (bind)
    int wt(const T *c, T *out) const;                     // out = W^T c
    int wt_pcg(const T *r, T *out) const;                 // out = W^T J^-1 r
    int wt_fold(const T *r, T *out, const FoldArgs &F) const;  // the fold's update, then out = W^T J^-1 r'
    // the last pass's coarse levels (pass F.e, operands F.rin, F.qin, F.bsh) beside out = W^T c
    // (c null: those levels alone)
    int wt_tail(const T *c, T *out, const FoldArgs &F) const;
    int proj(const T *u, T *out, int mode) const;         // kProjM: v = Gamma^T C Gamma P u; kProjA/CA: s = (C) mask Gamma P u
    int gt(const T *s, T *v, int mode) const;             // v = Gamma^T C s | Gamma^T mask s
    int pt(const T *v, T *x, const PassArgs &PA) const;   // x = P^T v (+ the scalar step of pass PA.k)
    // W x with an epilogue: the fine levels (fine) and the levels past kf (coarse)
    int fwd(const T *x, const FwdArgs &E, int epi, bool coarse = true, bool fine = true) const;
    int wnorm(const T *s) const;                          // sc[2].rho = sum C s^2
    int fit(const T *u, const T *a_prev, T *a, double gain, const T *a_m1 = nullptr) const;  // a_m1: closed loop
    int pol(const T *a_m1, const T *s, T *s_pol) const;   // s_pol = mask (s + Gamma P_DM a_m1)
    // least-squares fit of the layers u onto the DMs (n_cg CG steps), then the open-loop gain
    int fit_ls(const T *u, const T *a_prev, T *a, double gain, int n_cg, double eps) const;
    // out[l] = sum_layer x alpha D y, times 1 / gamma_l with `per_gamma` (the Cn^2 gradient)
    int prior_dot(const T *x, const T *y, double *out, bool per_gamma = false) const;
    int build_tables(int *over) const;                    // projection cell, transpose and rectangle tables
    int fill(T *x, long n, T val) const;
    int copy(T *dst, const T *src, long n) const;
    int init_scalars() const;
};

}  // namespace fewha
