// Launch interface of the FEWHA kernels (kernels.hip), used by the C ABI layer (api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include "fewha_internal.h"

namespace fewha {

// Operands of the forward transform's epilogues.
struct FwdArgs {
    void *out;          // destination coefficients (plain / prior / pcg)
    const void *cin;    // prior: c of y = W x + alpha D c
    const void *rk;     // pcg: r_k
    void *c;            // rhs: caller's c (zeroed on a cold start)
    int cold;           // rhs
};

// Operands of the inverse transform (with the fused Alg. 2 update in kInvUpdate mode).
struct InvArgs {
    const void *src;   // plain: c; first / update: r_{k-1} (update) or r_0 (first)
    void *out;         // layer nodal values
    const void *yv;    // update: y_{k-1}
    const void *qold;  // update: q_{k-2} (unused when k-1 is the first pass)
    void *qnew;        // update: q_{k-1}
    void *rnew;        // update: r_k
    void *c;           // update: iterate c (owned entries updated)
    int first_pass;    // update: pass k-1 was the first (p = z, q = y)
    int kprev;         // update: index of the pass whose reduction this launch consumes
    int nparts;        // update: number of FP64 partials of that pass
    double *resnorm;   // update: optional sqrt(rho) output
};

// Daubechies-3 analysis taps h and high-pass partner g_n = (-1)^n h_{5-n}.
template <typename T>
struct Taps {
    T h[6];
    T g[6];
};

template <typename T>
Taps<T> make_taps();

enum { kModeM = 0, kModeRhs = 1, kModeAdj = 2 };

// Epilogues of the forward transform: y = W x | y = W x + alpha D c | y = W x + alpha D J^-1 r with
// the PCG dot products | b = W x with the warm-restart residual update of Alg. 1.
enum { kEpiPlain = 0, kEpiPrior = 1, kEpiPcg = 2, kEpiRhs = 3 };

// Inverse-transform input modes: c as given | z = J^-1 r | Alg. 2 update, then z = J^-1 r_new.
enum { kInvPlain = 0, kInvFirst = 1, kInvUpdate = 2 };

// Enqueues the kernels of one plan on one stream; every call returns FEWHA_OK or FEWHA_ERR_HIP.
template <typename T>
struct Ops {
    const Plan &P;
    Bufs<T> B;
    hipStream_t st;

    int prepare() const;                                     // per-device kernel attributes (bind)
    int nparts() const;                                      // FP64 partials per forward transform
    int idwt(const T *c, T *out) const;                      // out = W^T c
    int idwt_first(const T *r, T *out) const;                // out = W^T J^-1 r
    // consume pass kprev's reduction (Alg. 2 scalars), apply its update (owned entries of p,
    // q_new, c, r_new written), then out = W^T J^-1 r_new
    int idwt_update(const T *r_old, const T *q_old, T *q_new, T *r_new, T *c, int kprev, double *resnorm,
                    T *out) const;
    template <int EPI>
    int fwd(const T *x, const FwdArgs &E) const;
    template <int EPI>
    size_t coarse_lds() const;
    int fdwt(const T *x, T *out) const;                      // out = W x
    int fdwt_prior(const T *x, const T *cin, T *out) const;  // out = W x + alpha D cin
    int fdwt_pcg(const T *x, const T *rk) const;             // y = W x + alpha D J^-1 r_k; (r, z), (y, z) partials
    int fdwt_rhs(const T *x, T *c, bool cold) const;         // b = W x; r = (b - b_prev) + r; b_prev = b
    // consume pass kprev's reduction and apply the final update of a solve (residual -> state)
    int update_last(T *c, const T *r_in, const T *q_old, T *q_new, int kprev, double *resnorm) const;
    int nodes(const T *in, T *v, int mode) const;            // Gamma^T C Gamma P u | Gamma^T C s | Gamma^T mask s
    int slopes(const T *u, T *s) const;                      // s = mask Gamma P u
    int pt(const T *v, T *x) const;                          // x = P^T v
    int wnorm(const T *s) const;                             // sc->rho = sum C^-1 s^2
    int fit(const T *u, const T *a_prev, T *a, double gain) const;
    int build_tables(int *over) const;                       // projection cell and transpose tables
    int fill(T *x, long n, T val) const;
    int copy(T *dst, const T *src, long n) const;
    int init_scalars() const;
};

}  // namespace fewha
