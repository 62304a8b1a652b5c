// Launch interface of the FEWHA kernels (kernels.hip), used by the C ABI layer (api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include "fewha_internal.h"

namespace fewha {

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

// Enqueues the kernels of one plan on one stream; every call returns FEWHA_OK or FEWHA_ERR_HIP.
template <typename T>
struct Ops {
    const Plan &P;
    Bufs<T> B;
    hipStream_t st;

    int idwt(const T *c, T *out, bool scale) const;          // out = W^T (J^-1 c if scale)
    int fdwt(const T *x, T *out) const;                      // out = W x
    int fdwt_prior(const T *x, const T *cin, T *out) const;  // out = W x + alpha D cin
    int fdwt_pcg(const T *x, int k, double *resnorm) const;  // y = W x + alpha D J^-1 r; Alg. 2 scalars
    int fdwt_rhs(const T *x, T *c, bool cold) const;         // b = W x; r = (b - b_prev) + r; b_prev = b
    int nodes(const T *in, T *v, int mode) const;            // Gamma^T C Gamma P u | Gamma^T C s | Gamma^T mask s
    int slopes(const T *u, T *s) const;                      // s = mask Gamma P u
    int pt(const T *v, T *x) const;                          // x = P^T v
    int update(T *c, int k) const;                           // p, q, c, r
    int wnorm(const T *s) const;                             // sc->rho = sum C^-1 s^2
    int fit(const T *u, const T *a_prev, T *a, double gain) const;
    int build_tables() const;                                // projection cell tables and ranges
    int fill(T *x, long n, T val) const;
    int copy(T *dst, const T *src, long n) const;
    int init_scalars() const;
};

}  // namespace fewha
