/*
 * fewha_oracle.c -- plain, slow FP64 CPU oracle of the FEWHA tomography hot path
 * (Stadler, Biasi, Manetti, Ramlau, "Real-time implementation of an iterative solver for
 * atmospheric tomography", arXiv 2009.00946).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its Python binding)
 * may link, load or call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with the GPU library.
 *
 * Everything is double precision, written as straightforward loops in the order the paper
 * states the method.  The outer loops over layers and over guide stars may run on OpenMP
 * threads (the paper's own CPU scheme parallelises the same loops, Sec. 3.3): each iteration
 * writes its own layer or sensor block, and every sum keeps its order, so results are bitwise
 * those of one thread (orc_set_threads; the default is OpenMP's):
 *   Sec. 2.1      Shack-Hartmann operator Gamma (Fried geometry) and the NGS / LGS
 *                 geometric propagation P (bilinear interpolation, cone effect);
 *   Eq. (fewha)   M = W Ahat^T C^-1 Ahat W^T + alpha D,  b = W Ahat^T C^-1 s, with an
 *                 orthonormal periodic Daubechies-3 wavelet transform W (W^-1 = W^T);
 *   Alg. 1        frame: right-hand side, warm-restart residual update, PCG, fitting, gain;
 *   Alg. 2        the PCG variant with one fused reduction point per iteration.
 * Readings of points the paper leaves open (node coordinates, the s^y typo, the prior D, the
 * preconditioner, fitting when there are more layers than DMs, loop bounds) are stated at
 * each function.
 *
 * Layouts (shared with the library only as data formats):
 *   coefficient / layer vectors: layers concatenated, each n x n row-major (row = y, col = x),
 *     wavelet coefficients in the Mallat in-place pyramid (top-left LL, top-right x-high,
 *     bottom-left y-high, bottom-right HH, recursing into LL);
 *   slope vectors: per guide star the s^x plane then the s^y plane, each n_s x n_s row-major;
 *   node vectors: per guide star (n_s+1) x (n_s+1) row-major;
 *   actuator vectors: DMs concatenated, each n_a x n_a row-major.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_GEOMETRY (-2)
#define ORC_ERR_BREAKDOWN (-6)

typedef struct { int n_sub; double theta_x, theta_y, gs_height, sigma; } orc_wfs;
typedef struct { double height, cn2_weight, spacing; int n; } orc_layer;
typedef struct { double height, pitch; int n_act; } orc_dm;

typedef struct {
    double D, obstruction, alpha_reg;
    int J, nw, nl, nd;
    orc_wfs *wfs;
    orc_layer *lay;
    orc_dm *dm;
    long *c_off, *s_off, *v_off, *a_off;
    long n_coef, n_slopes, n_nodes, n_act;
    int *dm_of_layer;
    double *prior; /* D per coefficient, without alpha_reg */
    double *jdiag; /* preconditioner diagonal per coefficient (after orc_build_precond) */
} orc_plan;

/* ------------------------------------------------------------------------------------ */
/* Daubechies-3 filter (orthonormal, compactly supported; Eq. (fewha) asks for such a W).  */
/* Closed form of the extremal-phase 6-tap filter with three vanishing moments.            */
/* ------------------------------------------------------------------------------------ */
void orc_db3(double *h)
{
    double q = sqrt(10.0), p = sqrt(5.0 + 2.0 * sqrt(10.0)), s = 16.0 * sqrt(2.0);
    h[0] = (1.0 + q + p) / s;
    h[1] = (5.0 + q + 3.0 * p) / s;
    h[2] = (10.0 - 2.0 * q + 2.0 * p) / s;
    h[3] = (10.0 - 2.0 * q - 2.0 * p) / s;
    h[4] = (5.0 + q - 3.0 * p) / s;
    h[5] = (1.0 + q - p) / s;
}

/* High-pass partner g_n = (-1)^n h_{5-n}. */
static void db3_pair(double *h, double *g)
{
    orc_db3(h);
    for (int n = 0; n < 6; n++) g[n] = ((n & 1) ? -1.0 : 1.0) * h[5 - n];
}

static int imod(long a, long m) { long r = a % m; return (int)(r < 0 ? r + m : r); }

/* One level of the periodic 1D analysis on an even length N >= 2:
 *   a[k] = sum_n h_n x[(2k+n) mod N],  d[k] = sum_n g_n x[(2k+n) mod N],  out = [a | d]. */
void orc_dwt1_fwd(const double *x, double *out, int N)
{
    double h[6], g[6];
    db3_pair(h, g);
    for (int k = 0; k < N / 2; k++) {
        double a = 0.0, d = 0.0;
        for (int n = 0; n < 6; n++) {
            a += h[n] * x[imod(2L * k + n, N)];
            d += g[n] * x[imod(2L * k + n, N)];
        }
        out[k] = a;
        out[N / 2 + k] = d;
    }
}

/* Exact transpose of orc_dwt1_fwd: every (k, n) pair adds its tap to x[(2k+n) mod N];
 * when N < 6 several taps land on one sample and are all summed. */
void orc_dwt1_inv(const double *in, double *x, int N)
{
    double h[6], g[6];
    db3_pair(h, g);
    for (int m = 0; m < N; m++) x[m] = 0.0;
    for (int k = 0; k < N / 2; k++)
        for (int n = 0; n < 6; n++)
            x[imod(2L * k + n, N)] += h[n] * in[k] + g[n] * in[N / 2 + k];
}

/* Multi-level 2D transform of one n x n layer: at each level the m x m top-left block is
 * analysed along x for every row, then along y for every column (m = n, n/2, ..., n/2^(J-1)). */
void orc_dwt2_fwd(const double *x, double *c, int n, int J)
{
    double *in = malloc(sizeof(double) * n), *out = malloc(sizeof(double) * n);
    memcpy(c, x, sizeof(double) * (size_t)n * n);
    for (int lev = 0; lev < J; lev++) {
        int m = n >> lev;
        for (int r = 0; r < m; r++) {
            for (int i = 0; i < m; i++) in[i] = c[(long)r * n + i];
            orc_dwt1_fwd(in, out, m);
            for (int i = 0; i < m; i++) c[(long)r * n + i] = out[i];
        }
        for (int col = 0; col < m; col++) {
            for (int i = 0; i < m; i++) in[i] = c[(long)i * n + col];
            orc_dwt1_fwd(in, out, m);
            for (int i = 0; i < m; i++) c[(long)i * n + col] = out[i];
        }
    }
    free(in);
    free(out);
}

/* W^T = W^-1: undo the levels from the coarsest, columns (y) first, then rows (x). */
void orc_dwt2_inv(const double *c, double *x, int n, int J)
{
    double *in = malloc(sizeof(double) * n), *out = malloc(sizeof(double) * n);
    memcpy(x, c, sizeof(double) * (size_t)n * n);
    for (int lev = J - 1; lev >= 0; lev--) {
        int m = n >> lev;
        for (int col = 0; col < m; col++) {
            for (int i = 0; i < m; i++) in[i] = x[(long)i * n + col];
            orc_dwt1_inv(in, out, m);
            for (int i = 0; i < m; i++) x[(long)i * n + col] = out[i];
        }
        for (int r = 0; r < m; r++) {
            for (int i = 0; i < m; i++) in[i] = x[(long)r * n + i];
            orc_dwt1_inv(in, out, m);
            for (int i = 0; i < m; i++) x[(long)r * n + i] = out[i];
        }
    }
    free(in);
    free(out);
}

/* W on every layer: FE nodal values -> wavelet coefficients. */
void orc_W(const orc_plan *P, const double *layers, double *c)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < P->nl; l++)
        orc_dwt2_fwd(layers + P->c_off[l], c + P->c_off[l], P->lay[l].n, P->J);
}

/* W^T on every layer: wavelet coefficients -> FE nodal values. */
void orc_Wt(const orc_plan *P, const double *c, double *layers)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < P->nl; l++)
        orc_dwt2_inv(c + P->c_off[l], layers + P->c_off[l], P->lay[l].n, P->J);
}

/* Level s (1 = finest detail, J = coarsest; LL also gets s = J) and orientation
 * o (0 LL, 1 x-high/y-low, 2 x-low/y-high, 3 HH) of Mallat position (row, col). */
void orc_level_of(int n, int J, int row, int col, int *s, int *o)
{
    int mJ = n >> J;
    if (row < mJ && col < mJ) { *s = J; *o = 0; return; }
    int lev = 1, m = n >> 1;
    while (row < m && col < m) { lev++; m >>= 1; }
    *s = lev;
    *o = (row < m) ? 1 : ((col < m) ? 2 : 3);
}

/* ------------------------------------------------------------------------------------ */
/* Geometry (Sec. 2.1).                                                                   */
/* ------------------------------------------------------------------------------------ */
static double subap(const orc_plan *P, int g) { return P->D / P->wfs[g].n_sub; }

/* Subaperture (i, j) is active iff its centre lies in the annulus [eps D/2, D/2]. */
int orc_active(const orc_plan *P, int g, int i, int j)
{
    double d = subap(P, g);
    double xc = (j + 0.5) * d - P->D / 2, yc = (i + 0.5) * d - P->D / 2;
    double r = sqrt(xc * xc + yc * yc);
    return r <= P->D / 2 && r >= P->obstruction * P->D / 2;
}

/* Cone factor: 1 - h/H for a laser guide star at height H, 1 for a natural one. */
static double cone(const orc_plan *P, int g, int l)
{
    return P->wfs[g].gs_height > 0 ? 1.0 - P->lay[l].height / P->wfs[g].gs_height : 1.0;
}

/* Continuous grid coordinate of a point (metres) on layer l: node index k sits at (k - n/2) delta. */
static double grid_coord(const orc_plan *P, int l, double X) { return X / P->lay[l].spacing + P->lay[l].n / 2; }

/* Bilinear cell and weights of a continuous coordinate u in [0, n-1]; the cell index is
 * clamped to n-2 so that u = n-1 uses the last cell with weight t = 1. */
static void cell(double u, int n, int *k0, double *t)
{
    int k = (int)floor(u);
    if (k > n - 2) k = n - 2;
    *k0 = k;
    *t = u - k;
}

/* Where WFS node (i, j) of guide star g meets layer l (P^NGS / P^LGS of Sec. 2.1):
 * X = sigma x_j + theta_x h_l, Y = sigma y_i + theta_y h_l, node x_j = -D/2 + j d. */
static void project(const orc_plan *P, int g, int l, int i, int j, double *u, double *v)
{
    double d = subap(P, g), s = cone(P, g, l), h = P->lay[l].height;
    double X = s * (-P->D / 2 + j * d) + P->wfs[g].theta_x * h;
    double Y = s * (-P->D / 2 + i * d) + P->wfs[g].theta_y * h;
    *u = grid_coord(P, l, X);
    *v = grid_coord(P, l, Y);
}

/* phi_g = sum_l P_gl U_l on every WFS node grid (bilinear interpolation). */
void orc_P(const orc_plan *P, const double *layers, double *phi)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < P->nw; g++) {
        int nv = P->wfs[g].n_sub + 1;
        for (int i = 0; i < nv; i++)
            for (int j = 0; j < nv; j++) {
                double acc = 0.0;
                for (int l = 0; l < P->nl; l++) {
                    int n = P->lay[l].n, k0, l0;
                    double u, v, t, tau;
                    project(P, g, l, i, j, &u, &v);
                    cell(u, n, &l0, &t);
                    cell(v, n, &k0, &tau);
                    const double *U = layers + P->c_off[l];
                    acc += (1 - tau) * (1 - t) * U[(long)k0 * n + l0] + (1 - tau) * t * U[(long)k0 * n + l0 + 1] +
                           tau * (1 - t) * U[(long)(k0 + 1) * n + l0] + tau * t * U[(long)(k0 + 1) * n + l0 + 1];
                }
                phi[P->v_off[g] + (long)i * nv + j] = acc;
            }
    }
}

/* P^T: each node value is spread back onto the four layer nodes with the same weights.  Layer
 * by layer (each layer receives its sums in guide-star, row, column order). */
void orc_Pt(const orc_plan *P, const double *phi, double *layers)
{
    memset(layers, 0, sizeof(double) * P->n_coef);
#pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < P->nl; l++) {
        int n = P->lay[l].n;
        double *U = layers + P->c_off[l];
        for (int g = 0; g < P->nw; g++) {
            int nv = P->wfs[g].n_sub + 1;
            for (int i = 0; i < nv; i++)
                for (int j = 0; j < nv; j++) {
                    double f = phi[P->v_off[g] + (long)i * nv + j], u, v, t, tau;
                    int k0, l0;
                    project(P, g, l, i, j, &u, &v);
                    cell(u, n, &l0, &t);
                    cell(v, n, &k0, &tau);
                    U[(long)k0 * n + l0] += (1 - tau) * (1 - t) * f;
                    U[(long)k0 * n + l0 + 1] += (1 - tau) * t * f;
                    U[(long)(k0 + 1) * n + l0] += tau * (1 - t) * f;
                    U[(long)(k0 + 1) * n + l0 + 1] += tau * t * f;
                }
        }
    }
}

/* Shack-Hartmann operator of Sec. 2.1 for guide star g (no mask), phi row = y, col = x:
 *   s^x_ij = ((phi_i,j+1 - phi_i,j) + (phi_i+1,j+1 - phi_i+1,j)) / 2
 *   s^y_ij = ((phi_i+1,j - phi_i,j) + (phi_i+1,j+1 - phi_i,j+1)) / 2
 * (the second s^y difference is read as a y-difference; the printed diagonal form would
 * not annihilate the Fried waffle mode). */
void orc_gamma(const orc_plan *P, int g, const double *phi, double *s)
{
    int ns = P->wfs[g].n_sub, nv = ns + 1;
    for (int i = 0; i < ns; i++)
        for (int j = 0; j < ns; j++) {
            double p00 = phi[(long)i * nv + j], p01 = phi[(long)i * nv + j + 1];
            double p10 = phi[(long)(i + 1) * nv + j], p11 = phi[(long)(i + 1) * nv + j + 1];
            s[(long)i * ns + j] = 0.5 * ((p01 - p00) + (p11 - p10));
            s[(long)ns * ns + (long)i * ns + j] = 0.5 * ((p10 - p00) + (p11 - p01));
        }
}

/* Gamma^T for guide star g: each slope is spread back onto its four corner nodes. */
void orc_gamma_t(const orc_plan *P, int g, const double *s, double *phi)
{
    int ns = P->wfs[g].n_sub, nv = ns + 1;
    memset(phi, 0, sizeof(double) * (size_t)nv * nv);
    for (int i = 0; i < ns; i++)
        for (int j = 0; j < ns; j++) {
            double sx = s[(long)i * ns + j], sy = s[(long)ns * ns + (long)i * ns + j];
            phi[(long)i * nv + j] += 0.5 * (-sx - sy);
            phi[(long)i * nv + j + 1] += 0.5 * (sx - sy);
            phi[(long)(i + 1) * nv + j] += 0.5 * (-sx + sy);
            phi[(long)(i + 1) * nv + j + 1] += 0.5 * (sx + sy);
        }
}

/* Pupil mask per slope (1 active, 0 inactive). */
void orc_slope_mask(const orc_plan *P, double *m)
{
    for (int g = 0; g < P->nw; g++) {
        int ns = P->wfs[g].n_sub;
        for (int i = 0; i < ns; i++)
            for (int j = 0; j < ns; j++) {
                double a = orc_active(P, g, i, j) ? 1.0 : 0.0;
                m[P->s_off[g] + (long)i * ns + j] = a;
                m[P->s_off[g] + (long)ns * ns + (long)i * ns + j] = a;
            }
    }
}

/* C_eta^-1 read as a diagonal: sigma_g^-2 on active slopes, 0 on inactive ones. */
void orc_slope_weights(const orc_plan *P, double *w)
{
    orc_slope_mask(P, w);
    for (int g = 0; g < P->nw; g++) {
        double iv = 1.0 / (P->wfs[g].sigma * P->wfs[g].sigma);
        long n2 = 2L * P->wfs[g].n_sub * P->wfs[g].n_sub;
        for (long k = 0; k < n2; k++) w[P->s_off[g] + k] *= iv;
    }
}

/* Ahat: FE layers -> masked slopes, s_g = mask Gamma_g P_g phi (Eq. (atmo)). */
void orc_apply_Ahat(const orc_plan *P, const double *layers, double *s)
{
    double *phi = malloc(sizeof(double) * P->n_nodes), *m = malloc(sizeof(double) * P->n_slopes);
    orc_P(P, layers, phi);
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < P->nw; g++) orc_gamma(P, g, phi + P->v_off[g], s + P->s_off[g]);
    orc_slope_mask(P, m);
    for (long k = 0; k < P->n_slopes; k++) s[k] *= m[k];
    free(phi);
    free(m);
}

/* Ahat^T: slopes -> FE layers (mask, Gamma^T, P^T). */
void orc_apply_Ahat_t(const orc_plan *P, const double *s, double *layers)
{
    double *phi = malloc(sizeof(double) * P->n_nodes), *m = malloc(sizeof(double) * P->n_slopes);
    double *sm = malloc(sizeof(double) * P->n_slopes);
    orc_slope_mask(P, m);
    for (long k = 0; k < P->n_slopes; k++) sm[k] = s[k] * m[k];
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < P->nw; g++) orc_gamma_t(P, g, sm + P->s_off[g], phi + P->v_off[g]);
    orc_Pt(P, phi, layers);
    free(phi);
    free(m);
    free(sm);
}

/* A = mask Gamma P W^T: wavelet coefficients -> slopes. */
void orc_apply_A(const orc_plan *P, const double *c, double *s)
{
    double *lay = malloc(sizeof(double) * P->n_coef);
    orc_Wt(P, c, lay);
    orc_apply_Ahat(P, lay, s);
    free(lay);
}

/* A^T = W P^T Gamma^T mask: slopes -> wavelet coefficients. */
void orc_apply_At(const orc_plan *P, const double *s, double *c)
{
    double *lay = malloc(sizeof(double) * P->n_coef);
    orc_apply_Ahat_t(P, s, lay);
    orc_W(P, lay, c);
    free(lay);
}

/* Right-hand side of Eq. (fewha): b = W Ahat^T C_eta^-1 s. */
void orc_rhs(const orc_plan *P, const double *s, double *b)
{
    double *w = malloc(sizeof(double) * P->n_slopes), *ws = malloc(sizeof(double) * P->n_slopes);
    orc_slope_weights(P, w);
    for (long k = 0; k < P->n_slopes; k++) ws[k] = w[k] * s[k];
    orc_apply_At(P, ws, b);
    free(w);
    free(ws);
}

/* Left-hand side of Eq. (fewha): y = W Ahat^T C_eta^-1 Ahat W^T c + alpha D c. */
void orc_apply_M(const orc_plan *P, const double *c, double *y)
{
    double *s = malloc(sizeof(double) * P->n_slopes), *w = malloc(sizeof(double) * P->n_slopes);
    orc_apply_A(P, c, s);
    orc_slope_weights(P, w);
    for (long k = 0; k < P->n_slopes; k++) s[k] *= w[k];
    orc_apply_At(P, s, y);
    for (long k = 0; k < P->n_coef; k++) y[k] += P->alpha_reg * P->prior[k] * c[k];
    free(s);
    free(w);
}

/* Prior D (diagonal approximation of C_phi^-1 in the wavelet domain, Eq. (fewha)), read as the
 * Kolmogorov scale law: D = gamma_l^-1 (delta_l / d_1)^(-5/3) 2^(-(11/3)(s-1)), with d_1 the
 * subaperture size of the first guide star and s the level of the coefficient. */
static void build_prior(orc_plan *P)
{
    double d1 = subap(P, 0);
    for (int l = 0; l < P->nl; l++) {
        int n = P->lay[l].n;
        double base = pow(P->lay[l].spacing / d1, -5.0 / 3.0) / P->lay[l].cn2_weight;
        for (int r = 0; r < n; r++)
            for (int q = 0; q < n; q++) {
                int s, o;
                orc_level_of(n, P->J, r, q, &s, &o);
                P->prior[P->c_off[l] + (long)r * n + q] = base * pow(2.0, -(11.0 / 3.0) * (s - 1));
            }
    }
}

void orc_prior(const orc_plan *P, double *d) { memcpy(d, P->prior, sizeof(double) * P->n_coef); }

/* Origin of band (s, o) inside an n x n Mallat block. */
static void band_origin(int n, int s, int o, int *r0, int *c0)
{
    int m = n >> s;
    *r0 = (o == 2 || o == 3) ? m : 0;
    *c0 = (o == 1 || o == 3) ? m : 0;
}

/* Modified Jacobi preconditioner (Sec. 3.4: diagonal, different weights for low and high
 * frequencies), read as J = alpha D + tau_{l,s,o}, where tau is the exact data-term diagonal
 * ||C_eta^(1/2) A W^T e_k||^2 at one representative coefficient k per (layer, level,
 * orientation): block-local position (m_s/2, m_s/2).  Every coefficient of that band gets it. */
int orc_build_precond(orc_plan *P)
{
    double *w = malloc(sizeof(double) * P->n_slopes);
    orc_slope_weights(P, w);
#pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < P->nl; l++) {
        double *e = calloc(P->n_coef, sizeof(double)), *s = malloc(sizeof(double) * P->n_slopes);
        int n = P->lay[l].n;
        for (int sl = 1; sl <= P->J; sl++)
            for (int o = 0; o < 4; o++) {
                if (o == 0 && sl != P->J) continue;
                int m = n >> sl, r0, c0;
                band_origin(n, sl, o, &r0, &c0);
                long k = P->c_off[l] + (long)(r0 + m / 2) * n + (c0 + m / 2);
                e[k] = 1.0;
                orc_apply_A(P, e, s);
                e[k] = 0.0;
                double tau = 0.0;
                for (long q = 0; q < P->n_slopes; q++) tau += w[q] * s[q] * s[q];
                for (int r = 0; r < n; r++)
                    for (int q = 0; q < n; q++) {
                        int ss, oo;
                        orc_level_of(n, P->J, r, q, &ss, &oo);
                        if (ss == sl && oo == o) {
                            long kk = P->c_off[l] + (long)r * n + q;
                            P->jdiag[kk] = P->alpha_reg * P->prior[kk] + tau;
                        }
                    }
            }
        free(e);
        free(s);
    }
    free(w);
    return ORC_OK;
}

/* Threads of the outer layer / guide-star loops (results do not depend on it). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

void orc_precond(const orc_plan *P, double *j) { memcpy(j, P->jdiag, sizeof(double) * P->n_coef); }

static double dot(const double *a, const double *b, long n)
{
    double s = 0.0;
    for (long k = 0; k < n; k++) s += a[k] * b[k];
    return s;
}

/* Alg. 2 (PCG for M c = b with the residual given), read as exactly n_iter passes:
 *   z = J^-1 r;  y = M z;  rho = (r, z);  mu = (y, z);
 *   first pass: beta = 0, alpha = rho / mu,          p = z,        q = y;
 *   later:      beta = rho / rho_old, alpha = rho / (mu - rho beta / alpha_old),
 *               p = z + beta p,  q = y + beta q;
 *   c += alpha p;  r -= alpha q.
 * rho = 0 ends the loop early (exact solution); a non-positive denominator is a breakdown.
 * resnorm (optional) receives sqrt(rho) of every pass that ran; *done the number of passes. */
int orc_pcg(const orc_plan *P, double *c, double *r, int n_iter, double *resnorm, int *done)
{
    long N = P->n_coef;
    double *z = malloc(sizeof(double) * N), *y = malloc(sizeof(double) * N);
    double *p = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
    double rho_old = 0.0, alpha_old = 0.0;
    int status = ORC_OK, k;
    for (k = 0; k < n_iter; k++) {
        for (long i = 0; i < N; i++) z[i] = r[i] / P->jdiag[i];
        double rho = dot(r, z, N);
        if (resnorm) resnorm[k] = sqrt(rho);
        if (rho == 0.0) break;
        orc_apply_M(P, z, y);
        double mu = dot(y, z, N);
        double beta = 0.0, den = mu;
        if (k > 0) {
            beta = rho / rho_old;
            den = mu - rho * beta / alpha_old;
        }
        if (!(den > 0.0)) { status = ORC_ERR_BREAKDOWN; break; }
        double alpha = rho / den;
        for (long i = 0; i < N; i++) {
            p[i] = (k == 0) ? z[i] : z[i] + beta * p[i];
            q[i] = (k == 0) ? y[i] : y[i] + beta * q[i];
            c[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        rho_old = rho;
        alpha_old = alpha;
    }
    if (done) *done = k;
    free(z);
    free(y);
    free(p);
    free(q);
    return status;
}

/* Alg. 1 without the closed-loop and fitting lines: b = W Ahat^T C^-1 s;
 * r = (b - b_prev) + r_prev (= b - M c); PCG; then b_prev = b, r_prev = r.
 * A cold start uses c = b_prev = r_prev = 0, so r = b. */
int orc_frame(const orc_plan *P, const double *s, double *c, double *b_prev, double *r_prev, int n_iter,
              int cold, double *resnorm)
{
    long N = P->n_coef;
    double *b = malloc(sizeof(double) * N);
    orc_rhs(P, s, b);
    if (cold) {
        memset(c, 0, sizeof(double) * N);
        memset(b_prev, 0, sizeof(double) * N);
        memset(r_prev, 0, sizeof(double) * N);
    }
    for (long i = 0; i < N; i++) r_prev[i] = (b[i] - b_prev[i]) + r_prev[i];
    int st = orc_pcg(P, c, r_prev, n_iter, resnorm, NULL);
    memcpy(b_prev, b, sizeof(double) * N);
    free(b);
    return st;
}

/* Actuator (i, j) of DM m sits at ((j - (n_a-1)/2) pitch, (i - (n_a-1)/2) pitch). */
static void actuator_on_layer(const orc_plan *P, int m, int l, int i, int j, double *u, double *v)
{
    double c = (P->dm[m].n_act - 1) / 2.0;
    *u = grid_coord(P, l, (j - c) * P->dm[m].pitch);
    *v = grid_coord(P, l, (i - c) * P->dm[m].pitch);
}

/* Fitting interpolation F (Alg. 1): every layer goes to the DM nearest in altitude (ties to
 * the lower DM) and is sampled on-axis at that DM's actuators by bilinear interpolation;
 * the layers sharing a DM are summed.  With one layer per DM on a co-located grid this is the
 * identity (Sec. 4.1). */
void orc_fit_interp(const orc_plan *P, const double *layers, double *a)
{
    memset(a, 0, sizeof(double) * P->n_act);
    for (int l = 0; l < P->nl; l++) {
        int m = P->dm_of_layer[l], na = P->dm[m].n_act, n = P->lay[l].n;
        const double *U = layers + P->c_off[l];
        for (int i = 0; i < na; i++)
            for (int j = 0; j < na; j++) {
                double u, v, t, tau;
                int k0, l0;
                actuator_on_layer(P, m, l, i, j, &u, &v);
                cell(u, n, &l0, &t);
                cell(v, n, &k0, &tau);
                a[P->a_off[m] + (long)i * na + j] +=
                    (1 - tau) * (1 - t) * U[(long)k0 * n + l0] + (1 - tau) * t * U[(long)k0 * n + l0 + 1] +
                    tau * (1 - t) * U[(long)(k0 + 1) * n + l0] + tau * t * U[(long)(k0 + 1) * n + l0 + 1];
            }
    }
}

/* Transpose of orc_fit_interp (for adjoint checks). */
void orc_fit_interp_t(const orc_plan *P, const double *a, double *layers)
{
    memset(layers, 0, sizeof(double) * P->n_coef);
    for (int l = 0; l < P->nl; l++) {
        int m = P->dm_of_layer[l], na = P->dm[m].n_act, n = P->lay[l].n;
        double *U = layers + P->c_off[l];
        for (int i = 0; i < na; i++)
            for (int j = 0; j < na; j++) {
                double u, v, t, tau, f = a[P->a_off[m] + (long)i * na + j];
                int k0, l0;
                actuator_on_layer(P, m, l, i, j, &u, &v);
                cell(u, n, &l0, &t);
                cell(v, n, &k0, &tau);
                U[(long)k0 * n + l0] += (1 - tau) * (1 - t) * f;
                U[(long)k0 * n + l0 + 1] += (1 - tau) * t * f;
                U[(long)(k0 + 1) * n + l0] += tau * (1 - t) * f;
                U[(long)(k0 + 1) * n + l0 + 1] += tau * t * f;
            }
    }
}

/* Alg. 1 fitting and open-loop gain: a = (1 - gain) a_prev + gain F W^T c (a_prev may be NULL = 0). */
void orc_fit(const orc_plan *P, const double *c, const double *a_prev, double gain, double *a)
{
    double *lay = malloc(sizeof(double) * P->n_coef), *at = malloc(sizeof(double) * P->n_act);
    orc_Wt(P, c, lay);
    orc_fit_interp(P, lay, at);
    for (long k = 0; k < P->n_act; k++) a[k] = (1.0 - gain) * (a_prev ? a_prev[k] : 0.0) + gain * at[k];
    free(lay);
    free(at);
}

/* ------------------------------------------------------------------------------------ */
/* Closed loop (Alg. 1): pseudo-open-loop slopes and the closed-loop control law.          */
/* ------------------------------------------------------------------------------------ */
/* DM m as the piecewise bilinear surface over its actuator grid (Sec. 4.1):
 *   S_m(X, Y) = sum_ij a_m,ij hat((X - x_j) / p) hat((Y - y_i) / p),  hat(t) = max(0, 1 - |t|),
 * actuator (i, j) at ((j - (n_a-1)/2) p, (i - (n_a-1)/2) p); zero beyond the outermost hats.
 * Evaluated here by visiting every actuator whose hat support contains the point. */
static double dm_surface(const orc_plan *P, int m, const double *a, double X, double Y)
{
    int na = P->dm[m].n_act;
    double p = P->dm[m].pitch, c = (na - 1) / 2.0, acc = 0.0;
    for (int i = 0; i < na; i++) {
        double wy = 1.0 - fabs(Y / p - (i - c));
        if (wy <= 0.0) continue;
        for (int j = 0; j < na; j++) {
            double wx = 1.0 - fabs(X / p - (j - c));
            if (wx <= 0.0) continue;
            acc += wx * wy * a[P->a_off[m] + (long)i * na + j];
        }
    }
    return acc;
}

/* Where WFS node (i, j) of guide star g meets the altitude h (metres), as for a layer. */
static void node_at_height(const orc_plan *P, int g, double h, int i, int j, double *X, double *Y)
{
    double d = subap(P, g), s = P->wfs[g].gs_height > 0 ? 1.0 - h / P->wfs[g].gs_height : 1.0;
    *X = s * (-P->D / 2 + j * d) + P->wfs[g].theta_x * h;
    *Y = s * (-P->D / 2 + i * d) + P->wfs[g].theta_y * h;
}

/* The DMs' correction as the sensors see it: s = mask Gamma_g sum_m P^DM_gm a_m (every ray passes
 * through every DM).  Reading: Alg. 1 prints the pseudo-open-loop update as s + Gamma a^(-1),
 * which leaves out the projection of the DM surfaces onto the sensor grids; it is read as this
 * operator applied to a^(-1). */
void orc_apply_Hdm(const orc_plan *P, const double *a, double *s)
{
    for (int g = 0; g < P->nw; g++) {
        int ns = P->wfs[g].n_sub, nv = ns + 1;
        double *phi = malloc(sizeof(double) * (size_t)nv * nv);
        for (int i = 0; i < nv; i++)
            for (int j = 0; j < nv; j++) {
                double acc = 0.0;
                for (int m = 0; m < P->nd; m++) {
                    double X, Y;
                    node_at_height(P, g, P->dm[m].height, i, j, &X, &Y);
                    acc += dm_surface(P, m, a, X, Y);
                }
                phi[(long)i * nv + j] = acc;
            }
        double *sg = s + P->s_off[g];
        orc_gamma(P, g, phi, sg);
        for (int i = 0; i < ns; i++)
            for (int j = 0; j < ns; j++)
                if (!orc_active(P, g, i, j)) sg[(long)i * ns + j] = sg[(long)ns * ns + (long)i * ns + j] = 0.0;
        free(phi);
    }
}

/* Transpose of orc_apply_Hdm (for adjoint checks). */
void orc_apply_Hdm_t(const orc_plan *P, const double *s, double *a)
{
    memset(a, 0, sizeof(double) * P->n_act);
    for (int g = 0; g < P->nw; g++) {
        int ns = P->wfs[g].n_sub, nv = ns + 1;
        double *sm = malloc(sizeof(double) * 2 * (size_t)ns * ns), *phi = malloc(sizeof(double) * (size_t)nv * nv);
        for (int i = 0; i < ns; i++)
            for (int j = 0; j < ns; j++) {
                int act = orc_active(P, g, i, j);
                sm[(long)i * ns + j] = act ? s[P->s_off[g] + (long)i * ns + j] : 0.0;
                sm[(long)ns * ns + (long)i * ns + j] = act ? s[P->s_off[g] + (long)ns * ns + (long)i * ns + j] : 0.0;
            }
        orc_gamma_t(P, g, sm, phi);
        for (int i = 0; i < nv; i++)
            for (int j = 0; j < nv; j++)
                for (int m = 0; m < P->nd; m++) {
                    int na = P->dm[m].n_act;
                    double X, Y, p = P->dm[m].pitch, c = (na - 1) / 2.0;
                    node_at_height(P, g, P->dm[m].height, i, j, &X, &Y);
                    for (int ai = 0; ai < na; ai++) {
                        double wy = 1.0 - fabs(Y / p - (ai - c));
                        if (wy <= 0.0) continue;
                        for (int aj = 0; aj < na; aj++) {
                            double wx = 1.0 - fabs(X / p - (aj - c));
                            if (wx > 0.0) a[P->a_off[m] + (long)ai * na + aj] += wx * wy * phi[(long)i * nv + j];
                        }
                    }
                }
        free(sm);
        free(phi);
    }
}

/* Pseudo-open-loop slopes of Alg. 1: s_pol = mask (s + H_dm a^(-1)). */
void orc_pol(const orc_plan *P, const double *s, const double *a_m1, double *s_pol)
{
    orc_apply_Hdm(P, a_m1, s_pol);
    double *m = malloc(sizeof(double) * P->n_slopes);
    orc_slope_mask(P, m);
    for (long k = 0; k < P->n_slopes; k++) s_pol[k] = m[k] * (s[k] + s_pol[k]);
    free(m);
}

/* Closed-loop control of Alg. 1: a^(1) = a^(0) + gain (F W^T c - a^(-1)). */
void orc_fit_closed(const orc_plan *P, const double *c, const double *a0, const double *a_m1, double gain, double *a)
{
    double *lay = malloc(sizeof(double) * P->n_coef), *at = malloc(sizeof(double) * P->n_act);
    orc_Wt(P, c, lay);
    orc_fit_interp(P, lay, at);
    for (long k = 0; k < P->n_act; k++) a[k] = a0[k] + gain * (at[k] - a_m1[k]);
    free(lay);
    free(at);
}

/* ------------------------------------------------------------------------------------ */
/* Least-squares DM fitting for more layers than DMs (Sec. 4.1 makes the fit a            */
/* minimisation of its own there, left unstated).  Reading: over the 25 probe directions of */
/* the quality evaluation grid (theta_x, theta_y in {-60, -30, 0, 30, 60} arcsec) and the   */
/* nodes of the first sensor's grid inside the pupil annulus, natural-star rays, minimise   */
/*   sum_theta sum_x (sum_l U_l(x + theta h_l) - sum_m S_m(x + theta h_m))^2 + eps |a|^2    */
/* with U_l and S_m the piecewise bilinear (hat) surfaces over the layer nodes and the      */
/* actuators (zero beyond their grids), by n_cg steps of plain CG on the normal equations   */
/* from a = 0.                                                                             */
/* ------------------------------------------------------------------------------------ */
#define ORC_NPROBE 25

static void probe_dir(int t, double *tx, double *ty)
{
    const double as = 3.14159265358979323846 / (180.0 * 3600.0);
    *tx = (-60.0 + 30.0 * (t % 5)) * as;
    *ty = (-60.0 + 30.0 * (t / 5)) * as;
}

/* Evaluation node j (per axis) of the fitting grid and whether node (i, j) is in the pupil. */
static double fit_node(const orc_plan *P, int j) { return -P->D / 2 + j * (P->D / P->wfs[0].n_sub); }
static int fit_in_pupil(const orc_plan *P, int i, int j)
{
    double x = fit_node(P, j), y = fit_node(P, i), r = sqrt(x * x + y * y);
    return r <= P->D / 2 && r >= P->obstruction * P->D / 2;
}

/* Hat surface of layer l at (X, Y): its node k at ((k - n/2) delta), zero beyond the grid. */
static double layer_surface(const orc_plan *P, int l, const double *layers, double X, double Y)
{
    int n = P->lay[l].n;
    double dl = P->lay[l].spacing, acc = 0.0;
    for (int i = 0; i < n; i++) {
        double wy = 1.0 - fabs(Y / dl - (i - n / 2));
        if (wy <= 0.0) continue;
        for (int j = 0; j < n; j++) {
            double wx = 1.0 - fabs(X / dl - (j - n / 2));
            if (wx > 0.0) acc += wx * wy * layers[P->c_off[l] + (long)i * n + j];
        }
    }
    return acc;
}

long orc_fit_points(const orc_plan *P) { long nv = P->wfs[0].n_sub + 1; return ORC_NPROBE * nv * nv; }

/* The target: y[t][i][j] = sum_l U_l(x_ij + theta_t h_l) on pupil nodes (0 elsewhere). */
void orc_ls_target(const orc_plan *P, const double *layers, double *y)
{
    int nv = P->wfs[0].n_sub + 1;
    for (int t = 0; t < ORC_NPROBE; t++) {
        double tx, ty;
        probe_dir(t, &tx, &ty);
        for (int i = 0; i < nv; i++)
            for (int j = 0; j < nv; j++) {
                double acc = 0.0;
                if (fit_in_pupil(P, i, j))
                    for (int l = 0; l < P->nl; l++)
                        acc += layer_surface(P, l, layers, fit_node(P, j) + tx * P->lay[l].height,
                                             fit_node(P, i) + ty * P->lay[l].height);
                y[((long)t * nv + i) * nv + j] = acc;
            }
    }
}

/* H a: y[t][i][j] = sum_m S_m(x_ij + theta_t h_m) on pupil nodes (0 elsewhere). */
void orc_ls_H(const orc_plan *P, const double *a, double *y)
{
    int nv = P->wfs[0].n_sub + 1;
    for (int t = 0; t < ORC_NPROBE; t++) {
        double tx, ty;
        probe_dir(t, &tx, &ty);
        for (int i = 0; i < nv; i++)
            for (int j = 0; j < nv; j++) {
                double acc = 0.0;
                if (fit_in_pupil(P, i, j))
                    for (int m = 0; m < P->nd; m++)
                        acc += dm_surface(P, m, a, fit_node(P, j) + tx * P->dm[m].height,
                                          fit_node(P, i) + ty * P->dm[m].height);
                y[((long)t * nv + i) * nv + j] = acc;
            }
    }
}

/* H^T y: every pupil node of every direction spreads its value onto the actuators whose hats
 * cover it. */
void orc_ls_Ht(const orc_plan *P, const double *y, double *a)
{
    int nv = P->wfs[0].n_sub + 1;
    memset(a, 0, sizeof(double) * P->n_act);
    for (int t = 0; t < ORC_NPROBE; t++) {
        double tx, ty;
        probe_dir(t, &tx, &ty);
        for (int i = 0; i < nv; i++)
            for (int j = 0; j < nv; j++) {
                if (!fit_in_pupil(P, i, j)) continue;
                double f = y[((long)t * nv + i) * nv + j];
                for (int m = 0; m < P->nd; m++) {
                    int na = P->dm[m].n_act;
                    double p = P->dm[m].pitch, c = (na - 1) / 2.0;
                    double X = fit_node(P, j) + tx * P->dm[m].height, Y = fit_node(P, i) + ty * P->dm[m].height;
                    for (int ai = 0; ai < na; ai++) {
                        double wy = 1.0 - fabs(Y / p - (ai - c));
                        if (wy <= 0.0) continue;
                        for (int aj = 0; aj < na; aj++) {
                            double wx = 1.0 - fabs(X / p - (aj - c));
                            if (wx > 0.0) a[P->a_off[m] + (long)ai * na + aj] += wx * wy * f;
                        }
                    }
                }
            }
    }
}

/* Least-squares fit of the layers W^T c onto the DMs: n_cg plain CG steps on
 * (H^T H + eps I) a = H^T y0 from a = 0 (y0 the target). */
void orc_fit_ls(const orc_plan *P, const double *c, int n_cg, double eps, double *a)
{
    long na = P->n_act, np = orc_fit_points(P);
    double *lay = malloc(sizeof(double) * P->n_coef), *y = malloc(sizeof(double) * np);
    double *r = malloc(sizeof(double) * na), *p = malloc(sizeof(double) * na), *q = malloc(sizeof(double) * na);
    orc_Wt(P, c, lay);
    orc_ls_target(P, lay, y);
    orc_ls_Ht(P, y, r);
    memset(a, 0, sizeof(double) * na);
    memcpy(p, r, sizeof(double) * na);
    double rr = dot(r, r, na);
    for (int k = 0; k < n_cg && rr > 0.0; k++) {
        orc_ls_H(P, p, y);
        orc_ls_Ht(P, y, q);
        for (long i = 0; i < na; i++) q[i] += eps * p[i];
        double al = rr / dot(p, q, na);
        for (long i = 0; i < na; i++) {
            a[i] += al * p[i];
            r[i] -= al * q[i];
        }
        double rn = dot(r, r, na), be = rn / rr;
        for (long i = 0; i < na; i++) p[i] = r[i] + be * p[i];
        rr = rn;
    }
    free(lay);
    free(y);
    free(r);
    free(p);
    free(q);
}

/* ------------------------------------------------------------------------------------ */
/* Plan: copy the configuration, check the geometry, lay out the vectors.                 */
/* ------------------------------------------------------------------------------------ */
void orc_destroy(orc_plan *P)
{
    if (!P) return;
    free(P->wfs);
    free(P->lay);
    free(P->dm);
    free(P->c_off);
    free(P->s_off);
    free(P->v_off);
    free(P->a_off);
    free(P->dm_of_layer);
    free(P->prior);
    free(P->jdiag);
    free(P);
}

static int in_grid(double u, int n) { return u >= 0.0 && u <= n - 1.0; }

int orc_create(const orc_wfs *wfs, int nw, const orc_layer *lay, int nl, const orc_dm *dm, int nd, double D,
               double obstruction, int J, double alpha_reg, orc_plan **out)
{
    *out = NULL;
    if (nw < 1 || nl < 1 || nd < 1 || J < 1 || !(D > 0) || !(obstruction >= 0 && obstruction < 1) ||
        !(alpha_reg > 0))
        return ORC_ERR_ARG;
    for (int l = 0; l < nl; l++) {
        int n = lay[l].n;
        if (n < 2 || (n & (n - 1)) || (n >> J) < 1 || !(lay[l].spacing > 0) || !(lay[l].cn2_weight > 0) ||
            lay[l].height < 0)
            return ORC_ERR_ARG;
    }
    for (int g = 0; g < nw; g++)
        if (wfs[g].n_sub < 1 || !(wfs[g].sigma > 0) || wfs[g].gs_height < 0) return ORC_ERR_ARG;
    for (int m = 0; m < nd; m++)
        if (dm[m].n_act < 2 || !(dm[m].pitch > 0)) return ORC_ERR_ARG;

    orc_plan *P = calloc(1, sizeof(orc_plan));
    P->D = D;
    P->obstruction = obstruction;
    P->alpha_reg = alpha_reg;
    P->J = J;
    P->nw = nw;
    P->nl = nl;
    P->nd = nd;
    P->wfs = malloc(sizeof(orc_wfs) * nw);
    memcpy(P->wfs, wfs, sizeof(orc_wfs) * nw);
    P->lay = malloc(sizeof(orc_layer) * nl);
    memcpy(P->lay, lay, sizeof(orc_layer) * nl);
    P->dm = malloc(sizeof(orc_dm) * nd);
    memcpy(P->dm, dm, sizeof(orc_dm) * nd);
    P->c_off = malloc(sizeof(long) * nl);
    P->s_off = malloc(sizeof(long) * nw);
    P->v_off = malloc(sizeof(long) * nw);
    P->a_off = malloc(sizeof(long) * nd);
    P->dm_of_layer = malloc(sizeof(int) * nl);
    for (int l = 0; l < nl; l++) {
        P->c_off[l] = P->n_coef;
        P->n_coef += (long)lay[l].n * lay[l].n;
    }
    for (int g = 0; g < nw; g++) {
        P->s_off[g] = P->n_slopes;
        P->n_slopes += 2L * wfs[g].n_sub * wfs[g].n_sub;
        P->v_off[g] = P->n_nodes;
        P->n_nodes += (long)(wfs[g].n_sub + 1) * (wfs[g].n_sub + 1);
    }
    for (int m = 0; m < nd; m++) {
        P->a_off[m] = P->n_act;
        P->n_act += (long)dm[m].n_act * dm[m].n_act;
    }
    /* nearest DM in altitude, ties to the lower one (the earlier one when heights are equal) */
    for (int l = 0; l < nl; l++) {
        int best = 0;
        for (int m = 1; m < nd; m++) {
            double dn = fabs(lay[l].height - dm[m].height), db = fabs(lay[l].height - dm[best].height);
            if (dn < db || (dn == db && dm[m].height < dm[best].height)) best = m;
        }
        P->dm_of_layer[l] = best;
    }
    /* every LGS above every layer; every projected WFS node and every actuator inside its grid */
    int bad = 0;
    for (int g = 0; g < nw && !bad; g++)
        for (int l = 0; l < nl && !bad; l++) {
            if (wfs[g].gs_height > 0 && !(lay[l].height < wfs[g].gs_height)) { bad = 1; break; }
            int nv = wfs[g].n_sub + 1;
            for (int i = 0; i < nv && !bad; i++)
                for (int j = 0; j < nv; j++) {
                    double u, v;
                    project(P, g, l, i, j, &u, &v);
                    if (!in_grid(u, lay[l].n) || !in_grid(v, lay[l].n)) { bad = 1; break; }
                }
        }
    for (int l = 0; l < nl && !bad; l++) {
        int m = P->dm_of_layer[l], na = dm[m].n_act;
        for (int i = 0; i < na && !bad; i++)
            for (int j = 0; j < na; j++) {
                double u, v;
                actuator_on_layer(P, m, l, i, j, &u, &v);
                if (!in_grid(u, lay[l].n) || !in_grid(v, lay[l].n)) { bad = 1; break; }
            }
    }
    if (bad) {
        orc_destroy(P);
        return ORC_ERR_GEOMETRY;
    }
    P->prior = malloc(sizeof(double) * P->n_coef);
    P->jdiag = malloc(sizeof(double) * P->n_coef);
    build_prior(P);
    for (long k = 0; k < P->n_coef; k++) P->jdiag[k] = 1.0;
    *out = P;
    return ORC_OK;
}

void orc_sizes(const orc_plan *P, long *out)
{
    out[0] = P->n_coef;
    out[1] = P->n_slopes;
    out[2] = P->n_nodes;
    out[3] = P->n_act;
}

void orc_dm_of_layer(const orc_plan *P, int *out) { memcpy(out, P->dm_of_layer, sizeof(int) * P->nl); }
