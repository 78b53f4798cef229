/*
 * oracle.h -- plain, slow FP64 CPU oracle for Gaussian-cubature potential
 * and field of constant-charge-density BEM triangles and rectangles
 * (Glueck & Hilk, arXiv:1606.03743).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this code; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no source, table or helper with the
 * GPU library.
 *
 * Geometry (host arrays, row-major, FP64):
 *   tri  [n_tri ][9] = A(3) B(3) C(3)                 (barycentric form, Eq. 3.3)
 *   rect [n_rect][9] = P0(3) e1(3) e2(3)  corner and two side vectors;
 *                      a = |e1| is the x side, b = |e2| the y side (Eq. 3.2)
 * Global element index: triangles [0, n_tri), then rectangles.
 * Densities sigma [n_rhs][n_E] in C/m^2.  Points [n][3].  Outputs in V, V/m.
 */
#ifndef BEMC_ORACLE_H
#define BEMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 1/(4 pi eps0) with CODATA-2022 eps0 = 8.8541878188e-12 F/m (SI units, Sec. 2 Eq. 2.1). */
double orc_coulomb_constant(void);

/* Triangle rules of App. A (n = 4, 7, 12, 19, 33): barycentric lam[n][3], weights w[n].
 * Returns n, or -1 for an unknown rule. */
int orc_tri_rule(int n, double* lam, double* w);

/* Rectangle rules in natural coordinates (Eq. 3.2), xy[n][2], w[n], sum w = 1.
 * gl_n > 0: tensor Gauss-Legendre gl_n x gl_n (gl_n <= 16); gl_n == 0: table of App. B
 * with table_n = 4, 7, 12, 17 or 33 points.  Returns the node count or -1. */
int orc_rect_rule(int gl_n, int table_n, double* xy, double* w);

/* Gauss-Legendre nodes and weights on [-1, 1] (n <= 64), by Newton iteration on P_n. */
int orc_gauss_legendre(int n, double* x, double* w);

/* Evaluation parameters. */
typedef struct {
    int tri_rule;      /* 4, 7, 12, 19, 33 */
    int rect_gl_n;     /* > 0: tensor Gauss-Legendre n x n */
    int rect_table_n;  /* used when rect_gl_n == 0: 4, 7, 12, 17, 33 */
    double near_dr;    /* distance-ratio threshold (3.0) */
    int max_depth;     /* subdivision depth cap */
    int dr_rules;      /* 1: far pairs take a rule by distance ratio (Sec. 4, rule choice by DR):
                          triangles 7 / 12 / 19 points for DR >= tri_dr[0] / tri_dr[1] /
                          tri_dr[2], else tri_rule; rectangles Tables B2 / B3 / B4 for
                          DR >= rect_dr[0..2], else the rectangle rule above */
    double tri_dr[3];
    double rect_dr[3];
} orc_params;

/* Counters of one call. */
typedef struct {
    int64_t near_pairs;   /* (point, element) pairs with D < near_dr * L */
    int64_t leaves;       /* rule applications made by the near-field subdivision */
    int64_t cap_hits;     /* leaves that were still near at the depth cap */
    int64_t on_surface;   /* pairs whose point lies on the element */
    int64_t max_depth;    /* deepest level reached */
} orc_stats;

/* Potential and field at n points from all elements with density sigma[n_E].
 * phi[n], E[n][3] (E may be NULL).  abs_phi[n] (optional) = sum over elements of
 * |phi_j|, abs_E[n] (optional) = sum over elements of |E_j| (per-element contributions,
 * used to normalise errors).  nthreads <= 0: OpenMP default.
 * Returns the number of threads used (> 0), or < 0 on invalid input. */
int orc_eval(const double* tri, int64_t n_tri, const double* rect, int64_t n_rect,
             const double* sigma, const orc_params* prm,
             const double* pts, int64_t n, double* phi, double* E,
             double* abs_phi, double* abs_E, orc_stats* st, int nthreads);

/* Field gradient dE_i/dx_j = -d^2 phi/dx_i dx_j at n points: each cubature point charge
 * of Eq. (4.1) contributes K q (delta_ij r^2 - 3 d_i d_j) / r^5 with d = P - Q (the
 * conclusions note that higher derivatives come from the same charges); the near-field
 * subdivision and rule choice are those of the field.  G[n][6] = xx, yy, zz, xy, xz, yz.
 * abs_G[n] (optional) = K sum_j |sigma_j| |G_j|_F; abs_T[n] (optional) = K times the sum,
 * over every point-charge term the evaluation adds (near-field leaves included), of
 * |q| sqrt(6) / r^3 (the Frobenius norm of one term): the scale of the rounding error of
 * the whole sum.  A point lying on an element has no gradient (the normal field jumps
 * there): its six values are NaN.  Returns threads used or < 0. */
int orc_eval_gradient(const double* tri, int64_t n_tri, const double* rect, int64_t n_rect,
                      const double* sigma, const orc_params* prm, const double* pts, int64_t n,
                      double* G, double* abs_G, double* abs_T, orc_stats* st, int nthreads);

/* Matrix-free collocation product: out[r][k] = potential at the centroid of element
 * rows[k] from all elements with density sigma[r][:], r < n_rhs.  The element's own
 * contribution is its on-element (self) integral.  abs_out[r][k] (optional) = K times the
 * sum over elements j of |sigma[r][j] phi_j| (the row's own per-element potentials, the
 * normaliser of errors of right-hand side r).  Returns threads used or < 0. */
int orc_collocation(const double* tri, int64_t n_tri, const double* rect, int64_t n_rect,
                    const double* sigma, int n_rhs, const orc_params* prm,
                    const int64_t* rows, int64_t n_rows, double* out, double* abs_out,
                    orc_stats* st, int nthreads);

/* Single element, single point, unit density, no Coulomb constant:
 * mode 0 = the rule at the element itself (no near/far switch),
 * mode 1 = full dispatch (far rule / subdivision / on-element rule);
 * mode | 2 also returns the field gradient: out[4..9] = xx, yy, zz, xy, xz, yz.
 * kind 0 triangle, 1 rectangle; geom[9] as above.  out[4] (or out[10]) = phi, Ex, Ey, Ez
 * (, gradient). */
int orc_element(int kind, const double* geom, const double* P, const orc_params* prm,
                int mode, double* out, orc_stats* st);

/* Centroid[3], area and average side length L of one element (Sec. 2, Eq. 3.2/3.3). */
int orc_element_geometry(int kind, const double* geom, double* centroid, double* area, double* L);

#ifdef __cplusplus
}
#endif
#endif
