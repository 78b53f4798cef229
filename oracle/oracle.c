/*
 * oracle.c -- plain, slow, FP64 CPU oracle (test infrastructure only).
 *
 * Computes what the GPU library computes, written out step by step after
 * Glueck & Hilk, "Electric potential and field calculation of charged BEM
 * triangles and rectangles by Gaussian cubature" (arXiv:1606.03743):
 *
 *   * an element of constant density sigma is replaced by the point charges
 *     q_i = w_i * sigma * area at its Gaussian points Q_i (Sec. 4, Eq. 4.1;
 *     cubature rule Sec. 3, Eq. 3.1, sum w_i = 1);
 *   * Gaussian points of triangles from barycentric coordinates (Eq. 3.3,
 *     rule tables A1-A5), of rectangles from natural coordinates (Eq. 3.2,
 *     tables B1-B5, or a tensor Gauss-Legendre n x n rule);
 *   * potential and field from the same points in one pass (Sec. 4);
 *   * distance ratio DR = D / L, D = |P - centroid|, L = average side length
 *     (Sec. 2).  Below DR 3 the paper switches to analytical integration
 *     (Sec. 1, Sec. 4); this implementation instead subdivides the element
 *     recursively (triangle: 4 midpoint children; rectangle: 2 x 2) until each
 *     child is at DR >= 3 of its own, with a depth cap;
 *   * a point lying on the element (collocation self-term, or an evaluation
 *     point on an electrode) is integrated exactly in polar coordinates about
 *     the point: the element is the fan of triangles (P, V_k, V_k+1), the
 *     radial integral cancels the 1/r singularity, and the angular integral
 *     over each edge has a closed form; the field there is the principal value
 *     (in-plane part; the element's own normal part is zero).
 *
 * Each element is integrated in coordinates relative to its first vertex (same
 * integrals, better conditioned close to the element).  Per point, the element
 * contributions are accumulated in element-index order with Neumaier-compensated
 * FP64 sums; the Coulomb constant is applied last.
 *
 * Rule tables are typed in here from the paper's appendices; Gauss-Legendre
 * nodes come from Newton iteration on the Legendre polynomial.  Nothing here
 * is shared with the GPU library.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_D 3.14159265358979323846264338327950288
#define EPS0_SI 8.8541878188e-12 /* CODATA 2022, F/m */

double orc_coulomb_constant(void) { return 1.0 / (4.0 * PI_D * EPS0_SI); }

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double* a, const double* b, double* o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* Neumaier-compensated sum */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes: Newton iteration on P_n, long double          */
/* ------------------------------------------------------------------ */
int orc_gauss_legendre(int n, double* x, double* w)
{
    if (n < 1 || n > 64) return -1;
    for (int k = 0; k < (n + 1) / 2; ++k) {
        /* k-th largest root; standard asymptotic first guess */
        long double z = cosl((long double)PI_D * (k + 0.75L) / (n + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 60; ++it) {
            long double p_prev = 1.0L, p = z; /* P_0, P_1 */
            for (int m = 2; m <= n; ++m) {
                long double p_next = ((2.0L * m - 1.0L) * z * p - (m - 1.0L) * p_prev) / m;
                p_prev = p;
                p = p_next;
            }
            /* P_n' = n (z P_n - P_{n-1}) / (z^2 - 1) */
            dp = n * (z * p - p_prev) / (z * z - 1.0L);
            long double step = p / dp;
            z -= step;
            if (fabsl(step) < 1e-19L) break;
        }
        /* final derivative at the converged root */
        {
            long double p_prev = 1.0L, p = z;
            for (int m = 2; m <= n; ++m) {
                long double p_next = ((2.0L * m - 1.0L) * z * p - (m - 1.0L) * p_prev) / m;
                p_prev = p;
                p = p_next;
            }
            dp = n * (z * p - p_prev) / (z * z - 1.0L);
        }
        long double wk = 2.0L / ((1.0L - z * z) * dp * dp);
        x[k] = (double)(-z);
        x[n - 1 - k] = (double)z;
        w[k] = (double)wk;
        w[n - 1 - k] = (double)wk;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
    return n;
}

/* ------------------------------------------------------------------ */
/* Rule tables (App. A triangles, App. B rectangles)                   */
/* ------------------------------------------------------------------ */
#define MAX_TRI_NODES 64
#define MAX_RECT_NODES 256

typedef struct { int n; double lam[MAX_TRI_NODES][3]; double w[MAX_TRI_NODES]; } tri_rule;
typedef struct { int n; double xy[MAX_RECT_NODES][2]; double w[MAX_RECT_NODES]; } rect_rule;

static void tri_put(tri_rule* r, double a, double b, double c, double w)
{
    r->lam[r->n][0] = a; r->lam[r->n][1] = b; r->lam[r->n][2] = c; r->w[r->n] = w; r->n++;
}
/* one point at the centroid */
static void tri_center(tri_rule* r, double w) { tri_put(r, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, w); }
/* (a,b,b): the three placements of the distinct coordinate */
static void tri_s21(tri_rule* r, double a, double b, double w)
{
    tri_put(r, a, b, b, w); tri_put(r, b, a, b, w); tri_put(r, b, b, a, w);
}
/* (a,b,c) and its two cyclic shifts (A,B,C)->(B,C,A)->(C,A,B) */
static void tri_cyc(tri_rule* r, double a, double b, double c, double w)
{
    tri_put(r, a, b, c, w); tri_put(r, b, c, a, w); tri_put(r, c, a, b, w);
}
/* all six permutations of (a,b,c) */
static void tri_s111(tri_rule* r, double a, double b, double c, double w)
{
    tri_put(r, a, b, c, w); tri_put(r, a, c, b, w); tri_put(r, b, a, c, w);
    tri_put(r, b, c, a, w); tri_put(r, c, a, b, w); tri_put(r, c, b, a, w);
}

static int build_tri_rule(int n, tri_rule* r)
{
    r->n = 0;
    switch (n) {
    case 4: /* Table A1, degree 3 */
        tri_center(r, -9.0 / 16.0);
        tri_s21(r, 3.0 / 5.0, 1.0 / 5.0, 25.0 / 48.0);
        break;
    case 7: { /* Table A2, degree 5: t = 1/3, s = (1-sqrt15)/7, r = (1+sqrt15)/7 */
        double q = sqrt(15.0), t = 1.0 / 3.0;
        double s = (1.0 - q) / 7.0, rr = (1.0 + q) / 7.0;
        tri_center(r, 9.0 / 40.0);
        tri_s21(r, t + 2.0 * t * s, t - t * s, (155.0 + q) / 1200.0);
        tri_s21(r, t + 2.0 * t * rr, t - t * rr, (155.0 - q) / 1200.0);
        break;
    }
    case 12: /* Table A3, degree 7, cyclic orbits only */
        tri_cyc(r, 0.06238226509439084, 0.06751786707392436, 0.8700998678316848, 0.05303405631486900);
        tri_cyc(r, 0.05522545665692000, 0.3215024938520156, 0.6232720494910644, 0.08776281742889622);
        tri_cyc(r, 0.03432430294509488, 0.6609491961867980, 0.3047265008681072, 0.05755008556995056);
        tri_cyc(r, 0.5158423343536001, 0.2777161669764050, 0.2064414986699949, 0.13498637401961758);
        break;
    case 19: /* Table A4, degree 9 */
        tri_center(r, 0.09713579628279610);
        tri_s21(r, 0.02063496160252593, 0.48968251919873704, 0.03133470022713983);
        tri_s21(r, 0.1258208170141290, 0.4370895914929355, 0.07782754100477543);
        tri_s21(r, 0.6235929287619356, 0.18820353561903219, 0.07964773892720910);
        tri_s21(r, 0.9105409732110941, 0.04472951339445297, 0.02557767565869810);
        tri_s111(r, 0.03683841205473626, 0.7411985987844980, 0.22196298916076573, 0.04328353937728940);
        break;
    case 33: /* Table A5, degree 12 */
        tri_s21(r, 0.4570749859701478, 0.27146250701492611, 0.06254121319590276);
        tri_s21(r, 0.1197767026828138, 0.44011164865859310, 0.04991833492806094);
        tri_s21(r, 0.0235924981089169, 0.48820375094554155, 0.02426683808145203);
        tri_s21(r, 0.7814843446812914, 0.10925782765935432, 0.02848605206887754);
        tri_s21(r, 0.9507072731273288, 0.02464636343633558, 0.00793164250997364);
        tri_s111(r, 0.1162960196779266, 0.2554542286385173, 0.62824975168355610, 0.04322736365941421);
        tri_s111(r, 0.02303415635526714, 0.2916556797383410, 0.68531016390639186, 0.02178358503860756);
        tri_s111(r, 0.02138249025617059, 0.1272797172335894, 0.85133779251024000, 0.01508367757651144);
        break;
    default:
        return -1;
    }
    return r->n;
}

static void rect_put(rect_rule* r, double x, double y, double w)
{
    r->xy[r->n][0] = x; r->xy[r->n][1] = y; r->w[r->n] = w; r->n++;
}
/* all sign changes (x,y), (x,-y), (-x,y), (-x,-y) */
static void rect_sign4(rect_rule* r, double x, double y, double w)
{
    rect_put(r, x, y, w); rect_put(r, x, -y, w); rect_put(r, -x, y, w); rect_put(r, -x, -y, w);
}
/* rotations by 0, 180, +-90 degrees: +-(x,y), +-(-y,x) */
static void rect_rot4(rect_rule* r, double x, double y, double w)
{
    rect_put(r, x, y, w); rect_put(r, -x, -y, w); rect_put(r, -y, x, w); rect_put(r, y, -x, w);
}

static int build_rect_rule(int gl_n, int table_n, rect_rule* r)
{
    r->n = 0;
    if (gl_n > 0) {
        double x[64], w[64];
        if (gl_n > 16 || orc_gauss_legendre(gl_n, x, w) < 0) return -1;
        /* tensor product; each 1-D weight sums to 2, so w_ij = w_i w_j / 4 sums to 1 */
        for (int i = 0; i < gl_n; ++i)
            for (int j = 0; j < gl_n; ++j) rect_put(r, x[i], x[j], w[i] * w[j] / 4.0);
        return r->n;
    }
    switch (table_n) {
    case 4: { /* Table B1, degree 3 */
        double s = 1.0 / sqrt(3.0);
        rect_sign4(r, s, s, 0.25);
        break;
    }
    case 7: { /* Table B2, degree 5 */
        double t = sqrt(14.0 / 15.0), rr = sqrt(3.0 / 5.0), s = sqrt(1.0 / 3.0);
        rect_put(r, 0.0, 0.0, 2.0 / 7.0);
        rect_put(r, 0.0, t, 5.0 / 63.0);
        rect_put(r, 0.0, -t, 5.0 / 63.0);
        rect_sign4(r, rr, s, 5.0 / 36.0);
        break;
    }
    case 12: { /* Table B3, degree 7 */
        double q = sqrt(583.0);
        double rr = sqrt(6.0 / 7.0);
        double s = sqrt((114.0 - 3.0 * q) / 287.0), t = sqrt((114.0 + 3.0 * q) / 287.0);
        double b1 = 49.0 / 810.0;
        double b2 = (178981.0 + 2769.0 * q) / 1888920.0;
        double b3 = (178981.0 - 2769.0 * q) / 1888920.0;
        rect_put(r, rr, 0.0, b1); rect_put(r, -rr, 0.0, b1);
        rect_put(r, 0.0, rr, b1); rect_put(r, 0.0, -rr, b1);
        rect_sign4(r, s, s, b2);
        rect_sign4(r, t, t, b3);
        break;
    }
    case 17: /* Table B4, degree 9 */
        rect_put(r, 0.0, 0.0, 0.131687242798353921);
        rect_rot4(r, 0.968849966361977720, 0.630680119731668854, 0.022219844542549678);
        rect_rot4(r, 0.750277099978900533, 0.927961645959569667, 0.028024900532399120);
        rect_rot4(r, 0.523735820214429336, 0.453339821135647190, 0.099570609815517519);
        rect_rot4(r, 0.076208328192617173, 0.852615729333662307, 0.067262834409945196);
        break;
    case 33: /* Table B5, degree 13 */
        rect_put(r, 0.0, 0.0, 0.075095528857806335);
        rect_rot4(r, 0.778809711554419422, 0.983486682439872263, 0.007497959716124783);
        rect_rot4(r, 0.957297699786307365, 0.859556005641638928, 0.009543605329270918);
        rect_rot4(r, 0.138183459862465353, 0.958925170287534857, 0.015106230954437494);
        rect_rot4(r, 0.941327225872925236, 0.390736216129461000, 0.019373184633276336);
        rect_rot4(r, 0.475808625218275905, 0.850076673699748575, 0.029711166825148901);
        rect_rot4(r, 0.755805356572081436, 0.647821637187010732, 0.032440887592500675);
        rect_rot4(r, 0.696250078491749413, 0.070741508996444936, 0.053335395364297350);
        rect_rot4(r, 0.342716556040406789, 0.409304561694038843, 0.064217687370491966);
        break;
    default:
        return -1;
    }
    return r->n;
}

int orc_tri_rule(int n, double* lam, double* w)
{
    tri_rule r;
    if (build_tri_rule(n, &r) < 0) return -1;
    for (int i = 0; i < r.n; ++i) {
        lam[3 * i + 0] = r.lam[i][0]; lam[3 * i + 1] = r.lam[i][1]; lam[3 * i + 2] = r.lam[i][2];
        w[i] = r.w[i];
    }
    return r.n;
}

int orc_rect_rule(int gl_n, int table_n, double* xy, double* w)
{
    rect_rule r;
    if (build_rect_rule(gl_n, table_n, &r) < 0) return -1;
    for (int i = 0; i < r.n; ++i) { xy[2 * i] = r.xy[i][0]; xy[2 * i + 1] = r.xy[i][1]; w[i] = r.w[i]; }
    return r.n;
}

/* ------------------------------------------------------------------ */
/* Element geometry (Sec. 2: centroid, average side length; Eq. 3.2/3.3) */
/* ------------------------------------------------------------------ */
typedef struct {
    int kind;        /* 0 triangle, 1 rectangle */
    double g[9];     /* A,B,C  or  P0,e1,e2 */
    double cen[3];
    double area;
    double L;
    double nrm[3];   /* unit normal */
} elem;

static int make_elem(int kind, const double* g, elem* e)
{
    e->kind = kind;
    memcpy(e->g, g, 9 * sizeof(double));
    for (int i = 0; i < 9; ++i)
        if (!isfinite(g[i])) return -1;
    if (kind == 0) {
        const double *A = g, *B = g + 3, *C = g + 6;
        double ab[3], ac[3], bc[3], cr[3];
        sub3(B, A, ab); sub3(C, A, ac); sub3(C, B, bc);
        cross3(ab, ac, cr);
        double c2 = norm3(cr);
        for (int k = 0; k < 3; ++k) e->cen[k] = (A[k] + B[k] + C[k]) / 3.0;
        e->area = 0.5 * c2;
        /* L = (a + b + c) / 3 */
        e->L = (norm3(bc) + norm3(ac) + norm3(ab)) / 3.0;
        if (!(e->area > 0.0)) return -2;
        for (int k = 0; k < 3; ++k) e->nrm[k] = cr[k] / c2;
    } else {
        const double *P0 = g, *e1 = g + 3, *e2 = g + 6;
        double a = norm3(e1), b = norm3(e2), cr[3];
        if (!(a > 0.0 && b > 0.0)) return -2;
        if (fabs(dot3(e1, e2)) > 1e-10 * a * b) return -3;
        cross3(e1, e2, cr);
        double c2 = norm3(cr);
        for (int k = 0; k < 3; ++k) e->cen[k] = P0[k] + 0.5 * e1[k] + 0.5 * e2[k];
        e->area = a * b;
        /* L = mean of the four sides = (a + b) / 2 */
        e->L = 0.5 * (a + b);
        for (int k = 0; k < 3; ++k) e->nrm[k] = cr[k] / c2;
    }
    return 0;
}

int orc_element_geometry(int kind, const double* geom, double* centroid, double* area, double* L)
{
    elem e;
    int rc = make_elem(kind, geom, &e);
    if (rc) return rc;
    memcpy(centroid, e.cen, 3 * sizeof(double));
    *area = e.area;
    *L = e.L;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Point-charge sum of one (sub-)element at P, unit density, Eq. 4.1   */
/* acc[4] += area * sum_i w_i (1/r_i, (P - Q_i)/r_i^3)                 */
/* ------------------------------------------------------------------ */
typedef struct {
    tri_rule tri;
    rect_rule rect;
    tri_rule tri_lv[3];   /* 7, 12, 19 points (distance-ratio-dependent choice) */
    rect_rule rect_lv[3]; /* Tables B2, B3, B4 */
    int grad;             /* also accumulate the field gradient (acc[4..9]) */
} rules;

static void apply_rules(const double* P, int kind, const double* g, double area, const tri_rule* TR,
                        const rect_rule* RR, int grad, double* acc);

static void apply_rule(const double* P, int kind, const double* g, double area, const rules* R, double* acc)
{
    apply_rules(P, kind, g, area, &R->tri, &R->rect, R->grad, acc);
}

/* Field gradient of one point charge w at Q (unit density, no constant), d = P - Q:
 * dE_i/dx_j = w (delta_ij r^2 - 3 d_i d_j) / r^5; accumulated as xx, yy, zz, xy, xz, yz. */
static void add_gradient(const double* d, double r, double w, double* G)
{
    double r2 = r * r, f5 = w / (r2 * r2 * r);
    G[0] += f5 * (r2 - 3.0 * d[0] * d[0]);
    G[1] += f5 * (r2 - 3.0 * d[1] * d[1]);
    G[2] += f5 * (r2 - 3.0 * d[2] * d[2]);
    G[3] -= 3.0 * f5 * d[0] * d[1];
    G[4] -= 3.0 * f5 * d[0] * d[2];
    G[5] -= 3.0 * f5 * d[1] * d[2];
}

static void apply_rules(const double* P, int kind, const double* g, double area, const tri_rule* TR,
                        const rect_rule* RR, int grad, double* acc)
{
    double G[6] = { 0, 0, 0, 0, 0, 0 }, T = 0.0;
    double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    if (kind == 0) {
        const double *A = g, *B = g + 3, *C = g + 6;
        for (int i = 0; i < TR->n; ++i) {
            const double* l = TR->lam[i];
            double Q[3], d[3];
            for (int k = 0; k < 3; ++k) Q[k] = l[0] * A[k] + l[1] * B[k] + l[2] * C[k];
            sub3(P, Q, d);
            double r = norm3(d);
            double inv = 1.0 / r;
            double f = TR->w[i] * inv * inv * inv;
            phi += TR->w[i] * inv;
            ex += f * d[0]; ey += f * d[1]; ez += f * d[2];
            if (grad) { add_gradient(d, r, TR->w[i], G); T += fabs(TR->w[i]) / (r * r * r); }
        }
    } else {
        const double *P0 = g, *e1 = g + 3, *e2 = g + 6;
        double cen[3];
        for (int k = 0; k < 3; ++k) cen[k] = P0[k] + 0.5 * e1[k] + 0.5 * e2[k];
        for (int i = 0; i < RR->n; ++i) {
            double x = RR->xy[i][0], y = RR->xy[i][1];
            double Q[3], d[3];
            /* Q = Q_cen + (a/2) x u_x + (b/2) y u_y = Q_cen + (x/2) e1 + (y/2) e2 */
            for (int k = 0; k < 3; ++k) Q[k] = cen[k] + 0.5 * x * e1[k] + 0.5 * y * e2[k];
            sub3(P, Q, d);
            double r = norm3(d);
            double inv = 1.0 / r;
            double f = RR->w[i] * inv * inv * inv;
            phi += RR->w[i] * inv;
            ex += f * d[0]; ey += f * d[1]; ez += f * d[2];
            if (grad) { add_gradient(d, r, RR->w[i], G); T += fabs(RR->w[i]) / (r * r * r); }
        }
    }
    acc[0] += area * phi; acc[1] += area * ex; acc[2] += area * ey; acc[3] += area * ez;
    if (grad) {
        for (int k = 0; k < 6; ++k) acc[4 + k] += area * G[k];
        acc[10] += area * sqrt(6.0) * T; /* |one term|_F = sqrt(6) |w| / r^3 */
    }
}

/* ------------------------------------------------------------------ */
/* Near field: recursive subdivision                                   */
/* ------------------------------------------------------------------ */
static void subdivide(int kind, const double* g, double ch[4][9])
{
    if (kind == 0) {
        const double *A = g, *B = g + 3, *C = g + 6;
        double mab[3], mbc[3], mca[3];
        for (int k = 0; k < 3; ++k) {
            mab[k] = 0.5 * (A[k] + B[k]);
            mbc[k] = 0.5 * (B[k] + C[k]);
            mca[k] = 0.5 * (C[k] + A[k]);
        }
        /* (A, mAB, mCA), (mAB, B, mBC), (mCA, mBC, C), (mBC, mCA, mAB) */
        for (int k = 0; k < 3; ++k) {
            ch[0][k] = A[k];   ch[0][3 + k] = mab[k]; ch[0][6 + k] = mca[k];
            ch[1][k] = mab[k]; ch[1][3 + k] = B[k];   ch[1][6 + k] = mbc[k];
            ch[2][k] = mca[k]; ch[2][3 + k] = mbc[k]; ch[2][6 + k] = C[k];
            ch[3][k] = mbc[k]; ch[3][3 + k] = mca[k]; ch[3][6 + k] = mab[k];
        }
    } else {
        const double *P0 = g, *e1 = g + 3, *e2 = g + 6;
        for (int k = 0; k < 3; ++k) {
            double h1 = 0.5 * e1[k], h2 = 0.5 * e2[k];
            /* children (0,0), (1,0), (0,1), (1,1) along (e1, e2) */
            ch[0][k] = P0[k];
            ch[1][k] = P0[k] + h1;
            ch[2][k] = P0[k] + h2;
            ch[3][k] = P0[k] + h1 + h2;
            for (int c = 0; c < 4; ++c) { ch[c][3 + k] = h1; ch[c][6 + k] = h2; }
        }
    }
}

typedef struct { int64_t near_pairs, leaves, cap_hits, on_surface, max_depth; } lstats;

static void near_recurse(const double* P, int kind, const double* g, int depth, const rules* R,
                         const orc_params* prm, double* acc, lstats* st)
{
    double ch[4][9];
    subdivide(kind, g, ch);
    for (int c = 0; c < 4; ++c) {
        elem e;
        make_elem(kind, ch[c], &e);
        double d[3];
        sub3(P, e.cen, d);
        double D2 = dot3(d, d);
        double thr = prm->near_dr * e.L;
        if (depth + 1 > st->max_depth) st->max_depth = depth + 1;
        if (!(D2 < thr * thr)) {
            apply_rule(P, kind, ch[c], e.area, R, acc);
            st->leaves++;
        } else if (depth + 1 >= prm->max_depth) {
            apply_rule(P, kind, ch[c], e.area, R, acc);
            st->leaves++;
            st->cap_hits++;
        } else {
            near_recurse(P, kind, ch[c], depth + 1, R, prm, acc, st);
        }
    }
}

/* ------------------------------------------------------------------ */
/* On-element point: exact integration in polar coordinates about P     */
/* ------------------------------------------------------------------ */
static int on_element(const double* P, const elem* e)
{
    double d[3];
    sub3(P, e->cen, d);
    if (fabs(dot3(d, e->nrm)) > 1e-12 * e->L) return 0;
    const double tol = 1e-12;
    if (e->kind == 0) {
        const double *A = e->g, *B = e->g + 3, *C = e->g + 6;
        double pa[3], pb[3], pc[3], c1[3];
        sub3(A, P, pa); sub3(B, P, pb); sub3(C, P, pc);
        double tot = 2.0 * e->area;
        cross3(pb, pc, c1); double la = dot3(c1, e->nrm) / tot;
        cross3(pc, pa, c1); double lb = dot3(c1, e->nrm) / tot;
        cross3(pa, pb, c1); double lc = dot3(c1, e->nrm) / tot;
        return la >= -tol && lb >= -tol && lc >= -tol;
    } else {
        const double *e1 = e->g + 3, *e2 = e->g + 6;
        double x = 2.0 * dot3(d, e1) / dot3(e1, e1);
        double y = 2.0 * dot3(d, e2) / dot3(e2, e2);
        return fabs(x) <= 1.0 + tol && fabs(y) <= 1.0 + tol;
    }
}

/* Polar coordinates about P (in the element's plane): along a ray at angle theta the
 * integrand 1/rho times the area element rho d rho d theta integrates to the ray length,
 * so the potential is the angular integral of the distance to the boundary; the in-plane
 * field is the principal value -int e(theta) ln rho(theta) d theta (the divergent ln eps
 * part multiplies int e d theta = 0).  For an edge whose line lies at distance h from P,
 * with unit normal n (from P to the line), unit direction t and end offsets t1 < t2 along
 * it (rho^2 = h^2 + t^2), both angular integrals have closed forms:
 *   potential  h [asinh(t/h)]_t1^t2
 *   field      -n [(t/rho)(1 + ln rho) - asinh(t/h)]_t1^t2  +  h t [(1 + ln rho)/rho]_t1^t2
 * The element's own normal field is zero at a point of the element (principal value). */
static void self_rule(const double* P, const elem* e, double* acc)
{
    double V[4][3];
    int nv;
    if (e->kind == 0) {
        nv = 3;
        for (int k = 0; k < 3; ++k) { V[0][k] = e->g[k]; V[1][k] = e->g[3 + k]; V[2][k] = e->g[6 + k]; }
    } else {
        nv = 4;
        const double *P0 = e->g, *e1 = e->g + 3, *e2 = e->g + 6;
        for (int k = 0; k < 3; ++k) {
            V[0][k] = P0[k];
            V[1][k] = P0[k] + e1[k];
            V[2][k] = P0[k] + e1[k] + e2[k];
            V[3][k] = P0[k] + e2[k];
        }
    }
    double phi = 0.0, E[3] = { 0.0, 0.0, 0.0 };
    for (int k = 0; k < nv; ++k) {
        const double* Va = V[k];
        const double* Vb = V[(k + 1) % nv];
        double tv[3], pa[3], pb[3], nv_[3];
        sub3(Vb, Va, tv);
        double len = norm3(tv);
        for (int c = 0; c < 3; ++c) tv[c] /= len;
        sub3(Va, P, pa);
        sub3(Vb, P, pb);
        double t1 = dot3(pa, tv), t2 = dot3(pb, tv);
        for (int c = 0; c < 3; ++c) nv_[c] = pa[c] - t1 * tv[c]; /* foot of the perpendicular, from P */
        double h = norm3(nv_);
        if (!(h > 1e-14 * e->L)) continue; /* P on this edge's line: the sector has no area */
        for (int c = 0; c < 3; ++c) nv_[c] /= h;
        double r1 = sqrt(h * h + t1 * t1), r2 = sqrt(h * h + t2 * t2);
        phi += h * (asinh(t2 / h) - asinh(t1 / h));
        double gn = (t2 / r2) * (1.0 + log(r2)) - asinh(t2 / h) - ((t1 / r1) * (1.0 + log(r1)) - asinh(t1 / h));
        double gt = h * ((1.0 + log(r2)) / r2 - (1.0 + log(r1)) / r1);
        for (int c = 0; c < 3; ++c) E[c] += -gn * nv_[c] + gt * tv[c];
    }
    acc[0] += phi; acc[1] += E[0]; acc[2] += E[1]; acc[3] += E[2];
}

/* ------------------------------------------------------------------ */
/* Dispatch for one (point, element) pair: unit density, no constant   */
/* ------------------------------------------------------------------ */
/* The same element with its first vertex (A, or the corner P0) moved to the origin, and
 * the field point moved with it.  Integrating in these coordinates forms P - Q_i from
 * numbers of the element's own size instead of absolute coordinates; near the element
 * (distances down to 1e-3 L and below) this removes the cancellation that absolute
 * coordinates far from the origin would cause.  The integrals are unchanged. */
static void to_local(const double* P, const elem* e, double* Pl, elem* le)
{
    *le = *e;
    const double* O = e->g;
    sub3(P, O, Pl);
    if (e->kind == 0) {
        for (int k = 0; k < 3; ++k) {
            le->g[k] = 0.0;
            le->g[3 + k] = e->g[3 + k] - O[k];
            le->g[6 + k] = e->g[6 + k] - O[k];
        }
    } else {
        for (int k = 0; k < 3; ++k) le->g[k] = 0.0;
    }
    sub3(e->cen, O, le->cen);
}

static void element_contribution(const double* P, const elem* e, const rules* R, const orc_params* prm,
                                 double* out, lstats* st)
{
    for (int k = 0; k < 11; ++k) out[k] = 0.0;
    double d[3];
    sub3(P, e->cen, d);
    double D2 = dot3(d, d);
    double thr = prm->near_dr * e->L;
    double Pl[3];
    elem le;
    to_local(P, e, Pl, &le);
    if (!(D2 < thr * thr)) { /* far: DR >= threshold */
        if (prm->dr_rules) {
            /* the coarsest rule whose distance-ratio limit the pair meets */
            const double* lim = e->kind == 0 ? prm->tri_dr : prm->rect_dr;
            for (int lv = 0; lv < 3; ++lv) {
                const double t = lim[lv] * e->L;
                if (D2 >= t * t) {
                    apply_rules(Pl, le.kind, le.g, le.area, &R->tri_lv[lv], &R->rect_lv[lv], R->grad, out);
                    return;
                }
            }
        }
        apply_rule(Pl, le.kind, le.g, le.area, R, out);
        return;
    }
    st->near_pairs++;
    if (on_element(Pl, &le)) {
        st->on_surface++;
        self_rule(Pl, &le, out);
        if (R->grad) /* the normal field jumps across the element: no gradient there */
            for (int k = 4; k < 11; ++k) out[k] = NAN;
        return;
    }
    if (prm->max_depth <= 0) {
        apply_rule(Pl, le.kind, le.g, le.area, R, out);
        st->leaves++;
        st->cap_hits++;
        return;
    }
    near_recurse(Pl, le.kind, le.g, 0, R, prm, out, st);
}

static int build_rules(const orc_params* prm, rules* R)
{
    if (build_tri_rule(prm->tri_rule, &R->tri) < 0) return -1;
    if (build_rect_rule(prm->rect_gl_n, prm->rect_table_n, &R->rect) < 0) return -1;
    if (!(prm->near_dr > 0.0)) return -1;
    R->grad = 0;
    const int tl[3] = { 7, 12, 19 }, rl[3] = { 7, 12, 17 };
    for (int lv = 0; lv < 3; ++lv) {
        build_tri_rule(tl[lv], &R->tri_lv[lv]);
        build_rect_rule(0, rl[lv], &R->rect_lv[lv]);
    }
    return 0;
}

static int build_elems(const double* tri, int64_t n_tri, const double* rect, int64_t n_rect, elem** out)
{
    int64_t n = n_tri + n_rect;
    elem* el = (elem*)malloc((size_t)(n > 0 ? n : 1) * sizeof(elem));
    if (!el) return -4;
    for (int64_t j = 0; j < n_tri; ++j)
        if (make_elem(0, tri + 9 * j, &el[j])) { free(el); return -2; }
    for (int64_t j = 0; j < n_rect; ++j)
        if (make_elem(1, rect + 9 * j, &el[n_tri + j])) { free(el); return -2; }
    *out = el;
    return 0;
}

static void merge_stats(orc_stats* st, const lstats* l)
{
    st->near_pairs += l->near_pairs;
    st->leaves += l->leaves;
    st->cap_hits += l->cap_hits;
    st->on_surface += l->on_surface;
    if (l->max_depth > st->max_depth) st->max_depth = l->max_depth;
}

int orc_eval(const double* tri, int64_t n_tri, const double* rect, int64_t n_rect,
             const double* sigma, const orc_params* prm,
             const double* pts, int64_t n, double* phi, double* E,
             double* abs_phi, double* abs_E, orc_stats* st, int nthreads)
{
    if (n_tri < 0 || n_rect < 0 || n < 0 || !prm) return -1;
    rules* R = (rules*)malloc(sizeof(rules));
    if (!R) return -4;
    if (build_rules(prm, R)) { free(R); return -1; }
    elem* el = NULL;
    int rc = build_elems(tri, n_tri, rect, n_rect, &el);
    if (rc) { free(R); return rc; }
    const int64_t ne = n_tri + n_rect;
    const double K = orc_coulomb_constant();
    orc_stats tot;
    memset(&tot, 0, sizeof(tot));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int used_threads = 1;
#pragma omp parallel
    {
        lstats ls;
        memset(&ls, 0, sizeof(ls));
#ifdef _OPENMP
#pragma omp single
        used_threads = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 4)
        for (int64_t p = 0; p < n; ++p) {
            const double* P = pts + 3 * p;
            nsum s0 = { 0, 0 }, s1 = { 0, 0 }, s2 = { 0, 0 }, s3 = { 0, 0 };
            double aphi = 0.0, aE = 0.0;
            for (int64_t j = 0; j < ne; ++j) {
                double c[11];
                element_contribution(P, &el[j], R, prm, c, &ls);
                double sg = sigma[j];
                nadd(&s0, sg * c[0]); nadd(&s1, sg * c[1]); nadd(&s2, sg * c[2]); nadd(&s3, sg * c[3]);
                aphi += fabs(sg * c[0]);
                aE += fabs(sg) * sqrt(c[1] * c[1] + c[2] * c[2] + c[3] * c[3]);
            }
            phi[p] = K * nval(&s0);
            if (E) { E[3 * p] = K * nval(&s1); E[3 * p + 1] = K * nval(&s2); E[3 * p + 2] = K * nval(&s3); }
            if (abs_phi) abs_phi[p] = K * aphi;
            if (abs_E) abs_E[p] = K * aE;
        }
#pragma omp critical
        merge_stats(&tot, &ls);
    }
    if (st) {
        memcpy(st, &tot, sizeof(tot));
    }
    (void)used_threads;
    free(el);
    free(R);
    return used_threads;
}

/* Field gradient dE_i/dx_j at each point: the derivative of the point-charge field of
 * Eq. (4.1) (conclusions: higher derivatives follow from the same point charges), with the
 * same near-field subdivision (Sec. 4) and rule choice as the field itself.  G is [n][6]
 * (xx, yy, zz, xy, xz, yz); abs_G[p] = K sum_j |sigma_j| |G_j|_F (Frobenius norm of the
 * element's tensor); abs_T[p] = K sum over every point-charge term summed (subdivision
 * leaves included) of |q| sqrt(6) / r^3, the magnitude scale of the rounding of the whole
 * sum.  A point on an element gets NaN. */
int orc_eval_gradient(const double* tri, int64_t n_tri, const double* rect, int64_t n_rect,
                      const double* sigma, const orc_params* prm, const double* pts, int64_t n,
                      double* G, double* abs_G, double* abs_T, orc_stats* st, int nthreads)
{
    if (n_tri < 0 || n_rect < 0 || n < 0 || !prm || !G) return -1;
    rules* R = (rules*)malloc(sizeof(rules));
    if (!R) return -4;
    if (build_rules(prm, R)) { free(R); return -1; }
    R->grad = 1;
    elem* el = NULL;
    int rc = build_elems(tri, n_tri, rect, n_rect, &el);
    if (rc) { free(R); return rc; }
    const int64_t ne = n_tri + n_rect;
    const double K = orc_coulomb_constant();
    orc_stats tot;
    memset(&tot, 0, sizeof(tot));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int used_threads = 1;
#pragma omp parallel
    {
        lstats ls;
        memset(&ls, 0, sizeof(ls));
#ifdef _OPENMP
#pragma omp single
        used_threads = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 4)
        for (int64_t p = 0; p < n; ++p) {
            const double* P = pts + 3 * p;
            nsum s[6];
            for (int k = 0; k < 6; ++k) { s[k].s = 0.0; s[k].c = 0.0; }
            double aG = 0.0, aT = 0.0;
            for (int64_t j = 0; j < ne; ++j) {
                double c[11];
                element_contribution(P, &el[j], R, prm, c, &ls);
                const double sg = sigma[j];
                double f2 = 0.0;
                for (int k = 0; k < 6; ++k) {
                    nadd(&s[k], sg * c[4 + k]);
                    f2 += (k < 3 ? 1.0 : 2.0) * c[4 + k] * c[4 + k];
                }
                aG += fabs(sg) * sqrt(f2);
                aT += fabs(sg) * c[10];
            }
            for (int k = 0; k < 6; ++k) G[6 * p + k] = K * nval(&s[k]);
            if (abs_G) abs_G[p] = K * aG;
            if (abs_T) abs_T[p] = K * aT;
        }
#pragma omp critical
        merge_stats(&tot, &ls);
    }
    if (st) memcpy(st, &tot, sizeof(tot));
    free(el);
    free(R);
    return used_threads;
}

int orc_collocation(const double* tri, int64_t n_tri, const double* rect, int64_t n_rect,
                    const double* sigma, int n_rhs, const orc_params* prm,
                    const int64_t* rows, int64_t n_rows, double* out, double* abs_out,
                    orc_stats* st, int nthreads)
{
    if (n_tri < 0 || n_rect < 0 || n_rows < 0 || n_rhs < 1 || n_rhs > 64 || !prm) return -1;
    rules* R = (rules*)malloc(sizeof(rules));
    if (!R) return -4;
    if (build_rules(prm, R)) { free(R); return -1; }
    elem* el = NULL;
    int rc = build_elems(tri, n_tri, rect, n_rect, &el);
    if (rc) { free(R); return rc; }
    const int64_t ne = n_tri + n_rect;
    for (int64_t k = 0; k < n_rows; ++k)
        if (rows[k] < 0 || rows[k] >= ne) { free(el); free(R); return -1; }
    const double K = orc_coulomb_constant();
    orc_stats tot;
    memset(&tot, 0, sizeof(tot));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int used_threads = 1;
#pragma omp parallel
    {
        lstats ls;
        memset(&ls, 0, sizeof(ls));
        nsum acc[64];
#ifdef _OPENMP
#pragma omp single
        used_threads = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < n_rows; ++k) {
            const double* P = el[rows[k]].cen;
            double ab[64];
            for (int r = 0; r < n_rhs; ++r) { acc[r].s = 0.0; acc[r].c = 0.0; ab[r] = 0.0; }
            for (int64_t j = 0; j < ne; ++j) {
                double c[11];
                element_contribution(P, &el[j], R, prm, c, &ls);
                for (int r = 0; r < n_rhs; ++r) {
                    const double t = sigma[(int64_t)r * ne + j] * c[0];
                    nadd(&acc[r], t);
                    ab[r] += fabs(t);
                }
            }
            for (int r = 0; r < n_rhs; ++r) {
                out[(int64_t)r * n_rows + k] = K * nval(&acc[r]);
                if (abs_out) abs_out[(int64_t)r * n_rows + k] = K * ab[r];
            }
        }
#pragma omp critical
        merge_stats(&tot, &ls);
    }
    if (st) memcpy(st, &tot, sizeof(tot));
    free(el);
    free(R);
    return used_threads;
}

int orc_element(int kind, const double* geom, const double* P, const orc_params* prm,
                int mode, double* out, orc_stats* st)
{
    rules* R = (rules*)malloc(sizeof(rules));
    if (!R) return -4;
    if (build_rules(prm, R)) { free(R); return -1; }
    R->grad = (mode & 2) ? 1 : 0;
    elem e;
    int rc = make_elem(kind, geom, &e);
    if (rc) { free(R); return rc; }
    lstats ls;
    memset(&ls, 0, sizeof(ls));
    double tmp[11];
    if ((mode & 1) == 0) {
        double Pl[3];
        elem le;
        to_local(P, &e, Pl, &le);
        for (int k = 0; k < 11; ++k) tmp[k] = 0.0;
        apply_rule(Pl, kind, le.g, le.area, R, tmp);
    } else {
        element_contribution(P, &e, R, prm, tmp, &ls);
    }
    for (int k = 0; k < (R->grad ? 10 : 4); ++k) out[k] = tmp[k];
    if (st) {
        memset(st, 0, sizeof(*st));
        merge_stats(st, &ls);
    }
    free(R);
    return 0;
}
