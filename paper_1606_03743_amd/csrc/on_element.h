// Field points lying on an element (device code shared by the near-pair cost pass and the
// kernel that evaluates such pairs).
//
// The Gaussian rules (Sec. 3) and their subdivision (Sec. 4) cannot reach a point on the
// element itself: 1/r is singular there.  For a flat element with constant density the
// integral about the point has a closed form (polar coordinates about the point, one term
// per edge), which these pairs take instead.  The test and the integral run in three
// dimensions relative to the element's first vertex.
#pragma once

#include "bemc_internal.h"

namespace bemc {

// Corners of element e relative to its first vertex (3 for a triangle, 4 for a rectangle).
__device__ __forceinline__ int element_corners(const Elements& el, int64_t e, bool tri, const double (&G)[9],
                                               double (&V)[4][3])
{
    if (tri) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            V[0][c] = 0.0; V[1][c] = G[3 + c] - G[c]; V[2][c] = G[6 + c] - G[c]; V[3][c] = 0.0;
        }
        return 3;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        V[0][c] = 0.0; V[1][c] = G[3 + c]; V[2][c] = G[3 + c] + G[6 + c]; V[3][c] = G[6 + c];
    }
    return 4;
}

// Does the point X lie on element e?  Within 1e-12 L of its plane and inside it (the edge
// tests of a triangle with a relative tolerance of 1e-12, the natural coordinates of a
// rectangle within 1 + 1e-12).  P receives X relative to the first vertex.
__device__ __forceinline__ bool point_on_element(const Elements& el, int64_t e, bool tri, const double (&X)[3],
                                                 double (&G)[9], double (&P)[3])
{
    const int64_t ne = el.ne;
#pragma unroll
    for (int c = 0; c < 9; ++c) G[c] = el.geom[(int64_t)c * ne + e];
#pragma unroll
    for (int c = 0; c < 3; ++c) P[c] = X[c] - G[c];
    const double L = el.L[e];
    const double nx = el.nrm[e], ny = el.nrm[ne + e], nz = el.nrm[2 * ne + e];
    const double dx = P[0] - (el.cen[e] - G[0]);
    const double dy = P[1] - (el.cen[ne + e] - G[1]);
    const double dz = P[2] - (el.cen[2 * ne + e] - G[2]);
    bool on = fabs(nx * dx + ny * dy + nz * dz) <= 1e-12 * L;
    if (!on) return false;
    if (tri) {
        double V[4][3];
        element_corners(el, e, true, G, V);
        const double twoA = 2.0 * el.area[e];
        for (int k = 0; k < 3 && on; ++k) {
            const double* Va = V[(k + 1) % 3];
            const double* Vb = V[(k + 2) % 3];
            const double ax = Va[0] - P[0], ay = Va[1] - P[1], az = Va[2] - P[2];
            const double bx = Vb[0] - P[0], by = Vb[1] - P[1], bz = Vb[2] - P[2];
            const double cxp = ay * bz - az * by, cyp = az * bx - ax * bz, czp = ax * by - ay * bx;
            on = (nx * cxp + ny * cyp + nz * czp) / twoA >= -1e-12;
        }
        return on;
    }
    const double x = 2.0 * (dx * G[3] + dy * G[4] + dz * G[5]) / (G[3] * G[3] + G[4] * G[4] + G[5] * G[5]);
    const double y = 2.0 * (dx * G[6] + dy * G[7] + dz * G[8]) / (G[6] * G[6] + G[7] * G[7] + G[8] * G[8]);
    return fabs(x) <= 1.0 + 1e-12 && fabs(y) <= 1.0 + 1e-12;
}

}  // namespace bemc
