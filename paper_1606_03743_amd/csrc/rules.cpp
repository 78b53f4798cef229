// Cubature rules of the GPU library (host side; expanded once and uploaded to
// constant memory).
//
// Triangle rules: barycentric coordinates and weights of App. A (Tables A1-A5), one
// entry per table row with the symmetry that row stands for (table captions):
//   CENTROID  (1/3, 1/3, 1/3)
//   S21       (a, b, b) and the placements of the distinct value: 3 points
//   CYCLIC    (a, b, c), (b, c, a), (c, a, b): 3 points          (Table A3 only)
//   S111      all six permutations of (a, b, c)
// Weights are normalised to sum 1 (Eq. 3.1).
//
// Rectangle rules: tensor Gauss-Legendre n x n on the natural coordinates of Eq. 3.2,
// weights w_i w_j / 4; Legendre roots by Newton iteration on the three-term recurrence.
#include <cmath>
#include <vector>

#include "bemc_internal.h"

namespace bemc {

namespace {

enum Orbit { CENTROID, S21, CYCLIC, S111 };

struct Row {
    Orbit orbit;
    double a, b, c, w;
};

void expand(const Row* rows, int nrows, std::vector<TriNode>& out)
{
    out.clear();
    for (int r = 0; r < nrows; ++r) {
        const Row& R = rows[r];
        switch (R.orbit) {
        case CENTROID:
            out.push_back({ 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, R.w });
            break;
        case S21:
            out.push_back({ R.a, R.b, R.b, R.w });
            out.push_back({ R.b, R.a, R.b, R.w });
            out.push_back({ R.b, R.b, R.a, R.w });
            break;
        case CYCLIC:
            out.push_back({ R.a, R.b, R.c, R.w });
            out.push_back({ R.b, R.c, R.a, R.w });
            out.push_back({ R.c, R.a, R.b, R.w });
            break;
        case S111: {
            const double v[3] = { R.a, R.b, R.c };
            static const int perm[6][3] = { { 0, 1, 2 }, { 0, 2, 1 }, { 1, 0, 2 }, { 1, 2, 0 }, { 2, 0, 1 }, { 2, 1, 0 } };
            for (auto& p : perm) out.push_back({ v[p[0]], v[p[1]], v[p[2]], R.w });
            break;
        }
        }
    }
}

}  // namespace

bool triangle_rule(int n, std::vector<TriNode>& out)
{
    const double q15 = std::sqrt(15.0);
    const double t = 1.0 / 3.0;
    switch (n) {
    case 4: {  // Table A1, degree 3 (negative centroid weight)
        const Row rows[] = { { CENTROID, 0, 0, 0, -9.0 / 16.0 }, { S21, 0.6, 0.2, 0, 25.0 / 48.0 } };
        expand(rows, 2, out);
        return true;
    }
    case 7: {  // Table A2, degree 5: s = (1 - sqrt15)/7, r = (1 + sqrt15)/7
        const double s = (1.0 - q15) / 7.0, r = (1.0 + q15) / 7.0;
        const Row rows[] = { { CENTROID, 0, 0, 0, 9.0 / 40.0 },
                             { S21, t * (1.0 + 2.0 * s), t * (1.0 - s), 0, (155.0 + q15) / 1200.0 },
                             { S21, t * (1.0 + 2.0 * r), t * (1.0 - r), 0, (155.0 - q15) / 1200.0 } };
        expand(rows, 3, out);
        return true;
    }
    case 12: {  // Table A3, degree 7, cyclic orbits
        const Row rows[] = {
            { CYCLIC, 0.06238226509439084, 0.06751786707392436, 0.8700998678316848, 0.05303405631486900 },
            { CYCLIC, 0.05522545665692000, 0.3215024938520156, 0.6232720494910644, 0.08776281742889622 },
            { CYCLIC, 0.03432430294509488, 0.6609491961867980, 0.3047265008681072, 0.05755008556995056 },
            { CYCLIC, 0.5158423343536001, 0.2777161669764050, 0.2064414986699949, 0.13498637401961758 },
        };
        expand(rows, 4, out);
        return true;
    }
    case 19: {  // Table A4, degree 9
        const Row rows[] = {
            { CENTROID, 0, 0, 0, 0.09713579628279610 },
            { S21, 0.02063496160252593, 0.48968251919873704, 0, 0.03133470022713983 },
            { S21, 0.1258208170141290, 0.4370895914929355, 0, 0.07782754100477543 },
            { S21, 0.6235929287619356, 0.18820353561903219, 0, 0.07964773892720910 },
            { S21, 0.9105409732110941, 0.04472951339445297, 0, 0.02557767565869810 },
            { S111, 0.03683841205473626, 0.7411985987844980, 0.22196298916076573, 0.04328353937728940 },
        };
        expand(rows, 6, out);
        return true;
    }
    case 33: {  // Table A5, degree 12
        const Row rows[] = {
            { S21, 0.4570749859701478, 0.27146250701492611, 0, 0.06254121319590276 },
            { S21, 0.1197767026828138, 0.44011164865859310, 0, 0.04991833492806094 },
            { S21, 0.0235924981089169, 0.48820375094554155, 0, 0.02426683808145203 },
            { S21, 0.7814843446812914, 0.10925782765935432, 0, 0.02848605206887754 },
            { S21, 0.9507072731273288, 0.02464636343633558, 0, 0.00793164250997364 },
            { S111, 0.1162960196779266, 0.2554542286385173, 0.62824975168355610, 0.04322736365941421 },
            { S111, 0.02303415635526714, 0.2916556797383410, 0.68531016390639186, 0.02178358503860756 },
            { S111, 0.02138249025617059, 0.1272797172335894, 0.85133779251024000, 0.01508367757651144 },
        };
        expand(rows, 8, out);
        return true;
    }
    default:
        return false;
    }
}

// Legendre roots on [-1, 1] by Newton's method; P_n and P_n' from the recurrence
// (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.  Weights 2 / ((1 - x^2) P_n'(x)^2).
bool gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    if (n < 1 || n > 64) return false;
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double r = std::cos(pi * (4.0L * i + 3.0L) / (4.0L * n + 2.0L));  // i-th largest root, first guess
        long double pn = 0, dpn = 1;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = r;
            for (int k = 1; k < n; ++k) {
                long double p2 = ((2.0L * k + 1.0L) * r * p1 - k * p0) / (k + 1.0L);
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 0) ? 1.0L : p1;
            long double pm1 = p0;
            dpn = n * (pm1 - r * pn) / (1.0L - r * r);
            long double dr = pn / dpn;
            r -= dr;
            if (std::fabs((double)dr) < 1e-19) {
                // refresh the derivative at the final root
                p0 = 1.0L; p1 = r;
                for (int k = 1; k < n; ++k) {
                    long double p2 = ((2.0L * k + 1.0L) * r * p1 - k * p0) / (k + 1.0L);
                    p0 = p1;
                    p1 = p2;
                }
                dpn = n * (p0 - r * p1) / (1.0L - r * r);
                break;
            }
        }
        const long double wi = 2.0L / ((1.0L - r * r) * dpn * dpn);
        x[n - 1 - i] = (double)r;
        x[i] = -(double)r;
        w[i] = w[n - 1 - i] = (double)wi;
    }
    if (n & 1) x[n / 2] = 0.0;
    return true;
}

bool rectangle_gauss_rule(int n, std::vector<RectNode>& out)
{
    std::vector<double> x, w;
    if (!gauss_legendre(n, x, w)) return false;
    out.clear();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) out.push_back({ x[i], x[j], 0.25 * w[i] * w[j] });
    return true;
}

}  // namespace bemc
