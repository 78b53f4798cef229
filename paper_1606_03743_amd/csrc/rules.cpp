// Cubature rules of the GPU library (host side; expanded once per rule change and
// copied to device memory as FP64 and FP32 node tables).
//
// Triangle rules: barycentric coordinates and weights of App. A (Tables A1-A5), one
// entry per table row with the symmetry that row stands for (table captions):
//   CENTROID  (1/3, 1/3, 1/3)
//   S21       (a, b, b) and the placements of the distinct value: 3 points
//   CYCLIC    (a, b, c), (b, c, a), (c, a, b): 3 points          (Table A3 only)
//   S111      all six permutations of (a, b, c)
// Weights are the printed digits; they sum to 1 (Eq. 3.1) to the printed precision.
//
// Rectangle rules: tensor Gauss-Legendre n x n on the natural coordinates of Eq. 3.2,
// weights w_i w_j / 4 (Legendre roots by Newton iteration on the three-term recurrence),
// or the tables of App. B.
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

// Rectangle rules of App. B in natural coordinates (Eq. 3.2).  Each entry is one table
// row; its orbit is given by the table caption: a single point, the four sign changes
// (Tables B1-B3), or the four rotations +-(x, y), +-(-y, x) (Tables B4, B5).
namespace {
enum RectOrbit { ONE, SIGNS, ROTATIONS };
struct RectRow {
    RectOrbit orbit;
    double x, y, w;
};
void expand_rect(const RectRow* rows, int nrows, std::vector<RectNode>& out)
{
    out.clear();
    for (int r = 0; r < nrows; ++r) {
        const RectRow& R = rows[r];
        if (R.orbit == ONE) {
            out.push_back({ R.x, R.y, R.w });
        } else if (R.orbit == SIGNS) {
            for (double sx : { 1.0, -1.0 })
                for (double sy : { 1.0, -1.0 }) out.push_back({ sx * R.x, sy * R.y, R.w });
        } else {
            out.push_back({ R.x, R.y, R.w });
            out.push_back({ -R.x, -R.y, R.w });
            out.push_back({ -R.y, R.x, R.w });
            out.push_back({ R.y, -R.x, R.w });
        }
    }
}
}  // namespace

bool rectangle_table_rule(int n, std::vector<RectNode>& out)
{
    switch (n) {
    case 4: {  // Table B1, degree 3
        const double s = std::sqrt(1.0 / 3.0);
        const RectRow rows[] = { { SIGNS, s, s, 0.25 } };
        expand_rect(rows, 1, out);
        return true;
    }
    case 7: {  // Table B2, degree 5
        const double t = std::sqrt(14.0 / 15.0), r = std::sqrt(3.0 / 5.0), s = std::sqrt(1.0 / 3.0);
        const RectRow rows[] = { { ONE, 0.0, 0.0, 2.0 / 7.0 }, { ONE, 0.0, t, 5.0 / 63.0 }, { ONE, 0.0, -t, 5.0 / 63.0 },
                                 { SIGNS, r, s, 5.0 / 36.0 } };
        expand_rect(rows, 4, out);
        return true;
    }
    case 12: {  // Table B3, degree 7
        const double q = std::sqrt(583.0);
        const double r = std::sqrt(6.0 / 7.0);
        const double s = std::sqrt((114.0 - 3.0 * q) / 287.0), t = std::sqrt((114.0 + 3.0 * q) / 287.0);
        const double b1 = 49.0 / 810.0, b2 = (178981.0 + 2769.0 * q) / 1888920.0, b3 = (178981.0 - 2769.0 * q) / 1888920.0;
        const RectRow rows[] = { { ONE, r, 0.0, b1 }, { ONE, -r, 0.0, b1 }, { ONE, 0.0, r, b1 }, { ONE, 0.0, -r, b1 },
                                 { SIGNS, s, s, b2 }, { SIGNS, t, t, b3 } };
        expand_rect(rows, 6, out);
        return true;
    }
    case 17: {  // Table B4, degree 9
        const RectRow rows[] = {
            { ONE, 0.0, 0.0, 0.131687242798353921 },
            { ROTATIONS, 0.968849966361977720, 0.630680119731668854, 0.022219844542549678 },
            { ROTATIONS, 0.750277099978900533, 0.927961645959569667, 0.028024900532399120 },
            { ROTATIONS, 0.523735820214429336, 0.453339821135647190, 0.099570609815517519 },
            { ROTATIONS, 0.076208328192617173, 0.852615729333662307, 0.067262834409945196 },
        };
        expand_rect(rows, 5, out);
        return true;
    }
    case 33: {  // Table B5, degree 13
        const RectRow rows[] = {
            { ONE, 0.0, 0.0, 0.075095528857806335 },
            { ROTATIONS, 0.778809711554419422, 0.983486682439872263, 0.007497959716124783 },
            { ROTATIONS, 0.957297699786307365, 0.859556005641638928, 0.009543605329270918 },
            { ROTATIONS, 0.138183459862465353, 0.958925170287534857, 0.015106230954437494 },
            { ROTATIONS, 0.941327225872925236, 0.390736216129461000, 0.019373184633276336 },
            { ROTATIONS, 0.475808625218275905, 0.850076673699748575, 0.029711166825148901 },
            { ROTATIONS, 0.755805356572081436, 0.647821637187010732, 0.032440887592500675 },
            { ROTATIONS, 0.696250078491749413, 0.070741508996444936, 0.053335395364297350 },
            { ROTATIONS, 0.342716556040406789, 0.409304561694038843, 0.064217687370491966 },
        };
        expand_rect(rows, 9, out);
        return true;
    }
    default:
        return false;
    }
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
