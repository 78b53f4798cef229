// HIP kernels for gfx950 (MI355X): Gaussian-cubature potential and field of charged
// BEM triangles and rectangles (Glueck & Hilk, arXiv:1606.03743).
//
//  far_eval_kernel     PPT field points per lane; element tiles are staged in LDS with
//                      their Gaussian points generated on the fly in each element's own
//                      frame (Eq. 3.2 / 3.3); FP64 distance-ratio test per pair (Sec. 2), near
//                      pairs compacted per wavefront into a dense list; far pairs summed as
//                      point charges (Sec. 4, Eq. 4.1), potential and field from the same
//                      nodes.  FP64 or mixed (FP32 node sums); one rule per element kind or
//                      the rule chosen by distance ratio; field or field gradient.
//  far_colloc_kernel   the same sum, potential only, at element centroids, for up to eight
//                      density vectors (matrix-free collocation product).
//  near_kernel         FP64 near field over the dense list: each lane walks the recursive
//                      subdivision of its pair depth first (triangle: four midpoint
//                      children; rectangle: 2 x 2) using lattice coordinates instead of a
//                      stack; a child at DR >= near_dr of its own (or at the depth cap) gets
//                      the element's rule; a point lying on its element gets the exact
//                      polar integral.  Each pair's result goes to its own slot in
//                      (point, element) order; the per-point sums are formed in that order
//                      afterwards (near_order.hip), so results are reproducible bit for bit.
#include "bemc_internal.h"

namespace bemc {

constexpr double kEps0 = 8.8541878188e-12;  // vacuum permittivity, CODATA 2022 (F/m)
double coulomb_constant() { return 1.0 / (4.0 * 3.14159265358979323846 * kEps0); }

namespace {

constexpr int kBlock = 256;       // 4 wavefronts
constexpr int kTileNodes = 1024;  // Gaussian-point slots of one LDS tile
constexpr int kMaxTileElems = 64;

__device__ __forceinline__ int tile_elems(int nn) { return nn >= 16 ? kTileNodes / nn : kMaxTileElems; }

// 1/sqrt(x) in FP64: hardware estimate (~24 bits) refined by one third-order step
// y (1 + e/2 + 3 e^2 / 8), e = 1 - x y^2 (relative error ~ e^3).
__device__ __forceinline__ double rsqrt64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ float rsqrt32(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of m below this lane
__device__ __forceinline__ unsigned lanes_below(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ unsigned long long bcast_u64(unsigned long long v, int src)
{
    const unsigned lo = __shfl((unsigned)v, src);
    const unsigned hi = __shfl((unsigned)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

// Wavefront-level compaction of near pairs: one atomic per wavefront, lane offsets by
// popcount.  Called with every lane of the wavefront active.
__device__ __forceinline__ void record_near(bool is_near, uint32_t p, uint32_t e, NearPair* list,
                                            unsigned long long cap, DevCounters* ctr)
{
    const unsigned long long m = __ballot(is_near);
    if (m == 0ull) return;
    const int first = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == first) base = atomicAdd(&ctr->near_count, (unsigned long long)__popcll(m));
    base = bcast_u64(base, first);
    if (is_near) {
        const unsigned long long pos = base + lanes_below(m);
        if (pos < cap) list[pos] = NearPair{ p, e };
    }
}

// ---------------------------------------------------------------- LDS staging ------
// Each element is summed in its own orthonormal frame: origin at the centroid, f1 and f2
// in its plane, f3 its unit normal.  A Gaussian point has in-plane coordinates (a, b) and
// a field point the coordinates (p1, p2, p3), so
//   r^2 = (p1 - a)^2 + (p2 - b)^2 + p3^2 = |p|^2 + (a^2 + b^2) - 2 (p1 a + p2 b):
// with a^2 + b^2 staged per node and |p|^2 = D^2 from the distance test, r^2 takes one addition and
// two FMAs per node (for DR >= 3 the expansion adds about a tenth of an ulp to the rounding
// of 1/r; the gradient keeps the two differences).  The sums are rotated back to the global axes once per pair.  For rectangles f1
// runs along the second side, so the nodes of a tensor Gauss-Legendre rule that share their
// first coordinate share b; for the 7 x 7 rule (p2 - b)^2 + p3^2 is formed once per group of
// seven and r^2 takes one difference and one FMA per node.
template <bool MIXED, int NRHS>
struct TileLds {
    using T = typename std::conditional<MIXED, float, double>::type;
    using T4 = typename std::conditional<MIXED, float4, double4>::type;
    T4 nd[kTileNodes];  // a, b, a^2 + b^2, weight (unit element charge)
    double cx[kMaxTileElems], cy[kMaxTileElems], cz[kMaxTileElems], thr2[kMaxTileElems];
    T f[9][kMaxTileElems];  // f1, f2, f3 (x, y, z each), in the precision of the node sums
    double q[NRHS][kMaxTileElems];
};

// Gaussian points of elements [t0, t0 + te) in their frames (Eq. 3.2 / 3.3): triangle
// (a, b) = la A' + lb B' + lc C' from the in-plane coordinates of the vertices relative to
// the centroid; rectangle a = x gamma + y alpha, b = x beta for the rule point (x, y) in
// [-1, 1]^2 (alpha = |e2| / 2; beta, gamma the components of e1 / 2 across and along e2).
// FP32 tiles hold the FP64 values rounded once; the mixed path also rotates in FP32.
template <bool TRI, bool MIXED, int NRHS>
__device__ __forceinline__ void stage_tile(TileLds<MIXED, NRHS>& s, const Elements& el, const RuleTables& R, int nn,
                                           int64_t t0, int te, int rhs0, int nrhs)
{
    const int64_t ne = el.ne;
    for (int k = threadIdx.x; k < te; k += kBlock) {
        const int64_t e = t0 + k;
        s.cx[k] = el.cen[e];
        s.cy[k] = el.cen[ne + e];
        s.cz[k] = el.cen[2 * ne + e];
        s.thr2[k] = el.thr2[e];
#pragma unroll
        for (int c = 0; c < 9; ++c) s.f[c][k] = (typename TileLds<MIXED, NRHS>::T)el.frame[(int64_t)c * ne + e];
        for (int r = 0; r < nrhs; ++r) s.q[r][k] = el.q[(int64_t)(rhs0 + r) * ne + e];
    }
    for (int k = threadIdx.x; k < te * nn; k += kBlock) {
        const int j = k / nn;
        const int i = k - j * nn;
        const int64_t e = t0 + j;
        double a, b, w;
        if (TRI) {
            const double la = R.tri[4 * i], lb = R.tri[4 * i + 1], lc = R.tri[4 * i + 2];
            w = R.tri[4 * i + 3];
            a = la * el.loc[e] + lb * el.loc[2 * ne + e] + lc * el.loc[4 * ne + e];
            b = la * el.loc[ne + e] + lb * el.loc[3 * ne + e] + lc * el.loc[5 * ne + e];
        } else {
            const double x = R.rect[4 * i], y = R.rect[4 * i + 1];
            w = R.rect[4 * i + 2];
            a = x * el.loc[e] + y * el.loc[2 * ne + e];
            b = x * el.loc[ne + e];
        }
        const double g = fma(a, a, b * b);
        if constexpr (MIXED) s.nd[k] = make_float4((float)a, (float)b, (float)g, (float)w);
        else s.nd[k] = make_double4(a, b, g, w);
    }
}

// ------------------------------------------------------------ far field: sums -------
// kFarField: per point phi, Ex, Ey, Ez.  kFarGrad: the field gradient dE_i/dx_j as xx, yy,
// zz, xy, xz, yz (each point charge contributes q (delta_ij r^2 - 3 d_i d_j) / r^5).
// kFarPhi: the potential only (collocation).
enum FarMode { kFarField = 0, kFarGrad = 1, kFarPhi = 2 };

template <int MODE>
struct Sums {
    static constexpr int kOut = MODE == kFarGrad ? 6 : (MODE == kFarField ? 4 : 1);   // outputs per point
    static constexpr int kNode = MODE == kFarGrad ? 7 : (MODE == kFarField ? 4 : 1);  // element sums per point
};

// Field points of one lane and their FP64 accumulators.
template <int PPT, int MODE>
struct PointSet {
    double x[PPT], y[PPT], z[PPT];
    bool valid[PPT];
    uint32_t idx[PPT];
    double acc[Sums<MODE>::kOut][PPT];
};

// Offsets of the lane's points from the element in hand, in its frame.
template <int PPT, typename T>
struct Local {
    T p1[PPT], p2[PPT], p3[PPT], h[PPT];  // h = p3^2
    T q1[PPT], q2[PPT], H[PPT];           // -2 p1, -2 p2, |p|^2 (expanded r^2 only)
};

// Runs term(i) for the nodes i = 0 .. n-1 of one element.  Long rules (and run-time
// counts) go in groups of four with a separate remainder: this keeps the accumulators in
// place, where an unrolled loop with a remainder makes the compiler copy them every
// iteration.  The short rules of the distance-ratio levels use a plain unrolled loop.
template <int NN, typename Term>
__device__ __forceinline__ void for_nodes(int n, Term term)
{
    if (NN > 0 && NN < 32) {
#pragma unroll 4
        for (int i = 0; i < n; ++i) term(i);
        return;
    }
    int i = 0;
#pragma unroll 1
    for (; i + 4 <= n; i += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) term(i + u);
    }
    for (; i < n; ++i) term(i);
}

// Element sums in the frame, per field point (unit element charge).  EXP: r^2 expanded;
// otherwise from the differences da = p1 - a, db = p2 - b (the gradient).
//   kFarField  (sum w/r, sum w a/r^3, sum w b/r^3, sum w/r^3) expanded, the field's in-plane
//              parts following as p1 sum w/r^3 - sum w a/r^3 and likewise for b;
//              (sum w/r, sum w da/r^3, sum w db/r^3, sum w/r^3) from differences;
//   kFarGrad   FP64: (sum w/r^3, sum w/r^5, sum w da/r^5, sum w db/r^5, sum w da^2/r^5,
//              sum w db^2/r^5, sum w da db/r^5), turned into the local tensor after the loop;
//              FP32: the local tensor itself, sum w/r^3 and sum w u_i u_j / r^3 over the unit
//              offset u = (da, db, p3)/r (xx, yy, zz, xy, xz, yz), so that no power of 1/r
//              above the third is formed in single precision;
//   kFarPhi    sum w/r.
template <int PPT, int MODE, bool EXP>
__device__ __forceinline__ void node_term64(const double4 Q, const Local<PPT, double>& L,
                                            double (&o)[Sums<MODE>::kNode][PPT])
{
    const double a = Q.x, b = Q.y, g = Q.z, w = Q.w;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if constexpr (MODE != kFarGrad) {
            double ri, ca, cb;  // ca, cb: a, b (expanded) or da, db
            if constexpr (EXP) {
                ri = rsqrt64(fma(L.q1[k], a, fma(L.q2[k], b, L.H[k] + g)));
                ca = a;
                cb = b;
            } else {
                ca = L.p1[k] - a;
                cb = L.p2[k] - b;
                ri = rsqrt64(fma(ca, ca, fma(cb, cb, L.h[k])));
            }
            if constexpr (MODE == kFarPhi) {
                o[0][k] = fma(w, ri, o[0][k]);
            } else {
                const double wr = w * ri;
                const double w3 = wr * (ri * ri);
                o[0][k] += wr;
                o[1][k] = fma(w3, ca, o[1][k]);
                o[2][k] = fma(w3, cb, o[2][k]);
                o[3][k] += w3;
            }
        } else {
            const double da = L.p1[k] - a, db = L.p2[k] - b;
            const double ri = rsqrt64(fma(da, da, fma(db, db, L.h[k])));
            const double ri2 = ri * ri;
            const double w3 = (w * ri) * ri2;
            const double w5 = w3 * ri2;
            const double ua = w5 * da, ub = w5 * db;
            o[0][k] += w3;
            o[1][k] += w5;
            o[2][k] += ua;
            o[3][k] += ub;
            o[4][k] = fma(ua, da, o[4][k]);
            o[5][k] = fma(ub, db, o[5][k]);
            o[6][k] = fma(ua, db, o[6][k]);
        }
    }
}

template <int PPT, int MODE, bool EXP>
__device__ __forceinline__ void node_term32(const float4 Q, const Local<PPT, float>& L,
                                            float (&o)[Sums<MODE>::kNode][PPT])
{
    const float a = Q.x, b = Q.y, g = Q.z, w = Q.w;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if constexpr (MODE != kFarGrad) {
            float ri, ca, cb;
            if constexpr (EXP) {
                ri = rsqrt32(fmaf(L.q1[k], a, fmaf(L.q2[k], b, L.H[k] + g)));
                ca = a;
                cb = b;
            } else {
                ca = L.p1[k] - a;
                cb = L.p2[k] - b;
                ri = rsqrt32(fmaf(ca, ca, fmaf(cb, cb, L.h[k])));
            }
            if constexpr (MODE == kFarPhi) {
                o[0][k] = fmaf(w, ri, o[0][k]);
            } else {
                const float wr = w * ri;
                const float w3 = wr * (ri * ri);
                o[0][k] += wr;
                o[1][k] = fmaf(w3, ca, o[1][k]);
                o[2][k] = fmaf(w3, cb, o[2][k]);
                o[3][k] += w3;
            }
        } else {
            const float da = L.p1[k] - a, db = L.p2[k] - b;
            const float ri = rsqrt32(fmaf(da, da, fmaf(db, db, L.h[k])));
            const float w3 = (w * ri) * (ri * ri);
            const float va = da * ri, vb = db * ri, vc = L.p3[k] * ri;
            const float ua = w3 * va, ub = w3 * vb, uc = w3 * vc;
            o[0][k] += w3;
            o[1][k] = fmaf(ua, va, o[1][k]);
            o[2][k] = fmaf(ub, vb, o[2][k]);
            o[3][k] = fmaf(uc, vc, o[3][k]);
            o[4][k] = fmaf(ua, vb, o[4][k]);
            o[5][k] = fmaf(ua, vc, o[5][k]);
            o[6][k] = fmaf(ub, vc, o[6][k]);
        }
    }
}

// Tensor rule in groups of G nodes with the same b: per group the lane forms db and
// (p2 - b)^2 + p3^2 once; per node one difference remains.  Field: the b-component and
// sum w/r^3 are gathered per group.  Gradient (the FP64 sums of node_term64): sum w/r^5
// and sum w da/r^5 are gathered per group, and the sums with db follow from them.
template <int G, int PPT, int MODE>
__device__ __forceinline__ void group_sum64(const double4* t, int base, const Local<PPT, double>& L,
                                            double (&o)[Sums<MODE>::kNode][PPT])
{
#pragma unroll 1
    for (int g = 0; g < G; ++g) {
        const int n0 = base + g * G;
        const double b = t[n0].y;
        double db[PPT], B[PPT], sg[PPT], xg[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            db[k] = L.p2[k] - b;
            B[k] = fma(db[k], db[k], L.h[k]);
            sg[k] = 0.0;
            xg[k] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const double a = t[n0 + i].x, w = t[n0 + i].w;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const double da = L.p1[k] - a;
                const double ri = rsqrt64(fma(da, da, B[k]));
                if constexpr (MODE == kFarPhi) {
                    o[0][k] = fma(w, ri, o[0][k]);
                } else if constexpr (MODE == kFarField) {
                    const double wr = w * ri;
                    const double w3 = wr * (ri * ri);
                    o[0][k] += wr;
                    o[1][k] = fma(w3, da, o[1][k]);
                    sg[k] += w3;
                } else {
                    const double ri2 = ri * ri;
                    const double w3 = (w * ri) * ri2;
                    const double w5 = w3 * ri2;
                    const double ua = w5 * da;
                    o[0][k] += w3;
                    sg[k] += w5;
                    xg[k] += ua;
                    o[4][k] = fma(ua, da, o[4][k]);
                }
            }
        }
        if constexpr (MODE == kFarField) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                o[2][k] = fma(sg[k], db[k], o[2][k]);
                o[3][k] += sg[k];
            }
        } else if constexpr (MODE == kFarGrad) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const double u = sg[k] * db[k];  // sum w db / r^5 of the group
                o[1][k] += sg[k];
                o[2][k] += xg[k];
                o[3][k] += u;
                o[5][k] = fma(u, db[k], o[5][k]);
                o[6][k] = fma(xg[k], db[k], o[6][k]);
            }
        }
    }
}

template <int G, int PPT, int MODE>
__device__ __forceinline__ void group_sum32(const float4* t, int base, const Local<PPT, float>& L,
                                            float (&o)[Sums<MODE>::kNode][PPT])
{
    static_assert(MODE != kFarGrad, "the gradient takes the node-by-node form");
#pragma unroll 1
    for (int g = 0; g < G; ++g) {
        const int n0 = base + g * G;
        const float b = t[n0].y;
        float db[PPT], B[PPT], sg[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            db[k] = L.p2[k] - b;
            B[k] = fmaf(db[k], db[k], L.h[k]);
            sg[k] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const float4 Q = t[n0 + i];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const float da = L.p1[k] - Q.x;
                const float ri = rsqrt32(fmaf(da, da, B[k]));
                if constexpr (MODE == kFarPhi) {
                    o[0][k] = fmaf(Q.w, ri, o[0][k]);
                } else {
                    const float wr = Q.w * ri;
                    const float w3 = wr * (ri * ri);
                    o[0][k] += wr;
                    o[1][k] = fmaf(w3, da, o[1][k]);
                    sg[k] += w3;
                }
            }
        }
        if constexpr (MODE == kFarField) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                o[2][k] = fmaf(sg[k], db[k], o[2][k]);
                o[3][k] += sg[k];
            }
        }
    }
}

// Sums of one element over its nodes [base, base + n) of the tile (Eq. 4.1, unit element
// charge) in the precision T of the tile (FP64, or FP32 for the mixed path).  NN > 0:
// compile-time node count; G > 0: tensor rule in groups of G.  Gradient: the result is the
// local tensor (sum w/r^3; sum w d_i d_j / r^5 for xx, yy, zz, xy, xz, yz, d = (da, db, p3)).
template <int NN, int G, bool MIXED, int PPT, int MODE, bool EXP, typename Lds, typename T>
__device__ __forceinline__ void element_sum(const Lds& s, int base, int n, const Local<PPT, T>& L,
                                            T (&o)[Sums<MODE>::kNode][PPT])
{
    constexpr int S = Sums<MODE>::kNode;
    T r[S][PPT];
#pragma unroll
    for (int c = 0; c < S; ++c)
#pragma unroll
        for (int k = 0; k < PPT; ++k) r[c][k] = T(0);
    const int nn = NN > 0 ? NN : n;
    constexpr bool GROUPS = G > 0 && (MODE != kFarGrad || !MIXED);
    if constexpr (!MIXED) {
        if constexpr (GROUPS) group_sum64<G, PPT, MODE>(s.nd, base, L, r);
        else for_nodes<NN>(nn, [&](int i) { node_term64<PPT, MODE, EXP>(s.nd[base + i], L, r); });
    } else {
        if constexpr (GROUPS) group_sum32<G, PPT, MODE>(s.nd, base, L, r);
        else for_nodes<NN>(nn, [&](int i) { node_term32<PPT, MODE, EXP>(s.nd[base + i], L, r); });
    }
    if constexpr (MODE == kFarField && EXP && !GROUPS) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            o[0][k] = r[0][k];
            o[1][k] = fma(L.p1[k], r[3][k], -r[1][k]);
            o[2][k] = fma(L.p2[k], r[3][k], -r[2][k]);
            o[3][k] = r[3][k];
        }
    } else if constexpr (MODE == kFarGrad && !MIXED) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            o[0][k] = r[0][k];
            o[1][k] = r[4][k];
            o[2][k] = r[5][k];
            o[3][k] = L.h[k] * r[1][k];
            o[4][k] = r[6][k];
            o[5][k] = L.p3[k] * r[2][k];
            o[6][k] = L.p3[k] * r[3][k];
        }
    } else {
#pragma unroll
        for (int c = 0; c < S; ++c)
#pragma unroll
            for (int k = 0; k < PPT; ++k) o[c][k] = r[c][k];
    }
}

// Offsets of the lane's points from element j of the tile: D^2 in FP64 (the distance test,
// Sec. 2) and the coordinates in the element's frame, in the precision of the node sums;
// EXP: with -2 p and |p|^2 for the expanded r^2; H2: with p3^2 (differences, rows).
template <bool EXP, bool H2 = !EXP, int PPT, typename Lds, typename T>
__device__ __forceinline__ void to_frame(const Lds& s, int j, const double (&x)[PPT], const double (&y)[PPT],
                                         const double (&z)[PPT], double (&D2)[PPT], Local<PPT, T>& L)
{
    const double cx = s.cx[j], cy = s.cy[j], cz = s.cz[j];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const double dx = x[k] - cx, dy = y[k] - cy, dz = z[k] - cz;
        D2[k] = fma(dx, dx, fma(dy, dy, dz * dz));
        const T u = (T)dx, v = (T)dy, w = (T)dz;
        L.p1[k] = fma(u, s.f[0][j], fma(v, s.f[1][j], w * s.f[2][j]));
        L.p2[k] = fma(u, s.f[3][j], fma(v, s.f[4][j], w * s.f[5][j]));
        L.p3[k] = fma(u, s.f[6][j], fma(v, s.f[7][j], w * s.f[8][j]));
        if constexpr (EXP) {  // |p|^2 = D^2: the rotation keeps the length (to rounding)
            L.q1[k] = T(-2) * L.p1[k];
            L.q2[k] = T(-2) * L.p2[k];
            L.H[k] = (T)D2[k];
        }
        if constexpr (H2) L.h[k] = L.p3[k] * L.p3[k];
    }
}

// acc += q * (element sums of point k), rotated to the global axes in the precision of the
// sums and accumulated in FP64
template <int PPT, int MODE, typename Lds, typename T>
__device__ __forceinline__ void add_element(PointSet<PPT, MODE>& P, int k, double q, const Lds& s, int j,
                                            const Local<PPT, T>& L, const T (&o)[Sums<MODE>::kNode][PPT])
{
    if constexpr (MODE == kFarField) {
        P.acc[0][k] = fma(q, (double)o[0][k], P.acc[0][k]);
        const T t3 = L.p3[k] * o[3][k];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T e = fma(s.f[c][j], o[1][k], fma(s.f[3 + c][j], o[2][k], s.f[6 + c][j] * t3));
            P.acc[1 + c][k] = fma(q, (double)e, P.acc[1 + c][k]);
        }
    } else {
        // global tensor M = F m F^T of the local one m (F: the frame vectors as columns);
        // dE_i/dx_j = q (delta_ij sum w/r^3 - 3 M_ij)
        const T m[3][3] = { { o[1][k], o[4][k], o[5][k] },
                            { o[4][k], o[2][k], o[6][k] },
                            { o[5][k], o[6][k], o[3][k] } };
        T U[3][3];  // U[a][c] = sum_b m[a][b] f_b[c]
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                U[a][c] = fma(m[a][0], s.f[c][j], fma(m[a][1], s.f[3 + c][j], m[a][2] * s.f[6 + c][j]));
        auto M = [&](int u, int v) -> double {
            return (double)fma(s.f[u][j], U[0][v], fma(s.f[3 + u][j], U[1][v], s.f[6 + u][j] * U[2][v]));
        };
        const double s3 = (double)o[0][k];
#pragma unroll
        for (int c = 0; c < 3; ++c) P.acc[c][k] = fma(q, fma(-3.0, M(c, c), s3), P.acc[c][k]);
        P.acc[3][k] = fma(-3.0 * q, M(0, 1), P.acc[3][k]);
        P.acc[4][k] = fma(-3.0 * q, M(0, 2), P.acc[4][k]);
        P.acc[5][k] = fma(-3.0 * q, M(1, 2), P.acc[5][k]);
    }
}

// group size of the tensor path for a rectangle rule of NN nodes (7 x 7 only)
template <bool TRI, int NN>
constexpr int tensor_group() { return (!TRI && NN == 49) ? 7 : 0; }

// One element kind over [e_begin, e_end) with one rule; NN > 0 is the compile-time node
// count, NN == 0 reads it at run time.
template <int NN, bool TRI, bool MIXED, int PPT, int MODE, typename Lds>
__device__ __forceinline__ void far_eval_range(const FarArgs& a, Lds& s, PointSet<PPT, MODE>& P, int64_t e_begin,
                                               int64_t e_end)
{
    using T = typename Lds::T;
    // the expanded r^2 (node loop without rows; the gradient keeps the differences)
    constexpr bool EXPAND = MODE != kFarGrad && tensor_group<TRI, NN>() == 0;
    const int nn = NN > 0 ? NN : (TRI ? a.rules.nt : a.rules.nr);
    const int TE = tile_elems(nn);
    for (int64_t t0 = e_begin; t0 < e_end; t0 += TE) {
        const int te = (int)min((int64_t)TE, e_end - t0);
        __syncthreads();
        stage_tile<TRI, MIXED>(s, a.el, a.rules, nn, t0, te, a.rhs, 1);
        __syncthreads();
        for (int j = 0; j < te; ++j) {
            const double thr2 = s.thr2[j], q = s.q[0][j];
            double D2[PPT];
            Local<PPT, T> L;
            to_frame<EXPAND>(s, j, P.x, P.y, P.z, D2, L);
            bool nr[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                nr[k] = P.valid[k] && (D2[k] < thr2);
                record_near(nr[k], P.idx[k], (uint32_t)(t0 + j), a.near_list, a.near_cap, a.ctr);
            }
            T o[Sums<MODE>::kNode][PPT];
            element_sum<NN, tensor_group<TRI, NN>(), MIXED, PPT, MODE, EXPAND>(s, j * nn, nn, L, o);
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (!nr[k]) add_element<PPT, MODE>(P, k, q, s, j, L, o);
        }
    }
}

// One element kind with the rule chosen by distance ratio (Sec. 4): the staged nodes of an
// element are the four levels back to back; a pair needs level l when D^2 >= c[l] (near_dr
// L)^2 (the last level otherwise).  The wavefront runs the finest level that any of its
// pairs needs, once, for all its lanes: a finer rule is at least as accurate at a larger
// distance ratio, and one level per wavefront costs less than each level a lane needs.
// N0..N3 > 0: compile-time counts.
template <int N0, int N1, int N2, int N3, bool TRI, bool MIXED, int PPT, int MODE, typename Lds>
__device__ __forceinline__ void far_eval_dr_range(const FarArgs& a, Lds& s, PointSet<PPT, MODE>& P, int64_t e_begin,
                                                  int64_t e_end, unsigned long long& terms)
{
    using T = typename Lds::T;
    const int* off = TRI ? a.lv.tri_off : a.lv.rect_off;
    const double* c = TRI ? a.lv.tri_c : a.lv.rect_c;
    const int o1 = off[1], o2 = off[2], o3 = off[3], nn = off[4];
    const double c0 = c[0], c1 = c[1], c2 = c[2];
    const int TE = tile_elems(nn);
    for (int64_t t0 = e_begin; t0 < e_end; t0 += TE) {
        const int te = (int)min((int64_t)TE, e_end - t0);
        __syncthreads();
        stage_tile<TRI, MIXED>(s, a.el, a.lv.tab, nn, t0, te, a.rhs, 1);
        __syncthreads();
        for (int j = 0; j < te; ++j) {
            const double thr2 = s.thr2[j], q = s.q[0][j];
            double D2[PPT];
            Local<PPT, T> L;
            to_frame<MODE != kFarGrad, true>(s, j, P.x, P.y, P.z, D2, L);
            bool nr[PPT];
            int lvl[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                nr[k] = P.valid[k] && (D2[k] < thr2);
                record_near(nr[k], P.idx[k], (uint32_t)(t0 + j), a.near_list, a.near_cap, a.ctr);
                lvl[k] = D2[k] >= c0 * thr2 ? 0 : (D2[k] >= c1 * thr2 ? 1 : (D2[k] >= c2 * thr2 ? 2 : 3));
                if (nr[k] || !P.valid[k]) lvl[k] = -1;  // contributes nothing
            }
            // the finest level any lane of the wavefront needs
            int mx = -1;
#pragma unroll
            for (int k = 0; k < PPT; ++k) mx = max(mx, lvl[k]);
            const int wl = __ballot(mx >= 3) ? 3 : (__ballot(mx >= 2) ? 2 : (__ballot(mx >= 1) ? 1 : (__ballot(mx >= 0) ? 0 : -1)));
            if (wl < 0) continue;
            T o[Sums<MODE>::kNode][PPT];
            const int b = j * nn;
            int nw;
            constexpr bool X = MODE != kFarGrad;
            if (wl == 0) { element_sum<N0, 0, MIXED, PPT, MODE, X>(s, b, o1, L, o); nw = o1; }
            else if (wl == 1) { element_sum<N1, 0, MIXED, PPT, MODE, X>(s, b + o1, o2 - o1, L, o); nw = o2 - o1; }
            else if (wl == 2) { element_sum<N2, 0, MIXED, PPT, MODE, X>(s, b + o2, o3 - o2, L, o); nw = o3 - o2; }
            else {
                element_sum<N3, tensor_group<TRI, N3>(), MIXED, PPT, MODE, X>(s, b + o3, nn - o3, L, o);
                nw = nn - o3;
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (lvl[k] >= 0) {
                    add_element<PPT, MODE>(P, k, q, s, j, L, o);
                    terms += (unsigned)nw;
                }
        }
    }
}

__device__ __forceinline__ void add_terms(unsigned long long terms, DevCounters* ctr)
{
    // wavefront sum, one atomic per wavefront
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned lo = __shfl_xor((unsigned)terms, o);
        const unsigned hi = __shfl_xor((unsigned)(terms >> 32), o);
        terms += ((unsigned long long)hi << 32) | lo;
    }
    if (lane_id() == 0 && terms) atomicAdd(&ctr->node_ints, terms);
}

// DR == false: one rule per kind, NT / NR nodes.  DR == true: levels (T0..T3 / R0..R3).
// GRAD: field gradient instead of potential and field.
template <bool DR, int NT, int NR, int T1, int T2, int T3, int R1, int R2, int R3, bool MIXED, int PPT, bool GRAD>
__global__ __launch_bounds__(kBlock) void far_eval_kernel(FarArgs a)
{
    constexpr int MODE = GRAD ? kFarGrad : kFarField;
    constexpr int NO = Sums<MODE>::kOut;
    __shared__ TileLds<MIXED, 1> s;
    PointSet<PPT, MODE> P;
    const int64_t base = (int64_t)blockIdx.x * (kBlock * PPT) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t p = base + (int64_t)k * kBlock;
        P.valid[k] = p < a.n;
        P.idx[k] = (uint32_t)p;
        P.x[k] = P.valid[k] ? a.pts[p] : 0.0;
        P.y[k] = P.valid[k] ? a.pts[a.n + p] : 0.0;
        P.z[k] = P.valid[k] ? a.pts[2 * a.n + p] : 0.0;
#pragma unroll
        for (int c = 0; c < NO; ++c) P.acc[c][k] = 0.0;
    }
    int64_t e_lo = a.elem_begin, e_hi = a.elem_end;
    if (a.n_split > 1) {
        e_lo = min(a.elem_begin + (int64_t)blockIdx.y * a.chunk, a.elem_end);
        e_hi = min(e_lo + a.chunk, a.elem_end);
    }
    const int64_t nt_end = min((int64_t)a.el.n_tri, e_hi);
    const int64_t nr_begin = max((int64_t)a.el.n_tri, e_lo);
    if (DR) {
        unsigned long long terms = 0;
        if (e_lo < nt_end) far_eval_dr_range<NT, T1, T2, T3, true, MIXED, PPT, MODE>(a, s, P, e_lo, nt_end, terms);
        if (nr_begin < e_hi) far_eval_dr_range<NR, R1, R2, R3, false, MIXED, PPT, MODE>(a, s, P, nr_begin, e_hi, terms);
        add_terms(terms, a.ctr);
    } else {
        if (e_lo < nt_end) far_eval_range<NT, true, MIXED, PPT, MODE>(a, s, P, e_lo, nt_end);
        if (nr_begin < e_hi) far_eval_range<NR, false, MIXED, PPT, MODE>(a, s, P, nr_begin, e_hi);
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (!P.valid[k]) continue;
        const int64_t p = base + (int64_t)k * kBlock;
        if (a.partial) {  // element-split launch: unscaled partial sums, reduced later in fixed order
            double* o = a.partial + (int64_t)blockIdx.y * NO * a.n;
#pragma unroll
            for (int c = 0; c < NO; ++c) o[c * a.n + p] = P.acc[c][k];
        } else if (GRAD) {
#pragma unroll
            for (int c = 0; c < NO; ++c) a.G[c * a.n + p] = a.K * P.acc[c][k];
        } else {
            a.phi[p] = a.K * P.acc[0][k];
            if (a.E) {
                a.E[p] = a.K * P.acc[1][k];
                a.E[a.n + p] = a.K * P.acc[2][k];
                a.E[2 * a.n + p] = a.K * P.acc[3][k];
            }
        }
    }
}

// ------------------------------------------------------- far field: collocation -----
template <int NN, bool TRI, bool MIXED, int PPT, typename Lds>
__device__ __forceinline__ void far_colloc_range(const FarArgs& a, Lds& s, const double (&px)[PPT],
                                                 const double (&py)[PPT], const double (&pz)[PPT],
                                                 const bool (&valid)[PPT], const uint32_t (&idx)[PPT],
                                                 double (&acc)[PPT][kMaxRhs], int64_t e_begin, int64_t e_end)
{
    using T = typename Lds::T;
    constexpr bool EXPAND = tensor_group<TRI, NN>() == 0;
    const int nn = NN > 0 ? NN : (TRI ? a.rules.nt : a.rules.nr);
    const int TE = tile_elems(nn);
    const int nrhs = a.n_rhs;
    for (int64_t t0 = e_begin; t0 < e_end; t0 += TE) {
        const int te = (int)min((int64_t)TE, e_end - t0);
        __syncthreads();
        stage_tile<TRI, MIXED>(s, a.el, a.rules, nn, t0, te, 0, nrhs);
        __syncthreads();
        for (int j = 0; j < te; ++j) {
            const double thr2 = s.thr2[j];
            double D2[PPT];
            Local<PPT, T> L;
            to_frame<EXPAND>(s, j, px, py, pz, D2, L);
            bool nr[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                nr[k] = valid[k] && (D2[k] < thr2);
                record_near(nr[k], idx[k], (uint32_t)(t0 + j), a.near_list, a.near_cap, a.ctr);
            }
            T o[1][PPT];
            element_sum<NN, tensor_group<TRI, NN>(), MIXED, PPT, kFarPhi, EXPAND>(s, j * nn, nn, L, o);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!nr[k]) {
                    const double v = (double)o[0][k];
#pragma unroll
                    for (int r = 0; r < kMaxRhs; ++r)
                        if (r < nrhs) acc[k][r] = fma(s.q[r][j], v, acc[k][r]);
                }
            }
        }
    }
}

template <int NT, int NR, bool MIXED, int PPT>
__global__ __launch_bounds__(kBlock) void far_colloc_kernel(FarArgs a)
{
    __shared__ TileLds<MIXED, kMaxRhs> s;
    const int64_t ne = a.el.ne;
    const int64_t base = (int64_t)blockIdx.x * (kBlock * PPT) + threadIdx.x;
    double px[PPT], py[PPT], pz[PPT];
    bool valid[PPT];
    uint32_t idx[PPT];
    double acc[PPT][kMaxRhs];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t p = base + (int64_t)k * kBlock;
        valid[k] = p < ne;
        idx[k] = (uint32_t)p;
        px[k] = valid[k] ? a.el.cen[p] : 0.0;
        py[k] = valid[k] ? a.el.cen[ne + p] : 0.0;
        pz[k] = valid[k] ? a.el.cen[2 * ne + p] : 0.0;
#pragma unroll
        for (int r = 0; r < kMaxRhs; ++r) acc[k][r] = 0.0;
    }
    int64_t e_lo = 0, e_hi = ne;
    if (a.n_split > 1) {
        e_lo = min((int64_t)blockIdx.y * a.chunk, ne);
        e_hi = min(e_lo + a.chunk, ne);
    }
    const int64_t nt = a.el.n_tri;
    const int64_t t_hi = min(nt, e_hi);
    if (e_lo < t_hi) far_colloc_range<NT, true, MIXED, PPT>(a, s, px, py, pz, valid, idx, acc, e_lo, t_hi);
    const int64_t r_lo = max(nt, e_lo);
    if (r_lo < e_hi) far_colloc_range<NR, false, MIXED, PPT>(a, s, px, py, pz, valid, idx, acc, r_lo, e_hi);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (!valid[k]) continue;
        const int64_t p = base + (int64_t)k * kBlock;
        if (a.partial) {  // element chunk blockIdx.y: unscaled partial sums [split][rhs][ne]
            double* o = a.partial + (int64_t)blockIdx.y * a.n_rhs * ne;
#pragma unroll
            for (int r = 0; r < kMaxRhs; ++r)
                if (r < a.n_rhs) o[(int64_t)r * ne + p] = acc[k][r];
        } else {
#pragma unroll
            for (int r = 0; r < kMaxRhs; ++r)
                if (r < a.n_rhs) a.phi[(int64_t)r * ne + p] = a.K * acc[k][r];
        }
    }
}

// --------------------------------------------------------------- near field ---------
struct NearState {
    int kind;        // 0 triangle, 1 rectangle
    int level;       // 0 = the element itself
    int i, j;        // lattice position at this level
    bool up;         // triangle orientation (up: vertices (i,j),(i+1,j),(i,j+1))
};

// Index of a child within its parent and the parent's lattice position.
__device__ __forceinline__ int child_index(NearState& s)
{
    const int a = s.i & 1, b = s.j & 1;
    int c;
    bool pup = true;
    if (s.kind == 1) {
        c = a + 2 * b;
    } else if (s.up) {
        if (a && b) { pup = false; c = 3; }
        else c = a ? 1 : (b ? 2 : 0);
    } else {
        if (!a && !b) { pup = true; c = 3; }
        else { pup = false; c = (a && b) ? 0 : (b ? 1 : 2); }
    }
    s.i >>= 1;
    s.j >>= 1;
    s.up = pup;
    s.level -= 1;
    return c;
}

// Child c of the node s (s becomes the child).
__device__ __forceinline__ void to_child(NearState& s, int c)
{
    const int i2 = 2 * s.i, j2 = 2 * s.j;
    s.level += 1;
    if (s.kind == 1) {
        s.i = i2 + (c & 1);
        s.j = j2 + (c >> 1);
    } else if (s.up) {  // up parent: up(2i,2j), up(2i+1,2j), up(2i,2j+1), down(2i,2j)
        s.i = i2 + (c == 1 ? 1 : 0);
        s.j = j2 + (c == 2 ? 1 : 0);
        s.up = (c != 3);
    } else {  // down parent: down(2i+1,2j+1), down(2i,2j+1), down(2i+1,2j), up(2i+1,2j+1)
        s.i = i2 + (c == 1 ? 0 : 1);
        s.j = j2 + (c == 2 ? 0 : 1);
        s.up = (c == 3);
    }
}

// Move to the next node of the depth-first walk after finishing node s; false when the
// walk has returned to the root.
__device__ __forceinline__ bool advance(NearState& s)
{
    while (s.level > 0) {
        const int c = child_index(s);  // s is now the parent
        if (c < 3) {
            to_child(s, c + 1);
            return true;
        }
    }
    return false;
}

// Vertices of a triangle node: root A, edge vectors eB = B - A, eC = C - A.
__device__ __forceinline__ void tri_node_vertices(const NearState& s, const double* A, const double* eB, const double* eC,
                                                  double V[3][3])
{
    const double h = ldexp(1.0, -s.level);
    double u[3], v[3];
    if (s.up) {
        u[0] = s.i; v[0] = s.j; u[1] = s.i + 1; v[1] = s.j; u[2] = s.i; v[2] = s.j + 1;
    } else {
        u[0] = s.i + 1; v[0] = s.j + 1; u[1] = s.i; v[1] = s.j + 1; u[2] = s.i + 1; v[2] = s.j;
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double uh = u[m] * h, vh = v[m] * h;
#pragma unroll
        for (int c = 0; c < 3; ++c) V[m][c] = fma(uh, eB[c], fma(vh, eC[c], A[c]));
    }
}

// Point-charge terms of one Gaussian point at offset r from the field point (unit weight
// w): field mode f = (w/r, w r/r^3); gradient mode f = (w/r^3, w r_i r_j / r^5 for xx, yy,
// zz, xy, xz, yz).
template <bool GRAD>
__device__ __forceinline__ void leaf_terms(double w, double rx, double ry, double rz, double (&f)[7])
{
    const double ri = rsqrt64(fma(rx, rx, fma(ry, ry, rz * rz)));
    const double wr = w * ri;
    if (!GRAD) {
        const double w3 = wr * ri * ri;
        f[0] += wr; f[1] = fma(w3, rx, f[1]); f[2] = fma(w3, ry, f[2]); f[3] = fma(w3, rz, f[3]);
    } else {
        const double ri2 = ri * ri, w3 = wr * ri2, w5 = w3 * ri2;
        const double ux = w5 * rx, uy = w5 * ry, uz = w5 * rz;
        f[0] += w3;
        f[1] = fma(ux, rx, f[1]); f[2] = fma(uy, ry, f[2]); f[3] = fma(uz, rz, f[3]);
        f[4] = fma(ux, ry, f[4]); f[5] = fma(ux, rz, f[5]); f[6] = fma(uy, rz, f[6]);
    }
}

// MODE: kNearEval (phi, E at field points), kNearColloc (phi at centroids, several density
// vectors), kNearGrad (field gradient at field points; NaN for a point on its element).
template <int MODE>
__global__ __launch_bounds__(kBlock) void near_kernel(NearArgs a)
{
    constexpr bool COLLOC = MODE == kNearColloc;
    constexpr bool GRAD = MODE == kNearGrad;
    const Elements& el = a.el;
    const int64_t ne = el.ne;
    const unsigned long long total = min(a.ctr->near_count, a.near_cap);
    const int lane = lane_id();

    unsigned long long n_leaves = 0, n_cap = 0, n_on = 0, n_limit = 0;
    int max_level = 0;

    bool active = false;
    NearState st{ 0, 0, 0, 0, true };
    uint32_t p = 0, e = 0;
    unsigned long long cur = 0;  // result slot of the pair in hand
    double P[3] = { 0, 0, 0 }, g0[3] = { 0, 0, 0 }, g1[3] = { 0, 0, 0 }, g2[3] = { 0, 0, 0 };
    double thr2 = 0.0, acc[6] = { 0, 0, 0, 0, 0, 0 };
    int64_t visits = 0;

    while (true) {
        // ---- refill: one atomic per wavefront for all lanes that need a pair
        const unsigned long long need = __ballot(!active);
        if (need) {
            const int first = __ffsll((long long)need) - 1;
            unsigned long long b = 0;
            if (lane == first) b = atomicAdd(&a.ctr->cursor, (unsigned long long)__popcll(need));
            b = bcast_u64(b, first);
            if (!active) {
                const unsigned long long w = b + lanes_below(need);
                if (w >= total) break;
                cur = a.slot[w];
                const NearPair pr = a.near_list[w];
                p = pr.point;
                e = pr.elem;
                if (COLLOC) {
                    P[0] = el.cen[p]; P[1] = el.cen[ne + p]; P[2] = el.cen[2 * ne + p];
                } else {
                    P[0] = a.pts[p]; P[1] = a.pts[a.n + p]; P[2] = a.pts[2 * a.n + p];
                }
                st.kind = (int64_t)e < el.n_tri ? 0 : 1;
                // Work relative to the element's first vertex (A or P0): P - Q is then formed
                // from numbers of the element's size, which keeps points very close to a small
                // element far from the origin accurate.
                double G[9];
#pragma unroll
                for (int c = 0; c < 9; ++c) G[c] = el.geom[(int64_t)c * ne + e];
#pragma unroll
                for (int c = 0; c < 3; ++c) P[c] -= G[c];
                if (st.kind == 0) {  // origin at A; edges B - A, C - A
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        g0[c] = 0.0; g1[c] = G[3 + c] - G[c]; g2[c] = G[6 + c] - G[c];
                        G[3 + c] = g1[c]; G[6 + c] = g2[c]; G[c] = 0.0;
                    }
                } else {             // origin at P0; sides e1, e2
#pragma unroll
                    for (int c = 0; c < 3; ++c) { g0[c] = 0.0; g1[c] = G[3 + c]; g2[c] = G[6 + c]; }
                }
                thr2 = el.thr2[e];
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] = 0.0;
                visits = 0;
                active = true;
                st.level = 0; st.i = 0; st.j = 0; st.up = true;

                // ---- point on the element: exact polar integral about the point
                const double L = el.L[e];
                const double nx = el.nrm[e], ny = el.nrm[ne + e], nz = el.nrm[2 * ne + e];
                const double dx = P[0] - (el.cen[e] - el.geom[e]);
                const double dy = P[1] - (el.cen[ne + e] - el.geom[ne + e]);
                const double dz = P[2] - (el.cen[2 * ne + e] - el.geom[2 * ne + e]);
                bool on = fabs(nx * dx + ny * dy + nz * dz) <= 1e-12 * L;
                double V[4][3];
                int nv;
                if (st.kind == 0) {
                    nv = 3;
#pragma unroll
                    for (int c = 0; c < 3; ++c) { V[0][c] = G[c]; V[1][c] = G[3 + c]; V[2][c] = G[6 + c]; V[3][c] = 0.0; }
                } else {
                    nv = 4;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        V[0][c] = 0.0; V[1][c] = G[3 + c];
                        V[2][c] = G[3 + c] + G[6 + c]; V[3][c] = G[6 + c];
                    }
                }
                if (on) {  // inside test
                    if (st.kind == 0) {
                        const double twoA = 2.0 * el.area[e];
                        for (int k = 0; k < 3 && on; ++k) {
                            const double* Va = V[(k + 1) % 3];
                            const double* Vb = V[(k + 2) % 3];
                            const double ax = Va[0] - P[0], ay = Va[1] - P[1], az = Va[2] - P[2];
                            const double bx = Vb[0] - P[0], by = Vb[1] - P[1], bz = Vb[2] - P[2];
                            const double cxp = ay * bz - az * by, cyp = az * bx - ax * bz, czp = ax * by - ay * bx;
                            on = (nx * cxp + ny * cyp + nz * czp) / twoA >= -1e-12;
                        }
                    } else {
                        const double x = 2.0 * (dx * G[3] + dy * G[4] + dz * G[5]) / (G[3] * G[3] + G[4] * G[4] + G[5] * G[5]);
                        const double y = 2.0 * (dx * G[6] + dy * G[7] + dz * G[8]) / (G[6] * G[6] + G[7] * G[7] + G[8] * G[8]);
                        on = fabs(x) <= 1.0 + 1e-12 && fabs(y) <= 1.0 + 1e-12;
                    }
                }
                if (on) {
                    // per edge at distance h with end offsets t1, t2 (rho^2 = h^2 + t^2):
                    //   potential h [asinh(t/h)],  field -n [(t/rho)(1 + ln rho) - asinh(t/h)] + h t [(1 + ln rho)/rho]
                    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                    for (int k = 0; k < nv; ++k) {
                        const double* Va = V[k];
                        const double* Vb = V[(k + 1) % nv];
                        double tv[3] = { Vb[0] - Va[0], Vb[1] - Va[1], Vb[2] - Va[2] };
                        const double len = sqrt(tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]);
                        tv[0] /= len; tv[1] /= len; tv[2] /= len;
                        const double pa[3] = { Va[0] - P[0], Va[1] - P[1], Va[2] - P[2] };
                        const double t1 = pa[0] * tv[0] + pa[1] * tv[1] + pa[2] * tv[2];
                        const double t2 = t1 + len;
                        double fn[3] = { pa[0] - t1 * tv[0], pa[1] - t1 * tv[1], pa[2] - t1 * tv[2] };
                        const double hh = sqrt(fn[0] * fn[0] + fn[1] * fn[1] + fn[2] * fn[2]);
                        if (!(hh > 1e-14 * L)) continue;
                        fn[0] /= hh; fn[1] /= hh; fn[2] /= hh;
                        const double r1 = sqrt(hh * hh + t1 * t1), r2 = sqrt(hh * hh + t2 * t2);
                        const double as = asinh(t2 / hh) - asinh(t1 / hh);
                        s0 += hh * as;
                        const double l1 = 1.0 + log(r1), l2 = 1.0 + log(r2);
                        const double gn = (t2 / r2) * l2 - (t1 / r1) * l1 - as;
                        const double gt = hh * (l2 / r2 - l1 / r1);
                        s1 += -gn * fn[0] + gt * tv[0];
                        s2 += -gn * fn[1] + gt * tv[1];
                        s3 += -gn * fn[2] + gt * tv[2];
                    }
                    const double inv_area = 1.0 / el.area[e];
                    acc[0] = s0 * inv_area; acc[1] = s1 * inv_area; acc[2] = s2 * inv_area; acc[3] = s3 * inv_area;
                    if (GRAD) {  // the normal field jumps across the element: no gradient there
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc[c] = __builtin_nan("");
                    }
                    n_on++;
                    active = false;  // finished: fall through to the write-out below
                    st.level = -1;
                } else if (a.max_depth <= 0) {
                    st.level = 0;  // evaluate the rule on the element itself (depth cap)
                } else {
                    st.level = 1; st.i = 0; st.j = 0; st.up = true;  // first child of the root
                }
            }
        }

        bool finished = false;
        if (active) {
            // ---- visit node st
            const double h = ldexp(1.0, -st.level);
            double cen[3];
            double V[3][3];
            if (st.kind == 0) {
                tri_node_vertices(st, g0, g1, g2, V);
#pragma unroll
                for (int c = 0; c < 3; ++c) cen[c] = (V[0][c] + V[1][c] + V[2][c]) * (1.0 / 3.0);
            } else {
                const double ih = st.i * h, jh = st.j * h;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    V[0][c] = fma(ih, g1[c], fma(jh, g2[c], g0[c]));  // corner
                    cen[c] = fma(0.5 * h, g1[c] + g2[c], V[0][c]);
                }
            }
            const double dx = P[0] - cen[0], dy = P[1] - cen[1], dz = P[2] - cen[2];
            const double D2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const bool is_near = D2 < thr2 * h * h;
            ++visits;
            if (st.level > max_level) max_level = st.level;
            if (!is_near || st.level >= a.max_depth || visits > a.visit_limit) {
                // leaf: the element's rule on this node, weights scaled by the area ratio h^2
                double f[7] = { 0, 0, 0, 0, 0, 0, 0 };
                if (st.kind == 0) {
                    for (int i = 0; i < a.rules.nt; ++i) {
                        const double la = a.rules.tri[4 * i], lb = a.rules.tri[4 * i + 1], lc = a.rules.tri[4 * i + 2];
                        const double w = a.rules.tri[4 * i + 3];
                        const double rx = P[0] - (la * V[0][0] + lb * V[1][0] + lc * V[2][0]);
                        const double ry = P[1] - (la * V[0][1] + lb * V[1][1] + lc * V[2][1]);
                        const double rz = P[2] - (la * V[0][2] + lb * V[1][2] + lc * V[2][2]);
                        leaf_terms<GRAD>(w, rx, ry, rz, f);
                    }
                } else {
                    const double hh = 0.5 * h;
                    for (int i = 0; i < a.rules.nr; ++i) {
                        const double x = a.rules.rect[4 * i] * hh, y = a.rules.rect[4 * i + 1] * hh;
                        const double w = a.rules.rect[4 * i + 2];
                        const double rx = P[0] - fma(x, g1[0], fma(y, g2[0], cen[0]));
                        const double ry = P[1] - fma(x, g1[1], fma(y, g2[1], cen[1]));
                        const double rz = P[2] - fma(x, g1[2], fma(y, g2[2], cen[2]));
                        leaf_terms<GRAD>(w, rx, ry, rz, f);
                    }
                }
                const double h2 = h * h;
                if (!GRAD) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] = fma(h2, f[c], acc[c]);
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[c] = fma(h2, fma(-3.0, f[1 + c], f[0]), acc[c]);
#pragma unroll
                    for (int c = 3; c < 6; ++c) acc[c] = fma(-3.0 * h2, f[1 + c], acc[c]);
                }
                n_leaves++;
                if (is_near) n_cap++;
                if (visits > a.visit_limit) {
                    n_limit++;
                    finished = true;
                } else {
                    finished = !advance(st);
                }
            } else {
                to_child(st, 0);
            }
        } else if (st.level == -1) {
            finished = true;  // on-element pair completed during refill
        }

        if (finished) {
            // the pair's own result slot(s); collocation keeps the unit-density potential
            // (the densities are applied per right-hand side when the sums are formed)
            const unsigned long long S = a.res_stride;
            if (COLLOC) {
                a.res[cur] = acc[0];
            } else {
                const double Kq = a.K * el.q[(int64_t)a.rhs * ne + e];
#pragma unroll
                for (int c = 0; c < (GRAD ? 6 : 4); ++c) a.res[c * S + cur] = Kq * acc[c];
            }
            active = false;
            st.level = 0;
        }
    }

    // per-lane counters -> one atomic per counter per lane that has something to add
    if (n_leaves) atomicAdd(&a.ctr->leaves, n_leaves);
    if (n_cap) atomicAdd(&a.ctr->cap_hits, n_cap);
    if (n_on) atomicAdd(&a.ctr->on_surface, n_on);
    if (n_limit) atomicAdd(&a.ctr->visit_limit_hits, n_limit);
    if (max_level) atomicMax(&a.ctr->max_depth, (unsigned long long)max_level);
}

// ---------------------------------------------------------------- small kernels -----
__global__ void charges_kernel(const double* sigma, const double* area, double* q, int64_t ne, int n_rhs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne * n_rhs) return;
    q[i] = sigma[i] * area[i % ne];
}

__global__ void reduce_split_kernel(const double* partial, int n_split, int64_t n, double K, double* phi, double* E)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double s[4] = { 0, 0, 0, 0 };
    for (int k = 0; k < n_split; ++k)  // fixed order: independent of timing
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c] += partial[((int64_t)k * 4 + c) * n + p];
    phi[p] = K * s[0];
    if (E) {
        E[p] = K * s[1];
        E[n + p] = K * s[2];
        E[2 * n + p] = K * s[3];
    }
}

// out[m][p] = K * sum over the element chunks k (fixed order) of partial[k][m][p]
__global__ void reduce_chunks_kernel(const double* partial, int n_split, int64_t rows, int64_t n, double K,
                                     double* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * n) return;
    double s = 0.0;
    for (int k = 0; k < n_split; ++k) s += partial[(int64_t)k * rows * n + i];
    out[i] = K * s;
}

__global__ void zero_counters_kernel(DevCounters* c)
{
    unsigned long long* w = reinterpret_cast<unsigned long long*>(c);
    const int i = threadIdx.x;
    if (i < (int)(sizeof(DevCounters) / sizeof(unsigned long long))) w[i] = 0ull;
}

template <bool DR, int NT, int NR, int T1, int T2, int T3, int R1, int R2, int R3, bool MIXED, int PPT, bool GRAD>
hipError_t far_eval_launch(const FarArgs& a, hipStream_t s)
{
    const int64_t per = (int64_t)kBlock * PPT;
    const int64_t blocks = (a.n + per - 1) / per;
    if (blocks > 0x7fffffff || a.n_split < 1 || a.n_split > 65535) return hipErrorInvalidValue;
    far_eval_kernel<DR, NT, NR, T1, T2, T3, R1, R2, R3, MIXED, PPT, GRAD>
        <<<dim3((unsigned)blocks, (unsigned)a.n_split), dim3(kBlock), 0, s>>>(a);
    return hipGetLastError();
}

// Field points per lane: two for the distance-ratio levels and the run-time rules; for the
// compiled long rules three in FP64 and one in the mixed path (on the 150k-element cylinder
// 1 % and 2 % faster than two; four was slower in both).
template <bool MIXED>
hipError_t far_eval_dispatch(const FarArgs& a, hipStream_t s)
{
    constexpr int PPT = 2;
    constexpr int PPT_LONG = MIXED ? 1 : 3;
    if (a.dr_rules) {
        const int* t = a.lv.tri_off;
        const int* r = a.lv.rect_off;
        const bool std_levels = t[1] == 7 && t[2] == 19 && t[3] == 38 && r[1] == 7 && r[2] == 19 && r[3] == 36;
        if (std_levels && t[4] - t[3] == 33 && r[4] - r[3] == 49)
            return far_eval_launch<true, 7, 7, 12, 19, 33, 12, 17, 49, MIXED, PPT, false>(a, s);
        return far_eval_launch<true, 0, 0, 0, 0, 0, 0, 0, 0, MIXED, PPT, false>(a, s);
    }
    const int nt = a.rules.nt, nr = a.rules.nr;
    if (nr == 49) {
        if (nt == 7) return far_eval_launch<false, 7, 49, 0, 0, 0, 0, 0, 0, MIXED, PPT_LONG, false>(a, s);
        if (nt == 12) return far_eval_launch<false, 12, 49, 0, 0, 0, 0, 0, 0, MIXED, PPT_LONG, false>(a, s);
        if (nt == 19) return far_eval_launch<false, 19, 49, 0, 0, 0, 0, 0, 0, MIXED, PPT_LONG, false>(a, s);
        if (nt == 33) return far_eval_launch<false, 33, 49, 0, 0, 0, 0, 0, 0, MIXED, PPT_LONG, false>(a, s);
    }
    if (nr == 33 && nt == 33)  // Table B5 for the rectangles
        return far_eval_launch<false, 33, 33, 0, 0, 0, 0, 0, 0, MIXED, PPT_LONG, false>(a, s);
    return far_eval_launch<false, 0, 0, 0, 0, 0, 0, 0, 0, MIXED, PPT, false>(a, s);
}

// Gradient: compile-time node counts for the default rules only; one point per lane for
// those in the mixed path (7 % faster than two on the 150k-element cylinder; FP64 is
// fastest with two).
template <bool MIXED>
hipError_t far_grad_dispatch(const FarArgs& a, hipStream_t s)
{
    constexpr int PPT = 2;
    constexpr int PPT_LONG = MIXED ? 1 : 2;
    if (a.dr_rules) {
        const int* t = a.lv.tri_off;
        const int* r = a.lv.rect_off;
        const bool std_levels = t[1] == 7 && t[2] == 19 && t[3] == 38 && r[1] == 7 && r[2] == 19 && r[3] == 36;
        if (std_levels && t[4] - t[3] == 33 && r[4] - r[3] == 49)
            return far_eval_launch<true, 7, 7, 12, 19, 33, 12, 17, 49, MIXED, PPT, true>(a, s);
        return far_eval_launch<true, 0, 0, 0, 0, 0, 0, 0, 0, MIXED, PPT, true>(a, s);
    }
    if (a.rules.nt == 33 && a.rules.nr == 49)
        return far_eval_launch<false, 33, 49, 0, 0, 0, 0, 0, 0, MIXED, PPT_LONG, true>(a, s);
    return far_eval_launch<false, 0, 0, 0, 0, 0, 0, 0, 0, MIXED, PPT, true>(a, s);
}

template <int NT, int NR, bool MIXED, int PPT>
hipError_t far_colloc_launch(const FarArgs& a, hipStream_t s)
{
    const int64_t per = (int64_t)kBlock * PPT;
    const int64_t blocks = (a.el.ne + per - 1) / per;
    if (blocks > 0x7fffffff || a.n_split < 1 || a.n_split > 65535) return hipErrorInvalidValue;
    far_colloc_kernel<NT, NR, MIXED, PPT><<<dim3((unsigned)blocks, (unsigned)a.n_split), dim3(kBlock), 0, s>>>(a);
    return hipGetLastError();
}

template <bool MIXED>
hipError_t far_colloc_dispatch(const FarArgs& a, hipStream_t s)
{
    constexpr int PPT = 2;
    if (a.rules.nr == 49 && a.rules.nt == 33) return far_colloc_launch<33, 49, MIXED, PPT>(a, s);
    return far_colloc_launch<0, 0, MIXED, PPT>(a, s);
}

}  // namespace

hipError_t launch_far_eval(const FarArgs& a, int precision, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    return precision == 1 ? far_eval_dispatch<true>(a, s) : far_eval_dispatch<false>(a, s);
}

hipError_t launch_far_colloc(const FarArgs& a, int precision, hipStream_t s)
{
    if (a.el.ne <= 0) return hipSuccess;
    return precision == 1 ? far_colloc_dispatch<true>(a, s) : far_colloc_dispatch<false>(a, s);
}

hipError_t launch_far_grad(const FarArgs& a, int precision, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    return precision == 1 ? far_grad_dispatch<true>(a, s) : far_grad_dispatch<false>(a, s);
}

hipError_t launch_near(const NearArgs& a, int mode, hipStream_t s)
{
    // persistent lanes; every lane leaves once the shared cursor passes the pair count
    const int blocks = 1024;
    if (mode == kNearColloc) near_kernel<kNearColloc><<<blocks, kBlock, 0, s>>>(a);
    else if (mode == kNearGrad) near_kernel<kNearGrad><<<blocks, kBlock, 0, s>>>(a);
    else near_kernel<kNearEval><<<blocks, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_charges(const double* sigma, const double* area, double* q, int64_t ne, int n_rhs, hipStream_t s)
{
    const int64_t tot = ne * n_rhs;
    if (tot <= 0) return hipSuccess;
    charges_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(sigma, area, q, ne, n_rhs);
    return hipGetLastError();
}

hipError_t launch_reduce_split(const double* partial, int n_split, int64_t n, double K, double* phi, double* E,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    reduce_split_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(partial, n_split, n, K, phi, E);
    return hipGetLastError();
}

hipError_t launch_reduce_chunks(const double* partial, int n_split, int64_t rows, int64_t n, double K, double* out,
                                hipStream_t s)
{
    const int64_t tot = rows * n;
    if (tot <= 0) return hipSuccess;
    reduce_chunks_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(partial, n_split, rows, n, K, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ solver support -------
// Potential of an element with unit density at its own centroid, K times the exact polar
// integral (per edge at distance h with end offsets t1, t2: h [asinh(t2/h) - asinh(t1/h)]):
// the diagonal of the collocation matrix.
__global__ void self_diag_kernel(Elements el, double K, double* __restrict__ diag)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ne = el.ne;
    if (e >= ne) return;
    double G[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) G[c] = el.geom[(int64_t)c * ne + e];
    double V[4][3];
    int nv;
    if (e < el.n_tri) {
        nv = 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) { V[0][c] = 0.0; V[1][c] = G[3 + c] - G[c]; V[2][c] = G[6 + c] - G[c]; V[3][c] = 0.0; }
    } else {
        nv = 4;
#pragma unroll
        for (int c = 0; c < 3; ++c) { V[0][c] = 0.0; V[1][c] = G[3 + c]; V[2][c] = G[3 + c] + G[6 + c]; V[3][c] = G[6 + c]; }
    }
    double P[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) P[c] = el.cen[c * ne + e] - G[c];
    double sum = 0.0;
    for (int k = 0; k < nv; ++k) {
        const double* Va = V[k];
        const double* Vb = V[(k + 1) % nv];
        double tv[3] = { Vb[0] - Va[0], Vb[1] - Va[1], Vb[2] - Va[2] };
        const double len = sqrt(tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]);
        tv[0] /= len; tv[1] /= len; tv[2] /= len;
        const double pa[3] = { Va[0] - P[0], Va[1] - P[1], Va[2] - P[2] };
        const double t1 = pa[0] * tv[0] + pa[1] * tv[1] + pa[2] * tv[2];
        const double fx = pa[0] - t1 * tv[0], fy = pa[1] - t1 * tv[1], fz = pa[2] - t1 * tv[2];
        const double h = sqrt(fx * fx + fy * fy + fz * fz);
        if (h > 0.0) sum += h * (asinh((t1 + len) / h) - asinh(t1 / h));
    }
    diag[e] = K * sum;
}

// partial[j][b] = sum over block b's share of V[j][i] * w[i], j < k (fixed order)
__global__ void multi_dot_kernel(const double* __restrict__ V, int k, int64_t n, const double* __restrict__ w,
                                 double* __restrict__ partial)
{
    __shared__ double red[256];
    for (int j = 0; j < k; ++j) {
        double acc = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
            acc = fma(V[(int64_t)j * n + i], w[i], acc);
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// y[i] = a * y[i] + sum_j c[j] V[j][i] / d[i]^p  (p = 0 or 1; d may be null when p = 0)
__global__ void combine_kernel(double* __restrict__ y, double a, const double* __restrict__ V, const double* __restrict__ c,
                               int k, int64_t n, const double* __restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s = fma(c[j], V[(int64_t)j * n + i], s);
    if (d) s /= d[i];
    y[i] = fma(a, y[i], s);
}

// y[i] = x[i] / d[i]
__global__ void divide_kernel(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ d, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = x[i] / d[i];
}

hipError_t launch_zero_counters(DevCounters* c, hipStream_t s)
{
    zero_counters_kernel<<<1, 64, 0, s>>>(c);
    return hipGetLastError();
}

hipError_t launch_self_diag(const Elements& el, double K, double* diag, hipStream_t s)
{
    if (el.ne <= 0) return hipSuccess;
    self_diag_kernel<<<(unsigned)((el.ne + 255) / 256), 256, 0, s>>>(el, K, diag);
    return hipGetLastError();
}

hipError_t launch_multi_dot(const double* V, int k, int64_t n, const double* w, double* partial, int blocks, hipStream_t s)
{
    multi_dot_kernel<<<blocks, 256, 0, s>>>(V, k, n, w, partial);
    return hipGetLastError();
}

hipError_t launch_combine(double* y, double a, const double* V, const double* c, int k, int64_t n, const double* d,
                          hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    combine_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y, a, V, c, k, n, d);
    return hipGetLastError();
}

hipError_t launch_divide(double* y, const double* x, const double* d, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    divide_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y, x, d, n);
    return hipGetLastError();
}

}  // namespace bemc
