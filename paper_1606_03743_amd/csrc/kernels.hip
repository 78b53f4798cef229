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
//                      the element's rule.  Lanes take pairs from a shared cursor, the most
//                      expensive first (near_order.hip).  Each pair's result goes to its
//                      own slot in (point, element) order; the per-point sums are formed in
//                      that order afterwards (near_order.hip), so results are reproducible
//                      bit for bit.
//                      Pairs whose point lies on the element (found by the cost pass, last in
//                      the order) get the exact polar integral, one lane per pair, after the
//                      walk loop: kept out of the loop so that the walk's register footprint
//                      stays near 128 VGPRs, and its workgroups fit beside the far kernels of
//                      other streams.
#include "bemc_internal.h"
#include "on_element.h"

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

// The lanes of the wavefront for which pred holds.  A comparison's own lane mask: __ballot
// takes an int, and turning the comparison into one and back costs two more vector
// instructions per call.
__device__ __forceinline__ unsigned long long lane_mask(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }

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
    const unsigned long long m = lane_mask(is_near);
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

// ------------------------------------------------------------- near-pair list -----
// Every (point, element) pair with D^2 < (near_dr L)^2 (the distance-ratio switch, Sec. 2)
// goes into the near-pair list, compacted per wavefront; pairs past the capacity are
// counted, not stored.  A workgroup takes kListPoints consecutive points (Morton order:
// neighbours in space) and one chunk of the elements (more chunks when the points are few),
// and bounds the points by a box; an element takes the per-point test only when its
// centroid lies within near_dr L of that box.  Collocation: the points are the centroids
// themselves (the same [3][n] layout).
constexpr int kListPPT = 2;
constexpr int kListPoints = kBlock * kListPPT;

__global__ __launch_bounds__(kBlock) void near_list_kernel(const double* __restrict__ pts, int64_t n, Elements el,
                                                           NearPair* __restrict__ list, unsigned long long cap,
                                                           DevCounters* __restrict__ ctr, int64_t chunk)
{
    __shared__ double wbox[kBlock / 64][6];
    __shared__ double box[6];
    __shared__ uint32_t cand[kBlock];
    __shared__ double4 cand_c[kBlock];  // the candidates' centroids and thresholds
    __shared__ int ncand;
    const int64_t ne = el.ne;
    double x[kListPPT], y[kListPPT], z[kListPPT];
    bool valid[kListPPT];
    uint32_t idx[kListPPT];
    double lo[3] = { INFINITY, INFINITY, INFINITY }, hi[3] = { -INFINITY, -INFINITY, -INFINITY };
#pragma unroll
    for (int k = 0; k < kListPPT; ++k) {
        const int64_t p = (int64_t)blockIdx.x * kListPoints + (int64_t)k * kBlock + threadIdx.x;
        valid[k] = p < n;
        idx[k] = (uint32_t)p;
        x[k] = valid[k] ? pts[p] : 0.0;
        y[k] = valid[k] ? pts[n + p] : 0.0;
        z[k] = valid[k] ? pts[2 * n + p] : 0.0;
        if (valid[k]) {
            lo[0] = fmin(lo[0], x[k]); lo[1] = fmin(lo[1], y[k]); lo[2] = fmin(lo[2], z[k]);
            hi[0] = fmax(hi[0], x[k]); hi[1] = fmax(hi[1], y[k]); hi[2] = fmax(hi[2], z[k]);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        for (int o = 32; o > 0; o >>= 1) {
            lo[c] = fmin(lo[c], __shfl_xor(lo[c], o));
            hi[c] = fmax(hi[c], __shfl_xor(hi[c], o));
        }
    const int wave = threadIdx.x / 64;
    if (lane_id() == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) { wbox[wave][c] = lo[c]; wbox[wave][3 + c] = hi[c]; }
    }
    if (threadIdx.x == 0) ncand = 0;
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = wbox[0][threadIdx.x];
        for (int w = 1; w < kBlock / 64; ++w) v = threadIdx.x < 3 ? fmin(v, wbox[w][threadIdx.x]) : fmax(v, wbox[w][threadIdx.x]);
        box[threadIdx.x] = v;
    }
    __syncthreads();
    const double b0 = box[0], b1 = box[1], b2 = box[2], b3 = box[3], b4 = box[4], b5 = box[5];
    // this workgroup's chunk of the elements (blockIdx.y)
    const int64_t e_begin = (int64_t)blockIdx.y * chunk, e_end = min(ne, e_begin + chunk);
    for (int64_t c0 = e_begin; c0 < e_end; c0 += kBlock) {
        const int64_t e = c0 + threadIdx.x;
        bool hit = false;
        double cx = 0.0, cy = 0.0, cz = 0.0, t2 = 0.0;
        if (e < e_end) {
            cx = el.cen[e]; cy = el.cen[ne + e]; cz = el.cen[2 * ne + e]; t2 = el.thr2[e];
            const double dx = fmax(fmax(b0 - cx, cx - b3), 0.0);
            const double dy = fmax(fmax(b1 - cy, cy - b4), 0.0);
            const double dz = fmax(fmax(b2 - cz, cz - b5), 0.0);
            hit = fma(dx, dx, fma(dy, dy, dz * dz)) < t2;
        }
        const unsigned long long m = lane_mask(hit);
        if (m) {
            int base = 0;
            if (lane_id() == 0) base = atomicAdd(&ncand, __popcll(m));
            base = __shfl(base, 0);
            if (hit) {
                cand[base + (int)lanes_below(m)] = (uint32_t)e;
                cand_c[base + (int)lanes_below(m)] = make_double4(cx, cy, cz, t2);
            }
        }
        __syncthreads();
        const int nc = ncand;
        for (int i = 0; i < nc; ++i) {
            const uint32_t ce = cand[i];
            const double4 cc = cand_c[i];  // one LDS read for the whole wavefront
            const double cx = cc.x, cy = cc.y, cz = cc.z, t2 = cc.w;
#pragma unroll
            for (int k = 0; k < kListPPT; ++k) {
                const double dx = x[k] - cx, dy = y[k] - cy, dz = z[k] - cz;
                const bool nr = valid[k] && fma(dx, dx, fma(dy, dy, dz * dz)) < t2;
                record_near(nr, idx[k], ce, list, cap, ctr);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) ncand = 0;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- LDS staging ------
// Each element is summed in its own orthonormal frame: origin at the centroid, f1 and f2
// in its plane, f3 its unit normal.  A Gaussian point has in-plane coordinates (a, b).
//
// Expanded form (triangles, Table B rectangles, the short distance-ratio levels): with
// d = P - centroid, |p|^2 = D^2 from the distance test and q1 = -2 f1.d, q2 = -2 f2.d,
//   r^2 = D^2 + (a^2 + b^2) + q1 a + q2 b,
// and the field follows from the node sums S3 = sum w/r^3, S1 = sum w a/r^3, S2 = sum w b/r^3
// as E = q (S3 d - f1 S1 - f2 S2), rotated once per pair.  When every weight is positive,
// the nodes are staged divided by w^2, (a, b, a^2 + b^2, 1) / w^2: the reciprocal square
// root of r^2 / w^2 is w/r itself, and (w/r)^3 times the staged values gives the three
// field sums, which saves the multiplication by the weight per node.
//
// Rows form (the 7 x 7 Gauss-Legendre rectangle rule, and the gradient): the point is
// rotated into the frame, p = (f1.d, f2.d, f3.d).  For rectangles f1 runs along the second
// side, so the nodes of a tensor Gauss-Legendre rule that share their first coordinate share
// b: (p2 - b)^2 + p3^2 is formed once per group of seven and r^2 takes one difference and
// one FMA per node.  The local field (sum w (p1 - a)/r^3, sum w (p2 - b)/r^3, p3 sum w/r^3)
// is rotated back with the frame.
enum FrameForm { kFrExp = 0, kFrRows = 1 };

template <bool MIXED, int NRHS>
struct TileLds {
    using T = typename std::conditional<MIXED, float, double>::type;
    using T4 = typename std::conditional<MIXED, float4, double4>::type;
    T4 nd[kTileNodes];  // (a, b, a^2 + b^2, w), or divided by w^2 as (a, b, a^2 + b^2, 1) / w^2
    double cx[kMaxTileElems], cy[kMaxTileElems], cz[kMaxTileElems], thr2[kMaxTileElems];
    T fr[9][kMaxTileElems];      // point rotation: expanded -2 f1, -2 f2; rows f1, f2, f3
    double qr[9][kMaxTileElems]; // rotation back scaled by the charge: expanded -q f1, -q f2;
                                 // rows q f1, q f2, q f3
    double q[NRHS][kMaxTileElems];
    T lc[6][kMaxTileElems];      // triangles: in-plane coordinates of A, B, C relative to the centroid
};

// Orbit structure of the compiled triangle rules (Tables A2-A5 as expanded on the host:
// the centroid first, then the S21 orbits with the distinct coordinate at A, B, C in turn,
// then the other orbits in groups of gs nodes).  A node of an S21 orbit lies on the line
// from the centroid to its vertex, at n = (l_k - l_other) u_k with u_k the vertex relative
// to the centroid, so d.n = s d.u_k needs one product per node once d.u_k is known per pair.
template <int NN> struct TriOrbits { static constexpr int nc = 0, n21 = 0, gs = 4; };
template <> struct TriOrbits<7> { static constexpr int nc = 1, n21 = 2, gs = 1; };    // Table A2
template <> struct TriOrbits<12> { static constexpr int nc = 0, n21 = 0, gs = 3; };   // Table A3 (cyclic)
template <> struct TriOrbits<19> { static constexpr int nc = 1, n21 = 4, gs = 6; };   // Table A4
template <> struct TriOrbits<33> { static constexpr int nc = 0, n21 = 5, gs = 6; };   // Table A5

// Staging form of the triangle nodes: levels back to back (one for a fixed rule), each with
// nc centroid nodes and n21 S21 nodes (three per orbit) in front.
struct TriForms {
    int nlev;
    int off[5];
    int nc[4], n21[4];
};

template <int NN, bool ORBITS>
__device__ __forceinline__ TriForms fixed_forms(int nn)
{
    TriForms t{ 1, { 0, nn, nn, nn, nn }, { 0, 0, 0, 0 }, { 0, 0, 0, 0 } };
    if (ORBITS) {
        t.nc[0] = TriOrbits<NN>::nc;
        t.n21[0] = 3 * TriOrbits<NN>::n21;
    }
    return t;
}

// Pair rows of the 7 x 7 Gauss-Legendre rectangle rule (node i*7 + j at natural coordinates
// (x_i, x_j)): the row of x_i has b = x_i beta and the nodes a = a0 + x_j alpha, a0 = x_i gamma,
// with x_{6-j} = -x_j, the same weight for j and 6 - j and x_3 = 0.  Four slots per row:
//   header (b, a0, w of the middle node, a0^2 + b^2), then per pair j = 0, 1, 2 with
//   s = x_{6-j} alpha: (s, s^2, w, w s).
constexpr int kPairRowSlots = 28;
__device__ __forceinline__ double4 pair_row_slot(const RuleTables& R, int prow, int m, double gamma, double beta,
                                                 double alpha)
{
    const int r = m >> 2, c = m & 3;
    if (c == 0) {
        const int i = prow + r * 7 + 3;
        const double x = R.rect[4 * i];
        const double b = x * beta, a0 = x * gamma;
        return make_double4(b, a0, R.rect[4 * i + 2], fma(a0, a0, b * b));
    }
    const int i = prow + r * 7 + 7 - c;  // j = 6 - (c - 1)
    const double sv = R.rect[4 * i + 1] * alpha, w = R.rect[4 * i + 2];
    return make_double4(sv, sv * sv, w, w * sv);
}

// Gaussian points of elements [t0, t0 + te) in their frames (Eq. 3.2 / 3.3): triangle
// (a, b) = la A' + lb B' + lc C' from the in-plane coordinates of the vertices relative to
// the centroid; rectangle a = x gamma + y alpha, b = x beta for the rule point (x, y) in
// [-1, 1]^2 (alpha = |e2| / 2; beta, gamma the components of e1 / 2 across and along e2).
// FP32 tiles hold the FP64 values rounded once.  QR: stage the rotation back (field only).
// The first nfold nodes of each element are staged divided by w^2 (positive weights only).
// Nodes from prow on are a 7 x 7 Gauss-Legendre rule staged as pair rows (pair_row_slot).
// Triangles: centroid and S21 nodes (TriForms, folded nodes only) are staged as
// (0, 0, 1/w^2, 0) and (s, |n|^2, 1, 0) / w^2 with n = s u_k.
template <bool TRI, bool MIXED, int NRHS, int FR, bool QR>
__device__ __forceinline__ void stage_tile(TileLds<MIXED, NRHS>& s, const Elements& el, const RuleTables& R, int nn,
                                           int64_t t0, int te, int rhs0, int nrhs, int nfold, int prow,
                                           const TriForms& tf)
{
    using T = typename TileLds<MIXED, NRHS>::T;
    const int64_t ne = el.ne;
    for (int k = threadIdx.x; k < te; k += kBlock) {
        const int64_t e = t0 + k;
        s.cx[k] = el.cen[e];
        s.cy[k] = el.cen[ne + e];
        s.cz[k] = el.cen[2 * ne + e];
        s.thr2[k] = el.thr2[e];
        for (int r = 0; r < nrhs; ++r) s.q[r][k] = el.q[(int64_t)(rhs0 + r) * ne + e];
        const double q = QR ? el.q[(int64_t)rhs0 * ne + e] : 0.0;
        if constexpr (FR == kFrExp) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double f = el.frame[(int64_t)c * ne + e];
                s.fr[c][k] = (T)(-2.0 * f);
                if (QR) s.qr[c][k] = -q * f;
                if (TRI) s.lc[c][k] = (T)el.loc[(int64_t)c * ne + e];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const double f = el.frame[(int64_t)c * ne + e];
                s.fr[c][k] = (T)f;
                if (QR) s.qr[c][k] = q * f;
            }
        }
    }
    for (int k = threadIdx.x; k < te * nn; k += kBlock) {
        const int j = k / nn;
        const int i = k - j * nn;
        const int64_t e = t0 + j;
        if (!TRI && i >= prow) {
            if (i - prow < kPairRowSlots) {
                const double4 v = pair_row_slot(R, prow, i - prow, el.loc[e], el.loc[ne + e], el.loc[2 * ne + e]);
                if constexpr (MIXED) s.nd[k] = make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
                else s.nd[k] = v;
            }
            continue;
        }
        double a, b, w;
        if (TRI) {
            const double la = R.tri[4 * i], lb = R.tri[4 * i + 1], lc = R.tri[4 * i + 2];
            w = R.tri[4 * i + 3];
            if (i < nfold) {
                // the level of node i (selects, not indexing: the forms stay in registers)
                int off_l = tf.off[0], nc_l = tf.nc[0], n21_l = tf.n21[0];
#pragma unroll
                for (int q = 1; q < 4; ++q)
                    if (q < tf.nlev && i >= tf.off[q]) { off_l = tf.off[q]; nc_l = tf.nc[q]; n21_l = tf.n21[q]; }
                const int il = i - off_l;
                if (il < nc_l + n21_l) {
                    const double iw2 = 1.0 / (w * w);
                    double v0 = 0.0, v1 = 0.0;
                    if (il >= nc_l) {  // S21: the distinct coordinate at vertex kk
                        const int kk = (il - nc_l) % 3;
                        const double lk = kk == 0 ? la : (kk == 1 ? lb : lc);
                        const double lk1 = kk == 0 ? lb : (kk == 1 ? lc : la);
                        const double sv = lk - lk1;
                        const double na = sv * el.loc[(int64_t)(2 * kk) * ne + e], nb = sv * el.loc[(int64_t)(2 * kk + 1) * ne + e];
                        v0 = sv * iw2;
                        v1 = fma(na, na, nb * nb) * iw2;
                    }
                    if constexpr (MIXED) s.nd[k] = make_float4((float)v0, (float)v1, (float)iw2, 0.0f);
                    else s.nd[k] = make_double4(v0, v1, iw2, 0.0);
                    continue;
                }
            }
            a = la * el.loc[e] + lb * el.loc[2 * ne + e] + lc * el.loc[4 * ne + e];
            b = la * el.loc[ne + e] + lb * el.loc[3 * ne + e] + lc * el.loc[5 * ne + e];
        } else {
            const double x = R.rect[4 * i], y = R.rect[4 * i + 1];
            w = R.rect[4 * i + 2];
            a = x * el.loc[e] + y * el.loc[2 * ne + e];
            b = x * el.loc[ne + e];
        }
        double g = fma(a, a, b * b);
        if (i < nfold) {
            const double iw2 = 1.0 / (w * w);
            a *= iw2;
            b *= iw2;
            g *= iw2;
            w = iw2;
        }
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

// The lane's points relative to the element in hand.
template <int PPT, typename T>
struct Local {
    T q1[PPT], q2[PPT], H[PPT];           // expanded: -2 f1.d, -2 f2.d, D^2
    T p1[PPT], p2[PPT], p3[PPT], h[PPT];  // rows: f1.d, f2.d, f3.d, p3^2
    double dx[PPT], dy[PPT], dz[PPT];     // d = P - centroid (FP64)
};

// Runs term(i) for the nodes i = 1 .. n-1 of one element (node 0 is peeled off by the
// caller, so that the sums start from its terms instead of from zero).  Long rules (and
// run-time counts) go in groups of four with a separate remainder: this keeps the
// accumulators in place, where an unrolled loop with a remainder makes the compiler copy
// them every iteration.  The short rules of the distance-ratio levels use a plain
// unrolled loop.
template <int NN, typename Term>
__device__ __forceinline__ void for_nodes(int n, Term term)
{
    if (NN > 0 && NN < 32) {
#pragma unroll 4
        for (int i = 1; i < n; ++i) term(i);
        return;
    }
    int i = 1;
#pragma unroll 1
    for (; i + 4 <= n; i += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) term(i + u);
    }
    for (; i < n; ++i) term(i);
}

// 1/sqrt(x) in the precision of T (FP64 refined, see rsqrt64)
__device__ __forceinline__ double rsqrtT(double x) { return rsqrt64(x); }
__device__ __forceinline__ float rsqrtT(float x) { return rsqrt32(x); }

// Node sums of one element per field point (unit element charge, Eq. 4.1), accumulated into
// o, whose sums start at -0.0 (so that adding the first node folds into an assignment).
//   kFarField, expanded: (sum w/r, sum w a/r^3, sum w b/r^3, sum w/r^3);
//              FOLD: the staged node is (a, b, g, 1) / w^2 and rsqrt(r^2 / w^2) = w/r;
//   kFarPhi,   expanded: sum w/r; FOLD in FP64: the potential of the node is y (1 + e/2 +
//              3 e^2 / 8) with y the hardware estimate of w/r and e = 1 - (r^2/w^2) y^2,
//              formed as one FMA of y with the factor (the same third-order step as rsqrt64);
//   kFarGrad   (differences da = p1 - a, db = p2 - b): FP64 (sum w/r^3, sum w/r^5,
//              sum w da/r^5, sum w db/r^5, sum w da^2/r^5, sum w db^2/r^5, sum w da db/r^5),
//              turned into the local tensor after the loop; FP32: the local tensor itself,
//              sum w/r^3 and sum w u_i u_j / r^3 over the unit offset u = (da, db, p3)/r (xx,
//              yy, zz, xy, xz, yz), so that no power of 1/r above the third is formed in
//              single precision.
template <int PPT, int MODE, bool FOLD, typename T, typename T4>
__device__ __forceinline__ void node_term(const T4 Q, const Local<PPT, T>& L, T (&o)[Sums<MODE>::kNode][PPT])
{
    constexpr bool F64 = std::is_same<T, double>::value;
    const T a = Q.x, b = Q.y, g = Q.z, w = Q.w;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if constexpr (MODE == kFarGrad) {
            const T da = L.p1[k] - a, db = L.p2[k] - b;
            const T ri = rsqrtT(fma(da, da, fma(db, db, L.h[k])));
            if constexpr (F64) {
                const T ri2 = ri * ri;
                const T w3 = (w * ri) * ri2;
                const T w5 = w3 * ri2;
                const T ua = w5 * da, ub = w5 * db;
                o[0][k] += w3;
                o[1][k] += w5;
                o[2][k] += ua;
                o[3][k] += ub;
                o[4][k] = fma(ua, da, o[4][k]);
                o[5][k] = fma(ub, db, o[5][k]);
                o[6][k] = fma(ua, db, o[6][k]);
            } else {
                const T w3 = (w * ri) * (ri * ri);
                const T va = da * ri, vb = db * ri, vc = L.p3[k] * ri;
                const T ua = w3 * va, ub = w3 * vb, uc = w3 * vc;
                o[0][k] += w3;
                o[1][k] = fma(ua, va, o[1][k]);
                o[2][k] = fma(ub, vb, o[2][k]);
                o[3][k] = fma(uc, vc, o[3][k]);
                o[4][k] = fma(ua, vb, o[4][k]);
                o[5][k] = fma(ua, vc, o[5][k]);
                o[6][k] = fma(ub, vc, o[6][k]);
            }
        } else if constexpr (FOLD) {
            const T x = fma(L.q1[k], a, fma(L.q2[k], b, fma(L.H[k], w, g)));  // r^2 / w^2
            if constexpr (MODE == kFarPhi) {
                if constexpr (F64) {
                    const double y = __builtin_amdgcn_rsq(x);
                    const double e = fma(-(x * y), y, 1.0);
                    o[0][k] = fma(y, fma(e, fma(e, 0.375, 0.5), 1.0), o[0][k]);
                } else {
                    o[0][k] += rsqrtT(x);
                }
            } else {
                const T wr = rsqrtT(x);  // w / r
                const T wr3 = (wr * wr) * wr;
                o[0][k] += wr;
                o[1][k] = fma(wr3, a, o[1][k]);
                o[2][k] = fma(wr3, b, o[2][k]);
                o[3][k] = fma(wr3, w, o[3][k]);
            }
        } else {
            const T ri = rsqrtT(fma(L.q1[k], a, fma(L.q2[k], b, L.H[k] + g)));
            if constexpr (MODE == kFarPhi) {
                o[0][k] = fma(w, ri, o[0][k]);
            } else {
                const T wr = w * ri;
                const T w3 = wr * (ri * ri);
                o[0][k] += wr;
                o[1][k] = fma(w3, a, o[1][k]);
                o[2][k] = fma(w3, b, o[2][k]);
                o[3][k] += w3;
            }
        }
    }
}

// Tensor rule in G groups of G nodes with the same b: per group the lane forms db and
// (p2 - b)^2 + p3^2 once; per node one difference remains.  Field: the b-component and
// sum w/r^3 are gathered per group.  Gradient (the FP64 sums of node_term): sum w/r^5 and
// sum w da/r^5 are gathered per group, and the sums with db follow from them.  The sums
// in o start at -0.0.
template <int G, int PPT, int MODE, typename T, typename T4>
__device__ __forceinline__ void group_body(const T4* t, int n0, const Local<PPT, T>& L, T (&o)[Sums<MODE>::kNode][PPT])
{
    const T b = t[n0].y;
    T db[PPT], B[PPT], sg[PPT], xg[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        db[k] = L.p2[k] - b;
        B[k] = fma(db[k], db[k], L.h[k]);
        sg[k] = T(-0.0);
        xg[k] = T(-0.0);
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const T a = t[n0 + i].x, w = t[n0 + i].w;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const T da = L.p1[k] - a;
            const T ri = rsqrtT(fma(da, da, B[k]));
            if constexpr (MODE == kFarPhi) {
                o[0][k] = fma(w, ri, o[0][k]);
            } else if constexpr (MODE == kFarField) {
                const T wr = w * ri;
                const T w3 = wr * (ri * ri);
                o[0][k] += wr;
                o[1][k] = fma(w3, da, o[1][k]);
                sg[k] += w3;
            } else {
                const T ri2 = ri * ri;
                const T w3 = (w * ri) * ri2;
                const T w5 = w3 * ri2;
                const T ua = w5 * da;
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
            const T u = sg[k] * db[k];  // sum w db / r^5 of the group
            o[1][k] += sg[k];
            o[2][k] += xg[k];
            o[3][k] += u;
            o[5][k] = fma(u, db[k], o[5][k]);
            o[6][k] = fma(xg[k], db[k], o[6][k]);
        }
    }
}

template <int G, int PPT, int MODE, typename T, typename T4>
__device__ __forceinline__ void group_sum(const T4* t, int base, const Local<PPT, T>& L, T (&o)[Sums<MODE>::kNode][PPT])
{
    static_assert(!(MODE == kFarGrad && std::is_same<T, float>::value), "the FP32 gradient takes the node form");
    group_body<G, PPT, MODE>(t, base, L, o);  // the first group starts the sums
#pragma unroll 1
    for (int g = 1; g < G; ++g) group_body<G, PPT, MODE>(t, base + g * G, L, o);
}

// One pair row of the 7 x 7 rule (slots n0 .. n0 + 3, see pair_row_slot) for potential and
// field, or the potential alone.  With da0 = p1 - a0 and C = |d - (a0 f1 + b f2)|^2, formed
// like the expanded form from D^2 (C = D^2 + a0^2 + b^2 - 2 (p1 a0 + p2 b): the rotation's
// rounding then enters only through the small products), the pair at a0 -+ s has
// r^2 = C + s^2 -+ 2 da0 s; its sums go in as w (1/r+ + 1/r-), w (1/r+^3 +
// 1/r-^3) and w s (1/r+^3 - 1/r-^3), the last one into SA.  Per row the field's local parts
// follow as E1 += da0 sg, E2 += (p2 - b) sg, S3 += sg with sg = sum over the row of w/r^3;
// E1 -= SA once per element.  FP64 potential only: each pair's 1/r as y (1 + e (1/2 + 3e/8))
// from the hardware estimate y (the third-order step of rsqrt64), the weight applied once.
template <int PPT, int MODE, typename T, typename T4>
__device__ __forceinline__ void pair_row(const T4* t, int n0, const Local<PPT, T>& L, T (&o)[Sums<MODE>::kNode][PPT],
                                         T (&SA)[PPT])
{
    constexpr bool F64 = std::is_same<T, double>::value;
    const T4 hd = t[n0];
    const T b = hd.x, a0 = hd.y, wc = hd.z, g0 = hd.w;
    T db[PPT], da0[PPT], C[PPT], mq[PPT], pq[PPT], sg[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        db[k] = L.p2[k] - b;
        da0[k] = L.p1[k] - a0;
        C[k] = fma(L.q1[k], a0, fma(L.q2[k], b, L.H[k] + g0));
        mq[k] = T(-2) * da0[k];
        pq[k] = T(2) * da0[k];
    }
    // the middle node (a = a0)
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if constexpr (MODE == kFarPhi) {
            if constexpr (F64) {
                const double y = __builtin_amdgcn_rsq(C[k]);
                const double e = fma(-(C[k] * y), y, 1.0);
                o[0][k] = fma(wc * y, fma(e, fma(e, 0.375, 0.5), 1.0), o[0][k]);
            } else {
                o[0][k] = fma(wc, rsqrtT(C[k]), o[0][k]);
            }
        } else {
            const T ri = rsqrtT(C[k]);
            o[0][k] = fma(wc, ri, o[0][k]);
            sg[k] = wc * ((ri * ri) * ri);
        }
    }
#pragma unroll
    for (int pi = 1; pi <= 3; ++pi) {
        const T4 Q = t[n0 + pi];
        const T sv = Q.x, s2 = Q.y, w = Q.z, ws = Q.w;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const T u = C[k] + s2;
            const T xp = fma(mq[k], sv, u), xm = fma(pq[k], sv, u);
            if constexpr (MODE == kFarPhi) {
                if constexpr (F64) {
                    const double yp = __builtin_amdgcn_rsq(xp), ym = __builtin_amdgcn_rsq(xm);
                    const double ep = fma(-(xp * yp), yp, 1.0), em = fma(-(xm * ym), ym, 1.0);
                    const double vp = fma(ep, fma(ep, 0.375, 0.5), 1.0), vm = fma(em, fma(em, 0.375, 0.5), 1.0);
                    o[0][k] = fma(w, fma(ym, vm, yp * vp), o[0][k]);
                } else {
                    o[0][k] = fma(w, rsqrtT(xp) + rsqrtT(xm), o[0][k]);
                }
            } else {
                const T rp = rsqrtT(xp), rm = rsqrtT(xm);
                const T r3p = (rp * rp) * rp, r3m = (rm * rm) * rm;
                o[0][k] = fma(w, rp + rm, o[0][k]);
                sg[k] = fma(w, r3p + r3m, sg[k]);
                SA[k] = fma(ws, r3p - r3m, SA[k]);
            }
        }
    }
    if constexpr (MODE == kFarField) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            o[1][k] = fma(da0[k], sg[k], o[1][k]);
            o[2][k] = fma(db[k], sg[k], o[2][k]);
            o[3][k] += sg[k];
        }
    }
}

// The 7 x 7 rule as seven pair rows; o (and SA) start at -0.0, the first row is peeled off.
template <int PPT, int MODE, typename T, typename T4>
__device__ __forceinline__ void pair_rows_sum(const T4* t, int base, const Local<PPT, T>& L,
                                              T (&o)[Sums<MODE>::kNode][PPT])
{
    T SA[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) SA[k] = T(-0.0);
    pair_row<PPT, MODE>(t, base, L, o, SA);
#pragma unroll 1
    for (int r = 1; r < 7; ++r) pair_row<PPT, MODE>(t, base + 4 * r, L, o, SA);
    if constexpr (MODE == kFarField) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) o[1][k] -= SA[k];
    }
}

// One folded node whose r^2 / w^2 is x: potential (and field sums S3 and, for S21 nodes, the
// vertex sum tv = sum (w/r)^3 s / w^2, from which S1 and S2 follow per pair).
template <int MODE, typename T>
__device__ __forceinline__ void folded_point(T x, T iw2, T sv, T& o0, T& o3, T& tv)
{
    if constexpr (MODE == kFarPhi) {
        if constexpr (std::is_same<T, double>::value) {
            const double y = __builtin_amdgcn_rsq(x);
            const double e = fma(-(x * y), y, 1.0);
            o0 = fma(y, fma(e, fma(e, 0.375, 0.5), 1.0), o0);
        } else {
            o0 += rsqrtT(x);
        }
    } else {
        const T wr = rsqrtT(x);  // w / r
        const T wr3 = (wr * wr) * wr;
        o0 += wr;
        tv = fma(wr3, sv, tv);
        o3 = fma(wr3, iw2, o3);
    }
}

// A compiled triangle rule with its orbit structure (TriOrbits), folded nodes: the centroid
// (r^2 = D^2), the S21 orbits (r^2 = D^2 + |n|^2 + s P_k with P_k = -2 d.u_k per pair; the
// field's in-plane sums per vertex), then the other orbits with the expanded form of
// node_term.  The sums in o start at -0.0; the first orbit of each kind is peeled off.
template <int NN, int PPT, int MODE, typename Lds, typename T>
__device__ __forceinline__ void tri_sum(const Lds& s, int j, int base, const Local<PPT, T>& L,
                                        T (&o)[Sums<MODE>::kNode][PPT])
{
    using O = TriOrbits<NN>;
    constexpr int NC = O::nc, N21 = O::n21, GS = O::gs, NG = NN - NC - 3 * N21;
    static_assert(NG % GS == 0, "orbit groups");
    constexpr int I3 = MODE == kFarPhi ? 0 : 3;  // index of S3 (unused for the potential alone)
    T Pk[3][PPT], Tk[3][PPT], dummy[PPT];
    if constexpr (N21 > 0) {
        const T ax = s.lc[0][j], ay = s.lc[1][j], bx = s.lc[2][j], by = s.lc[3][j];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            Pk[0][k] = fma(ax, L.q1[k], ay * L.q2[k]);
            Pk[1][k] = fma(bx, L.q1[k], by * L.q2[k]);
            Pk[2][k] = -(Pk[0][k] + Pk[1][k]);
#pragma unroll
            for (int c = 0; c < 3; ++c) Tk[c][k] = T(-0.0);
        }
    }
    if constexpr (NC > 0) {
        const T iw2 = s.nd[base].z;
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            folded_point<MODE, T>(L.H[k] * iw2, iw2, T(0), o[0][k], o[I3][k], dummy[k]);
    }
    if constexpr (N21 > 0) {
        auto orbit = [&](int ob) {
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                const auto Q = s.nd[base + NC + 3 * ob + kk];
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    folded_point<MODE, T>(fma(Q.x, Pk[kk][k], fma(L.H[k], Q.z, Q.y)), Q.z, Q.x, o[0][k], o[I3][k],
                                       Tk[kk][k]);
            }
        };
        orbit(0);
#pragma unroll 1
        for (int ob = 1; ob < N21; ++ob) orbit(ob);
    }
    if constexpr (NG > 0) {
        const int g0 = base + NC + 3 * N21;
        auto group = [&](int g) {
#pragma unroll
            for (int u = 0; u < GS; ++u) node_term<PPT, MODE, true>(s.nd[g0 + g * GS + u], L, o);
        };
        group(0);
#pragma unroll 1
        for (int g = 1; g < NG / GS; ++g) group(g);
    }
    if constexpr (N21 > 0 && MODE == kFarField) {
        const T l0 = s.lc[0][j], l1 = s.lc[1][j], l2 = s.lc[2][j], l3 = s.lc[3][j], l4 = s.lc[4][j], l5 = s.lc[5][j];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            o[1][k] = fma(l0, Tk[0][k], fma(l2, Tk[1][k], fma(l4, Tk[2][k], o[1][k])));
            o[2][k] = fma(l1, Tk[0][k], fma(l3, Tk[1][k], fma(l5, Tk[2][k], o[2][k])));
        }
    }
}

// Sums of one element over its nodes [base, base + n) of the tile (Eq. 4.1, unit element
// charge) in the precision T of the tile (FP64, or FP32 for the mixed path).  NN > 0:
// compile-time node count; G > 0: tensor rule in groups of G (rows form).  Field, expanded:
// (sum w/r, S1, S2, S3) in node coordinates; rows: (sum w/r, local E1, local E2 without p3,
// sum w/r^3).  Gradient: the local tensor (sum w/r^3; sum w d_i d_j / r^5 for xx, yy, zz,
// xy, xz, yz, d = (da, db, p3)).
template <int NN, int G, bool FOLD, bool TRI, int PPT, int MODE, typename Lds, typename T>
__device__ __forceinline__ void element_sum(const Lds& s, int j, int base, int n, const Local<PPT, T>& L,
                                            T (&o)[Sums<MODE>::kNode][PPT])
{
    constexpr int S = Sums<MODE>::kNode;
    constexpr bool MIXED = std::is_same<T, float>::value;
#pragma unroll
    for (int c = 0; c < S; ++c)
#pragma unroll
        for (int k = 0; k < PPT; ++k) o[c][k] = T(-0.0);
    const int nn = NN > 0 ? NN : n;
    constexpr bool GROUPS = G > 0 && (MODE != kFarGrad || !MIXED);
    if constexpr (GROUPS && MODE == kFarGrad) {
        group_sum<G, PPT, MODE>(s.nd, base, L, o);
    } else if constexpr (GROUPS) {
        static_assert(G == 7, "pair rows are built for the 7 x 7 rule");
        pair_rows_sum<PPT, MODE>(s.nd, base, L, o);
    } else if constexpr (TRI && FOLD && NN > 0 && MODE != kFarGrad) {
        tri_sum<NN, PPT, MODE>(s, j, base, L, o);
    } else {
        node_term<PPT, MODE, FOLD>(s.nd[base], L, o);
        for_nodes<NN>(nn, [&](int i) { node_term<PPT, MODE, FOLD>(s.nd[base + i], L, o); });
    }
    if constexpr (MODE == kFarGrad && !MIXED) {
        T r[S][PPT];
#pragma unroll
        for (int c = 0; c < S; ++c)
#pragma unroll
            for (int k = 0; k < PPT; ++k) r[c][k] = o[c][k];
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
    }
}

// Offsets of the lane's points from element j of the tile: D^2 in FP64 (the distance test,
// Sec. 2) and the coordinates the node sums need, in their precision.  Expanded: -2 f1.d,
// -2 f2.d and |p|^2 = D^2 (the rotation keeps the length, to rounding); rows: p = F d and
// p3^2; BOTH (rectangles with the rule chosen by distance ratio): rows, and the expanded
// coordinates from them.
template <int FR, bool BOTH, int PPT, typename Lds, typename T>
__device__ __forceinline__ void to_frame(const Lds& s, int j, const double (&x)[PPT], const double (&y)[PPT],
                                         const double (&z)[PPT], double (&D2)[PPT], Local<PPT, T>& L)
{
    const double cx = s.cx[j], cy = s.cy[j], cz = s.cz[j];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const double dx = x[k] - cx, dy = y[k] - cy, dz = z[k] - cz;
        L.dx[k] = dx;
        L.dy[k] = dy;
        L.dz[k] = dz;
        D2[k] = fma(dx, dx, fma(dy, dy, dz * dz));
        const T u = (T)dx, v = (T)dy, w = (T)dz;
        if constexpr (FR == kFrExp) {
            L.q1[k] = fma(u, s.fr[0][j], fma(v, s.fr[1][j], w * s.fr[2][j]));
            L.q2[k] = fma(u, s.fr[3][j], fma(v, s.fr[4][j], w * s.fr[5][j]));
            L.H[k] = (T)D2[k];
        } else {
            L.p1[k] = fma(u, s.fr[0][j], fma(v, s.fr[1][j], w * s.fr[2][j]));
            L.p2[k] = fma(u, s.fr[3][j], fma(v, s.fr[4][j], w * s.fr[5][j]));
            L.p3[k] = fma(u, s.fr[6][j], fma(v, s.fr[7][j], w * s.fr[8][j]));
            L.h[k] = L.p3[k] * L.p3[k];
            if constexpr (BOTH) {
                L.q1[k] = T(-2) * L.p1[k];
                L.q2[k] = T(-2) * L.p2[k];
                L.H[k] = (T)D2[k];
            }
        }
    }
}

// acc += the element's contribution to point k (charge q, sums o), in FP64.
//   expanded sums:  phi += q sum w/r;  E += (q S3) d - (q f1) S1 - (q f2) S2;
//   rows:           phi += q sum w/r;  E += (q f1) E1 + (q f2) E2 + (q f3) p3 S3;
//   gradient:       the global tensor M = F m F^T of the local one m (F: the frame vectors
//                   as columns), dE_i/dx_j += q (delta_ij sum w/r^3 - 3 M_ij).
template <int FR, int PPT, int MODE, typename Lds, typename T>
__device__ __forceinline__ void add_element(PointSet<PPT, MODE>& P, int k, double q, const Lds& s, int j,
                                            const Local<PPT, T>& L, const T (&o)[Sums<MODE>::kNode][PPT])
{
    if constexpr (MODE == kFarField) {
        P.acc[0][k] = fma(q, (double)o[0][k], P.acc[0][k]);
        if constexpr (FR == kFrExp) {
            const double s1 = (double)o[1][k], s2 = (double)o[2][k], qs3 = q * (double)o[3][k];
            P.acc[1][k] = fma(qs3, L.dx[k], fma(s.qr[0][j], s1, fma(s.qr[3][j], s2, P.acc[1][k])));
            P.acc[2][k] = fma(qs3, L.dy[k], fma(s.qr[1][j], s1, fma(s.qr[4][j], s2, P.acc[2][k])));
            P.acc[3][k] = fma(qs3, L.dz[k], fma(s.qr[2][j], s1, fma(s.qr[5][j], s2, P.acc[3][k])));
        } else {
            const double e1 = (double)o[1][k], e2 = (double)o[2][k], e3 = (double)(L.p3[k] * o[3][k]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                P.acc[1 + c][k] = fma(s.qr[c][j], e1, fma(s.qr[3 + c][j], e2, fma(s.qr[6 + c][j], e3, P.acc[1 + c][k])));
        }
    } else {
        const T m[3][3] = { { o[1][k], o[4][k], o[5][k] },
                            { o[4][k], o[2][k], o[6][k] },
                            { o[5][k], o[6][k], o[3][k] } };
        T U[3][3];  // U[a][c] = sum_b m[a][b] f_b[c]
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                U[a][c] = fma(m[a][0], s.fr[c][j], fma(m[a][1], s.fr[3 + c][j], m[a][2] * s.fr[6 + c][j]));
        auto M = [&](int u, int v) -> double {
            return (double)fma(s.fr[u][j], U[0][v], fma(s.fr[3 + u][j], U[1][v], s.fr[6 + u][j] * U[2][v]));
        };
        const double s3 = (double)o[0][k];
#pragma unroll
        for (int c = 0; c < 3; ++c) P.acc[c][k] = fma(q, fma(-3.0, M(c, c), s3), P.acc[c][k]);
        P.acc[3][k] = fma(-3.0 * q, M(0, 1), P.acc[3][k]);
        P.acc[4][k] = fma(-3.0 * q, M(0, 2), P.acc[4][k]);
        P.acc[5][k] = fma(-3.0 * q, M(1, 2), P.acc[5][k]);
    }
}

// group size of the rows form for a rectangle rule of NN nodes (7 x 7 only)
template <bool TRI, int NN>
constexpr int tensor_group() { return (!TRI && NN == 49) ? 7 : 0; }

// frame form of an element kind with a compiled rule of NN nodes
template <bool TRI, int NN, int MODE>
constexpr int frame_form() { return (MODE == kFarGrad || tensor_group<TRI, NN>() > 0) ? kFrRows : kFrExp; }

// One element kind over [e_begin, e_end) with one rule; NN > 0 is the compile-time node
// count, NN == 0 reads it at run time.  FOLD: the rule's weights are all positive (the
// nodes are staged divided by w^2).
template <int NN, bool TRI, bool MIXED, int PPT, int MODE, bool FOLD, typename Lds>
__device__ __forceinline__ void far_eval_range(const FarArgs& a, Lds& s, PointSet<PPT, MODE>& P, int64_t e_begin,
                                               int64_t e_end)
{
    using T = typename Lds::T;
    constexpr int FR = frame_form<TRI, NN, MODE>();
    constexpr bool FOLD_ = FOLD && FR == kFrExp;
    const int nn = NN > 0 ? NN : (TRI ? a.rules.nt : a.rules.nr);
    const int TE = tile_elems(nn);
    const TriForms tf = fixed_forms<NN, TRI && FOLD_>(nn);
    for (int64_t t0 = e_begin; t0 < e_end; t0 += TE) {
        const int te = (int)min((int64_t)TE, e_end - t0);
        __syncthreads();
        constexpr bool PROWS = tensor_group<TRI, NN>() > 0 && MODE != kFarGrad;
        stage_tile<TRI, MIXED, 1, FR, MODE == kFarField>(s, a.el, a.rules, nn, t0, te, a.rhs, 1, FOLD_ ? nn : 0,
                                                         PROWS ? 0 : nn, tf);
        __syncthreads();
        for (int j = 0; j < te; ++j) {
            const double thr2 = s.thr2[j], q = s.q[0][j];
            double D2[PPT];
            Local<PPT, T> L;
            to_frame<FR, FR == kFrRows && MODE != kFarGrad>(s, j, P.x, P.y, P.z, D2, L);
            bool nr[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                nr[k] = P.valid[k] && (D2[k] < thr2);  // listed by near_list_kernel
            }
            T o[Sums<MODE>::kNode][PPT];
            element_sum<NN, tensor_group<TRI, NN>(), FOLD_, TRI, PPT, MODE>(s, j, j * nn, nn, L, o);
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (!nr[k]) add_element<FR, PPT, MODE>(P, k, q, s, j, L, o);
        }
    }
}

// Expanded sums (node coordinates) of a rectangle level turned into the local field of the
// rows form: E1 = p1 S3 - S1, E2 = p2 S3 - S2.
template <int PPT, typename T>
__device__ __forceinline__ void exp_to_rows(const Local<PPT, T>& L, T (&o)[4][PPT])
{
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        o[1][k] = fma(L.p1[k], o[3][k], -o[1][k]);
        o[2][k] = fma(L.p2[k], o[3][k], -o[2][k]);
    }
}

// One element kind with the rule chosen by distance ratio (Sec. 4): the staged nodes of an
// element are the four levels back to back; a pair needs level l when D^2 >= c[l] (near_dr
// L)^2 (the last level otherwise).  The wavefront runs the finest level that any of its
// pairs needs, once, for all its lanes: a finer rule is at least as accurate at a larger
// distance ratio, and one level per wavefront costs less than each level a lane needs.
// N0..N3 > 0: compile-time counts (the levels' weights are then all positive).
// Triangles take the expanded form throughout; rectangles the rows form for a 7 x 7 last
// level, the expanded form (turned into the rows form's local field) for the others.
// Terms summed by the wavefront (w: pairs at each wavefront level) and at the pairs' own
// levels (n: pairs at levels 0, 1, 2 of nc in all), the levels having o1, o2 - o1, o3 - o2 and
// nn - o3 nodes.
__device__ __forceinline__ void add_terms(unsigned w0, unsigned w1, unsigned w2, unsigned w3, unsigned nc,
                                          unsigned n0, unsigned n1, unsigned n2, int o1, int o2, int o3, int nn,
                                          unsigned long long& terms, unsigned long long& terms_pair)
{
    terms += (unsigned long long)w0 * (unsigned)o1 + (unsigned long long)w1 * (unsigned)(o2 - o1) +
             (unsigned long long)w2 * (unsigned)(o3 - o2) + (unsigned long long)w3 * (unsigned)(nn - o3);
    terms_pair += (unsigned long long)n0 * (unsigned)o1 + (unsigned long long)n1 * (unsigned)(o2 - o1) +
                  (unsigned long long)n2 * (unsigned)(o3 - o2) +
                  (unsigned long long)(nc - n0 - n1 - n2) * (unsigned)(nn - o3);
}

template <int N0, int N1, int N2, int N3, bool TRI, bool MIXED, int PPT, int MODE, typename Lds>
__device__ __forceinline__ void far_eval_dr_range(const FarArgs& a, Lds& s, PointSet<PPT, MODE>& P, int64_t e_begin,
                                                  int64_t e_end, unsigned long long& terms,
                                                  unsigned long long& terms_pair)
{
    using T = typename Lds::T;
    constexpr bool GRAD = MODE == kFarGrad;
    constexpr int FR = (TRI && !GRAD) ? kFrExp : kFrRows;
    constexpr bool FOLD = N0 > 0 && !GRAD;
    const int* off = TRI ? a.lv.tri_off : a.lv.rect_off;
    const double* c = TRI ? a.lv.tri_c : a.lv.rect_c;
    const int o1 = off[1], o2 = off[2], o3 = off[3], nn = off[4];
    const double c0 = c[0], c1 = c[1], c2 = c[2];
    const int TE = tile_elems(nn);
    TriForms tf{ 4, { off[0], o1, o2, o3, nn }, { 0, 0, 0, 0 }, { 0, 0, 0, 0 } };
    if (TRI && FOLD) {
        tf.nc[0] = TriOrbits<N0>::nc; tf.n21[0] = 3 * TriOrbits<N0>::n21;
        tf.nc[1] = TriOrbits<N1>::nc; tf.n21[1] = 3 * TriOrbits<N1>::n21;
        tf.nc[2] = TriOrbits<N2>::nc; tf.n21[2] = 3 * TriOrbits<N2>::n21;
        tf.nc[3] = TriOrbits<N3>::nc; tf.n21[3] = 3 * TriOrbits<N3>::n21;
    }
    unsigned long long vmask[PPT];  // the lanes with a point, per point of the lane
#pragma unroll
    for (int k = 0; k < PPT; ++k) vmask[k] = lane_mask(P.valid[k]);
    for (int64_t t0 = e_begin; t0 < e_end; t0 += TE) {
        const int te = (int)min((int64_t)TE, e_end - t0);
        // the tile's pair counts (scalar, 32 bits: at most 64 PPT TE per tile): summed by the
        // wavefront at each of its levels, and at the pairs' own levels (all, level 0, 1, 2)
        unsigned w0 = 0, w1 = 0, w2 = 0, w3 = 0, nc = 0, n0 = 0, n1 = 0, n2 = 0;
        __syncthreads();
        // the 7 x 7 last level of the rectangles keeps its weights (rows form)
        const int nfold = !FOLD ? 0 : (tensor_group<TRI, N3>() > 0 ? o3 : nn);
        const int prow = (tensor_group<TRI, N3>() > 0 && !GRAD) ? o3 : nn;
        stage_tile<TRI, MIXED, 1, FR, !GRAD>(s, a.el, a.lv.tab, nn, t0, te, a.rhs, 1, nfold, prow, tf);
        __syncthreads();
        for (int j = 0; j < te; ++j) {
            const double thr2 = s.thr2[j], q = s.q[0][j];
            double D2[PPT];
            Local<PPT, T> L;
            to_frame<FR, !TRI && !GRAD>(s, j, P.x, P.y, P.z, D2, L);
            // the level each pair's distance ratio asks for, as wavefront masks straight from the
            // comparisons: pairs for which level 0 suffices, then level 1, level 2, and every far
            // pair (near pairs are listed by near_list_kernel and contribute nothing here); the
            // wavefront's level and the term counts are then scalar work on the masks
            const double lim0 = c0 * thr2, lim1 = c1 * thr2, lim2 = c2 * thr2;
            bool far[PPT];
            unsigned long long u0 = 0, u1 = 0, u2 = 0, u3 = 0;  // the lanes with a pair at each level
            unsigned ec = 0;                                      // the element's far pairs
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                // masks of plain comparisons only (the backend turns a mask of a combined
                // condition into a vector select and another comparison); the rest is scalar
                far[k] = P.valid[k] && !(D2[k] < thr2);
                const unsigned long long mf = vmask[k] & ~lane_mask(D2[k] < thr2);
                const unsigned long long m0 = mf & lane_mask(D2[k] >= lim0);
                const unsigned long long m1 = mf & lane_mask(D2[k] >= lim1) & ~m0;
                const unsigned long long m2 = mf & lane_mask(D2[k] >= lim2) & ~(m0 | m1);
                u0 |= m0; u1 |= m1; u2 |= m2; u3 |= mf & ~(m0 | m1 | m2);
                ec += (unsigned)__popcll(mf);
                n0 += (unsigned)__popcll(m0);
                n1 += (unsigned)__popcll(m1);
                n2 += (unsigned)__popcll(m2);
            }
            // the finest level any pair of the wavefront needs
            const int wl = u3 ? 3 : (u2 ? 2 : (u1 ? 1 : (u0 ? 0 : -1)));
            if (wl < 0) continue;
            nc += ec;
            T o[Sums<MODE>::kNode][PPT];
            const int b = j * nn;
            if (wl == 0) { element_sum<N0, 0, FOLD, TRI, PPT, MODE>(s, j, b, o1, L, o); w0 += ec; }
            else if (wl == 1) { element_sum<N1, 0, FOLD, TRI, PPT, MODE>(s, j, b + o1, o2 - o1, L, o); w1 += ec; }
            else if (wl == 2) { element_sum<N2, 0, FOLD, TRI, PPT, MODE>(s, j, b + o2, o3 - o2, L, o); w2 += ec; }
            else {
                constexpr int G3 = tensor_group<TRI, N3>();
                element_sum<N3, G3, FOLD && (TRI || G3 == 0), TRI, PPT, MODE>(s, j, b + o3, nn - o3, L, o);
                w3 += ec;
            }
            if constexpr (!TRI && !GRAD) {
                // rows form for the rotation back; the 7 x 7 last level is in it already
                if (!(wl == 3 && tensor_group<TRI, N3>() > 0)) exp_to_rows<PPT>(L, o);
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (far[k]) add_element<FR, PPT, MODE>(P, k, q, s, j, L, o);
        }
        add_terms(w0, w1, w2, w3, nc, n0, n1, n2, o1, o2, o3, nn, terms, terms_pair);
    }
}

// DR == false: one rule per kind, NT / NR nodes.  DR == true: levels (T0..T3 / R0..R3).
// GRAD: field gradient instead of potential and field.  Compiled node counts (NT, NR > 0)
// are used only for rules whose weights are all positive (their nodes are folded).
// The FP64 gradient with levels is held to three wavefronts per SIMD (167 registers, a few
// bytes of spill): left alone the compiler takes 220 and runs two, 3.6 % slower.
template <bool DR, int NT, int NR, int T1, int T2, int T3, int R1, int R2, int R3, bool MIXED, int PPT, bool GRAD>
__global__ __launch_bounds__(kBlock, (DR && GRAD && !MIXED) ? 3 : 1) void far_eval_kernel(FarArgs a)
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
        unsigned long long terms = 0, terms_pair = 0;
        if (e_lo < nt_end)
            far_eval_dr_range<NT, T1, T2, T3, true, MIXED, PPT, MODE>(a, s, P, e_lo, nt_end, terms, terms_pair);
        if (nr_begin < e_hi)
            far_eval_dr_range<NR, R1, R2, R3, false, MIXED, PPT, MODE>(a, s, P, nr_begin, e_hi, terms, terms_pair);
        // wavefront totals: one atomic per wavefront
        if (lane_id() == 0) {
            if (terms) atomicAdd(&a.ctr->node_ints, terms);
            if (terms_pair) atomicAdd(&a.ctr->node_ints_pair, terms_pair);
        }
    } else {
        if (e_lo < nt_end) far_eval_range<NT, true, MIXED, PPT, MODE, (NT > 0)>(a, s, P, e_lo, nt_end);
        if (nr_begin < e_hi) far_eval_range<NR, false, MIXED, PPT, MODE, (NR > 0)>(a, s, P, nr_begin, e_hi);
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
    constexpr int FR = frame_form<TRI, NN, kFarPhi>();
    constexpr bool FOLD = NN > 0 && FR == kFrExp;
    const int nn = NN > 0 ? NN : (TRI ? a.rules.nt : a.rules.nr);
    const int TE = tile_elems(nn);
    const int nrhs = a.n_rhs;
    const TriForms tf = fixed_forms<NN, TRI && FOLD>(nn);
    for (int64_t t0 = e_begin; t0 < e_end; t0 += TE) {
        const int te = (int)min((int64_t)TE, e_end - t0);
        __syncthreads();
        stage_tile<TRI, MIXED, kMaxRhs, FR, false>(s, a.el, a.rules, nn, t0, te, 0, nrhs, FOLD ? nn : 0,
                                                   tensor_group<TRI, NN>() > 0 ? 0 : nn, tf);
        __syncthreads();
        for (int j = 0; j < te; ++j) {
            const double thr2 = s.thr2[j];
            double D2[PPT];
            Local<PPT, T> L;
            to_frame<FR, FR == kFrRows>(s, j, px, py, pz, D2, L);
            bool nr[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                nr[k] = valid[k] && (D2[k] < thr2);  // listed by near_list_kernel
            }
            T o[1][PPT];
            element_sum<NN, tensor_group<TRI, NN>(), FOLD, TRI, PPT, kFarPhi>(s, j, j * nn, nn, L, o);
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

// The walk runs in the element's own frame (origin at the centroid, f1 and f2 in its plane,
// f3 its normal; built at upload): the field point is p = (p1, p2, p3), and a Gaussian point
// takes its offsets (da, db, dc) from the node coordinates in that frame.  The pair's local
// sums are rotated back once.  The frame of a sliver triangle is known only to eps times its
// aspect ratio, and the rounded centroid need not lie in the element's plane (a small element
// far from the origin: by a rounding of its coordinates), so the vertices keep their third
// coordinate in the frame (a rounding-level height) and a rectangle its corner relative to the
// centroid: with them the nodes are the exact combinations of the vertices, as in three
// dimensions.  A rectangle node's height varies across a cell only by rounding-level amounts
// (the sides' heights): the cell centre's height serves all its Gaussian points.
//
// Node geometry: a triangle node has a first vertex and two edge vectors (lattice position
// (i, j) in units of h = 2^-level along the root's edges B - A and C - A; an up node has
// vertices (i, j), (i+1, j), (i, j+1), a down node (i+1, j+1), (i, j+1), (i+1, j)); a
// rectangle node is the cell (i, j) of the h-grid along e1 and e2.
struct NearGeom {
    double ax, ay, az;  // triangle: root vertex A; rectangle: corner P0 (from the centroid)
    double ux, uy, uz;  // triangle: B - A; rectangle: e1 (in-plane, uz = 0)
    double vx, vy, vz;  // triangle: C - A; rectangle: e2 (in-plane, vz = 0)
};

// Node s: its first vertex (triangle) or centre (rectangle) and, for triangles, its edge
// vectors w1 = V1 - V0, w2 = V2 - V0; the node centroid c.
struct NodeGeom {
    double x0, y0, z0, w1x, w1y, w1z, w2x, w2y, w2z, cx, cy, cz;
};
__device__ __forceinline__ void node_geometry(const NearState& s, const NearGeom& g, double h, NodeGeom& n)
{
    if (s.kind == 0) {
        const double u = s.up ? s.i : s.i + 1, v = s.up ? s.j : s.j + 1, sg = s.up ? h : -h;
        n.x0 = fma(u * h, g.ux, fma(v * h, g.vx, g.ax));
        n.y0 = fma(u * h, g.uy, fma(v * h, g.vy, g.ay));
        n.z0 = fma(u * h, g.uz, fma(v * h, g.vz, g.az));
        n.w1x = sg * g.ux; n.w1y = sg * g.uy; n.w1z = sg * g.uz;
        n.w2x = sg * g.vx; n.w2y = sg * g.vy; n.w2z = sg * g.vz;
        n.cx = fma(1.0 / 3.0, n.w1x + n.w2x, n.x0);
        n.cy = fma(1.0 / 3.0, n.w1y + n.w2y, n.y0);
        n.cz = fma(1.0 / 3.0, n.w1z + n.w2z, n.z0);
    } else {
        const double ih = (s.i + 0.5) * h, jh = (s.j + 0.5) * h;
        n.cx = fma(ih, g.ux, fma(jh, g.vx, g.ax));
        n.cy = fma(ih, g.uy, fma(jh, g.vy, g.ay));
        n.cz = fma(ih, g.uz, fma(jh, g.vz, g.az));  // the height of the cell centre (rounding level)
        n.x0 = n.cx; n.y0 = n.cy; n.z0 = n.cz;
        n.w1x = n.w1y = n.w1z = n.w2x = n.w2y = n.w2z = 0.0;
    }
}

// Sums of one Gaussian point at offsets (da, db, dc) in the element's frame, weight w (unit
// element charge):
//   field:        f0 += w/r, (f1, f2, f3) += w (da, db, dc)/r^3;
//   collocation:  f0 += w/r;
//   gradient:     f0 += w/r^3, (f1 .. f6) += w (da^2, db^2, dc^2, da db, da dc, db dc)/r^5.
template <int MODE>
__device__ __forceinline__ void near_terms(double w, double da, double db, double dc, double (&f)[7])
{
    const double ri = rsqrt64(fma(da, da, fma(db, db, dc * dc)));
    const double wr = w * ri;
    if constexpr (MODE == kNearColloc) {
        f[0] += wr;
    } else if constexpr (MODE == kNearEval) {
        const double w3 = wr * (ri * ri);
        f[0] += wr;
        f[1] = fma(w3, da, f[1]);
        f[2] = fma(w3, db, f[2]);
        f[3] = fma(w3, dc, f[3]);
    } else {
        const double ri2 = ri * ri, w3 = wr * ri2, w5 = w3 * ri2;
        const double ua = w5 * da, ub = w5 * db, uc = w5 * dc;
        f[0] += w3;
        f[1] = fma(ua, da, f[1]);
        f[2] = fma(ub, db, f[2]);
        f[3] = fma(uc, dc, f[3]);
        f[4] = fma(ua, db, f[4]);
        f[5] = fma(ua, dc, f[5]);
        f[6] = fma(ub, dc, f[6]);
    }
}

// Pairs whose field point lies on the element (the trailing entries of the order, from
// *walk_end to the pair count): the exact integral about the point, one lane per pair; the
// walk kernel's lanes take them once the walks are done (grid-stride from `first`).  Per
// edge at distance h from the point with end offsets t1, t2 along it (rho^2 = h^2 + t^2):
// potential h [asinh(t/h)], field -n [(t/rho)(1 + ln rho) - asinh(t/h)] + h t [(1 + ln rho)/rho]
// (n the unit vector from the point's foot on the edge line towards the point's side).
template <int MODE>
__device__ __forceinline__ void on_element_pairs(const NearArgs& a, unsigned long long first, unsigned long long stride)
{
    constexpr bool COLLOC = MODE == kNearColloc;
    constexpr bool GRAD = MODE == kNearGrad;
    const Elements& el = a.el;
    const int64_t ne = el.ne;
    const unsigned long long total = min(a.ctr->near_count, a.near_cap);
    unsigned long long n_on = 0;
    for (unsigned long long w = *a.walk_end + first; w < total; w += stride) {
        const NearPair pr = a.opair[w];
        const unsigned long long cur = a.slot[a.order[w]];
        const int64_t e = pr.elem, p = pr.point;
        const bool tri = e < el.n_tri;
        double X[3];
        if (COLLOC) {
            X[0] = el.cen[p]; X[1] = el.cen[ne + p]; X[2] = el.cen[2 * ne + p];
        } else {
            X[0] = a.pts[p]; X[1] = a.pts[a.n + p]; X[2] = a.pts[2 * a.n + p];
        }
        double G[9], P[3], V[4][3];
        point_on_element(el, e, tri, X, G, P);  // (true: the cost pass put the pair here)
        const int nv = element_corners(el, e, tri, G, V);
        const double L = el.L[e];
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
        if (COLLOC) {
            a.res[cur] = s0 * inv_area;
        } else if (GRAD) {  // the normal field jumps across the element: no gradient there
            const double nan = __builtin_nan("");
            double2* r = reinterpret_cast<double2*>(a.res + 6 * cur);
            r[0] = make_double2(nan, nan);
            r[1] = make_double2(nan, nan);
            r[2] = make_double2(nan, nan);
        } else {
            const double Kq = a.K * el.q[(int64_t)a.rhs * ne + e];
            reinterpret_cast<double4*>(a.res)[cur] = make_double4(
                Kq * (s0 * inv_area), Kq * (s1 * inv_area), Kq * (s2 * inv_area), Kq * (s3 * inv_area));
        }
        n_on++;
    }
    if (n_on) atomicAdd(&a.ctr->on_surface, n_on);
}

constexpr unsigned kNearWindow = 64;  // entries of the order a wavefront claims at a time
constexpr int kNearWaves = kBlock / 64;
constexpr int kFront = 128;  // near nodes of one level of a breadth-first walk (per wavefront)
constexpr int kLeafQ = 128;  // leaves waiting for the rule: a batch of 64 and one chunk's more

// A pair's walk set-up from the element's record: the element kind, its node geometry in the
// element's frame, the field point in that frame (offset from the centroid: numbers of the
// element's size, accurate for points very close to a small element far from the origin)
// and the threshold (near_dr L)^2.
template <int MODE>
__device__ __forceinline__ void pair_setup(const NearArgs& a, uint32_t p, uint32_t e, int& kind, NearGeom& g,
                                           double& p1, double& p2, double& p3, double& thr2)
{
    const Elements& el = a.el;
    const int64_t ne = el.ne;
    double P[3];
    if (MODE == kNearColloc) {
        P[0] = el.cen[p]; P[1] = el.cen[ne + p]; P[2] = el.cen[2 * ne + p];
    } else {
        P[0] = a.pts[p]; P[1] = a.pts[a.n + p]; P[2] = a.pts[2 * a.n + p];
    }
    kind = (int64_t)e < el.n_tri ? 0 : 1;
    double R[kNearRec];  // centroid, frame F, loc, thr2
    {
        const double2* rec = reinterpret_cast<const double2*>(el.nrec + (int64_t)e * kNearRec);
#pragma unroll
        for (int c = 0; c < 11; ++c) {
            const double2 v = rec[c];
            R[2 * c] = v.x;
            R[2 * c + 1] = v.y;
        }
    }
    const double* F = R + 3;
    const double* lc = R + 12;
    const double dxc = P[0] - R[0], dyc = P[1] - R[1], dzc = P[2] - R[2];
    p1 = fma(F[0], dxc, fma(F[1], dyc, F[2] * dzc));
    p2 = fma(F[3], dxc, fma(F[4], dyc, F[5] * dzc));
    p3 = fma(F[6], dxc, fma(F[7], dyc, F[8] * dzc));
    if (kind == 0) {  // vertices A', B', C' in the frame
        g.ax = lc[0]; g.ay = lc[1]; g.az = lc[6];
        g.ux = lc[2] - g.ax; g.uy = lc[3] - g.ay; g.uz = lc[7] - g.az;
        g.vx = lc[4] - g.ax; g.vy = lc[5] - g.ay; g.vz = lc[8] - g.az;
    } else {  // e1 = (2 gamma, 2 beta, h1), e2 = (2 alpha, 0, h2); the corner P0 - c
        g.ux = 2.0 * lc[0]; g.uy = 2.0 * lc[1]; g.uz = lc[6];
        g.vx = 2.0 * lc[2]; g.vy = 0.0; g.vz = lc[7];
        g.ax = lc[3]; g.ay = lc[4]; g.az = lc[5];
    }
    thr2 = R[21];
}

// The distance test of node s: its scale h = 2^-level, its geometry, and whether the point is
// within near_dr times the node's own L of its centroid.
__device__ __forceinline__ bool visit_node(const NearState& s, const NearGeom& g, double p1, double p2, double p3,
                                           double thr2, double& h, NodeGeom& nd)
{
    h = ldexp(1.0, -s.level);
    node_geometry(s, g, h, nd);
    const double qx = p1 - nd.cx, qy = p2 - nd.cy, qz = p3 - nd.cz;
    const double D2 = fma(qx, qx, fma(qy, qy, qz * qz));
    return D2 < thr2 * h * h;
}

// The element's rule on leaf node nd (scale h), weights scaled by the area ratio h^2, added to
// acc (the sums of near_terms in the element's frame).
template <int MODE>
__device__ __forceinline__ void leaf_add(int kind, const NearGeom& g, double p1, double p2, double p3,
                                         const NodeGeom& nd, double h, const double4* __restrict__ tri_nodes,
                                         const double4* __restrict__ rect_nodes, int nt, int nr, double (&acc)[7])
{
    double f[7] = { 0, 0, 0, 0, 0, 0, 0 };
    if (kind == 0) {
        const double q1 = p1 - nd.x0, q2 = p2 - nd.y0, q3 = p3 - nd.z0;
#pragma unroll 4
        for (int i = 0; i < nt; ++i) {
            const double4 q = tri_nodes[i];
            const double lb = q.y, lc = q.z, w = q.w;
            const double da = fma(-lb, nd.w1x, fma(-lc, nd.w2x, q1));
            const double db = fma(-lb, nd.w1y, fma(-lc, nd.w2y, q2));
            const double dc = fma(-lb, nd.w1z, fma(-lc, nd.w2z, q3));
            near_terms<MODE>(w, da, db, dc, f);
        }
    } else {
        const double qx = p1 - nd.cx, qy = p2 - nd.cy, qz = p3 - nd.cz;
        const double H1x = h * (0.5 * g.ux), H1y = h * (0.5 * g.uy), H2x = h * (0.5 * g.vx);
#pragma unroll 4
        for (int i = 0; i < nr; ++i) {
            const double4 q = rect_nodes[i];
            const double x = q.x, y = q.y, w = q.z;
            const double da = fma(-x, H1x, fma(-y, H2x, qx));
            const double db = fma(-x, H1y, qy);
            near_terms<MODE>(w, da, db, qz, f);
        }
    }
    const double h2 = h * h;
    constexpr int NS = MODE == kNearGrad ? 7 : (MODE == kNearColloc ? 1 : 4);
#pragma unroll
    for (int c = 0; c < NS; ++c) acc[c] = fma(h2, f[c], acc[c]);
}

// The pair's own result record at its slot (32 bytes for the field, 48 for the gradient);
// collocation keeps the unit-density potential (the densities are applied per right-hand
// side when the sums are formed).
template <int MODE>
__device__ __forceinline__ void write_record(const NearArgs& a, uint32_t e, unsigned long long cur,
                                             const double (&acc)[7])
{
    const Elements& el = a.el;
    if (MODE == kNearColloc) {
        a.res[cur] = acc[0];
        return;
    }
    const double Kq = a.K * el.q[(int64_t)a.rhs * el.ne + e];
    double F[9];
    {
        const double* rec = el.nrec + (int64_t)e * kNearRec + 3;
#pragma unroll
        for (int c = 0; c < 9; ++c) F[c] = rec[c];
    }
    if (MODE == kNearGrad) {
        // local tensor m = sum w d d^T / r^5 (d = (da, db, dc)), global M = F^T m F,
        // dE_i/dx_j = q (delta_ij S3 - 3 M_ij)
        const double m[3][3] = { { acc[1], acc[4], acc[5] },
                                 { acc[4], acc[2], acc[6] },
                                 { acc[5], acc[6], acc[3] } };
        double U[3][3];  // U[r][v] = sum_b m[r][b] F[b][v]
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int v = 0; v < 3; ++v) U[r][v] = fma(m[r][0], F[v], fma(m[r][1], F[3 + v], m[r][2] * F[6 + v]));
        auto M = [&](int u, int v) { return fma(F[u], U[0][v], fma(F[3 + u], U[1][v], F[6 + u] * U[2][v])); };
        double2* r = reinterpret_cast<double2*>(a.res + 6 * cur);
        r[0] = make_double2(Kq * fma(-3.0, M(0, 0), acc[0]), Kq * fma(-3.0, M(1, 1), acc[0]));
        r[1] = make_double2(Kq * fma(-3.0, M(2, 2), acc[0]), -3.0 * Kq * M(0, 1));
        r[2] = make_double2(-3.0 * Kq * M(0, 2), -3.0 * Kq * M(1, 2));
    } else {
        // local field sum w (da, db, dc)/r^3, rotated back
        reinterpret_cast<double4*>(a.res)[cur] = make_double4(
            Kq * acc[0], Kq * fma(F[0], acc[1], fma(F[3], acc[2], F[6] * acc[3])),
            Kq * fma(F[1], acc[1], fma(F[4], acc[2], F[7] * acc[3])),
            Kq * fma(F[2], acc[1], fma(F[5], acc[2], F[8] * acc[3])));
    }
}

// A node of a breadth-first walk in one 64-bit word: i, j (24 bits each: depth cap <= 24),
// orientation, level.
__device__ __forceinline__ uint64_t pack_node(const NearState& s)
{
    return (uint64_t)(uint32_t)s.i | ((uint64_t)(uint32_t)s.j << 24) | ((uint64_t)(s.up ? 1 : 0) << 48) |
           ((uint64_t)(uint32_t)s.level << 49);
}
__device__ __forceinline__ NearState unpack_node(uint64_t v, int kind)
{
    NearState s;
    s.kind = kind;
    s.i = (int)(v & 0xffffffull);
    s.j = (int)((v >> 24) & 0xffffffull);
    s.up = ((v >> 48) & 1ull) != 0;
    s.level = (int)(v >> 49);
    return s;
}

// LDS written by some lanes of a wavefront, read by others: finish the writes first.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Move to the next node of a depth-first walk of the subtree below `root` (level) after
// finishing node s; false when the walk has returned to the subtree's root.
__device__ __forceinline__ bool advance_within(NearState& s, int root)
{
    while (s.level > root) {
        const int c = child_index(s);  // s is now the parent
        if (c < 3) {
            to_child(s, c + 1);
            return true;
        }
    }
    return false;
}

// One lane walks the subtree below the near node s (above the depth cap) depth first.
template <int MODE>
__device__ void walk_subtree(NearState s, const NearGeom& g, double p1, double p2, double p3, double thr2,
                             int max_depth, const double4* __restrict__ tri_nodes,
                             const double4* __restrict__ rect_nodes, int nt, int nr, double (&acc)[7],
                             unsigned long long& n_leaves, unsigned long long& n_cap, int& max_level)
{
    const int root = s.level;
    to_child(s, 0);
    while (true) {
        double h;
        NodeGeom nd;
        const bool near = visit_node(s, g, p1, p2, p3, thr2, h, nd);
        if (s.level > max_level) max_level = s.level;
        if (near && s.level < max_depth) {
            to_child(s, 0);
            continue;
        }
        leaf_add<MODE>(s.kind, g, p1, p2, p3, nd, h, tri_nodes, rect_nodes, nt, nr, acc);
        n_leaves++;
        if (near) n_cap++;
        if (!advance_within(s, root)) break;
    }
}

// A pair with a deep subdivision (the leading cost classes), walked by a whole wavefront
// breadth first: per level, the children of the level's near nodes are tested 64 at a time,
// the near ones (above the depth cap) form the next level, the others are leaves; leaves
// wait in LDS until 64 of them can take the rule loop together, one per lane.  A point very
// close to an element has a near region of some 65 nodes at every level (three node sizes
// around its foot), so its depth-first walk would take thousands of visits in one lane.
// Each lane sums its leaves in a fixed order; the lanes' sums are added by a fixed butterfly,
// so results are reproducible.  More near nodes in a level than kFront: the lane that found
// one walks its subtree depth first itself.  The visit limit ends the walk after the level in
// which the pair's visits pass it.
template <int MODE>
__device__ void heavy_pair(const NearArgs& a, unsigned long long w, uint64_t* front, uint64_t* leafq,
                           const double4* __restrict__ tri_nodes, const double4* __restrict__ rect_nodes, int nt,
                           int nr, int lane, unsigned long long& n_leaves, unsigned long long& n_cap,
                           unsigned long long& n_limit, int& max_level)
{
    const NearPair pr = a.opair[w];
    const unsigned long long cur = a.slot[a.order[w]];
    int kind;
    NearGeom g;
    double p1, p2, p3, thr2;
    pair_setup<MODE>(a, pr.point, pr.elem, kind, g, p1, p2, p3, thr2);
    double acc[7] = { 0, 0, 0, 0, 0, 0, 0 };
    // the same in every lane: the current level's near nodes (nF, in cur_f), the next level's
    // (nN), the next child of the level to test (base), the queued leaves (nq), the visits
    uint64_t* cur_f = front;
    uint64_t* nxt_f = front + kFront;
    int nF = 1, nN = 0, base = 0, nq = 0;
    long long visits = 0;
    bool done = false;
    if (a.max_depth <= 0) {  // the rule on the element itself (depth cap 0): the root is the leaf
        if (lane == 0) {
            const NearState s{ kind, 0, 0, 0, true };
            double h;
            NodeGeom nd;
            n_leaves++;
            if (visit_node(s, g, p1, p2, p3, thr2, h, nd)) n_cap++;
            leafq[0] = pack_node(s);
        }
        nq = 1;
        done = true;
    } else if (lane == 0) {
        cur_f[0] = pack_node(NearState{ kind, 0, 0, 0, true });
    }
    wave_lds_sync();
    while (true) {
        if (!done && base >= 4 * nF) {  // the level is tested: on to the next one
            uint64_t* t = cur_f;
            cur_f = nxt_f;
            nxt_f = t;
            nF = nN;
            nN = 0;
            base = 0;
            if (nF == 0) {
                done = true;
            } else if (visits > a.visit_limit) {  // the limit ends the walk here
                if (lane == 0) n_limit++;
                done = true;
            }
        }
        if (nq >= 64 || (done && nq > 0)) {  // a batch of leaves, one per lane
            const int k = min(nq, 64);
            if (lane < k) {
                const NearState t = unpack_node(leafq[lane], kind);
                double h;
                NodeGeom nd;
                (void)visit_node(t, g, p1, p2, p3, thr2, h, nd);
                leaf_add<MODE>(kind, g, p1, p2, p3, nd, h, tri_nodes, rect_nodes, nt, nr, acc);
            }
            const uint64_t rest = lane < nq - k ? leafq[k + lane] : 0ull;
            wave_lds_sync();
            if (lane < nq - k) leafq[lane] = rest;
            wave_lds_sync();
            nq -= k;
            continue;
        }
        if (done) break;
        // the next 64 children of the level's near nodes
        const int c = base + lane;
        const bool valid = c < 4 * nF;
        NearState s{ kind, 0, 0, 0, true };
        bool near = false;
        if (valid) {
            s = unpack_node(cur_f[c >> 2], kind);
            to_child(s, c & 3);
            double h;
            NodeGeom nd;
            near = visit_node(s, g, p1, p2, p3, thr2, h, nd);
            if (s.level > max_level) max_level = s.level;
        }
        visits += (long long)__popcll(lane_mask(valid));
        const bool desc = valid && near && s.level < a.max_depth;
        const bool leaf = valid && !desc;
        if (leaf) {
            n_leaves++;
            if (near) n_cap++;
        }
        // descending children: the next level (index order); past kFront a lane walks its
        // child's subtree itself
        const unsigned long long dm = lane_mask(desc);
        const int pos = nN + (int)lanes_below(dm);
        const bool spill = desc && pos >= kFront;
        if (desc && !spill) nxt_f[pos] = pack_node(s);
        nN = min(kFront, nN + (int)__popcll(dm));
        // leaves: the queue (fewer than 64 wait when a chunk adds at most 64)
        const unsigned long long lm = lane_mask(leaf);
        if (leaf) leafq[nq + (int)lanes_below(lm)] = pack_node(s);
        nq += (int)__popcll(lm);
        base += 64;
        wave_lds_sync();
        if (spill)
            walk_subtree<MODE>(s, g, p1, p2, p3, thr2, a.max_depth, tri_nodes, rect_nodes, nt, nr, acc, n_leaves,
                               n_cap, max_level);
    }
    wave_lds_sync();  // the queue and the levels are reused by the next pair
    // the lanes' sums added by a fixed butterfly (every lane ends with the same total)
#pragma unroll
    for (int c = 0; c < 7; ++c)
        for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o);
    if (lane == 0) write_record<MODE>(a, pr.elem, cur, acc);
}

// MODE: kNearEval (phi, E at field points), kNearColloc (phi at centroids, several density
// vectors), kNearGrad (field gradient at field points; NaN for a point on its element).
template <int MODE, bool DEEP>
__global__ __launch_bounds__(kBlock) void near_kernel(NearArgs a)
{
    // the walks: the leading entries of the order (the points lying on their element follow);
    // the first `heavy` of them have deep subdivisions (DEEP: walked breadth first, a wavefront
    // each; else depth first like the others)
    const unsigned long long total = *a.walk_end, heavy = DEEP ? *a.heavy_end : 0ull;
    const int lane = lane_id();
    // the rules' nodes in LDS: a leaf's loop reads them at one address for the whole wavefront
    // (from global memory every node would be a vector load and a wait for it)
    extern __shared__ double4 near_rule_nodes[];  // [nt] triangle (la, lb, lc, w), [nr] rectangle (x, y, w, 0)
    __shared__ uint64_t near_front[kNearWaves][2 * kFront];
    __shared__ uint64_t near_leafq[kNearWaves][kLeafQ];
    const int nt = a.rules.nt, nr = a.rules.nr;
    for (int i = threadIdx.x; i < nt + nr; i += kBlock) {
        const double* src = i < nt ? a.rules.tri + 4 * i : a.rules.rect + 4 * (i - nt);
        near_rule_nodes[i] = make_double4(src[0], src[1], src[2], src[3]);
    }
    __syncthreads();
    const double4* __restrict__ tri_nodes = near_rule_nodes;
    const double4* __restrict__ rect_nodes = near_rule_nodes + nt;

    unsigned long long n_leaves = 0, n_cap = 0, n_limit = 0;
    int max_level = 0;

    // ---- the deep pairs, one per wavefront at a time (no claim at all without them: a
    // launch's thousand wavefronts claiming one counter cost microseconds)
    while (DEEP && heavy > 0) {
        unsigned long long hw = 0;
        if (lane == 0) hw = atomicAdd(&a.ctr->heavy_cursor, 1ull);
        hw = bcast_u64(hw, 0);
        if (hw >= heavy) break;
        heavy_pair<MODE>(a, hw, near_front[threadIdx.x / 64], near_leafq[threadIdx.x / 64], tri_nodes, rect_nodes,
                         nt, nr, lane, n_leaves, n_cap, n_limit, max_level);
    }

    // ---- the other pairs, one per lane, depth first
    bool active = false;
    NearState st{ 0, 0, 0, 0, true };
    uint32_t e = 0;
    unsigned long long cur = 0;  // result slot of the pair in hand
    NearGeom g{};
    double p1 = 0.0, p2 = 0.0, p3 = 0.0;  // the field point in the element's frame
    double thr2 = 0.0, acc[7] = { 0, 0, 0, 0, 0, 0, 0 };
    int64_t visits = 0;
    // the wavefront's window of the order (the same in every lane): kNearWindow consecutive
    // entries claimed with one atomic, handed to its lanes as they need pairs; consecutive
    // entries are pairs of one cost class, so the lanes walk trees of one kind and similar size
    unsigned long long win = 0, win_end = 0;

    while (total > heavy) {
        // ---- refill from the window (a new window when it is used up)
        const unsigned long long need = lane_mask(!active);
        if (need) {
            if (win >= win_end) {
                const int first = __ffsll((long long)need) - 1;
                unsigned long long b = 0;
                if (lane == first) b = atomicAdd(&a.ctr->cursor, (unsigned long long)kNearWindow);
                win = heavy + bcast_u64(b, first);
                win_end = win + kNearWindow;
            }
            const unsigned rank = lanes_below(need);
            const unsigned long long avail = win_end - win, w = win + rank;
            win += min(avail, (unsigned long long)__popcll(need));
            // a lane without an entry (the window ran out) waits for the next one
            if (!active && rank < avail) {
                if (w >= total) break;
                const NearPair pr = a.opair[w];  // most expensive pairs first
                cur = a.slot[a.order[w]];
                e = pr.elem;
                pair_setup<MODE>(a, pr.point, pr.elem, st.kind, g, p1, p2, p3, thr2);
#pragma unroll
                for (int c = 0; c < 7; ++c) acc[c] = 0.0;
                visits = 0;
                active = true;
                st.i = 0; st.j = 0; st.up = true;
                if (a.max_depth <= 0) st.level = 0;  // evaluate the rule on the element itself (depth cap)
                else st.level = 1;                   // first child of the root
            }
        }

        if (!active) continue;
        // ---- visit nodes from st down to the next leaf (each lane on its own: internal nodes
        // cost a distance test, so the lanes then take the leaf loop together)
        double h;
        bool is_near;
        NodeGeom nd;
        while (true) {
            is_near = visit_node(st, g, p1, p2, p3, thr2, h, nd);
            ++visits;
            if (st.level > max_level) max_level = st.level;
            if (!(is_near && st.level < a.max_depth && visits <= a.visit_limit)) break;
            to_child(st, 0);
        }
        leaf_add<MODE>(st.kind, g, p1, p2, p3, nd, h, tri_nodes, rect_nodes, nt, nr, acc);
        n_leaves++;
        if (is_near) n_cap++;
        bool finished;
        if (visits > a.visit_limit) {
            n_limit++;
            finished = true;
        } else {
            finished = !advance(st);
        }
        if (!finished) continue;
        write_record<MODE>(a, e, cur, acc);
        active = false;
        st.level = 0;
    }

    // per-lane counters -> one atomic per counter per lane that has something to add
    if (n_leaves) atomicAdd(&a.ctr->leaves, n_leaves);
    if (n_cap) atomicAdd(&a.ctr->cap_hits, n_cap);
    if (n_limit) atomicAdd(&a.ctr->visit_limit_hits, n_limit);
    if (max_level) atomicMax(&a.ctr->max_depth, (unsigned long long)max_level);

    // then the pairs whose point lies on the element (after the walk loop: none of its
    // state is live here, so the closed form does not add to the walk's registers)
    on_element_pairs<MODE>(a, (unsigned long long)blockIdx.x * kBlock + threadIdx.x,
                           (unsigned long long)gridDim.x * kBlock);
}

// ---------------------------------------------------------------- small kernels -----
// One 192-byte record per element with what the near walk reads when it takes a pair (three
// 64-byte lines instead of 22 from the separate arrays): centroid, frame, loc, thr2.
__global__ void pack_near_records_kernel(Elements el, double* __restrict__ nrec)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t ne = el.ne;
    if (e >= ne) return;
    double r[kNearRec];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = el.cen[c * ne + e];
#pragma unroll
    for (int c = 0; c < 9; ++c) r[3 + c] = el.frame[c * ne + e];
#pragma unroll
    for (int c = 0; c < 9; ++c) r[12 + c] = el.loc[c * ne + e];
    r[21] = el.thr2[e];
    r[22] = 0.0;
    r[23] = 0.0;
    double2* out = reinterpret_cast<double2*>(nrec + e * kNearRec);
#pragma unroll
    for (int c = 0; c < kNearRec / 2; ++c) out[c] = make_double2(r[2 * c], r[2 * c + 1]);
}

__global__ void charges_kernel(const double* sigma, const double* area, double* q, int64_t ne, int n_rhs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne * n_rhs) return;
    q[i] = sigma[i] * area[i % ne];
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
    // a small evaluation (fewer than 1024 workgroups at three points per lane: under one
    // wavefront per SIMD and four per CU) takes one point per lane: more wavefronts hide the
    // latency of the dependent FP64 chains
    const bool small = !MIXED && (a.n + 3 * kBlock - 1) / (3 * kBlock) * a.n_split < 1024;
    if (small && nr == 49 && nt == 7) return far_eval_launch<false, 7, 49, 0, 0, 0, 0, 0, 0, MIXED, 1, false>(a, s);
    if (small && nr == 49 && nt == 33) return far_eval_launch<false, 33, 49, 0, 0, 0, 0, 0, 0, MIXED, 1, false>(a, s);
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

// Collocation points per lane: three in FP64, two in the mixed path (on the 200,000-element
// nested cylinders 1.5 % faster than two in FP64; one was slower in both, three slower mixed).
template <bool MIXED>
hipError_t far_colloc_dispatch(const FarArgs& a, hipStream_t s)
{
    constexpr int PPT = MIXED ? 2 : 3;
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
    // persistent lanes (no more than the list can hold pairs); every lane leaves once the
    // shared cursor passes the pair count
    const int blocks = (int)std::max<unsigned long long>(1, std::min<unsigned long long>(1024, (a.near_cap + kBlock - 1) / kBlock));
    const size_t lds = (size_t)(a.rules.nt + a.rules.nr) * sizeof(double4);
    if (mode == kNearColloc) near_kernel<kNearColloc, true><<<blocks, kBlock, lds, s>>>(a);
    else if (mode == kNearGrad) near_kernel<kNearGrad, true><<<blocks, kBlock, lds, s>>>(a);
    else if (a.deep) near_kernel<kNearEval, true><<<blocks, kBlock, lds, s>>>(a);
    else near_kernel<kNearEval, false><<<blocks, kBlock, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_near_list(const double* pts, int64_t n, const Elements& el, NearPair* list, unsigned long long cap,
                            DevCounters* ctr, hipStream_t s)
{
    if (n <= 0 || el.ne <= 0) return hipSuccess;
    const int64_t blocks = (n + kListPoints - 1) / kListPoints;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    // few point blocks (a small evaluation): split the elements into chunks (multiples of 16
    // elements), up to about 2048 workgroups in all
    const int64_t units = (el.ne + 15) / 16;
    const int64_t split = std::max<int64_t>(1, std::min<int64_t>({ (2048 + blocks - 1) / blocks, units, 65535 }));
    const int64_t chunk = ((units + split - 1) / split) * 16;
    const int64_t chunks = (el.ne + chunk - 1) / chunk;
    near_list_kernel<<<dim3((unsigned)blocks, (unsigned)chunks), kBlock, 0, s>>>(pts, n, el, list, cap, ctr, chunk);
    return hipGetLastError();
}

hipError_t launch_pack_near_records(const Elements& el, double* nrec, hipStream_t s)
{
    if (el.ne <= 0) return hipSuccess;
    pack_near_records_kernel<<<(unsigned)((el.ne + kBlock - 1) / kBlock), kBlock, 0, s>>>(el, nrec);
    return hipGetLastError();
}

hipError_t launch_charges(const double* sigma, const double* area, double* q, int64_t ne, int n_rhs, hipStream_t s)
{
    const int64_t tot = ne * n_rhs;
    if (tot <= 0) return hipSuccess;
    charges_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(sigma, area, q, ne, n_rhs);
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

__global__ void reset_near_count_kernel(DevCounters* c) { c->near_count = 0ull; }

// everything the list pass and the near stage count; the far field's term counts stay
__global__ void reset_near_stage_kernel(DevCounters* c)
{
    c->near_count = 0ull;
    c->cursor = 0ull;
    c->leaves = 0ull;
    c->cap_hits = 0ull;
    c->on_surface = 0ull;
    c->max_depth = 0ull;
    c->visit_limit_hits = 0ull;
    c->heavy_cursor = 0ull;
}

hipError_t launch_reset_near_stage(DevCounters* c, hipStream_t s)
{
    reset_near_stage_kernel<<<1, 1, 0, s>>>(c);
    return hipGetLastError();
}

hipError_t launch_reset_near_count(DevCounters* c, hipStream_t s)
{
    reset_near_count_kernel<<<1, 1, 0, s>>>(c);
    return hipGetLastError();
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
