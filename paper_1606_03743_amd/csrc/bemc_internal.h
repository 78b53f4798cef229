// Internal declarations shared by the host runtime and the kernels of the GPU library.
#pragma once

#include <hip/hip_runtime.h>

#include "bemc.h"

#include <cstdint>
#include <string>
#include <vector>

namespace bemc {

// ------------------------------------------------------------------ rules (host)
struct TriNode {
    double la, lb, lc, w;  // barycentric coordinates (Eq. 3.3) and weight
};
struct RectNode {
    double x, y, w;  // natural coordinates (Eq. 3.2) and weight
};
bool triangle_rule(int n, std::vector<TriNode>& out);
bool gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
bool rectangle_gauss_rule(int n, std::vector<RectNode>& out);
bool rectangle_table_rule(int n, std::vector<RectNode>& out);

constexpr int kMaxTriNodes = 64;
constexpr int kMaxRectNodes = 256;
constexpr int kMaxRhs = 8;
// rule choice by distance ratio: the last level (the context's rules) must be at least as
// fine as the third level (19-point triangle rule, Table B4)
constexpr int kMinDrTriNodes = 19;
constexpr int kMinDrRectNodes = 17;

// ------------------------------------------------------------------ device data
// Rule tables in device memory: triangle nodes as (la, lb, lc, w), rectangle nodes as
// (x, y, w, 0); FP32 copies for the mixed path.
struct RuleTables {
    const double* tri;    // [nt][4]  la, lb, lc, w
    const double* rect;   // [nr][4]  x, y, w, 0  (Gauss-Legendre n x n: node i n + j = (x_i, x_j))
    int nt, nr;
};

// Element arrays, SoA over the global element index (triangles first).
struct Elements {
    const double* geom;  // [9][ne]  input geometry: A,B,C  or  P0,e1,e2
    const double* cen;   // [3][ne]  centroid
    const double* thr2;  // [ne]     (near_dr * L)^2
    const double* frame; // [9][ne]  orthonormal frame f1, f2 (in the plane), f3 (normal);
                         //          rectangles: f1 along e2
    const double* loc;   // [9][ne]  tri: in-plane coordinates (f1, f2) of A-c, B-c, C-c, then their
                         //          f3 components (rounding-level heights, kept by the near field);
                         //          rect: gamma = f1.e1/2, beta = f2.e1/2, alpha = |e2|/2, the corner
                         //          P0 - c in the frame (3), the f3 components of e1 and e2, 0
    const double* nrec;  // [ne][kNearRec] the near walk's record of each element in one place:
                         //          centroid (3), frame (9), loc (9), thr2, 2 unused
    const double* L;     // [ne]     average side length
    const double* area;  // [ne]
    const double* nrm;   // [3][ne]  unit normal
    const double* q;     // [n_rhs][ne]  sigma * area
    int64_t ne;
    int n_tri;
    int n_rhs;
};

constexpr int kNearRec = 24;  // doubles per near-walk record (192 B)

// Rule choice by distance ratio: four levels per element kind, coarsest first
// (triangles 7/12/19/tri_rule points, rectangles Tables B2/B3/B4 then the rectangle rule).
// The level tables hold the nodes of all four levels back to back.
struct LevelRules {
    RuleTables tab;       // tri: [7 | 12 | 19 | nt] nodes, rect: [7 | 12 | 17 | nr] nodes
    int tri_off[5];       // node offsets of the levels within an element's staged nodes
    int rect_off[5];
    double tri_c[3];      // level l is used when D^2 >= tri_c[l] * (near_dr L)^2
    double rect_c[3];
};

struct NearPair {
    uint32_t point;
    uint32_t elem;
};

// Device counters of one evaluation.
struct DevCounters {
    unsigned long long near_count;  // near pairs found by the far kernel (may exceed capacity)
    unsigned long long cursor;      // work cursor of the near kernel
    unsigned long long leaves;
    unsigned long long cap_hits;
    unsigned long long on_surface;
    unsigned long long max_depth;
    unsigned long long visit_limit_hits;
    unsigned long long node_ints;  // point-charge terms summed (rule choice by distance ratio)
    unsigned long long node_ints_pair;  // the terms each far pair's own level would sum
    unsigned long long heavy_cursor;    // work cursor of the near kernel's deep pairs
};

// Arguments of the far-field kernels.
struct FarArgs {
    Elements el;
    RuleTables rules;
    const double* pts;       // [3][n] (eval)  -- unused for collocation
    int64_t n;               // field points (eval) or rows (collocation)
    int rhs;                 // density vector (eval)
    int n_rhs;               // collocation right-hand sides
    double K;                // Coulomb constant
    double* phi;             // [n] (eval) or out[n_rhs][ne] (collocation)
    double* E;               // [3][n] or null
    double* G;               // [6][n] field gradient (gradient mode)
    double* partial;         // element-split partial sums [n_split][rows][n] or null
    int64_t elem_begin, elem_end;  // element range of this launch
    int n_split;             // > 1: blockIdx.y takes elements [begin + y chunk, begin + (y+1) chunk)
    int64_t chunk;
    NearPair* near_list;
    unsigned long long near_cap;
    DevCounters* ctr;
    int dr_rules;            // 1: per-pair rule choice by distance ratio (levels below)
    LevelRules lv;
};

struct NearArgs {
    Elements el;
    RuleTables rules;
    const double* pts;  // [3][n] eval; null in collocation mode (points are centroids)
    int64_t n;
    int rhs;
    int n_rhs;
    double K;
    double* phi;        // eval: phi[n]; collocation: out[n_rhs][ne]
    double* E;          // eval only, may be null
    double* G;          // gradient mode: [6][n]
    const NearPair* near_list;   // as the far kernel appended it
    unsigned long long near_cap;
    const uint32_t* slot;        // result slot of each list entry
    const uint32_t* order;       // list indices in the order the lanes take them (costly first;
                                 // the pairs whose point lies on the element last)
    const NearPair* opair;       // the pairs in that order
    const uint32_t* walk_end;    // device: entries of order that subdivide (near_walk_end)
    const uint32_t* heavy_end;   // device: the leading entries with deep subdivisions (near_heavy_end)
    int deep;                    // field mode: 1 walks those breadth first, a wavefront each (more
                                 // registers); 0 walks every pair depth first in one lane
    double* res;                 // per-pair result records at the pairs' slots: [slot][4] field,
                                 // [slot][6] gradient, [slot] collocation
    DevCounters* ctr;
    double near_dr2;    // near_dr^2
    int max_depth;
    int64_t visit_limit;
};

// kernel launchers (kernels.hip)
hipError_t launch_far_eval(const FarArgs& a, int precision, hipStream_t s);
hipError_t launch_far_colloc(const FarArgs& a, int precision, hipStream_t s);
hipError_t launch_far_grad(const FarArgs& a, int precision, hipStream_t s);
enum NearMode { kNearEval = 0, kNearColloc = 1, kNearGrad = 2 };
hipError_t launch_near(const NearArgs& a, int mode, hipStream_t s);
hipError_t launch_charges(const double* sigma, const double* area, double* q, int64_t ne, int n_rhs, hipStream_t s);
// the near walk's records nrec[ne][kNearRec] from el.cen, el.frame, el.loc and el.thr2 (after an
// upload, and after the thresholds change)
hipError_t launch_pack_near_records(const Elements& el, double* nrec, hipStream_t s);
hipError_t launch_reduce_chunks(const double* partial, int n_split, int64_t rows, int64_t n, double K, double* out,
                                hipStream_t s);
hipError_t launch_zero_counters(DevCounters* c, hipStream_t s);
hipError_t launch_reset_near_count(DevCounters* c, hipStream_t s);  // near_count = 0 only
// the list pass's and the near stage's counters = 0 (before the near stage runs again)
hipError_t launch_reset_near_stage(DevCounters* c, hipStream_t s);
// near-pair list: every pair with D^2 < (near_dr L)^2 of the n points pts[3][n]
hipError_t launch_near_list(const double* pts, int64_t n, const Elements& el, NearPair* list, unsigned long long cap,
                            DevCounters* ctr, hipStream_t s);

hipError_t launch_self_diag(const Elements& el, double K, double* diag, hipStream_t s);
hipError_t launch_multi_dot(const double* V, int k, int64_t n, const double* w, double* partial, int blocks, hipStream_t s);
hipError_t launch_combine(double* y, double a, const double* V, const double* c, int k, int64_t n, const double* d,
                          hipStream_t s);
hipError_t launch_divide(double* y, const double* x, const double* d, int64_t n, hipStream_t s);

// workgroups per resident slot that element splitting aims for (dispatcher load balance)
constexpr int kSplitTargetBlocks = 16 * 1024;
constexpr int kMaxSplit = 64;

double coulomb_constant();
int solve_gmres(bemc_handle h, const Elements& el, const double* b, double* x, double tol, int max_iter, int m,
                int precision, bemc_solve_info* info, hipStream_t s, std::string& err);
int solve_refined(bemc_handle h, const Elements& el, const double* b, double* x, double tol, int max_iter, int m,
                  bemc_solve_info* info, hipStream_t s, std::string& err);

// Deterministic near-field accumulation (near_order.hip).  Per-point arrays hold n entries,
// the pair arrays the near-list capacity (< 2^32 pairs).
struct NearWork {
    uint32_t *count, *start, *cursor;  // [n] near pairs per point, segment starts, scatter cursors
    NearPair* grouped;                 // [capacity] pairs grouped by point, unordered within a point
    uint32_t* origin;                  // [capacity] list index of each grouped pair
    NearPair* sorted;                  // [capacity] pairs in (point, element) order
    uint32_t* slot;                    // [capacity] result slot (sorted position) of each list index
    double* res;                       // [capacity][rows] per-pair result records of the near kernel
    uint8_t* cost;                     // [capacity] cost class of each list index (near_cost_order)
    uint32_t* order;                   // [capacity] list indices, most expensive pairs first
    NearPair* opair;                   // [capacity] the pairs themselves in that order
    uint32_t* buckets;                 // [3][kCostClasses] count, start, cursor of each cost class
    void* temp;                        // scan workspace
    size_t temp_bytes;
};
// cost classes of near pairs: class 0 holds the pairs whose point lies on the element (exact
// integral, no subdivision); the others are deep (128 ..) or not, then rectangles (+ 64) or
// triangles, then 63 steps of the estimated subdivision depth.  The order runs most expensive
// class first: deep rectangles, deep triangles, the other rectangles, the other triangles.
constexpr int kCostClasses = 256;
constexpr int kOnElementClass = 0;
constexpr int kDeepClass = 128;      // first class of the deep pairs
constexpr int kDeepCost = 32;        // estimated-cost step from which a pair is deep (d <= L / 16)
size_t near_scan_temp_bytes(int64_t n);
hipError_t near_work_alloc(NearWork& w, int64_t n, unsigned long long pairs, int rows);  // frees w first
void near_work_free(NearWork& w);
// regroup the list (length read from ctr) into per-point segments sorted by element, and
// order the list indices by estimated subdivision cost (w.order) for the near kernel;
// pts [3][n] are the field points of the list (the centroids for collocation); cleared: w's
// per-point counts and cursors and its buckets are zero already (clear_call), else cleared here
hipError_t near_order(const NearPair* list, const DevCounters* ctr, unsigned long long cap, int64_t n,
                      const double* pts, const Elements& el, const NearWork& w, bool cleared, hipStream_t s);
// an evaluation's first launch: zeroes the counters and w's per-point counts and cursors (n
// points) and its buckets, so that near_order need not
hipError_t clear_call(DevCounters* ctr, const NearWork& w, int64_t n, hipStream_t s);
// the final rows of a field or gradient evaluation, in one pass per point: the far field
// (n_split > 1: K times the chunk partial sums partial[n_split][prow][n]; else far[rows][n])
// plus the point's near-pair records, stored at perm[p] (or p) of row 0 in d0 and of row
// r >= 1 in d1 + (r - 1) n
// ctr_out (device address of pinned host memory, or null): the call's counters ctr are copied
// there by the same launch, after every other kernel of the call
hipError_t near_finish(const NearWork& w, int64_t n, int mode, int rows, const double* partial, int n_split,
                       int prow, const double* far, double K, const uint32_t* perm, double* d0, double* d1,
                       const DevCounters* ctr, DevCounters* ctr_out, hipStream_t s);
// entries of w.order that the subdivision walk takes (device pointer; set by near_order)
inline const uint32_t* near_walk_end(const NearWork& w) { return w.buckets + kCostClasses + kOnElementClass; }
// entries of w.order with deep subdivisions (all classes from kDeepClass up come first)
inline const uint32_t* near_heavy_end(const NearWork& w) { return w.buckets + kCostClasses + (kDeepClass - 1); }
// add each point's segment of per-pair result records to its outputs (collocation; field and
// gradient evaluations use near_finish)
hipError_t near_reduce(const NearWork& w, int64_t n, int mode, double* phi, double* E,
                       double* G, const double* q, int64_t ne, int n_rhs, double K, const DevCounters* ctr,
                       DevCounters* ctr_out, hipStream_t s);
constexpr unsigned long long kMaxNearPairs = 0xffffffffull;  // 32-bit segment offsets

// Allocation-free evaluation (noalloc.hip): a static device array per GPU, carved into the
// buffers of one field evaluation of at most kNoAllocMaxPoints points and
// kNoAllocMaxNearPairs near pairs.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int64_t kNoAllocMaxPoints = 1 << 16;
constexpr unsigned long long kNoAllocMaxNearPairs = 1ull << 19;
constexpr size_t kNoAllocPartialDoubles = size_t(2) << 20;  // element-chunk partial sums (16 MiB)
constexpr size_t kNoAllocTempBytes = size_t(2) << 20;       // each of the sort and scan workspaces
constexpr int kNoAllocMaxDevices = 64;
// device address of this GPU's array (device current); taken once per device and kept
hipError_t noalloc_scratch(int device, void** ptr);

// Morton ordering of field points (order.hip).  Buffers sized for n points.  Evaluations of
// at most kOrderMinPoints points keep the caller's order: the sort's launches would cost more
// than the coherence it buys them.
constexpr int64_t kOrderMinPoints = 4096;
struct OrderWork {
    uint32_t *keys_in, *keys_out, *idx_in, *perm;
    void* temp;
    size_t temp_bytes;
    double* bbox;    // [1024][6]
    double* pts;     // [3][n] points in sorted order
    double* res;     // [6][n] far-field rows in processing order (phi, E or the gradient rows)
};
size_t order_temp_bytes(int64_t n);
hipError_t order_points(const double* pts, int64_t n, const OrderWork& w, hipStream_t s);

}  // namespace bemc
