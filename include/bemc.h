/*
 * bemc.h -- C ABI of the MI355X (gfx950) library for the electric potential and field
 * of charged BEM triangles and rectangles by Gaussian cubature
 * (F. Glueck, D. Hilk, arXiv:1606.03743).
 *
 * Method.  An element of constant charge density sigma is replaced by the point charges
 * q_i = w_i * sigma * area at the Gaussian points Q_i of a cubature rule (Sec. 4,
 * Eq. 4.1), and the potential and field at a field point P are the sums
 *     phi(P) = K sum_i q_i / |P - Q_i|,    E(P) = K sum_i q_i (P - Q_i) / |P - Q_i|^3,
 * K = 1 / (4 pi eps0) (SI units, Sec. 2 Eq. 2.1), both from the same points (Sec. 4).
 * Gaussian points come from barycentric coordinates for triangles (Eq. 3.3, rules of
 * Tables A1-A5) and from natural coordinates for rectangles (Eq. 3.2, tensor
 * Gauss-Legendre n x n).  Contributions of all elements are summed per field point
 * (Sec. 5, the integrating field solver).  The distance ratio DR = D / L, D = |P - centroid|,
 * L = average side length (Sec. 2), selects the path: for DR >= near_dr (3 by default,
 * the limit below which the paper's rules are not accurate enough, Sec. 1 and Sec. 4) the
 * rule is applied directly; below it the element is subdivided recursively (triangle:
 * four midpoint children; rectangle: 2 x 2) until every child is at DR >= near_dr of its
 * own, in FP64.  A field point lying on an element is integrated exactly in polar
 * coordinates about the point (principal value for the in-plane field, zero normal part).
 *
 * Conventions.
 *   * All entry points return BEMC_OK (0), a negative BEMC_E_* error, or (bemc_query_stats
 *     only) the positive warning BEMC_W_ON_SURFACE.  On error, bemc_last_error() gives a
 *     message for the calling thread.  No entry point aborts the process.
 *   * Evaluations (bemc_eval, bemc_eval_gradient, bemc_collocation_matvec) are enqueued on
 *     the caller's stream and return before they have run; the caller synchronizes the
 *     stream (or calls bemc_query_stats) before it reads the results.  Problems that show
 *     only on the device (an overflowing fixed near-pair list, the subdivision visit limit,
 *     points on elements) are reported by bemc_query_stats, and errors also by the next
 *     evaluation call that finds the earlier call finished.
 *   * "device" pointers are GPU memory of the context's device (e.g. torch tensors on
 *     cuda:N); "host" pointers are ordinary CPU memory.  The caller owns every buffer it
 *     passes; the library copies host inputs before returning.
 *   * stream arguments are hipStream_t (void* here so that the header needs no HIP
 *     include); NULL means the default stream.  Work is enqueued on that stream.
 *   * Element input format (host, FP64, row-major, 9 doubles per element):
 *       triangle  = A, B, C                      (vertices)
 *       rectangle = P0, e1, e2                   (corner and the two side vectors;
 *                                                 |e1| = a is the x side of Eq. 3.2)
 *     Global element index: triangles 0 .. n_tri-1, then rectangles.
 *   * Field points and fields are SoA on the device: pts[3][n] = x[n], y[n], z[n];
 *     E[3][n] likewise.  Units: metres, C/m^2, volts, V/m.
 *   * One context may be used from one host thread at a time.
 */
#ifndef BEMC_H
#define BEMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BEMC_OK 0
#define BEMC_E_INVALID_ARG -1
#define BEMC_E_DEGENERATE_ELEMENT -2 /* zero area or zero side length */
#define BEMC_E_NOT_RECTANGLE -3      /* |e1 . e2| > 1e-10 |e1| |e2| */
#define BEMC_E_NONFINITE -4          /* NaN or Inf in the geometry or densities */
#define BEMC_E_NO_GEOMETRY -5        /* evaluation before bemc_upload_geometry/densities */
#define BEMC_E_OUT_OF_MEMORY -6
#define BEMC_E_ADMISSION -7          /* serving: the query can never fit the memory budget */
#define BEMC_E_DEVICE -8             /* a HIP call failed; message in bemc_last_error() */
#define BEMC_E_LIMIT -9              /* a size exceeds the library's index range */
#define BEMC_W_ON_SURFACE 1          /* warning: some field point lies on an element */

/* precision of the bulk point-charge sums */
#define BEMC_FP64 0  /* everything in FP64 */
#define BEMC_MIXED 1 /* far-field node sums in FP32 (coordinates relative to the element
                        centroid in the element's own frame, FP32 reciprocal square
                        root), per-element partial sums scaled by
                        the element charge and accumulated per field point in FP64; the
                        distance-ratio classification, the near field and on-element
                        integrals stay FP64 */
#define BEMC_MIXED_REFINE 2 /* bemc_solve_densities only: corrections solved with mixed
                               products, residuals formed with FP64 products (iterative
                               refinement), so FP64 tolerances are reachable */

typedef struct bemc_context* bemc_handle;

/* Counters of the last bemc_eval / bemc_eval_gradient / bemc_collocation_matvec on a
 * context (a solve leaves those of its last product). */
typedef struct {
    int64_t pairs;          /* field points x elements */
    int64_t node_interactions; /* point-charge terms of the far-field sums: all pairs x the
                                  rule size with one rule per kind; with the rule chosen by
                                  distance ratio, the terms the far pairs really summed */
    int64_t near_pairs;     /* pairs with D < near_dr * L (handled in FP64) */
    int64_t leaves;         /* rule applications made by the subdivision */
    int64_t cap_hits;       /* leaves still near at the depth cap */
    int64_t on_surface;     /* pairs whose field point lies on the element */
    int64_t max_depth;      /* deepest subdivision level reached */
    int64_t near_capacity;  /* current size of the near-pair list */
    double far_ms;          /* far-field kernel time (HIP events around its launch) */
    double near_ms;         /* what follows it: chunk reduction, near-list regrouping, near
                               field and ordered sums (HIP events) */
    int64_t node_interactions_pair_rule; /* rule choice by distance ratio: the terms if every
                                            far pair summed its own level (a wavefront sums
                                            the finest level any of its pairs needs); else
                                            node_interactions */
} bemc_stats;

/* Message for the last non-OK status returned to this host thread ("" if none). */
const char* bemc_last_error(void);

/* Create a context on HIP device `device`; *out receives the handle.  Default rules:
 * 33-point triangle rule (Table A5), 7 x 7 Gauss-Legendre for rectangles, near_dr 3,
 * max_depth 24.  Errors: INVALID_ARG (no such device, out NULL), DEVICE. */
int bemc_create(int device, bemc_handle* out);

/* Release every device buffer of the context (waits for its pending work). */
int bemc_destroy(bemc_handle h);

/* Cubature rules and near-field parameters (Sec. 3, Tables A1-A5, B1-B5; Sec. 4
 * distance-ratio switch).  tri_rule in {4, 7, 12, 19, 33}; rect_rule in 1..16 for the
 * tensor Gauss-Legendre rule with rect_rule^2 points, or -4, -7, -12, -17, -33 for Table
 * B1..B5 (App. B); near_dr >= 2 (pairs with D < near_dr * L are subdivided; the far-field
 * sums expand r^2 about the centroid, whose rounding stays bounded at these distance
 * ratios, also in FP32); max_depth in 0..30.  Takes effect for subsequent evaluations;
 * node tables are rebuilt.
 * Errors: INVALID_ARG. */
int bemc_set_rules(bemc_handle h, int tri_rule, int rect_rule, double near_dr, int max_depth);

/* Rule choice by distance ratio for far pairs (Sec. 4: the fewest Gaussian points that
 * reach the accuracy floor at the pair's distance ratio; field limits somewhat above the
 * potential limits).  enable = 0 restores one rule per element kind.  When enabled, a far
 * triangle pair uses 7 / 12 / 19 points (Tables A2 / A3 / A4) for DR >= tri_dr[0] /
 * tri_dr[1] / tri_dr[2], else the triangle rule of bemc_set_rules; a far rectangle pair
 * uses Tables B2 / B3 / B4 for DR >= rect_dr[0..2], else the rectangle rule.  NULL
 * arrays select the defaults {100, 25, 10} and {150, 40, 15} (the paper's triangle
 * potential limits x 1.25; the rectangle tables' field-accuracy limits).  For each
 * element a wavefront of 128 points (neighbours: bemc_eval works on more than 4,096 points
 * in Morton order) uses the finest of the rules its pairs need (never
 * a coarser rule than a pair's own distance ratio asks for); results are returned in the
 * caller's order.  Near pairs and collocation are unaffected.  The rules of
 * bemc_set_rules must be at least as fine as the third level (>= 19 triangle points,
 * >= 17 rectangle points) while this is enabled.  Errors: INVALID_ARG (limits not
 * decreasing or below near_dr; rules too coarse). */
int bemc_set_dr_rules(bemc_handle h, int enable, const double* tri_dr, const double* rect_dr);

/* Upload the electrode geometry (host arrays in the element input format; either count
 * may be 0, n_tri + n_rect < 2^31).  Validates every element (finite, positive area,
 * orthogonal rectangle sides: |e1.e2| <= 1e-10 |e1||e2|; within that tolerance the element
 * is the parallelogram its sides span), computes centroids, areas, average side lengths L
 * (triangle (a + b + c)/3, Sec. 2; rectangle (a + b)/2), normals and an orthonormal frame
 * per element with the in-plane coordinates used for node generation, and keeps them
 * resident on the device.  Previously
 * uploaded densities are discarded.  Synchronous with respect to `stream`.
 * Errors: INVALID_ARG, NONFINITE, DEGENERATE_ELEMENT (index in the message),
 * NOT_RECTANGLE, LIMIT, OUT_OF_MEMORY, DEVICE. */
int bemc_upload_geometry(bemc_handle h, const double* tri, int64_t n_tri,
                         const double* rect, int64_t n_rect, void* stream);

/* Upload charge densities sigma[n_rhs][n_E] (C/m^2), 1 <= n_rhs <= 8, from host memory
 * (sigma_on_device = 0) or device memory (1).  Element charges q = sigma * area are
 * formed on the device.  Errors: NO_GEOMETRY, INVALID_ARG, NONFINITE (host input only),
 * OUT_OF_MEMORY, DEVICE. */
int bemc_upload_densities(bemc_handle h, const double* sigma, int n_rhs, int sigma_on_device,
                          void* stream);

/* Potential phi[n] (device) and, if E is not NULL, field E[3][n] (device) at the n field
 * points pts[3][n] (device), from density vector `rhs` (0 <= rhs < n_rhs).  Outputs are
 * overwritten.  precision = BEMC_FP64 or BEMC_MIXED.  n = 0 is a no-op.
 * More than 4,096 points are processed in Morton (Z-curve) order, which keeps the points
 * of a wavefront close together; fewer keep the caller's order (the sort would cost more
 * than it saves).  Results are returned in the caller's order.  With one rule per element
 * kind they do not depend on the processing order; with the rule choice by distance ratio
 * the rule level a wavefront picks does (an accuracy-level difference, never a coarser
 * rule than a pair needs).  The ordering workspace (about 110 bytes per point) is kept by
 * the context.
 * The call enqueues on `stream` the near-pair list (every pair with D < near_dr L, by a
 * classification pass), the far-field kernel (point-charge sums of the other pairs) and the
 * FP64 near field, and returns without waiting for them.  With a growing near-pair list
 * (the default, see bemc_set_near_capacity) the host reads the list pass's pair count --
 * a wait of about a millisecond, while the far field is already queued behind it -- and,
 * if the list was too short, grows it and repeats the list pass (never the far field)
 * before it enqueues the near field.  With a fixed list there is no host wait at all.
 * Results are reproducible bit for bit: far-field chunks are added in fixed order, and
 * each point's near pairs are summed in element order.  A field point lying on an
 * element gets the principal-value field there; bemc_query_stats then returns
 * BEMC_W_ON_SURFACE.  Consecutive calls on one context may use different streams (each
 * call waits on the device for the previous one).
 * Errors: NO_GEOMETRY, INVALID_ARG, LIMIT (n >= 2^31; or reported from an earlier call:
 * a fixed near-pair list overflowed, or a near pair needed more than 2^22 subdivision
 * steps), OUT_OF_MEMORY, DEVICE. */
int bemc_eval(bemc_handle h, const double* pts, int64_t n, int precision, int rhs,
              double* phi, double* E, void* stream);

/* Allocation-free variant of bemc_eval, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and asynchronous behaviour as bemc_eval, but the call
 * allocates nothing: its work buffers (point ordering, near-pair list and its regrouping,
 * element-chunk partial sums, counters) are carved from a static device array of 64 MiB
 * that each GPU the library runs on holds from the first context created on it until the
 * process ends.  Limits: n <= 65536 field points per call (larger n returns BEMC_E_LIMIT
 * at once) and 524288 near pairs (D < near_dr L) per call; more near pairs leave the near
 * field incomplete and are reported, as for a fixed list of bemc_set_near_capacity, by
 * bemc_query_stats and the next evaluation call (BEMC_E_LIMIT).  The element-chunk split
 * of the far field is capped by the array (results then differ from bemc_eval's in
 * summation grouping only, at rounding level).  All contexts on one GPU share that GPU's
 * array, which keeps the last call's contents: calls on one context are ordered (each
 * waits on the device for the previous one), but calls from different contexts on one
 * GPU that overlap on the device race -- the caller serialises them (one stream, or
 * events).  Errors: as bemc_eval; DEVICE when the array's address could not be taken. */
int bemc_eval_noalloc(bemc_handle h, const double* pts, int64_t n, int precision, int rhs,
                      double* phi, double* E, void* stream);

/* Field gradient dE_i/dx_j (V/m^2, symmetric and trace-free off the electrodes) at the n
 * field points pts[3][n] (device): G[6][n] (device, overwritten) holds the rows xx, yy, zz,
 * xy, xz, yz.  The derivative of the point-charge sums of Eq. (4.1): each Gaussian point
 * contributes K q (delta_ij r^2 - 3 d_i d_j) / r^5, d = P - Q (Sec. 7, conclusions: higher
 * derivatives of the field follow from the same point charges, e.g. for field maps with
 * Hermite interpolation).  Classification, near-field
 * subdivision, rule choice (including bemc_set_dr_rules) and precision handling are those
 * of bemc_eval; BEMC_MIXED forms the FP32 node sums from unit vectors d/r (no power of 1/r
 * above the third in FP32).  A field point lying on an element gets NaN in all six rows
 * (the normal field jumps there) and bemc_query_stats returns BEMC_W_ON_SURFACE.
 * Asynchronous like bemc_eval.  Errors: as bemc_eval. */
int bemc_eval_gradient(bemc_handle h, const double* pts, int64_t n, int precision, int rhs,
                       double* G, void* stream);

/* Matrix-free collocation product (BEM system matrix times densities, Sec. 5: the
 * matrix is never stored): out[r][i] = potential at the centroid of element i from the
 * densities sigma[r][:], r < n_rhs (1..8), for every element i.  sigma and out are device
 * arrays [n_rhs][n_E].  The element's own contribution is its exact on-element integral;
 * neighbours below near_dr are subdivided in FP64.  precision as in bemc_eval (far pairs
 * only).  Independent of the densities of bemc_upload_densities.  The near part depends
 * on the geometry and the rules only (it is formed for unit densities): consecutive
 * products on one context reuse the near-pair list and the near records of the first one,
 * until the geometry, the rules or the near-pair capacity change or a field or gradient
 * evaluation runs on the context; bemc_query_stats then repeats that product's near-field
 * counts, and its near time covers only the sums with the new densities.  Asynchronous like
 * bemc_eval.  Errors: NO_GEOMETRY, INVALID_ARG, LIMIT, OUT_OF_MEMORY, DEVICE. */
int bemc_collocation_matvec(bemc_handle h, const double* sigma, int n_rhs, int precision,
                            double* out, void* stream);

/* Result of bemc_solve_densities. */
typedef struct {
    int iterations;       /* collocation products used (all precisions) */
    int converged;        /* 1 if the relative residual reached tol */
    double rel_residual;  /* |potential - A sigma| / |potential|, from a final product */
    double seconds;
    int refinements;      /* BEMC_MIXED_REFINE: FP64 residual products (outer steps) */
} bemc_solve_info;

/* Charge densities from electrode potentials (the BEM linear-algebra step, Sec. 5): find
 * sigma[n_E] (device) with (A sigma)_i = potential[i] (device, volts at the centroid of
 * element i), A the operator of bemc_collocation_matvec.  Restarted GMRES (restart
 * 1..200) right-preconditioned by the diagonal of A (exact on-element potentials), started
 * from zero, stopped when the residual falls below tol * |potential| or after max_iter
 * products; precision BEMC_FP64 or BEMC_MIXED applies to the far pairs of each product
 * (BEMC_MIXED stalls near 1e-7, the accuracy of its products).  BEMC_MIXED_REFINE:
 * iterative refinement, r = potential - A sigma with FP64 products, each correction from
 * GMRES on mixed products to 1e-6 of |r|, until |r| <= tol |potential|.  Allocates
 * (restart + 7) n_E doubles of workspace.  Synchronous.  Errors: NO_GEOMETRY,
 * INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
int bemc_solve_densities(bemc_handle h, const double* potential, double* sigma, double tol, int max_iter,
                         int restart, int precision, bemc_solve_info* info, void* stream);

/* Size of the near-pair list (8 bytes per pair, plus 24 for its regrouping and 8 per
 * result row -- 4 for the field, 6 for the gradient -- allocated at the next evaluation;
 * 1 <= pairs <= 2^32 - 1).  grow != 0: the list starts at this size and grows to what an
 * evaluation needs (the default policy, starting at max(2^20, 8 n) pairs; the host reads
 * each evaluation's pair count before it enqueues the near field).  grow = 0: the size is
 * fixed and evaluations never wait on the host; an evaluation that finds more near pairs
 * evaluates the near field of those that fit only, and bemc_query_stats (and the next
 * evaluation call) reports BEMC_E_LIMIT.  Waits for the evaluations in flight.
 * Errors: INVALID_ARG, LIMIT, OUT_OF_MEMORY. */
int bemc_set_near_capacity(bemc_handle h, int64_t pairs, int grow);

/* Waits for the last evaluation on the context and returns its counters.  Returns
 * BEMC_W_ON_SURFACE when some of its field points lie on an element, BEMC_E_LIMIT (once)
 * when an evaluation since the last report overflowed a fixed near-pair list or hit the
 * subdivision visit limit, BEMC_E_DEVICE when one failed on the device.
 * Errors: INVALID_ARG. */
int bemc_query_stats(bemc_handle h, bemc_stats* out);

/* ---------------------------------------------------------------------------------
 * Serving: continuous batching of field-point queries against the resident geometry
 * and densities (density vector 0), mixed or FP64 precision, with the rules of the
 * context (including the distance-ratio rule choice when enabled).
 *
 * bemc_server_start launches a host scheduler thread that owns `n_streams` HIP streams
 * (default priority).  Submitted queries wait in arrival order; whenever a stream is
 * free the scheduler admits waiting queries in order while their points fit into
 * max_batch_points and their batch's device memory fits what the budget has left, packs
 * them into one batch (one far-field launch over all their points, element-split when
 * the batch is small so the GPU stays full; fixed-order reduction of the element chunks;
 * then the FP64 near field) and copies each query's results to its host buffers when the
 * batch completes.  Batches on different streams overlap on the device.  Device memory:
 * one allocation made at start (mem_budget_bytes, but at most twice what full batches on
 * every stream need) is handed out per batch on the host: a block for the batch's per-point
 * buffers and one for its near-pair list (16 pairs per point), taken at admission and given
 * back at completion.  The whole batch is enqueued at admission; when its list pass finds
 * more near pairs than the list holds, the far field is kept and the list grows -- a larger
 * block, the list pass and the near stage again.  A growth that does not fit waits while
 * another batch is running; otherwise the grown list goes outside the budget
 * (stream-ordered allocation, released with the batch), so at most one batch at a time
 * exceeds the budget, by its list.  With small_query_points > 0 and
 * at least two streams, queries of at most that many points wait in a queue of their
 * own, and one stream serves only that queue, so that short queries do not wait behind
 * long batches; the other streams take the long queue first and the short one when the
 * long one is empty.  A query's result depends on the other queries in its batch only
 * through the number of element chunks of the far-field launch (the summation grouping,
 * a rounding-level difference); with the rule choice by distance ratio also through the
 * rule each wavefront of neighbouring points picks (an accuracy-level difference).
 * --------------------------------------------------------------------------------- */

typedef struct {
    size_t mem_budget_bytes;   /* device bytes for in-flight batch buffers (at least one
                                  batch of max_batch_points: else INVALID_ARG) */
    int64_t max_batch_points;  /* points per batch (>= the largest admissible query) */
    int n_streams;             /* 1..8 concurrent batches */
    int precision;             /* BEMC_FP64 or BEMC_MIXED */
    int64_t small_query_points; /* > 0: queries of at most this many points form their own
                                   class with a stream of their own; 0: one class */
} bemc_server_config;

typedef struct {
    int done;                  /* 1 once results are in the host buffers */
    int status;                /* BEMC_OK or an error for this query */
    double submit_s, start_s, end_s; /* host clock (s since server start): submission,
                                        launch of its batch, results in host memory */
    int64_t batch_id;          /* batch the query ran in */
    int64_t batch_points;      /* points of that batch */
} bemc_query_info;

/* Start serving on the context (geometry and densities must be uploaded).
 * Errors: NO_GEOMETRY, INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
int bemc_server_start(bemc_handle h, const bemc_server_config* cfg);

/* Submit a query: pts_host[n][3] (host, AoS), results to phi_host[n] and, if not NULL,
 * E_host[n][3] (host, AoS).  Host buffers must stay valid until the query is done.
 * Never blocks.  *ticket receives the query id.  Errors: INVALID_ARG, ADMISSION (the
 * query can never fit the budget or max_batch_points; returned at once). */
int bemc_server_submit(bemc_handle h, const double* pts_host, int64_t n, double* phi_host,
                       double* E_host, uint64_t* ticket);

/* Non-blocking status of a query.  Errors: INVALID_ARG (unknown ticket, or a ticket whose
 * completion bemc_server_wait has already returned). */
int bemc_server_poll(bemc_handle h, uint64_t ticket, bemc_query_info* info);

/* Block until the query is done (timeout_s < 0: no limit).  Returns its status, or
 * BEMC_E_INVALID_ARG for an unknown ticket or when the timeout expired.  Once it has
 * returned a completed query, the server forgets the ticket (its record is released, so a
 * long-running server does not accumulate finished queries). */
int bemc_server_wait(bemc_handle h, uint64_t ticket, double timeout_s, bemc_query_info* info);

/* Finish all submitted queries, stop the scheduler and free the batch buffers. */
int bemc_server_stop(bemc_handle h);

/* Library facts for tests and tools: the Coulomb constant used, and the node count of
 * the triangle rule n (-1 if unknown). */
double bemc_coulomb_constant(void);
int bemc_rule_size(int tri_rule);

#ifdef __cplusplus
}
#endif
#endif /* BEMC_H */
