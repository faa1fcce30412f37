/*
 * pts.h -- C ABI of the MI355X (gfx950) library for pointwise signed distance
 * to point clouds, after "Points as Tori: Fast Pointwise Signed Distance for
 * Point Clouds" (Feng, Gkioulekas, Crane; ACM TOG 45(4), 2026).
 *
 * Problem statement (Algorithm 1): given oriented points (p_i, n_i) and, per
 * point, the six coefficients of a quadratic height function over the point's
 * supporting plane (Sec. 4.1, Eq. BivariatePolynomial), precompute one torus
 * per point ("precomputation", pts_cloud_build), then evaluate
 *
 *     phi(x) = sum_i g_i(x) w_i(x) / sum_i w_i(x),
 *     w_i(x) = exp(-lambda_x (|x - p_i| - sigma_x)),
 *     sigma_x = max_i |x - p_i| / 2,  lambda_x = C / sigma_x,
 *
 * at arbitrary query points ("inference", pts_eval), where g_i is the signed
 * distance to point i's torus (Sec. 4.2, Eqs. BasicFormulaShifted,
 * RelationshipBetweenLambdaAndRadius, SingleTorusSDF).  The sum runs over all
 * points.
 *
 * Conventions for every call:
 *  - Pointers marked "device" are HIP device pointers on the current device;
 *    the caller owns them.  Arrays are dense, row-major, float32 unless stated.
 *  - Calls enqueue work on `stream` (a hipStream_t; NULL = default stream) and
 *    return without waiting unless stated.  Results are valid after the stream
 *    has been synchronised.
 *  - Every call returns a status (PTS_OK = 0 on success).  On failure nothing
 *    has been enqueued, and pts_last_error() returns a message for the calling
 *    thread.  No C++ exception crosses this boundary.
 *  - A call that takes a record `rec` and a point count N requires N to be the
 *    count the record was built with.  The record lives in device memory and
 *    is not read back on the host to check this (that would block every
 *    call), so a different N is undefined behaviour: kernels would locate the
 *    record's sections for the wrong size.  pts_cloud_info_get returns the
 *    record's N.
 *  - No entry point allocates device memory except the server (pts_server_*),
 *    which allocates from its own budget; scratch memory is passed in by the
 *    caller, sized by the matching *_ws_bytes call.
 *
 * Input format of the coefficients (the paper's network output, Sec. 4.3):
 *   a = (a00, a01, a10, a11, a02, a20) per point, for
 *   Q_i(s,t) = sum a_nm s^n t^m over the frame (s_i, t_i, n_i), with
 *   n_i normalised internally and the frame fixed as
 *   e = (1,0,0) if |n_x| < 0.9 else (0,1,0),
 *   s = normalize(e - <e,n> n),  t = n x s.
 *   Curvature is signed along +n: a convex surface with outward normals has
 *   negative a02, a20 (a02 = a20 = -1/2 is the tangent unit sphere).
 */
#ifndef PTS_H
#define PTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PTS_OK 0
#define PTS_EINVAL 1      /* invalid argument (null pointer, size, layout)   */
#define PTS_EBUDGET 2     /* request does not fit the server's memory budget */
#define PTS_ENOMEM 3      /* device or pinned allocation failed (server only) */
#define PTS_EHIP 4        /* a HIP runtime call failed                       */
#define PTS_EBUSY 5       /* server busy: queue full, cloud or ticket in use  */
#define PTS_ECANCELLED 6  /* request cancelled                               */
#define PTS_ENOTFOUND 7   /* unknown cloud id or ticket                      */
#define PTS_ETIMEOUT 8    /* wait timed out                                  */

/* Library version (major * 100 + minor): 101 (1.01 adds pts_trace_bounded). */
int pts_version(void);

/* Message for the last non-zero status returned on the calling thread. */
const char* pts_last_error(void);

/* Parameters.  A NULL pointer means the defaults below. */
typedef struct pts_params {
  float C;           /* screening constant of Eq. (RelationshipBetweenLambdaAndRadius);
                        default 64 (Sec. 4.2).  0 < C <= 75.  phi does not
                        depend on the additive shift of Eq. (BasicFormulaShifted);
                        the FP32 kernels shift the exponents by s = min(C, 64)
                        instead of C, so the weights lie in [e^(s - 2C), e^s]:
                        the largest is at most e^64, which keeps the sums below
                        FLT_MAX while N * max|g| < 5e10 (coordinates in units
                        of the cloud), and the smallest stays a normal FP32
                        number (>= 2^-126) for C <= 75 (a query nearly
                        equidistant from every point would otherwise get 0/0).
                        Statistics report W with this shift. */
  float kfloor_rel;  /* curvature floor kappa_floor = kfloor_rel / D, D = bbox
                        diagonal of the cloud (D = 1 if it is 0); default 1e-6;
                        at least 1e-12 (radii reach D / kfloor_rel and the
                        anchored torus form squares them in FP32).
                        Applied at build time.  Principal curvatures smaller in
                        magnitude are raised to +-kappa_floor (sign(0) = -1),
                        which keeps planar and cylindrical points at finite,
                        very large torus radii (Sec. 6, "Sharp feature extraction"). */
  int splits;        /* 0 = automatic (up to 1024, see pts_eval_plan).  Otherwise
                        the number of point ranges a query's sum is split over
                        (power of two, <= 64); results depend on it only
                        through FP32 rounding order. */
  float offset;      /* default 0.  pts_eval, pts_eval_bounded and pts_eval_baseline
                        return phi - offset, the signed distance to the offset
                        surface phi = offset (Sec. 5.2, "Offset surfaces and
                        Booleans"), and pts_trace marches on it; gradients,
                        statistics and backward passes are those of phi itself.
                        Must be finite.  0 leaves every result bitwise unchanged.
                        pts_eval_radius and the server do not take it. */
} pts_params;

/* ---------------------------------------------------------------------------
 * Precomputation (Algorithm 1, first stage; torus fitting of Sec. 4.1).
 * ------------------------------------------------------------------------- */

/* Bytes of the opaque per-cloud record buffer for N points (N >= 1). */
int pts_record_bytes(int64_t N, size_t* out_bytes);

/* Fit one torus per point and lay the cloud out for evaluation.
 *   p [N,3], n [N,3], a [N,6]  device, float32 (layout above).
 *   rec                        device, rec_bytes >= pts_record_bytes(N);
 *                              256-byte aligned; written entirely.
 * The torus of point i (Sec. 4.1): principal curvatures kappa_+- = H +- sqrt(H^2-K)
 * (Eq. MeanAndGaussCurvatures; H^2-K < 0 from rounding is clamped to 0),
 * kappa_min / kappa_max by magnitude (ties: kappa_min = kappa_-), radii
 * r = 1/|kappa_max|, R = 1/|kappa_min| - sign(kappa_+ kappa_-) r, sign
 * (Eq. TorusSigns) +1 iff kappa_max < 0, center c = Q*(0,0) + n* / kappa_min
 * with kappa_min signed (this equals the printed center on elliptic points and
 * keeps saddle points on the correct side), axis u = n* x v_min with v_min
 * from Eq. (PrincipalDirections) (the longer of the two row solutions; the
 * frame vector s at umbilics).  Derivation runs in FP64; the record is FP32.
 * Blocks until the build has finished (it reads back a status word).
 * Errors: PTS_EINVAL for N < 1, null pointers, a short buffer, or a normal
 * with |n| <= 1e-20 or a non-finite input (detected on the device). */
int pts_cloud_build(const float* p, const float* n, const float* a, int64_t N,
                    const pts_params* prm, void* rec, size_t rec_bytes, void* stream);

/* Summary of a built record (copied to the host; blocks). */
typedef struct pts_cloud_info {
  int64_t N;          /* points */
  int64_t n_direct;   /* points evaluated with the direct torus formula */
  int64_t n_anchored; /* points with radius L > 4 D, evaluated in the anchored form */
  float bbox_lo[3], bbox_hi[3];
  float diag;         /* bbox diagonal D */
  float kfloor;       /* curvature floor used */
  int version;        /* record layout version: 4 (with the oriented unit boxes);
                         a record is built and read by the same library */
  int reserved;
} pts_cloud_info;
int pts_cloud_info_get(const void* rec, pts_cloud_info* out, void* stream);

/* Per-point torus in the caller's original point order, for inspection:
 * out [N,12] device float32 = (c.x, c.y, c.z, u.x, u.y, u.z, R, r, sign,
 * L = 1/|kappa_min|, anchored flag, 0).  Asynchronous. */
int pts_cloud_decode(const void* rec, int64_t N, float* out, void* stream);

/* ---------------------------------------------------------------------------
 * Inference (Algorithm 1, second stage; Sec. 4.2).
 * ------------------------------------------------------------------------- */

/* Launch plan pts_eval uses for N points and Q queries (a pure function of N,
 * Q and the parameters): queries per lane, number of point splits, and points
 * per split (a multiple of 64; splits * per_split >= N, every split
 * non-empty).  Many points get 8 splits, one per XCD, or 32 when an eighth of
 * the records would not fit an XCD's L2 (over about 420k points); few
 * queries get many short splits (down to 64 points, at most 1024): a
 * workgroup walks its split serially, so the split length sets the latency
 * of a small evaluation.  For inspection and tests; host only. */
int pts_eval_plan(int64_t N, int64_t Q, const pts_params* prm, int* qpl, int* splits,
                  int64_t* per_split);

/* Scratch bytes pts_eval needs for N points and Q queries (given params), when
 * no gradient is requested. */
int pts_eval_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes);

/* Scratch bytes for pts_eval with a gradient output and for pts_grad_x. */
int pts_grad_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes);

/* phi at Q queries.
 *   rec         device, built by pts_cloud_build for the same N.
 *   x [Q,3]     device float32 queries.
 *   sdf [Q]     device float32 output phi(x).
 *   grad [Q,3]  device float32 output grad phi(x), or NULL.  The gradient is
 *               the exact derivative of phi including the dependence of
 *               lambda_x on x: App. D holds lambda fixed; the extra term is
 *               (2C/M^2) e_* (1/W) sum_i w_i (g_i - phi) d_i, with M the largest
 *               distance and e_* the unit vector from that farthest point to x.
 *               Where a torus SDF is not differentiable (its axis, its core
 *               circle) and at a query on a point, the undefined factor is 0.
 *               Requires ws_bytes >= pts_grad_ws_bytes(N, Q, prm).
 *   stats [Q,6] device float32 output or NULL: (M, W, phi, e_*) with
 *               M = max_i |x - p_i|, W = sum_i exp(s - lambda_x |x-p_i|) with
 *               s = min(C, 64) (the shifted weight sum of Eq. BasicFormulaShifted,
 *               whose shift lambda_x sigma_x is C; see pts_params.C), phi, and
 *               e_* as above.  The input of pts_grad_x.
 *   ws          device scratch of ws_bytes >= pts_eval_ws_bytes(N, Q, prm).
 * A query with a NaN or infinite coordinate gives NaN.  Q = 0 is a no-op. */
int pts_eval(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, float* grad,
             float* stats, const pts_params* prm, void* ws, size_t ws_bytes, void* stream);

/* pts_eval without gradient or statistics, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and the same results, bit for bit,
 * as pts_eval(rec, N, x, Q, sdf, NULL, NULL, prm, ws, ws_bytes, stream), with
 * the workspace taken from a static device array of 64 MiB that the library
 * holds on every device it runs on until the process ends.  Nothing is
 * allocated by this call, ever.  The array's device address is looked up on
 * the first call on each device.
 *   rec, x [Q,3], sdf [Q]  as pts_eval (device; owned by the caller).
 * Errors as pts_eval, and PTS_EINVAL when the evaluation's workspace
 * (pts_eval_ws_bytes(N, Q, prm)) exceeds 64 MiB -- e.g. 2^20 queries with 8
 * point splits need 128 MiB; call pts_eval with a workspace then.  Every call
 * on one device uses the same array: calls that overlap on a device (two
 * streams, two threads) race and give wrong results; serialise them.  Each
 * call overwrites every byte it reads, so no clearing is needed between calls. */
int pts_eval_noalloc(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, const pts_params* prm,
                     void* stream);

/* Scratch bytes for pts_eval_bounded. */
int pts_eval_bounded_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes);

/* phi at Q queries with far point units skipped under a proven error bound:
 * |sdf[q] - phi(x_q)| <= eps in exact arithmetic (eps in the cloud's distance
 * units, >= 0), on top of the FP32 rounding pts_eval has.  The bound rests on
 * each torus passing through its anchor o_i = p_i + a00_i n_i (Sec. 4.1), so
 * |g_i(x)| <= |x - p_i| + max|a00|, and on the shifted weights of
 * Eq. (BasicFormulaShifted): n points at distance >= d_lo from x add at most
 * n exp(-lambda_x (d_lo - sigma_x)) to the denominator, d_lo taken from the
 * bounding sphere of a 4096-point block or the oriented box of a 64-point
 * unit (both built with the record).  A unit or block is skipped (by a whole
 * wavefront of queries, processed in Morton order) only while the skipped
 * bounds stay within eps times the denominator kept so far.
 *   bound [Q] (may be NULL)  the bound actually incurred, (G_s + |phi| D_s)/D_k
 *                            (<= eps up to FP32 rounding of the bound itself);
 *   kept [Q]  (may be NULL)  points evaluated for the query (N without skips).
 * eps = 0 skips nothing and returns the plain sum in another order.  Results
 * depend on the other queries of the call (they share wavefront votes) only
 * through which units are skipped, never beyond the bound.  ws_bytes >=
 * pts_eval_bounded_ws_bytes(N, Q, prm).  A NaN query gives NaN. */
int pts_eval_bounded(const void* rec, int64_t N, const float* x, int64_t Q, float eps, float* sdf,
                     float* bound, int32_t* kept, const pts_params* prm, void* ws, size_t ws_bytes,
                     void* stream);

/* The three stages of pts_eval without gradient or statistics as separate
 * calls, with the same arguments and workspace, for callers that time or
 * schedule them individually; the three in order give pts_eval's result bit
 * for bit (pts_eval itself skips the folding of the farthest-point sweep's
 * per-split maxima that pts_eval_far does when there are at most 16 of them,
 * and lets the blend sweep take their maximum):
 *   pts_eval_far      farthest-point sweep: M = max_i |x - p_i| per query and
 *                     point split (Eq. RelationshipBetweenLambdaAndRadius);
 *   pts_eval_blend    weighted sweep: per split, sum_i w_i g_i and sum_i w_i
 *                     (Eq. BasicFormulaShifted); needs pts_eval_far's output;
 *   pts_eval_combine  fixed-order sum over splits, phi = num / den.
 * Errors as pts_eval. */
int pts_eval_far(const void* rec, int64_t N, const float* x, int64_t Q, const pts_params* prm,
                 void* ws, size_t ws_bytes, void* stream);
int pts_eval_blend(const void* rec, int64_t N, const float* x, int64_t Q, const pts_params* prm,
                   void* ws, size_t ws_bytes, void* stream);
int pts_eval_combine(int64_t N, int64_t Q, float* sdf, const pts_params* prm, void* ws,
                     size_t ws_bytes, void* stream);

/* Backward with respect to the queries (App. D and the lambda_x term):
 * gx[q] = gout[q] * grad phi(x_q), from the statistics a pts_eval call wrote
 * for the same queries.  gout [Q] may be NULL (then 1).  Re-sweeps all points
 * once.  ws_bytes >= pts_grad_ws_bytes(N, Q, prm). */
int pts_grad_x(const void* rec, int64_t N, const float* x, int64_t Q, const float* gout,
               const float* stats, float* gx, const pts_params* prm, void* ws, size_t ws_bytes,
               void* stream);

/* Scratch bytes for pts_laplacian. */
int pts_laplacian_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes);

/* Second-order quantities of phi at Q queries (App. D gives the Laplacian for
 * a fixed lambda; here lambda_x = 2C/M moves with x as in pts_eval's
 * gradient), from the statistics a pts_eval call wrote for the same queries:
 *   lap [Q]    Laplacian of phi: the fixed-lambda Laplacian plus
 *              2 kappa grad V . e_* + kappa^2 F_ll, kappa = 2C/M^2,
 *              V = (1/W) sum_i w_i (g_i - phi) d_i, F_ll = <(g - phi) d^2> - 2 <d> V
 *              (1/M is harmonic in 3D, so lambda_x adds no Laplacian of its own);
 *   grad [Q,3] grad phi (the quantity pts_eval computes, here from the same
 *              sweep);
 *   eik [Q]    eikonal residual |grad phi| - 1 (its absolute value, averaged
 *              over queries, is the eikonal term of Eq. LossFunction, Sec. 4.3).
 * Each output may be NULL; at least one must be given.  One query-major sweep
 * over all points with 22 weighted sums per query, then a fixed-order
 * combine; deterministic.  On a torus's axis, core circle and at a query on a
 * point the undefined factor is 0, as for the gradient.  Per-pair arithmetic
 * in FP32; the weighted sums are carried and combined in FP64 because the
 * formula cancels terms of size 2C/M down to the Laplacian.
 * ws_bytes >= pts_laplacian_ws_bytes(N, Q, prm). */
int pts_laplacian(const void* rec, int64_t N, const float* x, int64_t Q, const float* stats, float* lap,
                  float* grad, float* eik, const pts_params* prm, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Offsets and Booleans of signed distances (Sec. 5.2, "Offset surfaces and
 * Booleans"): elementwise on values already evaluated, e.g. two clouds' phi
 * at the same queries.
 * ------------------------------------------------------------------------- */

#define PTS_OP_OFFSET 0    /* out = a - c            (offset surface a = c) */
#define PTS_OP_UNION 1     /* out = min(a, b)                                 */
#define PTS_OP_INTERSECT 2 /* out = max(a, b)                                 */
#define PTS_OP_SUBTRACT 3  /* out = max(a, -b)        (a minus b)             */

/* out [n] = op(a, b) on device float32 arrays (b unused, may be NULL, for
 * PTS_OP_OFFSET; c used only there).  A NaN in an operand gives NaN.  The
 * results are exact signed distances where the operands are, up to the usual
 * caveat of min/max compositions (exact outside the union and inside the
 * intersection; a bound elsewhere).  out may alias a or b. */
int pts_compose(const float* a, const float* b, int64_t n, int op, float c, float* out, void* stream);

/* ---------------------------------------------------------------------------
 * Baselines of the accuracy comparison (Sec. 5.2, "Signed distance accuracy"),
 * evaluated over the same record and skeleton as pts_eval.
 * ------------------------------------------------------------------------- */

#define PTS_BASELINE_SSPD 0 /* smoothed signed planar distance, Eq. (SmoothedSignedPlanarDistance) */
#define PTS_BASELINE_SHC 1  /* signed Hopf-Cole distance, Eq. (ScreenedWindingNumber) */

/* Per-point area weights A_i of both baselines, area [N] device float32 in the
 * caller's point order (NULL restores A_i = 1, the value pts_cloud_build sets).
 * The torus blend does not use them. */
int pts_set_areas(void* rec, int64_t N, const float* area, void* stream);

/* A baseline at Q queries, with the per-query sigma_x = M/2 and
 * lambda_x = 2C/M of Eq. (RelationshipBetweenLambdaAndRadius) and unit normals
 * (the input normals scaled to length 1), w_i = A_i exp(-lambda_x (d_i - sigma_x)):
 *   PTS_BASELINE_SSPD  phi = sum w_i <x - p_i, n_i> / sum w_i;
 *   PTS_BASELINE_SHC   s = sum w_i (lambda_x d_i + 1) <x - p_i, n_i> / (2 pi d_i^3),
 *                      phi = sign(s) (-log|s| / lambda_x + sigma_x), sign(0) = +1.
 * sdf [Q] device float32 output.  ws_bytes >= pts_eval_ws_bytes(N, Q, prm)
 * (the same workspace as pts_eval).  A NaN query gives NaN; for SHC a query
 * at distance 0 from a point (in the record's FP32 coordinates) gives NaN and
 * one within ~1e-5 (relative to the cloud's size) of a point may overflow FP32
 * to an infinite distance.  An unknown kind is PTS_EINVAL.  Deterministic. */
int pts_eval_baseline(const void* rec, int64_t N, const float* x, int64_t Q, int kind, float* sdf,
                      const pts_params* prm, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Backward with respect to the per-point coefficients (the representation is
 * differentiable, Sec. 6): ga[i] = dL/da_i for L = sum_q gout[q] phi(x_q).
 * ------------------------------------------------------------------------- */

/* Scratch bytes for pts_backward_params. */
int pts_backward_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes);

/* dL/da [N,6] (device float32, the caller's point order and coefficient order
 * (a00, a01, a10, a11, a02, a20)).
 *   rec, p, n, a  the record and the inputs it was built from (device);
 *   x [Q,3]       queries; stats [Q,6] from pts_eval at the same queries;
 *   gout [Q]      upstream gradient dL/dphi (NULL = 1).
 * The weights of Eq. (BasicFormulaShifted) do not depend on a, so
 * dL/da_i = sum_q gout_q (w_qi/W_q) dg_i(x_q)/da_i: a point-major sweep
 * accumulates dL/d(c, u, R, r) per point and an FP64 chain rule through the
 * torus fit of Sec. 4.1 maps it to a.  Derivatives through a floored
 * curvature are 0, and at umbilics d sqrt(H^2 - K) is taken as 0.  A NaN query
 * makes every point's gradient NaN.  Deterministic (fixed-order reductions). */
int pts_backward_params(const void* rec, int64_t N, const float* p, const float* n, const float* a,
                        const float* x, int64_t Q, const float* gout, const float* stats, float* ga,
                        const pts_params* prm, void* ws, size_t ws_bytes, void* stream);

/* Scratch bytes for pts_backward_points (any combination of outputs). */
int pts_backward_points_ws_bytes(int64_t N, int64_t Q, const pts_params* prm, size_t* out_bytes);

/* dL/da [N,6], dL/dp [N,3] and dL/dn [N,3] for L = sum_q gout[q] phi(x_q)
 * (device float32, the caller's point order; each output may be NULL, at
 * least one must be given).  Arguments as pts_backward_params.
 *   ga  as pts_backward_params (the same values, bit for bit).
 *   gn  through the torus fit of Sec. 4.1 on the (not necessarily unit)
 *       input normal: its normalisation, the tangent frame built from it and
 *       the anchor o = p + a00 n.  The choice of the frame's seed axis (x-hat
 *       unless |n_x| >= 0.9) is piecewise constant and not differentiated.
 *   gp  the torus moves rigidly with its point, so its share is minus the
 *       force on the anchor; the weights of Eq. (BasicFormulaShifted) add
 *       sum_q gout_q (w_qi/W_q) lambda_q (g_i - phi_q) e_qi with
 *       e = (x - p_i)/|x - p_i|, and the farthest point p_* of each query
 *       (which sets M, hence sigma_x and lambda_x of
 *       Eq. RelationshipBetweenLambdaAndRadius) adds
 *       -gout_q (2C/M^2) V_q e_*, V_q = (1/W) sum_j w_j (g_j - phi_q) d_j.
 *       Ties for the farthest point go to the lowest record slot (the
 *       build's spatial order).
 * With gp the call re-runs the culled farthest-point sweep and one weighted
 * query sweep before the point sweep.  Deterministic (fixed-order reductions,
 * no atomics).  ws_bytes >= pts_backward_points_ws_bytes(N, Q, prm). */
int pts_backward_points(const void* rec, int64_t N, const float* p, const float* n, const float* a,
                        const float* x, int64_t Q, const float* gout, const float* stats, float* ga,
                        float* gp, float* gn, const pts_params* prm, void* ws, size_t ws_bytes,
                        void* stream);

/* ---------------------------------------------------------------------------
 * Sphere tracing (Sec. 5.3, "Direct visualization of point cloud surfaces").
 * ------------------------------------------------------------------------- */

/* Scratch bytes for pts_trace with R rays. */
int pts_trace_ws_bytes(int64_t N, int64_t R, const pts_params* prm, size_t* out_bytes);

/* March R rays x(t) = origin + t dir (dir unit length; device [R,3] float32)
 * through phi: t = 0; up to `steps` evaluations; a ray stops with a hit when
 * |phi(x)| < eps, else t += phi(x) and it stops with a miss once t > tmax.
 * Outputs (device): t_out [R] float32 (final t), hit_out [R] int32 (1 = hit),
 * steps_out [R] int32 or NULL (steps taken before stopping; `steps` if the
 * budget ran out), normal_out [R,3] float32 or NULL (grad phi / |grad phi| at
 * hits, 0 elsewhere).  Each step evaluates the active rays with the pts_eval
 * kernels.  The point splits depend on N only -- the march uses the largest
 * power of two <= 64 that leaves every split two 512-point tiles
 * (pts_params.splits > 0 sets it), the normals at most 8 of them -- so a ray's
 * result does not depend on the other rays.  Blocks: it reads back the active-ray count after
 * every step.  phi overestimates |distance| away from the surface for finite
 * C (Sec. 6), so rays can overshoot thin features. */
int pts_trace(const void* rec, int64_t N, const float* origin, const float* dir, int64_t R, int steps,
              float eps, float tmax, float* t_out, float* normal_out, int32_t* hit_out,
              int32_t* steps_out, const pts_params* prm, void* ws, size_t ws_bytes, void* stream);

/* Scratch bytes for pts_trace_bounded with R rays (enough for any number of
 * rays still marching). */
int pts_trace_bounded_ws_bytes(int64_t N, int64_t R, const pts_params* prm, size_t* out_bytes);

/* pts_trace with every step's phi from the error-bounded evaluation of
 * pts_eval_bounded at eval_eps (finite, >= 0, the cloud's distance units):
 * each step's phi is within eval_eps of pts_trace's (plus FP32 rounding), so
 * with eval_eps well below eps the march takes the same steps up to
 * differences of order steps x eval_eps in t, and a ray near the hit
 * threshold may stop one step apart.  The normals at hits are pts_trace's
 * (the exact gradient).  A ray's phi depends on the rays marching beside it
 * (they share the evaluation's wavefront votes) only within eval_eps.
 * Arguments otherwise as pts_trace; ws_bytes >= pts_trace_bounded_ws_bytes. */
int pts_trace_bounded(const void* rec, int64_t N, const float* origin, const float* dir, int64_t R, int steps,
                      float eps, float tmax, float eval_eps, float* t_out, float* normal_out, int32_t* hit_out,
                      int32_t* steps_out, const pts_params* prm, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Radius-limited evaluation (Sec. 4.2, "Acceleration and adaptive lambda"):
 * the paper's accelerated form of Eq. (BasicFormulaShifted) with a constant
 * lambda per cloud.  It is a different function from pts_eval's all-points phi.
 *
 *   D      = mean over points of the mean distance to their 64 nearest other
 *            points (all others if N <= 64; D = 1 if N = 1),
 *   lambda = 1e3 / D,   R_eval = 2 C / lambda,   sigma = R_eval / 2,
 *   phi(x) = sum_{|x-p_i| <= R_eval} g_i w_i / sum w_i,
 *            w_i = exp(-lambda (|x - p_i| - sigma));
 *   if no point lies within R_eval: the same blend over the 32 nearest points
 *   (all if N < 32), shifted by the nearest distance instead of sigma.
 * A cloud whose every point has 64 or more coincident copies has D = 0, an
 * infinite lambda and NaN results; it has no scale for this form.
 * ------------------------------------------------------------------------- */

typedef struct pts_radius_info {
  double D;       /* mean 64-nearest-neighbour distance */
  float lam;      /* lambda = 1e3 / D */
  float reval;    /* 2 C / lambda */
  int ready;      /* 1 after pts_radius_prepare */
  int reserved;
} pts_radius_info;

/* Compute D, lambda and R_eval for a built record (stored in the record;
 * pts_params.C sets C).  Asynchronous; uses the record's own build scratch. */
int pts_radius_prepare(void* rec, int64_t N, const pts_params* prm, void* stream);

/* Read them back (blocks). */
int pts_radius_info_get(const void* rec, pts_radius_info* out, void* stream);

/* Scratch bytes for pts_eval_radius with Q queries (16 bytes per query plus
 * radix-sort histograms). */
int pts_eval_radius_ws_bytes(int64_t N, int64_t Q, size_t* out_bytes);

/* Radius-limited phi at Q queries (device x [Q,3] -> sdf [Q]); count [Q]
 * int32 or NULL: number of points blended, negated when the 32-nearest
 * fallback was used, 0 for a query with a non-finite coordinate (phi NaN).
 * phi is NaN everywhere if pts_radius_prepare has not run on the record.
 * The queries are evaluated in Morton order of the cloud's bounding box (a
 * device radix sort in ws), which only changes the order of work: each
 * query's result depends on that query alone.  ws_bytes >=
 * pts_eval_radius_ws_bytes(N, Q).  Q = 0 is a no-op. */
int pts_eval_radius(const void* rec, int64_t N, const float* x, int64_t Q, float* sdf, int32_t* count, void* ws,
                    size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: a resident-cloud server with continuous batching.
 *
 * The server keeps many clouds' records resident on the device and answers
 * requests (phi at queries, or a sphere trace) from client threads.  A
 * scheduler thread admits queued requests in arrival order while fewer than
 * max_inflight are running and their device buffers fit the memory budget,
 * packs runnable work (query requests and the next step of every trace
 * request) into one launch of the evaluation kernels, and keeps up to two
 * such launches in flight on two streams, so requests that arrive while the
 * device is busy are admitted and start as soon as memory and a launch slot
 * free up.  A launch takes at most quantum_pairs of work, so a long request
 * (a trace step of many rays, many queries on a large cloud) runs as several
 * launches and a request behind it waits about one quantum.  Trace requests
 * advance one step at a time and are repacked until every ray has stopped;
 * then normals are computed at the hit rays.  The two launches overlap on the device only if HIP maps the two
 * streams to different hardware queues; with HIP's default of 4 queues per
 * process that depends on how many streams the process created earlier, so
 * a process that runs a server beside other GPU work should start with
 * GPU_MAX_HW_QUEUES=8 or more in its environment (results do not depend on
 * it, latency does).
 *
 * A query request of Q queries on a cloud of N points is evaluated with
 * pts_eval's automatic plan for (N, Q) -- or, if one launch of max_batch_work
 * workgroups cannot hold it, with the largest power-of-two split <= 64 that
 * fits -- and a trace request with the point split pts_server_cloud_plan
 * reports, a function of N only (the march split of pts_trace).  Results are
 * bitwise the same alone or in any mix, and equal pts_eval (default splits,
 * or the fitting split) and pts_trace (default splits) with the same C,
 * kfloor_rel.
 *
 * All device memory (records, request buffers, launch descriptors) comes from
 * one allocation of hbm_budget_bytes made at creation; that is the budget
 * requests are admitted against.  Host buffers named in a request are plain
 * host memory: inputs are copied before pts_server_submit returns, outputs are
 * written before the request is reported finished and must stay valid until
 * then.  All entry points are thread-safe.
 * ------------------------------------------------------------------------- */

typedef struct pts_server pts_server;

typedef struct pts_server_cfg {
  size_t hbm_budget_bytes;  /* device memory of the server; 0 = 4 GiB */
  int max_inflight;         /* requests admitted at once; 0 = 64 */
  int max_queue;            /* queued (not yet admitted) requests; 0 = 2^20 */
  int64_t max_batch_work;   /* workgroups per packed launch (512 queries x one
                               point split each); 0 = 131072.  A request needing
                               more than this is rejected with PTS_EINVAL. */
  float C;                  /* as pts_params; 0 = 64 */
  float kfloor_rel;         /* as pts_params; 0 = 1e-6 */
  int mock;                 /* 1 = no device: a cost model stands in for the
                               kernels (pairs / mock_pairs_per_s seconds per
                               launch) and outputs are filled with a pattern
                               (query requests: cloud + 1e-3 (j mod 1000); trace
                               requests: t = cloud, hit = j mod 2, normals 0, and
                               every ray stops after min(steps, 3) steps).  For
                               testing the scheduler on hosts without a GPU. */
  int mock_fail_count;      /* mock only: query requests of exactly this count
                               fail with PTS_EHIP (0 = never) */
  double mock_pairs_per_s;  /* mock only; 0 = 1e12 */
  double quantum_pairs;     /* query x point pairs one packed launch takes on
                               (about that many / 1.1e12 seconds of device
                               time); 0 = 4e9.  A request with more work is
                               spread over several launches in chunks of
                               512-query blocks (results do not depend on
                               it), so a request that arrives behind it waits
                               about one quantum for a launch slot. */
} pts_server_cfg;

#define PTS_REQ_EVAL 0
#define PTS_REQ_TRACE 1

typedef struct pts_request {
  int kind;           /* PTS_REQ_EVAL or PTS_REQ_TRACE */
  int cloud;          /* id from pts_server_add_cloud */
  int64_t count;      /* queries (EVAL) or rays (TRACE); 0 finishes at once */
  const float* in0;   /* host [count,3]: queries (EVAL) or ray origins (TRACE) */
  const float* in1;   /* host [count,3]: unit ray directions (TRACE) */
  float* out_sdf;     /* host [count]: phi (EVAL) or final t (TRACE) */
  float* out_normal;  /* host [count,3] or NULL (TRACE): normals at hits, 0 elsewhere */
  int32_t* out_hit;   /* host [count] (TRACE): 1 = hit */
  int32_t* out_steps; /* host [count] or NULL (TRACE): as pts_trace's steps_out */
  int steps;          /* TRACE: evaluation budget per ray (>= 0) */
  float eps, tmax;    /* TRACE: hit threshold and exit distance, as pts_trace */
  int reserved;
} pts_request;

/* Request states reported by pts_server_poll. */
#define PTS_STATE_QUEUED 0
#define PTS_STATE_RUNNING 1
#define PTS_STATE_DONE 2
#define PTS_STATE_FAILED 3
#define PTS_STATE_CANCELLED 4

typedef struct pts_server_stats {
  uint64_t submitted, completed, failed, cancelled, rejected;
  uint64_t launches;            /* packed launches issued */
  uint64_t overlapped_launches; /* launches issued while another was in flight */
  int64_t max_batch_requests;   /* most requests packed into one launch */
  double pairs;                 /* query x point pairs evaluated (all sweeps count once) */
  double busy_s;                /* sum of launch durations (device time) */
  double p50_ms, p99_ms, max_ms;/* latency, submit -> result written, all requests */
  double p50_eval_ms, p99_eval_ms, p50_trace_ms, p99_trace_ms;
  size_t bytes_resident;        /* cloud records */
  size_t bytes_inflight;        /* buffers of admitted requests */
  size_t bytes_reserved;        /* launch descriptors */
  int inflight, queued;
} pts_server_stats;

/* Create a server (cfg NULL = defaults); allocates its budget on the current
 * device and starts the scheduler thread.  PTS_ENOMEM if the budget cannot be
 * allocated or does not hold the launch descriptors. */
int pts_server_create(const pts_server_cfg* cfg, pts_server** out);

/* Upload and build a cloud (host p [N,3], n [N,3], a [N,6], as
 * pts_cloud_build) into the server's memory; blocks until built.
 * PTS_EBUDGET if its record (plus the inputs while building) does not fit. */
int pts_server_add_cloud(pts_server* srv, const float* p, const float* n, const float* a, int64_t N,
                         int* id);

/* Split and point count a cloud's requests are evaluated with. */
int pts_server_cloud_plan(pts_server* srv, int id, int64_t* N, int* splits);

/* Remove a cloud; PTS_EBUSY while requests on it are queued or running. */
int pts_server_remove_cloud(pts_server* srv, int id);

/* Queue a request.  PTS_EINVAL for a malformed request, PTS_ENOTFOUND for an
 * unknown cloud, PTS_EBUDGET if its buffers can never fit next to the
 * resident clouds, PTS_EBUSY if the queue is full. */
int pts_server_submit(pts_server* srv, const pts_request* req, uint64_t* ticket);

/* Current state (PTS_STATE_*) of a request. */
int pts_server_poll(pts_server* srv, uint64_t ticket, int* state);

/* Wait until a request has finished (timeout_ms < 0: no limit).  Returns the
 * request's status: PTS_OK, PTS_ECANCELLED, or the error it failed with;
 * PTS_ETIMEOUT if it is still queued or running at the limit. */
int pts_server_wait(pts_server* srv, uint64_t ticket, int timeout_ms);

/* Cancel a request.  A queued one finishes at once; a running one finishes,
 * with its outputs unwritten, once its current launch has completed. */
int pts_server_cancel(pts_server* srv, uint64_t ticket);

/* Forget a finished request (its ticket becomes unknown). PTS_EBUSY if it
 * has not finished or another thread is still inside pts_server_wait on it
 * (release it once that wait has returned). */
int pts_server_release(pts_server* srv, uint64_t ticket);

/* Counters and latency percentiles since creation or the last reset. */
int pts_server_stats_get(pts_server* srv, pts_server_stats* out);
int pts_server_stats_reset(pts_server* srv);

/* Stop the server: queued and running requests finish as PTS_ECANCELLED, the
 * scheduler drains the device, and all memory is freed.  NULL is a no-op. */
int pts_server_destroy(pts_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* PTS_H */
