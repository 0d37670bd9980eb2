/*
 * tsqbx.h -- C ABI of libtsqbx.so: target-specific QBX (TSQBX) near-field
 * evaluation of Laplace layer potentials on AMD MI355X (gfx950), in FP64.
 *
 * The operation (Wala & Kloeckner, "Optimization of fast algorithms for
 * global quadrature by expansion using target-specific expansions"):
 *
 * For every target t with its QBX center c = c(t) (targets are associated
 * with expansion balls, Sec. 3.2, stage 1 of Algorithm 1) and every source y
 * of the center's near-field list L(c) (the sources of U_b, W_b close and
 * X_b close for the box b owning c, Sec. 3.3; stages 3, 5(a) and 6(a) of
 * Algorithm 1), with strength q_y = w_y sigma_y (eq. pt-pot):
 *
 *   single layer  out_slp[t]    = sum_{y in L(c)} q_y G^(p)(t, y)
 *   double layer  out_dlp[t]    = sum_{y in L(c)} q_y nu_y . grad_y G^(p)(t, y)
 *   S'            out_sprime[t] = sum_{y in L(c)} q_y nu_t . grad_t G^(p)(t, y)
 *
 *   G^(p)(t, y) = 1/(4 pi) sum_{n=0..p} |t-c|^n / |y-c|^{n+1} P_n(cos gamma)
 *
 * with gamma the angle between t-c and y-c (eq. tsqbx, Sec. 2.7, and the
 * first formula of App. A), grad_y the source gradient and grad_t the target
 * gradient of App. A (S' is the normal derivative of the single layer at the
 * target, with nu_t the caller's unit normal at t).  P_n is
 * the Legendre polynomial; the expansion has p+1 terms, n = 0..p (Sec. 2.3:
 * a p-th order expansion keeps the first p+1 terms).  The factor 1/(4 pi) is
 * that of the Laplace Green's function (eq. laplace-green-function).  nu_y is
 * the outward unit normal at y, so with centers inside the surface the double
 * layer is the interior-side value.
 *
 * The result is the L^{qbx,near} term of Algorithm 1; TSQBX_ACCUMULATE adds
 * it into the output so that a caller can sum it with far-field terms
 * (stage 9).
 *
 * Conventions shared by every entry point:
 *  - Every function returns a tsqbx_status.  On error nothing is written to
 *    any output and tsqbx_last_error() describes the failure (per thread).
 *  - The caller owns every array it passes.  Handles are owned by the library
 *    until their destroy call; destroy(NULL) is a no-op returning TSQBX_OK.
 *  - Coordinates are [n][3] row-major float64 (numpy (n, 3) C order).
 *  - Outputs are indexed by the caller's target order.
 *  - Preconditions not checked: |y - c| > 0 for every listed pair, and
 *    finite inputs.  |t - c| < |y - c| is needed for the truncated series to
 *    approximate the kernel (App. A), not for the sum to be defined.
 *  - Tracing: every call that launches work, builds a geometry or a plan, or
 *    waits on a server opens a roctx range named after the function
 *    (rocprofv3 --marker-trace); the library links librocprofiler-sdk-roctx.
 */
#ifndef TSQBX_H
#define TSQBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSQBX_OK = 0,
  TSQBX_E_INVALID = -1, /* malformed argument: NULL pointer, bad layer mask, bad CSR */
  TSQBX_E_RANGE = -2,   /* index or order outside its range (p > TSQBX_P_MAX, index >= n) */
  TSQBX_E_NOMEM = -3,   /* host or device allocation failed */
  TSQBX_E_DEVICE = -4,  /* a HIP runtime call failed (message names it) */
  TSQBX_E_BUDGET = -5,  /* a request can never fit the server's device-memory budget */
  TSQBX_E_STATE = -6,   /* call not valid in the object's current state */
  TSQBX_E_TIMEOUT = -7, /* a wait ran out of time; the work is still pending */
  TSQBX_E_CANCELED = -8 /* a served request was withdrawn before it ran */
} tsqbx_status;

/* Layer bitmask: which potentials to evaluate. */
enum { TSQBX_SLP = 1u, TSQBX_DLP = 2u, TSQBX_SPRIME = 4u };

/* Added to a layer mask in the tuning calls: the bucket of the Helmholtz
 * kernels (tsqbx_eval_helmholtz). */
enum { TSQBX_HELMHOLTZ = 64u };

/* Flags. */
enum {
  TSQBX_ACCUMULATE = 1u, /* eval: add into the outputs instead of overwriting */
  TSQBX_NO_REORDER = 2u, /* geometry_create: keep the caller's source/target order on device */
  TSQBX_PER_TARGET = 4u  /* plain Laplace eval: one wave per target even where targets share a
                            center's list (by default, with one target per wave, 1.5 or more
                            targets per list on average and at most 16 on any, one wave walks a
                            list once for up to four of its targets; the results are the same
                            bits either way) */
};

/* Highest supported expansion order. */
#define TSQBX_P_MAX 32

/* A geometry holds fewer than this many sources (2^27: device byte offsets of
 * per-source records stay within 32 bits). */
#define TSQBX_MAX_SOURCES 134217728LL

typedef struct tsqbx_ctx tsqbx_ctx;
typedef struct tsqbx_geometry tsqbx_geometry;
typedef struct tsqbx_plan tsqbx_plan;
typedef struct tsqbx_server tsqbx_server;

/*
 * Geometry: sources with weights (eq. pt-pot), normals for the double layer,
 * QBX centers with their near-field source lists in CSR form, targets, the
 * target -> center association and target normals for S'.  All pointers are
 * host pointers.
 */
typedef struct {
  int64_t n_sources;           /* N >= 0 */
  const double *sources;       /* [N][3] source points y */
  const double *weights;       /* [N] quadrature x area weights w_y */
  const double *normals;       /* [N][3] outward unit normals, or NULL (then no TSQBX_DLP) */
  int64_t n_centers;           /* M >= 0 */
  const double *centers;       /* [M][3] expansion centers c */
  const int64_t *list_offsets; /* [M+1], offsets[0] = 0, nondecreasing */
  const int32_t *list_sources; /* [offsets[M]] source indices in [0, N); repeats count twice */
  int64_t n_targets;           /* T >= 0 */
  const double *targets;       /* [T][3] target points t */
  const int32_t *target_center;/* [T] center of each target in [0, M); NULL: T == M (or T == 0), target i uses center i */
  const double *target_normals;/* [T][3] unit normals at the targets, or NULL (then no TSQBX_SPRIME) */
} tsqbx_geometry_desc;

typedef struct {
  int64_t n_sources, n_centers, n_targets;
  int64_t nnz;          /* list entries */
  int64_t pairs;        /* sum over targets of the length of their center's list */
  int64_t max_list;     /* longest list */
  size_t device_bytes;  /* device memory held by the geometry */
  int has_normals;
  int has_target_normals;
} tsqbx_geometry_info;

/* Library version as major*10000 + minor*100 + patch. */
int tsqbx_version(void);

/* Message of the last failed call on this thread ("" if none).  The string
 * stays valid until the next failing call on the same thread. */
const char *tsqbx_last_error(void);

/* Host-only check of a geometry description (touches no device): CSR shape,
 * index ranges, target->center map.  Returns TSQBX_OK, TSQBX_E_INVALID or
 * TSQBX_E_RANGE.  geometry_create performs the same checks. */
int tsqbx_validate_geometry(const tsqbx_geometry_desc *desc);

/* Host-only preview of the device layout tsqbx_geometry_create builds for
 * desc (touches no device; same checks as tsqbx_validate_geometry).  Sources
 * are ordered along a Morton curve, targets by the Morton key of their
 * center (then center, then index), unless flags has TSQBX_NO_REORDER.  Each
 * distinct center that a target uses gets one row, in order of first use in
 * the target order; a row holds its center's list (Sec. 3.3 near-field sets)
 * in device source numbers, sorted ascending and padded to a multiple of 16
 * entries with the padding index N.  Outputs (each nullable):
 *   source_order [N]   device position -> caller source index
 *   target_order [T]   device position -> caller target index
 *   target_row   [T]   device position -> row
 *   row_offsets  [row_offsets_cap >= n_rows + 1] padded row offsets
 *   rows         [rows_cap >= nnz] the padded rows
 * info (required) receives n_rows, nnz (padded entries), pairs (list
 * entries over all targets) and max_list.  Buffers too small for rows or
 * offsets give TSQBX_E_RANGE with info filled in. */
typedef struct {
  int64_t n_rows, nnz, pairs, max_list;
} tsqbx_layout_info;
int tsqbx_geometry_layout(const tsqbx_geometry_desc *desc, unsigned flags, int64_t *source_order,
                          int64_t *target_order, int64_t *target_row, int64_t *row_offsets,
                          int64_t row_offsets_cap, int32_t *rows, int64_t rows_cap,
                          tsqbx_layout_info *info);

/* Create a geometry from arrays in device memory: every pointer of desc is
 * a device pointer (the offsets and lists may come straight from
 * tsqbx_ball_lists or tsqbx_knn_lists), with the meaning and layout of
 * tsqbx_geometry_create.  The Morton orders, rows, remap, padding and sort
 * run on the device, on hip_stream; the call returns when the geometry is
 * complete, and the result equals tsqbx_geometry_create's on the same
 * arrays bit for bit (tsqbx_geometry_read_layout shows it).  Only the counts
 * (8 bytes for the list total, 4 bytes for the row count) and the list
 * length of each target (8 T bytes, for plans) come back to the host.  The
 * checks of tsqbx_validate_geometry run on the device (TSQBX_E_INVALID,
 * TSQBX_E_RANGE); TSQBX_NO_REORDER is not supported (TSQBX_E_INVALID).
 * The caller's arrays may be freed once the call returns. */
int tsqbx_geometry_create_device(tsqbx_ctx *ctx, const tsqbx_geometry_desc *desc,
                                 unsigned flags, void *hip_stream, tsqbx_geometry **out);
/* Read a geometry's device layout back into host buffers, in the form of
 * tsqbx_geometry_layout (same outputs, each nullable, same errors for small
 * buffers).  Synchronous. */
int tsqbx_geometry_read_layout(const tsqbx_geometry *geom, int64_t *source_order,
                               int64_t *target_order, int64_t *target_row, int64_t *row_offsets,
                               int64_t row_offsets_cap, int32_t *rows, int64_t rows_cap,
                               tsqbx_layout_info *info);

/* Check (p, layers) against a geometry's capabilities without a launch:
 * p in [0, TSQBX_P_MAX], layers a nonempty subset of SLP|DLP|SPRIME, DLP
 * needs source normals and SPRIME target normals.  geom may be NULL (then the
 * normals checks are skipped). */
int tsqbx_check_request(const tsqbx_geometry *geom, int p, unsigned layers);

/* Context on one HIP device (device ordinal as hipSetDevice takes it). */
int tsqbx_ctx_create(int device, tsqbx_ctx **out);
int tsqbx_ctx_destroy(tsqbx_ctx *ctx);

/* Copy a geometry into device memory.  The library reorders sources and
 * targets along a Morton curve for locality (unless TSQBX_NO_REORDER) and
 * sorts each list ascending; outputs are still in the caller's order.  The
 * caller may free its arrays when the call returns.  The arrays are checked
 * on the host; a reordered geometry of 2^20 list entries or more is then
 * uploaded as given and laid out on the device (the layout of
 * tsqbx_geometry_create_device, identical to the host's), using temporary
 * device memory of about the input's size during the call. */
int tsqbx_geometry_create(tsqbx_ctx *ctx, const tsqbx_geometry_desc *desc, unsigned flags,
                          tsqbx_geometry **out);
int tsqbx_geometry_destroy(tsqbx_geometry *geom);
int tsqbx_geometry_get_info(const tsqbx_geometry *geom, tsqbx_geometry_info *out);

/* Plain evaluation, host pointers, synchronous.  sigma: [N] density in the
 * caller's source order; out_slp / out_dlp / out_sprime: [T], required for
 * each requested layer (may be NULL for a layer not requested). */
int tsqbx_eval(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p, unsigned layers,
               const double *sigma, double *out_slp, double *out_dlp, double *out_sprime,
               unsigned flags);

/* Plain evaluation, device pointers, asynchronous on hip_stream (a
 * hipStream_t passed as void*, NULL = the null stream).  The buffers must stay
 * valid until the stream work completes.  Calls on one geometry use that
 * geometry's own staging buffer, so two of them must not overlap in time on
 * different streams (calls on the same stream are ordered and safe). */
int tsqbx_eval_async(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p, unsigned layers,
                     const double *d_sigma, double *d_out_slp, double *d_out_dlp,
                     double *d_out_sprime, unsigned flags, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * tsqbx_eval_async with the strengths staged in a static device array of the
 * library instead of the geometry's staging buffer; the call allocates
 * nothing.  The array holds TSQBX_NOALLOC_SCRATCH_BYTES on every GPU that
 * loads the library, until the process ends.  A request needs
 * 32 (N + 1) bytes, rounded up to a multiple of 256, plus 24 (N + 1) with
 * TSQBX_DLP (N = sources), at most that size (N + 1 <= 299592 with the
 * double layer, 524288 without); a larger one gives TSQBX_E_RANGE and
 * launches nothing.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (each call writes all it reads): calls that
 * overlap in time on one GPU (on different streams, or unordered across
 * threads) race and give wrong results; calls on one stream are ordered and
 * safe.  Results equal tsqbx_eval_async's bit for bit; arguments, flags and
 * the other errors as for tsqbx_eval_async. */
#define TSQBX_NOALLOC_SCRATCH_BYTES (16u << 20)
int tsqbx_eval_async_noalloc(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p, unsigned layers,
                             const double *d_sigma, double *d_out_slp, double *d_out_dlp,
                             double *d_out_sprime, unsigned flags, void *hip_stream);

/* The same evaluation in two steps on device pointers: tsqbx_stage_async
 * forms the strengths q_y = w_y sigma_y (and q_y nu_y when layers include
 * TSQBX_DLP) in the geometry's staging buffer (eq. pt-pot); then
 * tsqbx_eval_staged_async sums the near field from them, as often as wanted
 * (for instance several orders or layer masks on one density).  Both run
 * asynchronously on hip_stream; the staging buffer is the one
 * tsqbx_eval_async uses, with the same overlap rule.  tsqbx_stage_async
 * checks layers as tsqbx_check_request does (any valid p).
 * tsqbx_eval_staged_async returns TSQBX_E_STATE when the geometry has not
 * been staged, or when it asks for the double layer and the last staging did
 * not include it; other errors as for tsqbx_eval_async.  The results equal
 * those of tsqbx_eval_async bit for bit. */
int tsqbx_stage_async(tsqbx_ctx *ctx, const tsqbx_geometry *geom, unsigned layers,
                      const double *d_sigma, void *hip_stream);
int tsqbx_eval_staged_async(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p, unsigned layers,
                            double *d_out_slp, double *d_out_dlp, double *d_out_sprime,
                            unsigned flags, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Conventional QBX, Laplace single layer (Sec. 2.3; the first approach of
 * Sec. 2.4): the comparator of the target-specific evaluation, O((p+1)^2)
 * work per (source, center) instead of O(p+1) per (source, target).
 *
 * Local coefficients of a center c (eq. local-coeffs summed over its list
 * with q_y = w_y sigma_y, eq. pt-pot):
 *   L_n^m(c) = sum_{y in L(c)} q_y Y_n^{-m}(y - c) / ((2n+1) |y - c|^{n+1}),
 * n = 0..p, Y_n^m of eq. sph-harm with P_n^{|m|} taken without the
 * Condon-Shortley factor, so that L_n^{-m} = conj(L_n^m) for real sigma.
 * Evaluation at a target t of center c (eq. local-expansion truncated after
 * n = p):  u(t) = sum_n sum_{|m|<=n} L_n^m |t - c|^n Y_n^m(t - c), which
 * equals the target-specific single layer of tsqbx_eval (eq. tsqbx) up to
 * rounding.
 *
 * d_coeffs: [n_centers][(p+1)^2] float64, device memory, compact real
 * layout: degree n at offset n^2 holds Re L_n^0, then Re L_n^m, Im L_n^m for
 * m = 1..n.  Only the rows of centers that at least one target uses are
 * written or read; the others are left untouched.  d_sigma [N] (caller's
 * source order) and d_out [T] (caller's target order) are device pointers;
 * work runs asynchronously on hip_stream and the buffers must stay valid
 * until it completes.  TSQBX_ACCUMULATE adds into d_coeffs (form) or d_out
 * (evaluate, form-and-evaluate) instead of overwriting.  Errors as for
 * tsqbx_eval_async: p outside [0, TSQBX_P_MAX] is TSQBX_E_RANGE, a NULL buffer
 * that would be touched is TSQBX_E_INVALID.  The form and the
 * form-and-evaluate calls use the geometry's staging buffer, as
 * tsqbx_eval_async does (same overlap rule).
 * ------------------------------------------------------------------------- */
/* P2QBXL: form the coefficients of every center that a target uses. */
int tsqbx_qbxl_form_async(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p,
                          const double *d_sigma, double *d_coeffs, unsigned flags,
                          void *hip_stream);
/* QBXL2P: evaluate given coefficients at every target. */
int tsqbx_qbxl_eval_async(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p,
                          const double *d_coeffs, double *d_out, unsigned flags,
                          void *hip_stream);
/* Both in one launch; the coefficients stay on chip and are not written. */
int tsqbx_eval_conventional_async(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p,
                                  const double *d_sigma, double *d_out, unsigned flags,
                                  void *hip_stream);

/* ---------------------------------------------------------------------------
 * Helmholtz kernel (App. A, Helmholtz case), real wavenumber k > 0:
 *
 *   G_k^(p)(t, y) = (i k / 4 pi) sum_{n=0..p} (2n+1) j_n(k|t-c|) h_n(k|y-c|) P_n(cos gamma)
 *
 * with j_n the spherical Bessel and h_n the spherical Hankel function of the
 * first kind: the p-th order target-specific expansion of
 * exp(ik|t-y|) / (4 pi |t-y|).  layers: TSQBX_SLP (q_y G_k^(p)), TSQBX_DLP
 * (q_y nu_y . grad_y G_k^(p), App. A's source gradient; the two operators of
 * the paper's Brakhage-Werner experiment) and TSQBX_SPRIME
 * (q_y nu_t . grad_t G_k^(p), App. A's target gradient dotted with the
 * geometry's target normal; at t = c its limit, the n = 1 term
 * (i k / 4 pi) k h_1(k|y-c|) (nu_t . (y-c)/|y-c|)).  Densities and outputs
 * are complex, stored as interleaved (re, im) float64 pairs (C99 double
 * complex, numpy complex128): sigma [N][2] in the caller's source order,
 * out_slp / out_dlp / out_sprime [T][2] in the caller's target order (NULL
 * for a layer not requested).  The first call on a geometry allocates its
 * Helmholtz staging (64 (N + 1) + 264 T bytes), the first S' call a further
 * 528 T bytes.  Errors as for tsqbx_eval (S' without target normals is
 * TSQBX_E_INVALID); k <= 0 or not finite gives TSQBX_E_RANGE.
 * ------------------------------------------------------------------------- */
int tsqbx_eval_helmholtz(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p, unsigned layers,
                         double k, const double *sigma, double *out_slp, double *out_dlp,
                         double *out_sprime, unsigned flags);
/* The same on device pointers, asynchronous on hip_stream. */
int tsqbx_eval_helmholtz_async(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p,
                               unsigned layers, double k, const double *d_sigma,
                               double *d_out_slp, double *d_out_dlp, double *d_out_sprime,
                               unsigned flags, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Near-field lists on the device.  For every center c the sources y inside
 * the closed ball of radius r about c (the near-field source set of Sec. 3.3,
 * taken as a ball), in ascending source index: the CSR that
 * tsqbx_geometry_desc takes.  Membership is decided in FP64 as
 * dx = y_x - c_x (likewise y, z), d2 = (dx*dx + dy*dy) + dz*dz, each operation
 * rounded on its own, member iff d2 <= r*r.
 *
 * d_sources [N][3], d_centers [M][3]: device pointers, row-major float64.
 * d_offsets [M+1] (int64, device) is always written.  d_indices (int32,
 * device, `capacity` entries) receives the entries when they fit; *nnz
 * receives their number in any case, and a call with too small a capacity
 * returns TSQBX_E_RANGE (call again with a larger buffer).  A ball holding
 * more than 8192 sources gives TSQBX_E_RANGE.  Work runs on hip_stream; the
 * call allocates its own scratch (about 56 N + 8 M bytes plus a hash table
 * of 2N to 4N cells x 28 bytes) and returns when the lists are written.
 * ------------------------------------------------------------------------- */
int tsqbx_ball_lists(tsqbx_ctx *ctx, int64_t n_sources, const double *d_sources,
                     int64_t n_centers, const double *d_centers, double radius,
                     int64_t *d_offsets, int32_t *d_indices, int64_t capacity, int64_t *nnz,
                     void *hip_stream);

/* Nearest-neighbour near-field lists on the device: for every center c the
 * d_counts[c] sources nearest to c (the near-field source set of Sec. 3.3,
 * taken as the k_c nearest sources), in ascending source index.  "Nearest"
 * is the order of (d2, source index) with d2 formed in FP64 exactly as for
 * tsqbx_ball_lists, so equal distances go to the smaller index and the
 * result is unique.
 *
 * d_counts [M] (int32, device): 0 <= k_c <= min(N, 8192), else
 * TSQBX_E_RANGE.  Offsets, capacity and nnz as for tsqbx_ball_lists
 * (nnz = sum of the counts).  The call allocates its own scratch (about
 * 56 N bytes plus a hash table of 2N to 4N cells x 28 bytes) and returns
 * when the lists are written.  Work grows with the number of grid cells
 * between a center and its k_c-th neighbour, so centers far from every
 * source are slow (never wrong).
 * ------------------------------------------------------------------------- */
int tsqbx_knn_lists(tsqbx_ctx *ctx, int64_t n_sources, const double *d_sources,
                    int64_t n_centers, const double *d_centers, const int32_t *d_counts,
                    int64_t *d_offsets, int32_t *d_indices, int64_t capacity, int64_t *nnz,
                    void *hip_stream);

/* ---------------------------------------------------------------------------
 * Launch tuning.  A target's result depends only on its list, whether the
 * single layer is evaluated alone (it then runs its own recurrence; with DLP or
 * SPRIME every layer comes from one derivative recurrence) and group_lanes: it
 * is bitwise identical across every other setting, and across the plain,
 * batched and served paths at equal group_lanes.
 * ------------------------------------------------------------------------- */
typedef struct {
  int waves_per_block;   /* 1, 2, 4, or 8 for the plain Laplace kernel only (its
                            default with one target per wave); plans and
                            servers run blocks of at most 4, and a Helmholtz
                            key refuses 8 */
  int group_lanes;       /* lanes that share one target: 64, 32 or 16 */
  int unroll;            /* independent pairs in flight per lane: 1, 2 or 4 */
  int xcd_remap;         /* 1: give each XCD a contiguous range of targets */
} tsqbx_tuning;

/* The tuning the library uses for (p, layers) and a typical list length
 * (layers | TSQBX_HELMHOLTZ for the Helmholtz kernels). */
int tsqbx_get_tuning(tsqbx_ctx *ctx, int p, unsigned layers, int64_t mean_list,
                     tsqbx_tuning *out);
/* Override it (all later launches on ctx for this (p, layers) bucket). */
int tsqbx_set_tuning(tsqbx_ctx *ctx, int p, unsigned layers, int64_t mean_list,
                     const tsqbx_tuning *tuning);

/* Time every candidate tuning on geom (device-resident sigma of ones) and
 * install the fastest for its (p, layers, list-length) bucket.  *out receives
 * it; best_ms (nullable) the kernel time.  The geometry's staging buffer is
 * overwritten, so tsqbx_eval_staged_async needs a new tsqbx_stage_async. */
int tsqbx_autotune(tsqbx_ctx *ctx, const tsqbx_geometry *geom, int p, unsigned layers,
                   tsqbx_tuning *out, double *best_ms);

/* ---------------------------------------------------------------------------
 * Batched evaluation: many (geometry, p, layers) items in one persistent
 * kernel launch, captured once into a HIP graph and replayed.
 * ------------------------------------------------------------------------- */
typedef struct {
  const tsqbx_geometry *geom;
  int p;
  unsigned layers;
  const double *d_sigma;   /* device [N] */
  double *d_out_slp;       /* device [T] or NULL */
  double *d_out_dlp;       /* device [T] or NULL */
  double *d_out_sprime;    /* device [T] or NULL */
} tsqbx_item;

typedef struct {
  int64_t n_items;
  int64_t n_units;       /* work units the persistent kernel schedules */
  int64_t pairs;
  int64_t pair_terms;    /* sum over items of pairs x (p+1) x layer count */
  int grid_blocks;
  int waves_per_block;
  size_t device_bytes;   /* plan-owned device memory */
} tsqbx_plan_info;

/* Host-only preview of the static schedule a Laplace plan runs (touches no
 * device; the batch decomposition of the batched path).  Item i has
 * n_targets[i] targets whose list lengths follow one another in row_len (in
 * the geometry's device order of targets; all items concatenated), order
 * p[i] and layer mask layers[i].  Items are taken largest first (pairs times
 * the cost of one pair) and cut into units, runs of consecutive targets of
 * one item, dealt to at most max_waves waves of group_lanes-lane groups
 * (16, 32 or 64) at about equal estimated cost.  On return *n_units units
 * fill units[k] = (item, first target, count) ([units_cap][3] int32) and
 * wave w works through units wave_begin[w] .. wave_begin[w+1]-1
 * (wave_begin: max_waves + 1 entries; *n_waves waves used).  A units buffer
 * that is too small gives TSQBX_E_RANGE with *n_units set; NULL inputs or a
 * bad group width TSQBX_E_INVALID; p, layers as tsqbx_check_request. */
int tsqbx_schedule_preview(int64_t n_items, const int64_t *n_targets, const int64_t *row_len,
                           const int32_t *p, const uint32_t *layers, int group_lanes,
                           int max_waves, int32_t *units, int64_t units_cap, int64_t *n_units,
                           int32_t *wave_begin, int32_t *n_waves);

/* Build a plan.  Items' geometries and device buffers must outlive the plan;
 * the same geometry may appear in several items (each item gets its own
 * staging).  flags: TSQBX_ACCUMULATE applies to every item. */
int tsqbx_plan_create(tsqbx_ctx *ctx, int64_t n_items, const tsqbx_item *items,
                      unsigned flags, tsqbx_plan **out);

/* Batched Helmholtz evaluation (the kernel of tsqbx_eval_helmholtz): one
 * item per (geometry, p, layers, k) with complex density and outputs,
 * interleaved (re, im) float64 on the device as for
 * tsqbx_eval_helmholtz_async.  The plan stages every item's density and
 * per-target j_n tables and evaluates all items in one persistent launch
 * (one target per wave), captured into a HIP graph on the first
 * tsqbx_plan_execute; the result of every item equals
 * tsqbx_eval_helmholtz_async with group_lanes 64 bit for bit.  Errors as for
 * tsqbx_eval_helmholtz and tsqbx_plan_create; execute, get_info and destroy
 * are the plan calls above.  The plan holds per item 64 (N + 1) + 264 T
 * bytes (and 528 T more for S'). */
typedef struct {
  const tsqbx_geometry *geom;
  int p;
  unsigned layers;           /* TSQBX_SLP | TSQBX_DLP | TSQBX_SPRIME */
  double k;                  /* wavenumber, > 0 and finite */
  const double *d_sigma;     /* [N][2] complex, caller's source order */
  double *d_out_slp;         /* [T][2] complex, caller's target order */
  double *d_out_dlp;
  double *d_out_sprime;
} tsqbx_helm_item;
int tsqbx_plan_create_helmholtz(tsqbx_ctx *ctx, int64_t n_items, const tsqbx_helm_item *items,
                                unsigned flags, tsqbx_plan **out);
/* Run every item once on hip_stream (graph replay after the first call). */
int tsqbx_plan_execute(tsqbx_plan *plan, void *hip_stream);
int tsqbx_plan_get_info(const tsqbx_plan *plan, tsqbx_plan_info *out);
int tsqbx_plan_destroy(tsqbx_plan *plan);

/* Launch shape and static schedule of a plan's persistent kernel (the batch
 * decomposition; the paper leaves the evaluation's schedule to the
 * implementation).  A target's result depends only on group_lanes (as for
 * tsqbx_tuning): a plan equals tsqbx_eval_async at the same group_lanes bit
 * for bit whatever the other fields are. */
typedef struct {
  int group_lanes;       /* lanes per target: 64, 32 or 16 */
  int unroll;            /* pairs in flight per lane: 2, or 1 with 64 lanes */
  int waves_per_block;   /* 1, 2 or 4 */
  int oversubscription;  /* schedule ranges per resident wave slot (6 per SIMD), 1..32 */
  int step_cost;         /* fixed cost of one wave-step in the schedule's cost model,
                            in the units of one pair's instruction count, 0..100000 */
} tsqbx_plan_tuning;

/* The tuning a plan runs with: taken at creation from the context's table
 * for the plan's bucket (set by tsqbx_plan_autotune or tsqbx_tuning_load:
 * kernel, orders present, layers, list length and size, each rounded to a
 * power of two), else the defaults. */
int tsqbx_plan_get_tuning(const tsqbx_plan *plan, tsqbx_plan_tuning *out);
/* Rebuild the schedule for another tuning (TSQBX_E_INVALID if a field is out
 * of range).  Waits for the device to finish the plan's earlier work; the
 * next tsqbx_plan_execute captures a new graph. */
int tsqbx_plan_set_tuning(tsqbx_plan *plan, const tsqbx_plan_tuning *tuning);

/* Durations of a plan's kernels: the plan's launches run reps + 1 times on
 * hip_stream without the graph (the first run untimed), each kernel between
 * its own pair of HIP events; out receives the mean per-run milliseconds.
 * Synchronous.  Each run writes (or, with TSQBX_ACCUMULATE, adds to) the
 * outputs as tsqbx_plan_execute does.  reps in [1, 1000]. */
typedef struct {
  double stage_ms;       /* staging of every item's density (Helmholtz: and the j_n tables) */
  double eval_ms;        /* the persistent evaluation kernel */
  int reps;
} tsqbx_plan_timing;
int tsqbx_plan_profile(tsqbx_plan *plan, int reps, void *hip_stream, tsqbx_plan_timing *out);

/* Time the plan's evaluation kernel (tsqbx_plan_profile, 3 runs each) over
 * its candidate tunings, one field at a time: group_lanes with unroll, then
 * waves_per_block, oversubscription and step_cost, each starting from the best
 * so far; keep the fastest, install it in the context's table for the plan's
 * bucket (later plans of that bucket start from it) and return it in *out
 * (nullable) with its time in *best_ms (nullable).  Synchronous; runs the
 * plan about 60 times, so outputs of a TSQBX_ACCUMULATE plan must be reset
 * afterwards.  A later tsqbx_plan_set_tuning may choose another group width
 * and with it other bits (see tsqbx_plan_tuning). */
int tsqbx_plan_autotune(tsqbx_plan *plan, void *hip_stream, tsqbx_plan_tuning *out,
                        double *best_ms);

/* Persist the context's tuning tables (plain-kernel tunings from
 * tsqbx_autotune / tsqbx_set_tuning, and plan tunings) to a text file of JSON
 * lines, each tagged with the device's architecture name and the HIP runtime
 * version; tsqbx_tuning_load reads such a file and installs the entries made
 * on the same architecture and runtime (*n_loaded, nullable, counts them) and
 * skips the others.  TSQBX_E_INVALID for a file that cannot be opened or a
 * line that is not of this form. */
int tsqbx_tuning_save(tsqbx_ctx *ctx, const char *path);
int tsqbx_tuning_load(tsqbx_ctx *ctx, const char *path, int *n_loaded);

/* ---------------------------------------------------------------------------
 * Serving: requests against device-resident geometries, admitted under a
 * device-memory budget and batched continuously: requests that arrive while
 * others run are launched in the next step on another stream, so their work
 * overlaps on the device.
 * ------------------------------------------------------------------------- */
typedef struct {
  uint64_t submitted, admitted, completed, failed, rejected;
  uint64_t steps;               /* batched launches */
  size_t bytes_in_flight, peak_bytes_in_flight, budget_bytes;
  int64_t pair_terms_completed;
  double latency_p50_ms, latency_p90_ms, latency_p99_ms, latency_max_ms;
  double queue_p50_ms, queue_p99_ms; /* submit -> launch */
  double busy_s;                /* wall time with at least one step on the device */
  double host_launch_s;         /* scheduler time spent issuing steps */
} tsqbx_server_stats;

/* hbm_budget: bytes of per-request device memory that may be in flight
 * (staging records, density, outputs); max_slots: requests in flight. */
int tsqbx_server_create(tsqbx_ctx *ctx, size_t hbm_budget, int max_slots,
                        tsqbx_server **out);
/* Bytes a request on geom with these layers reserves from the budget. */
int tsqbx_server_request_bytes(const tsqbx_geometry *geom, unsigned layers, size_t *out);
/* Queue a request.  sigma_host is copied before the call returns; the output
 * buffers must stay valid until the ticket completes.  Thread-safe. */
int tsqbx_server_submit(tsqbx_server *srv, const tsqbx_geometry *geom, int p, unsigned layers,
                        const double *sigma_host, double *out_slp_host, double *out_dlp_host,
                        double *out_sprime_host, uint64_t *ticket);
/* As tsqbx_server_submit, without copying: sigma_host and the outputs must be
 * pinned host memory (hipHostMalloc, or a pinned torch tensor) and stay valid
 * and unmodified until the ticket completes.  Densities are uploaded and
 * outputs downloaded by DMA straight from and into these buffers.  Returns
 * TSQBX_E_INVALID if a buffer is not pinned host memory. */
int tsqbx_server_submit_pinned(tsqbx_server *srv, const tsqbx_geometry *geom, int p,
                               unsigned layers, const double *sigma_host, double *out_slp_host,
                               double *out_dlp_host, double *out_sprime_host, uint64_t *ticket);
/* Queue a Helmholtz request (the kernel of tsqbx_eval_helmholtz, real
 * wavenumber k > 0): sigma_host [N][2] and the outputs [T][2] are complex,
 * interleaved (re, im), in the caller's orders; sigma_host is copied before
 * the call returns, the outputs must stay valid until the ticket completes.
 * Helmholtz and Laplace requests share the server's steps; each is evaluated
 * with the server's one launch shape, so its result does not depend on what
 * it is batched with.  Errors as for tsqbx_eval_helmholtz and
 * tsqbx_server_submit.  Thread-safe. */
int tsqbx_server_submit_helmholtz(tsqbx_server *srv, const tsqbx_geometry *geom, int p,
                                  unsigned layers, double k, const double *sigma_host,
                                  double *out_slp_host, double *out_dlp_host,
                                  double *out_sprime_host, uint64_t *ticket);
/* The same without copies: sigma_host and the outputs are the caller's
 * pinned host buffers (as for tsqbx_server_submit_pinned), unmodified and
 * valid until the ticket completes. */
int tsqbx_server_submit_helmholtz_pinned(tsqbx_server *srv, const tsqbx_geometry *geom, int p,
                                         unsigned layers, double k, const double *sigma_host,
                                         double *out_slp_host, double *out_dlp_host,
                                         double *out_sprime_host, uint64_t *ticket);
/* Bytes a Helmholtz request of order p with these layers reserves. */
int tsqbx_server_request_bytes_helmholtz(const tsqbx_geometry *geom, int p, unsigned layers,
                                         size_t *out);
/* *done = 1 once the outputs are written (0 while pending).  Returns the
 * request's error status if it failed.  The server remembers the tickets of
 * pending requests and of the last 4096 completed ones (a long-running server
 * holds bounded host memory); an older ticket gives TSQBX_E_INVALID, as an
 * unknown one does. */
int tsqbx_server_poll(tsqbx_server *srv, uint64_t ticket, int *done);
/* Block until the ticket completes or timeout_s passes (TSQBX_E_TIMEOUT).
 * Tickets as for tsqbx_server_poll (one being waited on is not forgotten). */
int tsqbx_server_wait(tsqbx_server *srv, uint64_t ticket, double timeout_s);
/* Block until every submitted request has completed. */
int tsqbx_server_drain(tsqbx_server *srv, double timeout_s);
/* The server's launch and step shape: the persistent kernel's group width
 * and pairs in flight per lane (16/2, 32/2, 64/1 or 64/2) and waves per
 * block (1, 2 or 4), the wave-steps per work unit (1..64), the requests per
 * step (1..256), and dma_min_sources: densities in pinned memory of
 * geometries with at least this many sources are uploaded by DMA instead of
 * being read by the staging kernel over PCIe (0: never).  A request's result
 * depends on group_lanes only.  The defaults: 16, 2, 4, 8, 32, 0. */
typedef struct {
  int group_lanes, unroll, waves_per_block;
  int unit_steps, step_requests;
  int64_t dma_min_sources;
} tsqbx_server_tuning;
int tsqbx_server_get_tuning(tsqbx_server *srv, tsqbx_server_tuning *out);
/* Install a tuning; only before the first submission (TSQBX_E_STATE after
 * it, so that every request of a server is summed with one group width);
 * TSQBX_E_RANGE for an unsupported shape. */
int tsqbx_server_set_tuning(tsqbx_server *srv, const tsqbx_server_tuning *tuning);
/* Time candidate tunings on bursts of n_requests requests cycling over the
 * n (geometry, order, layer mask, density) tuples (the path of
 * tsqbx_server_submit_pinned; results discarded): one field at a time from
 * the best so far (group width and pairs in flight, then waves per block
 * {1, 2, 4}, unit steps {4, 8, 16}, requests per step {16, 32, 64}), best of
 * two bursts each after a warm-up burst, a candidate replacing the best only
 * when 3 % faster.  sigmas: n densities in pinned host memory (the caller's
 * own, so that reads over PCIe cost what they will), or NULL for densities
 * of ones in one shared buffer.  dma_min_sources is left as it is.  Installs
 * the result, returns it in *out and its burst time in *best_ms (both
 * nullable), and resets the statistics.  Only before the first submission
 * (TSQBX_E_STATE), and not concurrently with submissions on this server. */
int tsqbx_server_autotune(tsqbx_server *srv, int64_t n, const tsqbx_geometry *const *geoms,
                          const int *p, const unsigned *layers, const double *const *sigmas,
                          int n_requests, tsqbx_server_tuning *out, double *best_ms);
/* Withdraw a request that is still queued (not yet admitted to a step): it
 * completes with TSQBX_E_CANCELED, its outputs untouched, and counts as
 * failed.  TSQBX_E_STATE once it has been admitted or has ended,
 * TSQBX_E_INVALID for an unknown ticket.  Thread-safe. */
int tsqbx_server_cancel(tsqbx_server *srv, uint64_t ticket);
/* Counters since creation; latency and queueing percentiles over the last
 * 65536 completed requests. */
int tsqbx_server_get_stats(tsqbx_server *srv, tsqbx_server_stats *out);
/* Stop accepting requests, finish the ones in flight, free everything. */
int tsqbx_server_destroy(tsqbx_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* TSQBX_H */
