/*
 * vsht.h -- C interface of the MI355X (gfx950) vector spherical harmonic
 * transform library.
 *
 * The library computes the two transforms of Le Gia, Li and Wang, "FaVeST:
 * fast vector spherical harmonic transforms" for tangent fields T: S^2 -> C^3:
 *
 *   forward  (Definition 4.1, eq. (fwdvsht2)), for 1 <= l <= L, |m| <= l:
 *       a_{l,m} = sum_{k=1}^{N} w_k Y^div_{l,m}(x_k)^* T_k
 *       b_{l,m} = sum_{k=1}^{N} w_k Y^curl_{l,m}(x_k)^* T_k
 *   adjoint  (Definition 4.2, eq. (SLvec)), at every point x_i of the plan:
 *       T(x_i) = sum_{l=1}^{L} sum_{m=-l}^{l} a_{l,m} Y^div_{l,m}(x_i) + b_{l,m} Y^curl_{l,m}(x_i)
 *
 * with Y^div, Y^curl the vector spherical harmonics of Definition 3.1 (built
 * from 4pi-orthonormal scalar harmonics with the Condon-Shortley phase; the
 * negative orders satisfy Y_{l,-m} = (-1)^m conj(Y_{l,m})).  The quadrature
 * rule Q_N = {(w_k, x_k)} is the one of Section 4.1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Points    host array xyz[n][3] of binary64 unit vectors, row-major.
 * Weights   host array w[n] of binary64 (the quadrature weights).
 * Field T   device array of n x 3 complex numbers, row-major, each complex as
 *           (re, im) adjacent: complex128 for VSHT_FP64, complex64 otherwise.
 * Coeffs    device arrays a, b of vsht_num_coeffs(L) = L(L+2) complex numbers
 *           in the order l = 1..L, m = -l..l, i.e. a[l*l + l + m - 1]
 *           (same complex type as T).  There is no l = 0 entry.
 * Streams   `stream` is a hipStream_t passed as void* (NULL = the null
 *           stream).  Every call enqueues work on that stream and returns
 *           without waiting; buffers must stay valid until the stream has
 *           finished.  A plan must not run on two streams at the same time
 *           (it owns one workspace); create one plan per concurrent stream.
 * Ownership The plan deep-copies points and weights at creation and owns its
 *           device tables and workspace; the caller owns T, a and b.
 * Errors    Every function returns a vsht_status and never throws; on an
 *           error the outputs are unspecified.  vsht_last_error() returns a
 *           thread-local description of the last error on the calling thread.
 *           A buffer that does not start on a whole complex element (16
 *           bytes for complex128, 8 for complex64) is refused with
 *           VSHT_EINVAL before any work is enqueued.
 *
 * Point sets
 * ----------
 * The fast path needs iso-latitude rings: the points are grouped into
 * consecutive runs with bitwise-equal z (one run per ring), each run holding
 * n_phi >= 1 points at longitudes phi_0 + 2 pi j / n_phi, j = 0..n_phi-1 (in
 * this order), and no ring at a pole (weights may differ from point to point;
 * a ring of equal weights takes a faster path).  Rings whose
 * z values are exact negatives of each other are paired (north/south).  The
 * Gauss-Legendre product grids of Section 5.1 are of this kind.  Other point
 * sets are "scattered".
 *
 * Scattered points (the arbitrary points of eq. (expan)) are evaluated through
 * the double Fourier sphere: the synthesis runs on equispaced colatitudes of
 * the doubled circle, a DFT in theta gives the exact 2-D Fourier coefficients
 * of the spin-frame components, and every point gathers a window of an
 * oversampled grid with the exponential-of-semicircle kernel (width 14 grid
 * points in binary64, 8 otherwise; relative error near 1e-13 resp. 1e-6).
 * VSHT_OPT_SCATTERED_DIRECT selects the direct O(n L^2) evaluation instead; L
 * above 1279 always uses it (the grid's DFTs then no longer fit the kernels).  The forward transforms at scattered points run
 * the conjugate transpose of the grid path (spreading instead of gathering);
 * a plan on the direct path serves the adjoint only (VSHT_EUNSUPPORTED).
 */
#ifndef VSHT_H
#define VSHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vsht_plan_s *vsht_plan_t;

typedef enum {
    VSHT_OK = 0,
    VSHT_EINVAL = 1,      /* invalid argument (sizes, null pointers, non-unit or non-finite points) */
    VSHT_ENOWEIGHTS = 2,  /* forward called on a plan created without weights */
    VSHT_ENOMEM = 3,      /* host or device allocation failed */
    VSHT_EDEVICE = 4,     /* a HIP call failed; vsht_last_error() has the detail */
    VSHT_EUNSUPPORTED = 5 /* valid request the library cannot serve (e.g. forward on scattered points) */
} vsht_status;

typedef enum {
    VSHT_FP64 = 0,   /* complex128 I/O, binary64 arithmetic throughout */
    VSHT_FP32 = 1,   /* complex64 I/O, binary32 contraction and FFT, binary64 Legendre recurrence */
    VSHT_BF16X3 = 2, /* complex64 I/O, Legendre contraction as three bf16 split products with
                        binary32 accumulation, binary64 Legendre recurrence */
    VSHT_BF16X6 = 3  /* as VSHT_BF16X3 with three bf16 parts per operand and six products
                        (the dropped terms are below binary32 rounding) */
} vsht_precision;

/* Flags of vsht_opts. */
enum {
    VSHT_OPT_SCATTERED_DIRECT = 1, /* scattered points: direct evaluation (O(n L^2)) instead of
                                      the double-Fourier-sphere grid */
    VSHT_OPT_NO_FOLD = 2           /* ring grids: do not fold north/south mirror rings into pairs
                                      (every ring is its own pair; same results, about twice the
                                      Legendre work) */
};

typedef struct {
    int precision;          /* a vsht_precision value */
    int device;             /* HIP device ordinal; -1 = the calling thread's current device */
    int flags;              /* VSHT_OPT_* */
    double nfft_eps;        /* scattered grid path: target relative accuracy of the window
                               gather, 0 for the default (about 1e-13 in binary64, 1e-7 in
                               binary32); picks the window width w = ceil(-log10 eps) + 1 rounded
                               up to even, within [4, 16].  VSHT_EINVAL outside [0, 1). */
    const char *tune_cache; /* batch plans: a text file in which vsht_batch_autotune keeps the
                               fastest launch shape per (device architecture, precision, field
                               shapes); a later autotune of the same batch reads it instead of
                               timing.  NULL: no cache. */
} vsht_opts;

/* Plan kinds reported by vsht_plan_info. */
typedef enum { VSHT_PLAN_RINGS = 0, VSHT_PLAN_SCATTERED = 1, VSHT_PLAN_BATCH = 2 } vsht_plan_kind;

typedef struct {
    int L;
    int precision;
    int kind;           /* vsht_plan_kind */
    int64_t n_points;
    int64_t n_rings;    /* rings found (0 for scattered) */
    int64_t n_pairs;    /* north/south ring pairs incl. unpaired rings (0 for scattered) */
    int64_t max_nphi;   /* longest ring */
    int has_weights;
    size_t workspace_bytes;
    size_t table_bytes;
    int64_t nfft_grid;  /* scattered plans: grid size of the double-Fourier-sphere path (0: direct) */
} vsht_plan_info_t;

/* Number of coefficients of each kind for bandlimit L: L(L+2) (L >= 1), else 0. */
int64_t vsht_num_coeffs(int L);

/* Device workspace the plan owns (bytes; the *_many calls add their per-field
 * workspace on first use).  0 for NULL. */
size_t vsht_workspace_bytes(vsht_plan_t plan);

/* Create a plan for bandlimit L >= 1 on n points.
 *   xyz     host, n x 3 binary64 unit vectors (| |x| - 1 | <= 1e-12), finite.
 *   w       host, n binary64 weights, or NULL for an adjoint-only plan.
 *   opts    NULL for defaults (VSHT_FP64, current device).
 *   out     receives the plan on success.
 * Requirements: n >= 1; a plan with weights needs n >= 2 (Section 4.1, the
 * quadrature rule has N >= 2 nodes).  Returns VSHT_EINVAL on a violation,
 * VSHT_EUNSUPPORTED for L > 4096, VSHT_ENOMEM / VSHT_EDEVICE on allocation or
 * HIP failures.  The same limit holds for the fields of a batch plan.  Every
 * (order, ring) starts its Legendre recurrence at the first 32-degree block in
 * which the function reaches 2^-64, from a state computed with a carried
 * exponent, so seeds Lambda_{m,m} below binary64's range (L above ~1700) are
 * served exactly; terms below 2^-64 are dropped. */
vsht_status vsht_plan(int L, int64_t n, const double *xyz, const double *w,
                      const vsht_opts *opts, vsht_plan_t *out);

/* Forward transform (Definition 4.1, eq. (fwdvsht2)): T (device, n x 3) ->
 * a, b (device, L(L+2) each).  VSHT_ENOWEIGHTS if the plan has no weights,
 * VSHT_EUNSUPPORTED on a scattered plan on the direct path. */
vsht_status vsht_forward(vsht_plan_t plan, const void *T, void *a, void *b, void *stream);

/* Forward transform with unit weights, i.e. the exact adjoint (Hermitian
 * transpose) of vsht_adjoint as a linear map C^{2K} -> C^{3n}: the sum of
 * Definition 4.1, eq. (fwdvsht2), with every w_k = 1,
 *   a_{l,m} = sum_k Y^div_{l,m}(x_k)^* T_k, b likewise,
 * which transposes the synthesis of Definition 4.2, eq. (SLvec).
 * Used as the backward of the adjoint in automatic differentiation.  Works on
 * plans with or without weights; VSHT_EUNSUPPORTED on a scattered plan on the
 * direct path. */
vsht_status vsht_forward_unweighted(vsht_plan_t plan, const void *T, void *a, void *b,
                                    void *stream);

/* Adjoint transform (Definition 4.2, eq. (SLvec)): a, b (device) -> T
 * (device, n x 3) at every point of the plan, in the plan's point order. */
vsht_status vsht_adjoint(vsht_plan_t plan, const void *a, const void *b, void *T, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): vsht_forward on a ring plan
 * with its intermediate buffers (ring-Fourier buffer, coefficient triangle, and
 * for plans over 1024 ring pairs the partial triangles) in a static device array
 * of VSHT_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends, instead of the plan's workspace.  Same arguments,
 * layouts and results as vsht_forward (the same kernels).  The call performs
 * no allocation: no hipMalloc/hipFree, no events, no stage timing.
 *   VSHT_EUNSUPPORTED  scattered plans, or a plan that needs more than
 *                      VSHT_STATIC_SCRATCH_BYTES (vsht_last_error gives the size);
 *                      FP64 plans fit up to the GL grid at L = 1024.
 *   VSHT_ENOWEIGHTS    plan without weights.
 * All calls on one GPU share the array: calls that overlap on one GPU (on
 * different streams, or from several threads) race and give wrong results. */
#define VSHT_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
vsht_status vsht_forward_static(vsht_plan_t plan, const void *T, void *a, void *b, void *stream);

/* Scalar transforms on ring plans, with the same stages (scalar coefficients
 * f_{l,m}, 0 <= l <= L, |m| <= l, at index l^2 + l + m; vsht_num_sht_coeffs(L)
 * = (L+1)^2 of them; complex128 for VSHT_FP64, complex64 otherwise).
 *   vsht_sht_forward: the discrete forward scalar transform (FwdSHT, Section
 *     4.1, eq. (Flm)) f (device, n values, the plan's point order) -> flm
 *     (device), f_{l,m} = sum_k w_k f_k Y_{l,m}(x_k)^*.  VSHT_ENOWEIGHTS without
 *     weights.
 *   vsht_sht_adjoint: the adjoint scalar transform (AdjSHT, Section 4.2, eq.
 *     (SLscalar)) flm (device) -> f (device, n values), f_k = S_L(f_{l,m})(x_k).
 * Y_{l,m} is the orthonormal spherical harmonic with the Condon-Shortley phase.
 * VSHT_EUNSUPPORTED on scattered plans.  The workspace is the plan's (calls
 * on one plan are serialised by their stream). */
int64_t vsht_num_sht_coeffs(int L);
vsht_status vsht_sht_forward(vsht_plan_t plan, const void *f, void *flm, void *stream);
vsht_status vsht_sht_adjoint(vsht_plan_t plan, const void *flm, void *f, void *stream);

/* Flags of the *_many calls. */
enum {
    VSHT_UNIT_WEIGHTS = 1, /* forward: unit weights (S^H, as vsht_forward_unweighted) */
    VSHT_TIMES_WEIGHTS = 2 /* adjoint: T_k = w_k (S(a, b))_k, the Hermitian transpose of vsht_forward */
};

/* count fields through one plan, one after another on `stream`.  The fields
 * are contiguous: T holds count blocks of n x 3 complex values, a and b count
 * blocks of L(L+2) each.  vsht_forward_many computes the forward transform of
 * eq. (fwdvsht2) for every block (with VSHT_UNIT_WEIGHTS: with w_k = 1);
 * vsht_adjoint_many the adjoint of eq. (SLvec) (with VSHT_TIMES_WEIGHTS: each
 * output point multiplied by its weight, which makes it the Hermitian
 * transpose of the weighted forward; needs a plan with weights).  These are
 * the backward maps of the differentiable transforms: the gradient of the
 * adjoint is the unit-weight forward and the gradient of the forward the
 * weighted adjoint.  count = 0 does nothing.  VSHT_EINVAL for count < 0 or an
 * unknown flag; other errors as vsht_forward / vsht_adjoint. */
vsht_status vsht_forward_many(vsht_plan_t plan, int64_t count, const void *T, void *a, void *b,
                              int flags, void *stream);
vsht_status vsht_adjoint_many(vsht_plan_t plan, int64_t count, const void *a, const void *b, void *T,
                              int flags, void *stream);

/* Describe a plan (host-side; no device work). */
vsht_status vsht_plan_info(vsht_plan_t plan, vsht_plan_info_t *info);

/* Stages of the pipeline, for vsht_get_stage_times. */
typedef enum {
    VSHT_STAGE_RING_FWD = 0,   /* Cartesian -> (theta, phi), longitude DFT, N/S fold */
    VSHT_STAGE_LEG_FWD = 1,    /* Legendre analysis (contraction over ring pairs) */
    VSHT_STAGE_RECOMBINE = 2,  /* three-term recombination -> a, b */
    VSHT_STAGE_PREP = 3,       /* a, b -> spin-frame scalar coefficients */
    VSHT_STAGE_LEG_ADJ = 4,    /* Legendre synthesis */
    VSHT_STAGE_RING_ADJ = 5,   /* N/S unfold, inverse longitude DFT, -> Cartesian */
    VSHT_STAGE_SCATTERED = 6,  /* adjoint evaluation at scattered points */
    VSHT_NUM_STAGES = 7
} vsht_stage;

/* Profiling aid.  With enable != 0 every later call records a pair of HIP
 * events around each kernel on the caller's stream (a small overhead);
 * vsht_get_stage_times waits for those events and returns, per stage, the
 * summed duration in milliseconds (ms[s]) and the number of launches
 * (count[s]) since the previous read, then clears them.  nstages entries are
 * written (at most VSHT_NUM_STAGES).  Disabling drops pending records. */
vsht_status vsht_set_stage_timing(vsht_plan_t plan, int enable);
vsht_status vsht_get_stage_times(vsht_plan_t plan, double *ms, int64_t *count, int nstages);

/* ---------------------------------------------------------------------------
 * Batches: many independent fields, each with its own bandlimit L[f] and its
 * own iso-latitude ring grid (xyz[f], n[f] points, weights w[f]), one
 * precision for all.  Every stage of the transforms of eq. (SLvec) and eq.
 * (fwdvsht2) runs as one launch covering all fields (work items of the larger
 * fields first), and the launches of a call are captured once into a HIP graph
 * and replayed.  The per-field arrays a, b, T, a2, b2 are host arrays of
 * nfields device pointers (layouts as for single plans).  When a call passes
 * different buffers than the previous one, the library uploads the new
 * addresses and waits for `stream` once; calls with the same buffers only
 * replay the graph.  A batch plan must not run on two streams at the same
 * time.  The single-plan calls return VSHT_EINVAL on a batch plan.
 *
 * vsht_plan_batch   nfields >= 1; every field must be a ring grid with
 *                   weights (else VSHT_EINVAL / VSHT_EUNSUPPORTED, with the
 *                   field named in vsht_last_error).
 * vsht_batch_adjoint    a[f], b[f] -> T[f]   (eq. (SLvec))
 * vsht_batch_forward    T[f] -> a[f], b[f]   (eq. (fwdvsht2))
 * vsht_batch_roundtrip  a[f], b[f] -> T[f], then T[f] -> a2[f], b2[f], one graph.
 * vsht_batch_set_config / get_config   launch shape: adj_nw (1, 2 or 4; kept
 *                   for the call's shape and without effect: the synthesis
 *                   workgroups always hold four waves), fwd_merge (1: one
 *                   analysis launch at the widest workgroup; 0: one per tile
 *                   count), lpt (1: longest work items first), ring_nt (256 or
 *                   512 threads per ring workgroup; rings whose DFT is longer
 *                   than 2048 always take 512), chains (1: with three fields or
 *                   more, the fields are split by cost (L+1)^3 into up to three
 *                   classes, the cheapest up to 1/8 of the total, the next up to
 *                   1/2, the rest, and each class runs its stages as a parallel
 *                   branch of the graph, so that small fields finish early; 0:
 *                   all fields in one sequence of stages).  Chains are switched
 *                   off in this build: chains = 1 returns VSHT_EUNSUPPORTED.
 *                   Results do not depend on the shape.  Waits for the device.
 * vsht_batch_autotune  times every shape on the caller's buffers (roundtrip,
 *                   `reps` replays each), keeps the fastest and writes its time
 *                   per roundtrip in milliseconds to *best_ms (may be NULL).
 *                   Synchronous; overwrites T, a2, b2.
 * vsht_batch_field_times  per field, the device wall-clock time (microseconds,
 *                   from the earliest start in the batch) when its first work
 *                   item of the last call started and its last work item
 *                   ended; arrays of nfields.  Waits for the device.
 * ------------------------------------------------------------------------- */
vsht_status vsht_plan_batch(int nfields, const int *L, const int64_t *n, const double *const *xyz,
                            const double *const *w, const vsht_opts *opts, vsht_plan_t *out);
vsht_status vsht_batch_adjoint(vsht_plan_t plan, const void *const *a, const void *const *b, void *const *T,
                               void *stream);
vsht_status vsht_batch_forward(vsht_plan_t plan, const void *const *T, void *const *a, void *const *b,
                               void *stream);
vsht_status vsht_batch_roundtrip(vsht_plan_t plan, const void *const *a, const void *const *b, void *const *T,
                                 void *const *a2, void *const *b2, void *stream);
vsht_status vsht_batch_set_config(vsht_plan_t plan, int adj_nw, int fwd_merge, int lpt, int ring_nt,
                                  int chains);
vsht_status vsht_batch_get_config(vsht_plan_t plan, int *adj_nw, int *fwd_merge, int *lpt, int *ring_nt,
                                  int *chains);
vsht_status vsht_batch_autotune(vsht_plan_t plan, const void *const *a, const void *const *b, void *const *T,
                                void *const *a2, void *const *b2, int reps, double *best_ms, void *stream);
vsht_status vsht_batch_field_times(vsht_plan_t plan, double *start_us, double *end_us);

/* Release a plan and everything it owns (waits for the device first).
 * Passing NULL is allowed and returns VSHT_OK. */
vsht_status vsht_plan_destroy(vsht_plan_t plan);

/* Static description of a status code. */
const char *vsht_status_string(vsht_status s);

/* Thread-local detail of the last error raised on the calling thread ("" if none). */
const char *vsht_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VSHT_H */
