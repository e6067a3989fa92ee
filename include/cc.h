/*
 * cc.h -- C ABI of the MI355X (gfx950) connected-component (CC) N-body
 * integrator library, after Janes, Pelupessy & Portegies Zwart,
 * "A connected component-based method for efficiently integrating multiscale
 * N-body systems" (arXiv:1407.7105).
 *
 * Conventions for every entry point:
 *   - State is structure-of-arrays FP64 in DEVICE memory owned by the caller:
 *     positions x,y,z, velocities vx,vy,vz and masses m (m > 0), n particles,
 *     indexed 0..n-1 (the "particle index").  The library never frees or keeps
 *     caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work on it; calls documented as "syncs" wait for their own work before
 *     returning.  Calls never synchronise the device as a whole.
 *   - Return value: CC_OK (0) or a negative cc_status.  The message of the last
 *     failing call on a context is cc_last_error(ctx).  Arguments are checked on
 *     the host before any launch; a rejected call leaves the state untouched.
 *   - A context belongs to one device and one host thread at a time; calls on
 *     one context must not overlap.  Different contexts are independent.
 *   - Floating-point: every FP64 operation of the plain path is a single
 *     correctly rounded IEEE-754 operation in the order the paper's formulas
 *     are written (no contraction), so partitions, kicks and whole steps are
 *     reproducible run to run and match an FP64 reference that uses the same
 *     order bit for bit.
 */
#ifndef CC_MI355X_H
#define CC_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CC_OK = 0,
    CC_ERR_ARG = -1,        /* bad size, pointer, parameter, dt, t_end/dt not a positive integer, mass <= 0 */
    CC_ERR_NONFINITE = -2,  /* NaN/Inf in the state, or r^2 + eps^2 == 0 in a kick */
    CC_ERR_DEPTH = -3,      /* recursion deeper than params.max_depth */
    CC_ERR_DEVICE = -4,     /* HIP runtime error; see cc_last_error */
    CC_ERR_OOM = -5         /* device or pinned-host allocation failed */
} cc_status;

typedef enum {
    CC_FP64 = 0,            /* plain path: every sweep in FP64 */
    CC_MIXED = 1            /* FP32 pair forces on FP64 coordinate differences, Kahan-
                               compensated per tile and summed in FP64 across tiles, and
                               the FP32 screen in front of the FP64 one; FP64 state,
                               drift and every connectivity decision */
} cc_precision;

typedef enum {
    CC_ORDER_FAST = 0,      /* kick sums split over parallel tiles and combined in a
                               fixed order: deterministic run to run, equal to the
                               sequential sum up to rounding */
    CC_ORDER_EXACT = 1      /* every particle sums its partners sequentially in
                               ascending particle index: bit-identical to a plain
                               sequential FP64 evaluation of the same formulas */
} cc_kick_order;

typedef enum {
    CC_SCREEN_FP64 = 0,     /* edge test screened by a division-free FP64 form with a
                               certified error bound (the default) */
    CC_SCREEN_FP32 = 1      /* FP32 screen on FP32-rounded differences first, then the
                               FP64 screen; on gfx950 without packed FP32 this is slower */
} cc_screen;

typedef struct cc_ctx cc_ctx;

typedef struct {
    double *x, *y, *z;      /* positions q_i (device) */
    double *vx, *vy, *vz;   /* velocities v_i = p_i / m_i (device) */
    const double *m;        /* masses m_i > 0 (device, read-only) */
} cc_state;

typedef struct {
    double eta;             /* time-step accuracy parameter of eq. 19 (> 0, <= 1) */
    double eps2;            /* Plummer softening squared of eq. 3 (>= 0) */
    double G;               /* gravitational constant (> 0; 1 in N-body units) */
    int32_t max_depth;      /* recursion cap (levels below the global step), >= 0 */
    int32_t precision;      /* cc_precision */
    int32_t small_max;      /* largest component integrated on chip (3..1024;
                               0 = library default, 128) */
    int32_t kick_order;     /* cc_kick_order */
    int32_t screen;         /* cc_screen for the grid-wide sweep; either
                               screen leaves undecided pairs to the literal FP64 formula,
                               so partitions do not depend on it */
    int32_t kepler;         /* 0: plain CC; 1: CC_KEPLER (Sec. 2.2, last paragraph; Sec. 3.2):
                               a component of two particles is advanced over its half step
                               by the two-body Kepler solution of eq. 10 (universal
                               variables) instead of being recursed into; needs eps2 == 0 */
    int32_t hold;           /* 0: the CC split; 1: the HOLD split of Sec. 2.1 (eqs. 11-17): a
                               particle is fast when its time step tau(i) = min_j tau(i,j) is
                               below h, i.e. when it belongs to a non-trivial component; the
                               fast particles of a set are recursed into as ONE set F and every
                               pair with a slow member is kicked.  Not with kepler. */
    int32_t plain;          /* 0: batched (default): two-body components, small components and
                               all-small ensembles run in persistent on-chip launches beside the
                               grid-wide recursion; 1: plain path, every set of two or more bodies
                               is split and kicked by the grid-wide kernels, one level visit at a
                               time (the reference for the batching comparison; small_max is
                               ignored; not with kepler) */
} cc_params;

typedef struct {
    uint64_t tau_pairs;     /* pair time steps evaluated (all launches) */
    uint64_t tau_pairs_alg; /* pair time steps the split needs: n-1 per fully
                               connected set, n(n-1)/2 otherwise (Sec. 2.3); the HOLD
                               split always needs n(n-1)/2 */
    uint64_t kick_pairs;    /* unordered pairs kicked (label_i != label_j) */
    uint64_t drifts;        /* single-particle half-step drifts */
    uint64_t components;    /* non-trivial components produced by all splits */
    uint64_t splits;        /* calls of the split (evolve_cc invocations) */
    int64_t max_depth_seen; /* deepest recursion level (global step = 0) */
    double t_reached;       /* integration time completed without error */
    uint64_t kepler_solves; /* two-body components advanced by the Kepler solution */
} cc_stats;

/* Create a context on HIP device `hip_device` with parameters *p (copied).
 * Scratch memory is allocated on demand and kept for reuse. */
int cc_create(cc_ctx **out, int32_t hip_device, const cc_params *p);

/* Release a context and all its device memory.  NULL is a no-op. */
void cc_destroy(cc_ctx *ctx);

/* Replace the parameters of a context (same validation as cc_create). */
int cc_set_params(cc_ctx *ctx, const cc_params *p);

/* Message for the last failing call on ctx ("" if none).  Owned by ctx. */
const char *cc_last_error(const cc_ctx *ctx);

/* Pair time step tau(i,j) of eq. 19 (Sec. 2.2):
 *   tau = min( eta t_ff / (1 - eta t_ff'/2), eta t_fb / (1 - eta t_fb'/2) )
 * with r^2 = |q_i - q_j|^2 + eps^2, mu = G (m_i + m_j), t_ff = sqrt(r^3/mu),
 * t_ff' = (3/2) t_ff (q.u)/r^2, t_fb = r/|u|, t_fb' = (q.u)/(r|u|)(1 + mu/(r|u|^2)),
 * u = v_i - v_j; a term with a non-positive denominator (or |u| = 0 for the
 * fly-by term) gives +INF; r^2 == 0 gives 0.
 * pi, pj: device int32[npairs] in [0,n); tau_out: device double[npairs].
 * npairs == 0 is a no-op.  Asynchronous. */
int cc_pair_timesteps(cc_ctx *ctx, const cc_state *s, int64_t n,
                      const int32_t *pi, const int32_t *pj, int64_t npairs,
                      double *tau_out, void *stream);

/* Connected components of the time-step graph with an edge (i,j) iff
 * tau(i,j) < h (eq. 20, Sec. 2.2-2.3).  label_out (device int32[n]) receives
 * for each particle the smallest particle index of its component; a particle
 * is a trivial component iff no other particle shares its label.  If
 * n_nontrivial_out is not NULL it receives the number of components with at
 * least two particles (host int64).  The call syncs on `stream` (it reads
 * back the error flag).  h must be > 0 and finite. */
int cc_split_labels(cc_ctx *ctx, const cc_state *s, int64_t n, double h,
                    int32_t *label_out, int64_t *n_nontrivial_out, void *stream);

/* Kick operator K_h (eqs. 8-9) for every unordered pair i<j with
 * label[i] != label[j] (label: device int32[n], or NULL for every pair):
 *   v_i += h * sum_j G m_j (q_j - q_i) / (|q_j - q_i|^2 + eps^2)^(3/2),
 * each particle's sum taken over j in ascending index order.  With
 * params.precision == CC_MIXED the pair forces are FP32 on FP64 coordinate
 * differences, Kahan-compensated over each 256-partner tile and summed in
 * FP64 across tiles.  Fails with CC_ERR_NONFINITE (state untouched) if a
 * kicked pair has r^2 + eps^2 == 0; the call syncs (it reads back the error
 * flag before it applies the kick). */
int cc_kick(cc_ctx *ctx, cc_state *s, int64_t n, const int32_t *label, double h, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cc_kick
 * with its scratch (the three acceleration sums and the error flag) in a
 * static device array of the library (1.5 MiB per device, held until the
 * process ends), so the call allocates nothing on the device or the host.
 * Same arguments, results and errors as cc_kick (bit-identical output), for
 * 1 <= n <= CC_KICK_STATIC_MAX_N; a larger n fails with CC_ERR_ARG before
 * any launch.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (several host threads, or several streams in flight)
 * race and must not be issued.  Syncs on `stream` (it reads back the error
 * flag before it applies the kick). */
#define CC_KICK_STATIC_MAX_N 65536
int cc_kick_static(cc_ctx *ctx, cc_state *s, int64_t n, const int32_t *label, double h, void *stream);

/* Drift operator D_h (eq. 6): q_i += h v_i for every i with mask[i] != 0
 * (mask: device uint8[n], or NULL for every particle).  Asynchronous. */
int cc_drift(cc_ctx *ctx, cc_state *s, int64_t n, const uint8_t *mask, double h, void *stream);

/* The CC integrator (eqs. 26-31, Fig. 2): t_end/dt global steps of
 *   evolve_cc(H, h): split at h; evolve_cc(C_k, h/2) for every non-trivial
 *   component; drift R by h/2; kick every pair in different components by h;
 *   drift R by h/2; evolve_cc(C_k, h/2) again with the same partition,
 * starting with h = dt on all n particles (with params.hold the components of
 * a set are merged into one set F before the recursion, Sec. 2.1).
 * dt > 0, t_end/dt a positive
 * integer (t_end is the duration).  Updates x..vz in place; syncs.
 * On error the state is restored to the start of the failing global step and
 * out->t_reached tells how far the integration got.  out may be NULL. */
int cc_evolve(cc_ctx *ctx, cc_state *s, int64_t n, double dt, double t_end,
              cc_stats *out, void *stream);

/* Independent clusters: particles [offsets[c], offsets[c+1]) form cluster c
 * (offsets: host int64[ncl+1], strictly increasing, offsets[0] = 0), each
 * integrated as by cc_evolve with no forces between clusters.
 * out_per_cluster: host array of ncl records (may be NULL).  Syncs.  On error
 * every cluster is restored to the start of the failing global step. */
int cc_evolve_batch(cc_ctx *ctx, cc_state *s, const int64_t *offsets, int32_t ncl,
                    double dt, double t_end, cc_stats *out_per_cluster, void *stream);

/* Integrals of motion (eqs. 1-3) with compensated FP64 sums, written to the
 * host array out[12]: kinetic, potential, P[3], L[3], centre of mass[3], total
 * mass.  Syncs. */
int cc_diagnostics(cc_ctx *ctx, const cc_state *s, int64_t n, double *out, void *stream);

/* Autotuner for the launch shapes of the batched recursion.  Times one global
 * step of the given state (device SoA as for cc_evolve; only read: every trial
 * runs on a copy) while it varies, one at a time from the best so far, the
 * largest component run on chip (small_max in {64, 128, 256, 512}), the sweep
 * launches that give each tile a whole workgroup (up to {0, 512, 2048, 8192}
 * tiles) and the kick blocks per compute unit ({8, 16, 32, 64}); keeps the
 * fastest in the context (params.small_max is overwritten) and reports it in
 * *out (may be NULL).  Partitions and results in the EXACT kick order do not
 * depend on the choice.  Allocates a copy of the state; syncs. */
typedef struct {
    int32_t small_max;          /* chosen on-chip size limit */
    int32_t sweep_split_tiles;  /* chosen: sweep launches up to this many tiles use one workgroup per tile */
    int32_t kick_groups_per_cu; /* chosen: kick launches aim at this many blocks per compute unit */
    double ms_per_step;         /* best time of one global step with the choice */
    int32_t trials;             /* configurations timed */
} cc_tune;
int cc_autotune(cc_ctx *ctx, const cc_state *s, int64_t n, double dt, cc_tune *out, void *stream);

/* Per-kernel timing for roofline reporting.  While enabled, every launch made
 * by cc_evolve / cc_evolve_batch is bracketed by HIP events on its stream and
 * the pair time steps and kicked pairs it processed are counted per kernel
 * family. */
typedef struct {
    char name[32];          /* kernel family */
    uint64_t launches;
    double ms;              /* summed event time of the family's launches */
    uint64_t tau_pairs;     /* pair time steps evaluated by the family */
    uint64_t kick_pairs;    /* unordered pairs kicked by the family */
} cc_kernel_time;

/* Enable (1) or disable (0) timing; enabling clears the record.  Syncs. */
int cc_timing_enable(cc_ctx *ctx, int32_t enable);
/* Copies up to max records (host array) and returns how many families exist.
 * Syncs. */
int cc_timing_report(cc_ctx *ctx, cc_kernel_time *out, int32_t max);

#ifdef __cplusplus
}
#endif
#endif
