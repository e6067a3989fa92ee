/*
 * cc_oracle.h -- reference (oracle) implementation of the connected-component
 * Hamiltonian-splitting integrator of Janes, Pelupessy & Portegies Zwart,
 * "A connected component-based method for efficiently integrating multiscale
 * N-body systems" (arXiv:1407.7105).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * used to check the GPU library.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header or
 * constant with the GPU library and must never be used as a fallback for it.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math, no -march=native) so that
 * every floating-point operation is a single IEEE-754 binary64 operation.
 *
 * Every array is host memory owned by the caller.  State is structure-of-arrays
 * in the caller's particle order; "index" below always means that order.
 */
#ifndef CC_ORACLE_H
#define CC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CCO_OK = 0,
    CCO_ERR_ARG = -1,       /* bad argument (sizes, pointers, dt, t_end/dt) */
    CCO_ERR_NONFINITE = -2, /* NaN/Inf in the state, non-positive mass, or r^2+eps^2 == 0 in a kick */
    CCO_ERR_DEPTH = -3,     /* recursion deeper than max_depth */
    CCO_ERR_OOM = -5        /* host allocation failed */
};

typedef struct {
    double *x, *y, *z;      /* positions q_i */
    double *vx, *vy, *vz;   /* velocities v_i = p_i / m_i */
    const double *m;        /* masses m_i > 0 */
} cco_state;

typedef struct {
    double eta;             /* time-step accuracy parameter (Sec. 2.2, eq. 19) */
    double eps2;            /* Plummer softening squared (eq. 3) */
    double G;               /* gravitational constant (1 in N-body units) */
    int max_depth;          /* recursion cap; deeper calls fail with CCO_ERR_DEPTH */
    int kepler;             /* 1: CC_KEPLER (Sec. 2.2, Sec. 3.2): a component of two particles is
                               advanced by the Kepler solution instead of being recursed into;
                               needs eps2 == 0 */
    int hold;               /* 1: the HOLD split of Sec. 2.1 (eqs. 11-17) instead of the CC split:
                               the fast set F = {i : tau(i) < h}, tau(i) = min_j tau(i,j), is
                               recursed into as one set; pairs with a slow member are kicked
                               (not with kepler) */
} cco_params;

typedef struct {
    uint64_t tau_evals;     /* evaluations of the pair time-step formula */
    uint64_t kick_pairs;    /* unordered pairs kicked (each pair once) */
    uint64_t drifts;        /* single-particle drift operations */
    uint64_t components;    /* non-trivial components produced by all splits */
    uint64_t splits;        /* calls of the split */
    int64_t max_depth_seen; /* deepest recursion level reached (top = 0) */
    double t_reached;       /* integration time completed without error */
    uint64_t kepler_solves; /* two-body components advanced by the Kepler solution (CC_KEPLER) */
} cco_stats;

/* Interaction time step tau(i,j) (eq. 19): the smaller of the symmetrised
 * free-fall and fly-by steps eta*t / (1 - eta*t'/2); see cco_tau_parts. */
double cco_tau(const cco_params *p, const cco_state *s, int64_t i, int64_t j);

/* The four ingredients of eq. 19 for one pair: out[0]=t_ff, out[1]=d t_ff/dt,
 * out[2]=t_fb (+INF when the relative velocity is zero), out[3]=d t_fb/dt
 * (0 when the relative velocity is zero), out[4]=tau. */
void cco_tau_parts(const cco_params *p, const cco_state *s, int64_t i, int64_t j, double out[5]);

/* tau for a list of pairs (pi[k], pj[k]). */
int cco_pair_timesteps(const cco_params *p, const cco_state *s, int64_t n,
                       const int32_t *pi, const int32_t *pj, int64_t npairs, double *tau_out);

/* Connected components of the time-step graph {tau(i,j) < h} (eq. 20) over the
 * index set I[0..nI) (ascending), by breadth-first search (Sec. 2.3).
 * label_out[k] = smallest index in the component of I[k]. */
int cco_split_bfs(const cco_params *p, const cco_state *s, const int64_t *I, int64_t nI,
                  double h, int64_t *label_out, uint64_t *tau_evals);

/* Same partition, computed independently with a union-find over all pairs. */
int cco_split_uf(const cco_params *p, const cco_state *s, const int64_t *I, int64_t nI,
                 double h, int64_t *label_out);

/* Partition of all n particles (I = 0..n-1) by BFS; returns the number of
 * non-trivial components in *n_nontrivial. */
int cco_split_labels(const cco_params *p, const cco_state *s, int64_t n, double h,
                     int32_t *label_out, int64_t *n_nontrivial, uint64_t *tau_evals);

/* Kick operator (eqs. 8-9) for every pair k<l of I with label[k] != label[l]
 * (label == NULL: every pair).  Velocities change by h * acceleration. */
int cco_kick(const cco_params *p, cco_state *s, const int64_t *I, int64_t nI,
             const int64_t *label, double h, uint64_t *kick_pairs);

/* Drift operator (eq. 6): x_i += h v_i for every i in I with mask[i] != 0
 * (mask indexed by particle index; NULL: every i). */
int cco_drift(cco_state *s, const int64_t *I, int64_t nI, const uint8_t *mask, double h);

/* Whole integrator: t_end/dt global steps of evolve_cc(all particles, dt)
 * (Fig. 2).  On error the state is restored to the last completed global step
 * and st->t_reached says how far it got. */
int cco_evolve(const cco_params *p, cco_state *s, int64_t n, double dt, double t_end, cco_stats *st);

/* Independent clusters: particles [off[c], off[c+1]) form cluster c, evolved
 * on its own.  st is an array of ncl stats records. */
int cco_evolve_batch(const cco_params *p, cco_state *s, const int64_t *off, int32_t ncl,
                     double dt, double t_end, cco_stats *st);

/* Acceleration of particle i from all j != i, summed in ascending j:
 * a_i = sum_j G m_j (q_j - q_i) / (|q_j - q_i|^2 + eps^2)^(3/2). */
int cco_accel(const cco_params *p, const cco_state *s, int64_t n,
              const int64_t *idx, int64_t nidx, double *ax, double *ay, double *az);

/* Same with Neumaier-compensated sums (reference for tolerance checks). */
int cco_accel_compensated(const cco_params *p, const cco_state *s, int64_t n,
                          const int64_t *idx, int64_t nidx, double *ax, double *ay, double *az);

/* Two-body (Kepler) flow of eq. 10 with eps = 0 for time dt: the relative
 * motion r = q_j - q_i, v = v_j - v_i under mu = G (m_i + m_j), by the
 * universal-variable formulation (Bate, Mueller & White 1971), and the centre
 * of mass moving uniformly.  rv[6] = (r, v) is advanced in place.  Returns
 * CCO_ERR_ARG for mu <= 0 or a non-finite dt, CCO_ERR_NONFINITE for r = 0. */
int cco_kepler(double mu, double rv[6], double dt);

/* Conserved quantities with compensated sums (eqs. 1-3):
 * out[0]=kinetic, out[1]=potential, out[2..4]=linear momentum,
 * out[5..7]=angular momentum, out[8..10]=centre of mass, out[11]=total mass. */
int cco_diagnostics(const cco_params *p, const cco_state *s, int64_t n, double out[12]);

#ifdef __cplusplus
}
#endif
#endif
