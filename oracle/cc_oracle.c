/*
 * cc_oracle.c -- reference (oracle) implementation of the connected-component
 * (CC) Hamiltonian-splitting integrator, arXiv:1407.7105.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow FP64 CPU code that the GPU library
 * is checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares nothing with the GPU library.
 *
 * Every function states the passage of the paper it follows.  Where the paper
 * is silent the reading taken is stated at the point of use:
 *   - the free-fall and fly-by times of eq. 19 are only referenced (to an
 *     earlier paper); they are taken as t_ff = sqrt(r^3 / (G (m_i+m_j))) and
 *     t_fb = r / |v|, with their exact time derivatives along the relative
 *     two-body motion;
 *   - the symmetrisation acts on the scaled step eta*t, i.e. each term is
 *     eta t / (1 - (1/2) eta dt/dt): that is the first-order solution of
 *     h = (tau(t) + tau(t+h)) / 2, the time symmetry the paper claims for the
 *     criterion (abstract, Sec. 1); with eta applied only after the
 *     symmetrisation an eccentric Kepler orbit drifts secularly in energy;
 *   - a symmetrised term whose denominator 1 - (1/2) dt/dt is not positive
 *     gives no bound (+INF); with zero relative velocity the fly-by term gives
 *     no bound; a pair at zero separation (r^2 + eps^2 == 0) has tau = 0;
 *   - the edge test is strict, tau(i,j) < h (eq. 20);
 *   - the three kick terms of eq. 31 commute, so they are applied as the
 *     single operator K_{h, V_R + V_CC + V_CR} of eq. 30: one sweep over the
 *     pairs in different components, ascending i then ascending j, velocities
 *     updated after the sweep;
 *   - components are labelled by their smallest particle index and recursed
 *     into in ascending label order; members keep ascending index order;
 *   - recursion deeper than max_depth is an error (the paper's recursion has
 *     no bound when two unsoftened particles meet).
 *
 * Build with -O2 -ffp-contract=off and without fast-math: every operation in
 * this file is then one correctly rounded IEEE-754 binary64 operation.
 */
#include "cc_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Pair time step, eq. 19.                                                   */
/* ------------------------------------------------------------------------ */

/*
 * tau(i,j) = min( eta t_ff / (1 - eta t_ff'/2), eta t_fb / (1 - eta t_fb'/2) )
 * (eq. 19, with the free-fall and fly-by steps eta*t symmetrised)
 *
 * With q = q_i - q_j, u = v_i - v_j, r^2 = |q|^2 + eps^2, mu = G (m_i + m_j):
 *   t_ff  = sqrt(r^3 / mu)                         free-fall time
 *   t_ff' = (3/2) t_ff (q.u) / r^2                 since dr/dt = (q.u)/r
 *   t_fb  = r / |u|                                fly-by time
 *   t_fb' = (q.u)/(r |u|) * (1 + mu / (r |u|^2))   using du/dt = -mu q / r^3
 * For a step s(t) = eta t(t), the symmetrised form s / (1 - s'/2) is the
 * first-order solution of h = (s(t) + s(t+h)) / 2, which makes the criterion
 * approximately time-symmetric.  Operations are evaluated strictly left to
 * right.
 */
static void tau_parts(const cco_params *p, const cco_state *s, int64_t i, int64_t j,
                      double out[5])
{
    const double dx = s->x[i] - s->x[j];
    const double dy = s->y[i] - s->y[j];
    const double dz = s->z[i] - s->z[j];
    const double dvx = s->vx[i] - s->vx[j];
    const double dvy = s->vy[i] - s->vy[j];
    const double dvz = s->vz[i] - s->vz[j];

    const double r2 = ((dx * dx + dy * dy) + dz * dz) + p->eps2;
    const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
    const double rv = (dx * dvx + dy * dvy) + dz * dvz;
    const double mu = p->G * (s->m[i] + s->m[j]);

    if (r2 == 0.0) {
        /* coincident unsoftened pair: no finite step resolves it */
        out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = 0.0; out[4] = 0.0;
        return;
    }
    const double r = sqrt(r2);

    const double eta = p->eta;
    const double tff = sqrt((r2 * r) / mu);
    const double dtff = ((1.5 * tff) * rv) / r2;
    const double dff = 1.0 - (0.5 * eta) * dtff;
    const double sff = (dff > 0.0) ? (eta * tff) / dff : INFINITY;

    double tfb = INFINITY, dtfb = 0.0, sfb = INFINITY;
    if (v2 > 0.0) {
        const double v = sqrt(v2);
        tfb = r / v;
        dtfb = (rv / (r * v)) * (1.0 + mu / (r * v2));
        const double dfb = 1.0 - (0.5 * eta) * dtfb;
        sfb = (dfb > 0.0) ? (eta * tfb) / dfb : INFINITY;
    }
    out[0] = tff;
    out[1] = dtff;
    out[2] = tfb;
    out[3] = dtfb;
    out[4] = (sfb < sff) ? sfb : sff;
}

double cco_tau(const cco_params *p, const cco_state *s, int64_t i, int64_t j)
{
    double o[5];
    tau_parts(p, s, i, j, o);
    return o[4];
}

void cco_tau_parts(const cco_params *p, const cco_state *s, int64_t i, int64_t j, double out[5])
{
    tau_parts(p, s, i, j, out);
}

int cco_pair_timesteps(const cco_params *p, const cco_state *s, int64_t n,
                       const int32_t *pi, const int32_t *pj, int64_t npairs, double *tau_out)
{
    if (!p || !s || n < 1 || npairs < 0 || (npairs > 0 && (!pi || !pj || !tau_out)))
        return CCO_ERR_ARG;
    for (int64_t k = 0; k < npairs; k++) {
        if (pi[k] < 0 || pi[k] >= n || pj[k] < 0 || pj[k] >= n) return CCO_ERR_ARG;
    }
    for (int64_t k = 0; k < npairs; k++) tau_out[k] = cco_tau(p, s, pi[k], pj[k]);
    return CCO_OK;
}

/* ------------------------------------------------------------------------ */
/* Connected components of the time-step graph (eq. 20, Sec. 2.3).          */
/* ------------------------------------------------------------------------ */

/*
 * Breadth-first search as described in Sec. 2.3: take a particle X whose
 * component is known and give that component to every still unassigned
 * particle U with tau(X,U) < h; repeat from each newly assigned particle.  Only
 * unassigned particles are tested, so a set whose pairs all lie below h is
 * split with n-1 evaluations.  A new component starts at the smallest
 * unassigned position, so root[k] is the smallest position in k's component.
 */
static int split_bfs_pos(const cco_params *p, const cco_state *s, const int64_t *I, int64_t n,
                         double h, int64_t *root, uint64_t *tau_evals)
{
    int64_t *unas = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!unas || !queue) { free(unas); free(queue); return CCO_ERR_OOM; }
    uint64_t evals = 0;
    int64_t nun = n;
    for (int64_t k = 0; k < n; k++) unas[k] = k;

    while (nun > 0) {
        const int64_t r = unas[0];
        memmove(unas, unas + 1, sizeof(int64_t) * (size_t)(nun - 1));
        nun--;
        root[r] = r;
        int64_t head = 0, tail = 0;
        queue[tail++] = r;
        while (head < tail && nun > 0) {
            const int64_t X = queue[head++];
            int64_t keep = 0;
            for (int64_t u = 0; u < nun; u++) {
                const int64_t U = unas[u];
                evals++;
                if (cco_tau(p, s, I[X], I[U]) < h) {
                    root[U] = r;
                    queue[tail++] = U;
                } else {
                    unas[keep++] = U;
                }
            }
            nun = keep;
        }
    }
    free(unas);
    free(queue);
    if (tau_evals) *tau_evals += evals;
    return CCO_OK;
}

int cco_split_bfs(const cco_params *p, const cco_state *s, const int64_t *I, int64_t nI,
                  double h, int64_t *label_out, uint64_t *tau_evals)
{
    if (!p || !s || !I || nI < 1 || !label_out) return CCO_ERR_ARG;
    int64_t *root = (int64_t *)malloc(sizeof(int64_t) * (size_t)nI);
    if (!root) return CCO_ERR_OOM;
    int rc = split_bfs_pos(p, s, I, nI, h, root, tau_evals);
    if (rc == CCO_OK)
        for (int64_t k = 0; k < nI; k++) label_out[k] = I[root[k]];
    free(root);
    return rc;
}

static int64_t uf_find(int64_t *parent, int64_t a)
{
    while (parent[a] != a) a = parent[a];
    return a;
}

/* Union-find over every pair with tau < h; the smaller root always becomes the
 * parent, so each tree's root is its smallest position. */
int cco_split_uf(const cco_params *p, const cco_state *s, const int64_t *I, int64_t nI,
                 double h, int64_t *label_out)
{
    if (!p || !s || !I || nI < 1 || !label_out) return CCO_ERR_ARG;
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)nI);
    if (!parent) return CCO_ERR_OOM;
    for (int64_t k = 0; k < nI; k++) parent[k] = k;
    for (int64_t a = 0; a < nI; a++) {
        for (int64_t b = a + 1; b < nI; b++) {
            if (cco_tau(p, s, I[a], I[b]) < h) {
                int64_t ra = uf_find(parent, a), rb = uf_find(parent, b);
                if (ra < rb) parent[rb] = ra;
                else if (rb < ra) parent[ra] = rb;
            }
        }
    }
    for (int64_t k = 0; k < nI; k++) label_out[k] = I[uf_find(parent, k)];
    free(parent);
    return CCO_OK;
}

int cco_split_labels(const cco_params *p, const cco_state *s, int64_t n, double h,
                     int32_t *label_out, int64_t *n_nontrivial, uint64_t *tau_evals)
{
    if (!p || !s || n < 1 || !label_out) return CCO_ERR_ARG;
    int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *lab = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!I || !lab || !cnt) { free(I); free(lab); free(cnt); return CCO_ERR_OOM; }
    for (int64_t k = 0; k < n; k++) I[k] = k;
    int rc = cco_split_bfs(p, s, I, n, h, lab, tau_evals);
    if (rc == CCO_OK) {
        int64_t nt = 0;
        for (int64_t k = 0; k < n; k++) { label_out[k] = (int32_t)lab[k]; cnt[lab[k]]++; }
        for (int64_t k = 0; k < n; k++) if (cnt[k] >= 2) nt++;
        if (n_nontrivial) *n_nontrivial = nt;
    }
    free(I); free(lab); free(cnt);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Kick and drift operators (eqs. 6, 8, 9).                                  */
/* ------------------------------------------------------------------------ */

/*
 * K_h for the potential terms V_kl of all pairs k<l of I whose labels differ:
 * each pair changes both velocities, by equal and opposite momenta (eqs. 8-9),
 * F_kl = G m_k m_l (q_l - q_k) / (|q_l - q_k|^2 + eps^2)^(3/2).  The
 * accelerations are summed first and the velocities updated once.
 */
int cco_kick(const cco_params *p, cco_state *s, const int64_t *I, int64_t nI,
             const int64_t *label, double h, uint64_t *kick_pairs)
{
    if (!p || !s || !I || nI < 1) return CCO_ERR_ARG;
    double *ax = (double *)calloc((size_t)nI, sizeof(double));
    double *ay = (double *)calloc((size_t)nI, sizeof(double));
    double *az = (double *)calloc((size_t)nI, sizeof(double));
    if (!ax || !ay || !az) { free(ax); free(ay); free(az); return CCO_ERR_OOM; }
    uint64_t pairs = 0;
    int rc = CCO_OK;
    for (int64_t a = 0; a < nI && rc == CCO_OK; a++) {
        const int64_t i = I[a];
        for (int64_t b = a + 1; b < nI; b++) {
            if (label && label[a] == label[b]) continue;
            const int64_t j = I[b];
            const double dx = s->x[j] - s->x[i];
            const double dy = s->y[j] - s->y[i];
            const double dz = s->z[j] - s->z[i];
            const double r2 = ((dx * dx + dy * dy) + dz * dz) + p->eps2;
            if (r2 == 0.0) { rc = CCO_ERR_NONFINITE; break; }
            const double f = p->G / (r2 * sqrt(r2));
            const double mjf = s->m[j] * f;
            const double mif = s->m[i] * f;
            ax[a] += mjf * dx; ay[a] += mjf * dy; az[a] += mjf * dz;
            ax[b] -= mif * dx; ay[b] -= mif * dy; az[b] -= mif * dz;
            pairs++;
        }
    }
    if (rc == CCO_OK) {
        for (int64_t a = 0; a < nI; a++) {
            const int64_t i = I[a];
            s->vx[i] += h * ax[a];
            s->vy[i] += h * ay[a];
            s->vz[i] += h * az[a];
        }
        if (kick_pairs) *kick_pairs += pairs;
    }
    free(ax); free(ay); free(az);
    return rc;
}

/* D_{h,T_i}: q_i(t+h) = q_i(t) + h v_i(t)   (eq. 6). */
int cco_drift(cco_state *s, const int64_t *I, int64_t nI, const uint8_t *mask, double h)
{
    if (!s || !I || nI < 0) return CCO_ERR_ARG;
    for (int64_t a = 0; a < nI; a++) {
        const int64_t i = I[a];
        if (mask && !mask[i]) continue;
        s->x[i] += h * s->vx[i];
        s->y[i] += h * s->vy[i];
        s->z[i] += h * s->vz[i];
    }
    return CCO_OK;
}

/* ------------------------------------------------------------------------ */
/* Two-body flow (eq. 10), universal variables (Bate, Mueller & White 1971).  */
/* ------------------------------------------------------------------------ */

/*
 * Stumpff functions c2(z) = (1 - cos sqrt z)/z and c3(z) = (sqrt z - sin sqrt z)/z^(3/2)
 * (continued through z <= 0 with cosh/sinh).  |z| < 1: their power series
 * c2 = sum (-z)^k/(2k+2)!, c3 = sum (-z)^k/(2k+3)!, with no cancellation;
 * otherwise c2 in the form 2 sin^2(sqrt(z)/2)/z, which has none either.
 */
static const double TWO_PI = 6.283185307179586476925286766559005768;

static void stumpff(double z, double *c2, double *c3)
{
    if (fabs(z) < 1.0) {
        double t2 = 0.5, t3 = 1.0 / 6.0, s2 = 0.0, s3 = 0.0;
        for (int k = 0; k < 20; k++) {
            s2 += t2;
            s3 += t3;
            t2 *= -z / ((2.0 * k + 3.0) * (2.0 * k + 4.0));
            t3 *= -z / ((2.0 * k + 4.0) * (2.0 * k + 5.0));
        }
        *c2 = s2;
        *c3 = s3;
    } else if (z > 0.0) {
        const double w = sqrt(z);
        const double sh = sin(0.5 * w);
        *c2 = 2.0 * sh * sh / z;
        *c3 = (w - sin(w)) / (z * w);
    } else {
        const double w = sqrt(-z);
        const double sh = sinh(0.5 * w);
        *c2 = 2.0 * sh * sh / (-z);
        *c3 = (sinh(w) - w) / (-z * w);
    }
}

/*
 * Kepler's equation in the universal variable x for the relative orbit with
 * |r0| = r0n, sigma0 = r0.v0 / sqrt(mu), alpha = 2/r0n - |v0|^2/mu:
 *   sqrt(mu) t(x) = sigma0 x^2 c2(alpha x^2) + (1 - alpha r0n) x^3 c3(alpha x^2) + r0n x,
 * whose derivative is the radius, r(x) = sigma0 x (1 - alpha x^2 c3)
 * + (1 - alpha r0n) x^2 c2 + r0n > 0: t(x) increases, so x is found by
 * Newton's method kept inside a bracket (a bisection step whenever Newton
 * would leave it).  A bound orbit is first reduced by whole periods.  Then
 * the Lagrange coefficients f, g, f', g' give r = f r0 + g v0 and
 * v = f' r0 + g' v0.
 */
int cco_kepler(double mu, double rv[6], double dt)
{
    if (!(mu > 0.0) || !isfinite(mu) || !isfinite(dt)) return CCO_ERR_ARG;
    const double r0[3] = {rv[0], rv[1], rv[2]}, v0[3] = {rv[3], rv[4], rv[5]};
    const double r0n = sqrt((r0[0] * r0[0] + r0[1] * r0[1]) + r0[2] * r0[2]);
    if (!(r0n > 0.0)) return CCO_ERR_NONFINITE;
    if (dt == 0.0) return CCO_OK;
    const double v0sq = (v0[0] * v0[0] + v0[1] * v0[1]) + v0[2] * v0[2];
    const double rdv = (r0[0] * v0[0] + r0[1] * v0[1]) + r0[2] * v0[2];
    const double smu = sqrt(mu);
    const double sigma0 = rdv / smu;
    const double alpha = 2.0 / r0n - v0sq / mu;
    double t = dt;
    if (alpha > 0.0) {
        /* bound: the flow has period 2 pi / sqrt(mu alpha^3) */
        const double period = TWO_PI / sqrt(mu * alpha * alpha * alpha);
        t = fmod(dt, period);
        if (t < 0.0) t += period;   /* into [0, period): the flow backwards is the flow forwards */
    }
    const double target = smu * t;
    const double one_ar = 1.0 - alpha * r0n;
    double c2 = 0.5, c3 = 1.0 / 6.0;
    /* sqrt(mu) t(x); a non-finite value (overflow far beyond the root) counts
     * as +-infinity, t(x) being increasing */
#define TFUN(X, OUT)                                                                   \
    do {                                                                               \
        double c2_, c3_;                                                               \
        stumpff(alpha * (X) * (X), &c2_, &c3_);                                        \
        (OUT) = (sigma0 * (X) * (X) * c2_ + one_ar * (X) * (X) * (X) * c3_) + r0n * (X); \
        if (!isfinite(OUT)) (OUT) = (X) > 0.0 ? INFINITY : -INFINITY;                  \
    } while (0)
    /* bracket [lo, hi] around the root: a bound orbit's reduced time lies
     * within one period, x in [0, 2 pi / sqrt(alpha)]; otherwise start from the
     * hyperbolic estimate of x and double, but never past |x| sqrt(-alpha) = 700
     * (where the hyperbolic functions would overflow; the root lies far below) */
    double lo = 0.0, hi = 0.0, x;
    if (alpha > 0.0) {
        hi = TWO_PI / sqrt(alpha);
        x = smu * alpha * t;
    } else {
        double g = 0.0;
        if (alpha < 0.0) {
            const double a = 1.0 / alpha;
            const double sg = t >= 0.0 ? 1.0 : -1.0;
            const double arg = (-2.0 * mu * alpha * t) / (rdv + sg * sqrt(-mu * a) * (1.0 - r0n * alpha));
            if (arg > 0.0 && isfinite(arg)) g = sg * sqrt(-a) * log(arg);
        }
        if (!(g * t > 0.0)) g = target / r0n;
        const double cap = alpha < 0.0 ? 700.0 / sqrt(-alpha) : INFINITY;
        double ag = fmin(fabs(g), cap);
        for (int k = 0; k < 2100; k++) {
            double fv;
            const double xs = t >= 0.0 ? ag : -ag;
            TFUN(xs, fv);
            if (t >= 0.0 ? fv >= target : fv <= target) break;
            if (ag >= cap) break;
            ag = fmin(2.0 * ag, cap);
        }
        if (t >= 0.0) hi = ag;
        else lo = -ag;
        x = g;
    }
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    for (int it = 0; it < 400; it++) {
        double tf;
        TFUN(x, tf);
        stumpff(alpha * x * x, &c2, &c3);
        const double zz = alpha * x * x;
        const double rr = (sigma0 * x * (1.0 - zz * c3) + one_ar * x * x * c2) + r0n;
        const double res = tf - target;
        if (res > 0.0) hi = x;
        else lo = x;
        double xn = x - res / rr;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        const double dx = xn - x;
        x = xn;
        if (fabs(dx) <= 4.0 * DBL_EPSILON * fabs(x) || hi - lo <= 4.0 * DBL_EPSILON * fabs(x)) break;
    }
#undef TFUN
    const double z = alpha * x * x;
    stumpff(z, &c2, &c3);
    const double f = 1.0 - (x * x / r0n) * c2;
    const double g = t - (x * x * x / smu) * c3;
    double r[3];
    for (int c = 0; c < 3; c++) r[c] = f * r0[c] + g * v0[c];
    const double rn = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    const double fd = (smu / (rn * r0n)) * (z * x * c3 - x);
    const double gd = 1.0 - (x * x / rn) * c2;
    for (int c = 0; c < 3; c++) {
        rv[c] = r[c];
        rv[3 + c] = fd * r0[c] + gd * v0[c];
    }
    return CCO_OK;
}

/* E_{h, H_ij} for the two-body Hamiltonian of particles i and j (eq. 10):
 * the relative motion by the Kepler flow, the centre of mass uniformly. */
static int kepler_pair(const cco_params *p, cco_state *s, int64_t i, int64_t j, double h)
{
    const double mi = s->m[i], mj = s->m[j];
    const double M = mi + mj;
    double rv[6] = {s->x[j] - s->x[i], s->y[j] - s->y[i], s->z[j] - s->z[i],
                    s->vx[j] - s->vx[i], s->vy[j] - s->vy[i], s->vz[j] - s->vz[i]};
    const double X = (mi * s->x[i] + mj * s->x[j]) / M, Y = (mi * s->y[i] + mj * s->y[j]) / M,
                 Z = (mi * s->z[i] + mj * s->z[j]) / M;
    const double VX = (mi * s->vx[i] + mj * s->vx[j]) / M, VY = (mi * s->vy[i] + mj * s->vy[j]) / M,
                 VZ = (mi * s->vz[i] + mj * s->vz[j]) / M;
    const int rc = cco_kepler(p->G * M, rv, h);
    if (rc != CCO_OK) return rc == CCO_ERR_ARG ? CCO_ERR_NONFINITE : rc;
    const double X1 = X + h * VX, Y1 = Y + h * VY, Z1 = Z + h * VZ;
    const double fi = mj / M, fj = mi / M;
    s->x[i] = X1 - fi * rv[0]; s->y[i] = Y1 - fi * rv[1]; s->z[i] = Z1 - fi * rv[2];
    s->x[j] = X1 + fj * rv[0]; s->y[j] = Y1 + fj * rv[1]; s->z[j] = Z1 + fj * rv[2];
    s->vx[i] = VX - fi * rv[3]; s->vy[i] = VY - fi * rv[4]; s->vz[i] = VZ - fi * rv[5];
    s->vx[j] = VX + fj * rv[3]; s->vy[j] = VY + fj * rv[4]; s->vz[j] = VZ + fj * rv[5];
    return CCO_OK;
}

/* ------------------------------------------------------------------------ */
/* The CC integrator (eqs. 26-31, Fig. 2).                                   */
/* ------------------------------------------------------------------------ */

/*
 * evolve_cc(H, h) of Fig. 2 for the particle set I (ascending indices):
 *   (C_1..C_K, R) = split_cc(H, h)
 *   for C_i: evolve_cc(C_i, h/2)
 *   drift(R, h/2); kick(R,R,h); kick(C,C,h); kick(C,R,h); drift(R, h/2)
 *   for C_i: evolve_cc(C_i, h/2)
 * The partition found at h is used for both halves; each inner call splits its
 * own set again on the state it sees.
 */
static int evolve_rec(const cco_params *p, cco_state *s, const int64_t *I, int64_t n,
                      double h, int64_t depth, cco_stats *st);

/* E_{h, H_C} for a non-trivial component C (eq. 27): with CC_KEPLER a
 * component of two particles is the two-body Hamiltonian of eq. 10 and is
 * advanced by its Kepler solution (Sec. 2.2, last paragraph; Sec. 3.2);
 * everything else recurses. */
static int evolve_component(const cco_params *p, cco_state *s, const int64_t *I, int64_t n,
                            double h, int64_t depth, cco_stats *st)
{
    if (p->kepler && n == 2) {
        st->kepler_solves++;
        return kepler_pair(p, s, I[0], I[1], h);
    }
    return evolve_rec(p, s, I, n, h, depth, st);
}

static int evolve_rec(const cco_params *p, cco_state *s, const int64_t *I, int64_t n,
                      double h, int64_t depth, cco_stats *st)
{
    if (depth > p->max_depth) return CCO_ERR_DEPTH;
    if (depth > st->max_depth_seen) st->max_depth_seen = depth;

    int64_t *root = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *memb = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!root || !cnt || !start || !fill || !memb) {
        free(root); free(cnt); free(start); free(fill); free(memb);
        return CCO_ERR_OOM;
    }

    int rc = split_bfs_pos(p, s, I, n, h, root, &st->tau_evals);
    st->splits++;
    if (rc != CCO_OK) goto out;

    /* group members by component (ascending root, members ascending) */
    for (int64_t k = 0; k < n; k++) cnt[root[k]]++;
    {
        int64_t acc = 0;
        for (int64_t r = 0; r < n; r++) { start[r] = acc; fill[r] = acc; acc += cnt[r]; }
    }
    for (int64_t k = 0; k < n; k++) memb[fill[root[k]]++] = I[k];
    for (int64_t r = 0; r < n; r++) if (cnt[r] >= 2) st->components++;

    const double half = 0.5 * h;

    /* E_{h/2, H_C}: every non-trivial component independently (eq. 27) */
    for (int64_t r = 0; r < n && rc == CCO_OK; r++)
        if (cnt[r] >= 2) rc = evolve_component(p, s, memb + start[r], cnt[r], half, depth + 1, st);
    if (rc != CCO_OK) goto out;

    /* D_{h/2, T_R} */
    for (int64_t k = 0; k < n; k++) {
        if (cnt[root[k]] != 1) continue;
        const int64_t i = I[k];
        s->x[i] += half * s->vx[i];
        s->y[i] += half * s->vy[i];
        s->z[i] += half * s->vz[i];
        st->drifts++;
    }

    /* K_{h, V_R + V_CC + V_CR}: every pair in different components (eq. 30) */
    rc = cco_kick(p, s, I, n, root, h, &st->kick_pairs);
    if (rc != CCO_OK) goto out;

    /* D_{h/2, T_R} */
    for (int64_t k = 0; k < n; k++) {
        if (cnt[root[k]] != 1) continue;
        const int64_t i = I[k];
        s->x[i] += half * s->vx[i];
        s->y[i] += half * s->vy[i];
        s->z[i] += half * s->vz[i];
        st->drifts++;
    }

    /* E_{h/2, H_C} again with the same partition */
    for (int64_t r = 0; r < n && rc == CCO_OK; r++)
        if (cnt[r] >= 2) rc = evolve_component(p, s, memb + start[r], cnt[r], half, depth + 1, st);

out:
    free(root); free(cnt); free(start); free(fill); free(memb);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The HOLD split (Sec. 2.1, eqs. 11-17).                                    */
/* ------------------------------------------------------------------------ */

/*
 * evolve_hold(H, h) for the particle set I (ascending):
 *   tau(i) = min over j in I of tau(i,j)            particle time step
 *   S = {i : tau(i) >= h}, F = {i : tau(i) < h}     (eqs. 11-12)
 *   E_{h/2, H_F}                                    recursion at h/2 (eq. 14)
 *   D_{h/2, T_S} K_{h, V_S + V_SF} D_{h/2, T_S}     (eqs. 15-17)
 *   E_{h/2, H_F}
 * tau(i) < h holds exactly when some tau(i,j) < h, which needs every pair
 * (the HOLD split evaluates all interactions, Sec. 2.3).  F is recursed into
 * as one closed set.  The recursion ends when F is empty.
 */
static int evolve_hold(const cco_params *p, cco_state *s, const int64_t *I, int64_t n,
                       double h, int64_t depth, cco_stats *st)
{
    if (depth > p->max_depth) return CCO_ERR_DEPTH;
    if (depth > st->max_depth_seen) st->max_depth_seen = depth;
    st->splits++;
    double *taui = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *lab = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!taui || !lab || !F) { free(taui); free(lab); free(F); return CCO_ERR_OOM; }
    for (int64_t k = 0; k < n; k++) taui[k] = INFINITY;
    for (int64_t a = 0; a < n; a++) {
        for (int64_t b = a + 1; b < n; b++) {
            const double t = cco_tau(p, s, I[a], I[b]);
            st->tau_evals++;
            if (t < taui[a]) taui[a] = t;
            if (t < taui[b]) taui[b] = t;
        }
    }
    /* labels for the kick: every fast particle carries -1, a slow one its
     * position, so a pair is kicked unless both members are fast */
    int64_t nf = 0;
    for (int64_t k = 0; k < n; k++) {
        if (taui[k] < h) { lab[k] = -1; F[nf++] = I[k]; }
        else lab[k] = k;
    }
    const double half = 0.5 * h;
    int rc = CCO_OK;
    if (nf > 0) {
        st->components++;
        rc = evolve_hold(p, s, F, nf, half, depth + 1, st);
    }
    if (rc == CCO_OK) {
        for (int64_t k = 0; k < n; k++) {
            if (lab[k] < 0) continue;
            const int64_t i = I[k];
            s->x[i] += half * s->vx[i]; s->y[i] += half * s->vy[i]; s->z[i] += half * s->vz[i];
            st->drifts++;
        }
        rc = cco_kick(p, s, I, n, lab, h, &st->kick_pairs);
    }
    if (rc == CCO_OK) {
        for (int64_t k = 0; k < n; k++) {
            if (lab[k] < 0) continue;
            const int64_t i = I[k];
            s->x[i] += half * s->vx[i]; s->y[i] += half * s->vy[i]; s->z[i] += half * s->vz[i];
            st->drifts++;
        }
        if (nf > 0) rc = evolve_hold(p, s, F, nf, half, depth + 1, st);
    }
    free(taui); free(lab); free(F);
    return rc;
}

static int check_params(const cco_params *p)
{
    if (!p) return CCO_ERR_ARG;
    if (!(p->eta > 0.0) || !isfinite(p->eta)) return CCO_ERR_ARG;
    if (!(p->eps2 >= 0.0) || !isfinite(p->eps2)) return CCO_ERR_ARG;
    if (!(p->G > 0.0) || !isfinite(p->G)) return CCO_ERR_ARG;
    if (p->max_depth < 0) return CCO_ERR_ARG;
    if (p->kepler != 0 && p->kepler != 1) return CCO_ERR_ARG;
    if (p->kepler && p->eps2 != 0.0) return CCO_ERR_ARG;   /* the Kepler solution is for 1/r */
    if (p->hold != 0 && p->hold != 1) return CCO_ERR_ARG;
    if (p->hold && p->kepler) return CCO_ERR_ARG;          /* the Kepler option belongs to the CC split */
    return CCO_OK;
}

/* positions and velocities finite, masses finite and positive */
static int check_state(const cco_state *s, int64_t lo, int64_t hi)
{
    for (int64_t i = lo; i < hi; i++) {
        if (!(s->m[i] > 0.0) || !isfinite(s->m[i])) return CCO_ERR_ARG;
        if (!isfinite(s->x[i]) || !isfinite(s->y[i]) || !isfinite(s->z[i]) ||
            !isfinite(s->vx[i]) || !isfinite(s->vy[i]) || !isfinite(s->vz[i]))
            return CCO_ERR_NONFINITE;
    }
    return CCO_OK;
}

static int step_count(double dt, double t_end, int64_t *nsteps)
{
    if (!(dt > 0.0) || !isfinite(dt) || !(t_end > 0.0) || !isfinite(t_end)) return CCO_ERR_ARG;
    const double q = t_end / dt;
    if (!(q >= 1.0) || q != floor(q) || q > 2147483647.0) return CCO_ERR_ARG;
    *nsteps = (int64_t)q;
    return CCO_OK;
}

/* Global steps of evolve_cc(all, dt) over particles [lo, hi). */
static int evolve_range(const cco_params *p, cco_state *s, int64_t lo, int64_t hi,
                        double dt, int64_t nsteps, cco_stats *st)
{
    const int64_t n = hi - lo;
    int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *snap = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    if (!I || !snap) { free(I); free(snap); return CCO_ERR_OOM; }
    for (int64_t k = 0; k < n; k++) I[k] = lo + k;
    double *arr[6] = {s->x, s->y, s->z, s->vx, s->vy, s->vz};

    int rc = CCO_OK;
    st->t_reached = 0.0;
    for (int64_t step = 0; step < nsteps; step++) {
        rc = check_state(s, lo, hi);
        if (rc != CCO_OK) break;
        for (int c = 0; c < 6; c++) memcpy(snap + (size_t)c * n, arr[c] + lo, sizeof(double) * (size_t)n);
        rc = p->hold ? evolve_hold(p, s, I, n, dt, 0, st) : evolve_rec(p, s, I, n, dt, 0, st);
        if (rc == CCO_OK) rc = check_state(s, lo, hi);
        if (rc != CCO_OK) {
            for (int c = 0; c < 6; c++) memcpy(arr[c] + lo, snap + (size_t)c * n, sizeof(double) * (size_t)n);
            break;
        }
        st->t_reached = (double)(step + 1) * dt;
    }
    free(I);
    free(snap);
    return rc;
}

int cco_evolve(const cco_params *p, cco_state *s, int64_t n, double dt, double t_end, cco_stats *st)
{
    cco_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    if (check_params(p) != CCO_OK || !s || n < 1) return CCO_ERR_ARG;
    int64_t nsteps;
    if (step_count(dt, t_end, &nsteps) != CCO_OK) return CCO_ERR_ARG;
    return evolve_range(p, s, 0, n, dt, nsteps, st);
}

int cco_evolve_batch(const cco_params *p, cco_state *s, const int64_t *off, int32_t ncl,
                     double dt, double t_end, cco_stats *st)
{
    if (check_params(p) != CCO_OK || !s || !off || ncl < 1 || !st) return CCO_ERR_ARG;
    for (int32_t c = 0; c < ncl; c++) memset(&st[c], 0, sizeof(cco_stats));
    for (int32_t c = 0; c < ncl; c++)
        if (off[c] < 0 || off[c + 1] <= off[c]) return CCO_ERR_ARG;
    int64_t nsteps;
    if (step_count(dt, t_end, &nsteps) != CCO_OK) return CCO_ERR_ARG;
    int rc = CCO_OK;
    for (int32_t c = 0; c < ncl; c++) {
        int r = evolve_range(p, s, off[c], off[c + 1], dt, nsteps, &st[c]);
        if (r != CCO_OK && rc == CCO_OK) rc = r;
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                              */
/* ------------------------------------------------------------------------ */

typedef struct { double s, c; } nsum;   /* Neumaier running sum */

static void nsum_add(nsum *a, double v)
{
    const double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum *a) { return a->s + a->c; }

int cco_accel(const cco_params *p, const cco_state *s, int64_t n,
              const int64_t *idx, int64_t nidx, double *ax, double *ay, double *az)
{
    if (!p || !s || n < 1 || nidx < 0 || (nidx > 0 && (!idx || !ax || !ay || !az))) return CCO_ERR_ARG;
    for (int64_t k = 0; k < nidx; k++) {
        const int64_t i = idx[k];
        if (i < 0 || i >= n) return CCO_ERR_ARG;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            const double dx = s->x[j] - s->x[i];
            const double dy = s->y[j] - s->y[i];
            const double dz = s->z[j] - s->z[i];
            const double r2 = ((dx * dx + dy * dy) + dz * dz) + p->eps2;
            if (r2 == 0.0) return CCO_ERR_NONFINITE;
            const double f = p->G / (r2 * sqrt(r2));
            const double mjf = s->m[j] * f;
            sx += mjf * dx; sy += mjf * dy; sz += mjf * dz;
        }
        ax[k] = sx; ay[k] = sy; az[k] = sz;
    }
    return CCO_OK;
}

int cco_accel_compensated(const cco_params *p, const cco_state *s, int64_t n,
                          const int64_t *idx, int64_t nidx, double *ax, double *ay, double *az)
{
    if (!p || !s || n < 1 || nidx < 0 || (nidx > 0 && (!idx || !ax || !ay || !az))) return CCO_ERR_ARG;
    for (int64_t k = 0; k < nidx; k++) {
        const int64_t i = idx[k];
        if (i < 0 || i >= n) return CCO_ERR_ARG;
        nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            const double dx = s->x[j] - s->x[i];
            const double dy = s->y[j] - s->y[i];
            const double dz = s->z[j] - s->z[i];
            const double r2 = ((dx * dx + dy * dy) + dz * dz) + p->eps2;
            if (r2 == 0.0) return CCO_ERR_NONFINITE;
            const double f = p->G / (r2 * sqrt(r2));
            const double mjf = s->m[j] * f;
            nsum_add(&sx, mjf * dx); nsum_add(&sy, mjf * dy); nsum_add(&sz, mjf * dz);
        }
        ax[k] = nsum_get(&sx); ay[k] = nsum_get(&sy); az[k] = nsum_get(&sz);
    }
    return CCO_OK;
}

/* H = sum T_i + sum_{i<j} V_ij (eqs. 1-3) and the other integrals of motion. */
int cco_diagnostics(const cco_params *p, const cco_state *s, int64_t n, double out[12])
{
    if (!p || !s || n < 1 || !out) return CCO_ERR_ARG;
    nsum ek = {0, 0}, ep = {0, 0}, px = {0, 0}, py = {0, 0}, pz = {0, 0};
    nsum lx = {0, 0}, ly = {0, 0}, lz = {0, 0}, cx = {0, 0}, cy = {0, 0}, cz = {0, 0}, mt = {0, 0};
    for (int64_t i = 0; i < n; i++) {
        const double m = s->m[i];
        const double v2 = (s->vx[i] * s->vx[i] + s->vy[i] * s->vy[i]) + s->vz[i] * s->vz[i];
        nsum_add(&ek, 0.5 * m * v2);
        nsum_add(&px, m * s->vx[i]); nsum_add(&py, m * s->vy[i]); nsum_add(&pz, m * s->vz[i]);
        nsum_add(&lx, m * (s->y[i] * s->vz[i] - s->z[i] * s->vy[i]));
        nsum_add(&ly, m * (s->z[i] * s->vx[i] - s->x[i] * s->vz[i]));
        nsum_add(&lz, m * (s->x[i] * s->vy[i] - s->y[i] * s->vx[i]));
        nsum_add(&cx, m * s->x[i]); nsum_add(&cy, m * s->y[i]); nsum_add(&cz, m * s->z[i]);
        nsum_add(&mt, m);
        for (int64_t j = i + 1; j < n; j++) {
            const double dx = s->x[j] - s->x[i];
            const double dy = s->y[j] - s->y[i];
            const double dz = s->z[j] - s->z[i];
            const double r2 = ((dx * dx + dy * dy) + dz * dz) + p->eps2;
            nsum_add(&ep, -p->G * m * s->m[j] / sqrt(r2));
        }
    }
    const double M = nsum_get(&mt);
    out[0] = nsum_get(&ek);
    out[1] = nsum_get(&ep);
    out[2] = nsum_get(&px); out[3] = nsum_get(&py); out[4] = nsum_get(&pz);
    out[5] = nsum_get(&lx); out[6] = nsum_get(&ly); out[7] = nsum_get(&lz);
    out[8] = nsum_get(&cx) / M; out[9] = nsum_get(&cy) / M; out[10] = nsum_get(&cz) / M;
    out[11] = M;
    return CCO_OK;
}
