// cc_device.h -- device-side building blocks of the CC integrator on gfx950.
//
// Everything here is compiled with -ffp-contract=off and without fast-math:
// each FP64 expression below is evaluated as written, one correctly rounded
// IEEE-754 operation at a time, so results are reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccg {

struct DevParams {
    double eta, eps2, G;
    int32_t max_depth;
    int32_t pad;
};

// A set of particles evolved by one evolve_cc call: slots [start, start+n)
// of the working arrays, recursion level `depth` (global step = 0), and the
// cluster it belongs to (for per-cluster statistics).
struct Seg {
    int32_t start, n, cluster, depth;
};

// Statistics slots (per cluster, uint64 each).
enum StatIdx {
    ST_TAU = 0,       // pair time steps evaluated
    ST_TAU_ALG = 1,   // pair time steps the split needs (n-1 or n(n-1)/2)
    ST_KICK = 2,      // unordered pairs kicked
    ST_DRIFT = 3,     // single-particle half-step drifts
    ST_COMP = 4,      // non-trivial components found
    ST_SPLIT = 5,     // evolve_cc calls (splits)
    ST_MAXD = 6,      // deepest level (atomicMax)
    ST_N = 8
};

// Error bits raised by kernels.
enum ErrBits { EB_DEPTH = 1, EB_NONFINITE = 2, EB_MASS = 4, EB_CAPACITY = 8, EB_BUDGET = 16 };

// Work budgets that turn a runaway recursion (or a corrupted structure) into
// an error instead of an endless kernel: leaves of one two-particle walk,
// level visits of one on-chip item, steps of one union-find walk.
constexpr uint64_t PAIR_LEAF_BUDGET = 1ull << 28;
constexpr uint64_t ITEM_VISIT_BUDGET = 1ull << 24;
constexpr int FIND_BUDGET = 1 << 22;

// Working state: structure of arrays plus the original particle index.
struct SoA {
    double *x, *y, *z, *vx, *vy, *vz, *m;
    int32_t *orig;
};

// ---------------------------------------------------------------------------
// Pair time step tau(i,j) (eq. 19), symmetrised free-fall and fly-by steps:
//   tau = min( eta t_ff / (1 - eta t_ff'/2), eta t_fb / (1 - eta t_fb'/2) )
//   t_ff = sqrt(r^3/mu), t_ff' = (3/2) t_ff (q.u)/r^2,
//   t_fb = r/|u|,        t_fb' = (q.u)/(r|u|) (1 + mu/(r|u|^2)),
// r^2 = |q|^2 + eps^2, mu = G (m_i + m_j); non-positive denominator -> +INF,
// |u| = 0 -> no fly-by bound, r^2 = 0 -> 0.  (dx,..) = q_i - q_j (either sign:
// the value is symmetric bit for bit).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tau_pair(double dx, double dy, double dz, double dvx, double dvy,
                                           double dvz, double msum, const DevParams &p)
{
    const double r2 = ((dx * dx + dy * dy) + dz * dz) + p.eps2;
    const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
    const double rv = (dx * dvx + dy * dvy) + dz * dvz;
    const double mu = p.G * msum;
    if (r2 == 0.0) return 0.0;
    const double r = sqrt(r2);
    const double eta = p.eta;
    const double tff = sqrt((r2 * r) / mu);
    const double dtff = ((1.5 * tff) * rv) / r2;
    const double dff = 1.0 - (0.5 * eta) * dtff;
    const double sff = (dff > 0.0) ? (eta * tff) / dff : __builtin_inf();
    double sfb = __builtin_inf();
    if (v2 > 0.0) {
        const double v = sqrt(v2);
        const double tfb = r / v;
        const double dtfb = (rv / (r * v)) * (1.0 + mu / (r * v2));
        const double dfb = 1.0 - (0.5 * eta) * dtfb;
        sfb = (dfb > 0.0) ? (eta * tfb) / dfb : __builtin_inf();
    }
    return (sfb < sff) ? sfb : sff;
}

// Edge test tau(i,j) < h of eq. 20.  min(a,b) < h  <=>  a < h || b < h, so the
// fly-by term is only formed when the free-fall term does not already decide;
// every value that is formed is the same rounded value as in tau_pair.
__device__ __forceinline__ bool edge_pair(double dx, double dy, double dz, double dvx, double dvy,
                                          double dvz, double msum, const DevParams &p, double h)
{
    const double r2 = ((dx * dx + dy * dy) + dz * dz) + p.eps2;
    if (r2 == 0.0) return 0.0 < h;
    const double mu = p.G * msum;
    const double rv = (dx * dvx + dy * dvy) + dz * dvz;
    const double r = sqrt(r2);
    const double eta = p.eta;
    const double tff = sqrt((r2 * r) / mu);
    const double dtff = ((1.5 * tff) * rv) / r2;
    const double dff = 1.0 - (0.5 * eta) * dtff;
    if (dff > 0.0 && (eta * tff) / dff < h) return true;
    const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
    if (!(v2 > 0.0)) return false;
    const double v = sqrt(v2);
    const double tfb = r / v;
    const double dtfb = (rv / (r * v)) * (1.0 + mu / (r * v2));
    const double dfb = 1.0 - (0.5 * eta) * dtfb;
    return dfb > 0.0 && (eta * tfb) / dfb < h;
}

// Acceleration term of one partner j on particle i (eqs. 8-9):
// a_i += G m_j (q_j - q_i) / (|q_j - q_i|^2 + eps^2)^(3/2).  Returns false if
// r^2 + eps^2 == 0.
__device__ __forceinline__ bool accel_term(double xi, double yi, double zi, double xj, double yj,
                                           double zj, double mj, double eps2, double G, double &ax,
                                           double &ay, double &az)
{
    const double dx = xj - xi;
    const double dy = yj - yi;
    const double dz = zj - zi;
    const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
    const double f = G / (r2 * sqrt(r2));
    const double mjf = mj * f;
    ax += mjf * dx;
    ay += mjf * dy;
    az += mjf * dz;
    return r2 != 0.0;
}

// ---------------------------------------------------------------------------
// Two-particle evolve_cc, the recursion of Fig. 2 for a component {a, b}:
// split at h is either one component (recurse twice at h/2) or two singletons
// (drift h/2, kick h, drift h/2).  Walked iteratively: `second` holds one bit
// per level, set while that level's second half runs.  a must be the particle
// with the smaller original index (the kick is written in that orientation).
// ---------------------------------------------------------------------------
struct Body {
    double x, y, z, vx, vy, vz, m;
};

struct PairCounters {
    uint64_t tau, kick, drift, comp, split;
    int32_t maxd;
};

// Returns 0, or EB_DEPTH / EB_BUDGET (leaving a, b at their entry values).
__device__ inline int evolve_pair(Body &a, Body &b, double H, int32_t depth0, const DevParams &p,
                                  PairCounters &c)
{
    const Body a0 = a, b0 = b;
    uint64_t second = 0;
    uint64_t leaves = 0;
    int lvl = 0;
    double h = H;
    const double msum = a.m + b.m;
    for (;;) {
        const int32_t depth = depth0 + lvl;
        if (depth > p.max_depth) {
            a = a0;
            b = b0;
            return EB_DEPTH;
        }
        if (depth > c.maxd) c.maxd = depth;
        c.split++;
        c.tau++;
        const bool e = edge_pair(a.x - b.x, a.y - b.y, a.z - b.z, a.vx - b.vx, a.vy - b.vy, a.vz - b.vz,
                                 msum, p, h);
        if (e && lvl < 63) {
            c.comp++;
            lvl++;
            h = 0.5 * h;
            second &= ~(1ull << lvl);
            continue;
        }
        if (e) {  // deeper than the walker can track: treat as the depth cap
            a = a0;
            b = b0;
            return EB_DEPTH;
        }
        if (++leaves > PAIR_LEAF_BUDGET) {
            a = a0;
            b = b0;
            return EB_BUDGET;
        }
        // leaf: D_{h/2} K_h D_{h/2} on two singletons
        const double hh = 0.5 * h;
        a.x += hh * a.vx; a.y += hh * a.vy; a.z += hh * a.vz;
        b.x += hh * b.vx; b.y += hh * b.vy; b.z += hh * b.vz;
        {
            const double dx = b.x - a.x;
            const double dy = b.y - a.y;
            const double dz = b.z - a.z;
            const double r2 = ((dx * dx + dy * dy) + dz * dz) + p.eps2;
            const double f = p.G / (r2 * sqrt(r2));
            const double mbf = b.m * f;
            const double maf = a.m * f;
            const double aax = 0.0 + mbf * dx, aay = 0.0 + mbf * dy, aaz = 0.0 + mbf * dz;
            const double bax = 0.0 - maf * dx, bay = 0.0 - maf * dy, baz = 0.0 - maf * dz;
            a.vx += h * aax; a.vy += h * aay; a.vz += h * aaz;
            b.vx += h * bax; b.vy += h * bay; b.vz += h * baz;
        }
        a.x += hh * a.vx; a.y += hh * a.vy; a.z += hh * a.vz;
        b.x += hh * b.vx; b.y += hh * b.vy; b.z += hh * b.vz;
        c.kick++;
        c.drift += 4;
        // advance to the next sibling
        while (lvl > 0 && ((second >> lvl) & 1ull)) {
            second &= ~(1ull << lvl);
            lvl--;
            h = 2.0 * h;
        }
        if (lvl == 0) return 0;
        second |= (1ull << lvl);
    }
}

}  // namespace ccg
