// cc_device.h -- device-side building blocks of the CC integrator on gfx950.
//
// Everything here is compiled with -ffp-contract=off and without fast-math:
// each FP64 expression below is evaluated as written, one correctly rounded
// IEEE-754 operation at a time, so results are reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define CC_SCREEN64_FN __device__ __forceinline__
#define CC_SCREEN64_RSQ(x) __builtin_amdgcn_rsq(x)
#include "cc_screen64.h"
#define CC_KEPLER_FN __device__ inline
#include "cc_kepler.h"
#define CC_SCREEN32_FN __device__ __forceinline__
#include "cc_screen32.h"

namespace ccg {

struct DevParams {
    double eta, eps2, G;
    int32_t max_depth;
    int32_t kepler;  // CC_KEPLER: two-particle components by the Kepler solution
    int32_t hold;    // the HOLD split: all fast particles of a set form one set
};

// A set of particles evolved by one evolve_cc call: slots [start, start+n)
// of the working arrays, recursion level `depth` (global step = 0), and the
// cluster it belongs to (for per-cluster statistics).
struct Seg {
    int32_t start, n, cluster, depth;
};

// One block of the tiled kick: i tile `itile` (256 slots) of segment `seg`
// against partners [j0, j0 + nj) of the same segment (offsets within it).
struct KickBlock {
    int32_t seg, itile, j0, nj;
};

// The partial accelerations of the kick live in slots of 3 x 256 doubles:
// first one slot per kick block, then one per group sum.  An i tile's kick
// is the in-order sum of slots [src, src + n).
struct KickTile {
    int32_t src, n;
};

// A group sum: slots [src, src + n) added in order into slot dst (n is at
// most KICK_FANIN).  Tiles with more kick blocks than that are reduced in
// two stages, so that no sum runs long.
struct KickJob {
    int32_t src, n, dst, pad;
};
constexpr int KICK_FANIN = 16;

// Granularity of the kick's j ranges (partners per block are a multiple).
constexpr int KICK_JW = 32;

// Statistics slots (per cluster, uint64 each).
enum StatIdx {
    ST_TAU = 0,       // pair time steps evaluated
    ST_TAU_ALG = 1,   // pair time steps the split needs (n-1 or n(n-1)/2)
    ST_KICK = 2,      // unordered pairs kicked
    ST_DRIFT = 3,     // single-particle half-step drifts
    ST_COMP = 4,      // non-trivial components found
    ST_SPLIT = 5,     // evolve_cc calls (splits)
    ST_MAXD = 6,      // deepest level (atomicMax)
    ST_KEPLER = 7,    // two-body components advanced by the Kepler solution
    ST_N = 8
};

// Error bits raised by kernels.
enum ErrBits { EB_DEPTH = 1, EB_NONFINITE = 2, EB_MASS = 4, EB_CAPACITY = 8, EB_BUDGET = 16 };

// Work budgets that turn a runaway recursion (or a corrupted structure) into
// an error within seconds instead of an endless kernel.
//   - leaves of one two-particle walk in one launch: the hardest binaries of
//     the 262 144-body workload (a = 1e-5, e up to 0.999, the heaviest masses)
//     need about 2^22 leaves over h = 1/128 (some 1800 orbits of about 2000
//     leaves at eta = 0.01); 2^24 leaves take about 10 s on one lane;
//   - level visits of one on-chip item in one launch (a visit is one split or
//     one kick of a level in LDS, a few microseconds for a wavefront team):
//     the HOLD split keeps sets of three or more fast bodies deep in the
//     hierarchy (a hard binary with any third fast body): a cluster of the
//     fractal ensemble workload makes some 1.8 million splits in one step at
//     dt = 1/64 under HOLD, each two or three visits;
//   - steps of one union-find walk: links point to smaller slots only, so a
//     walk ends within the set size (at most 1024 in LDS; the global sets of
//     the workloads hold at most 2^18 slots and path halving keeps the walks
//     far shorter); retries of one union, each lost to another thread's link.
constexpr uint64_t PAIR_LEAF_BUDGET = 1ull << 24;
constexpr uint64_t ITEM_VISIT_BUDGET = 1ull << 23;
constexpr int FIND_BUDGET = 1 << 20;
constexpr int UNITE_RETRIES = 1 << 16;
constexpr int LDS_FIND_BUDGET = 1 << 11;

// The global union-find keeps one parent entry per 128-byte line: its
// coherent loads, path-halving stores and compare-and-swaps come from every
// tile of a sweep at once, and packed entries would make a few hundred lines
// the serialisation point of the whole launch (slot a lives at a * stride).
constexpr int PARENT_STRIDE = 32;

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

// The FP32 screen of the mixed path (cc_screen32.h, shared with a host test).
typedef ccs::ScreenParams32 ScreenParams;
using ccs::edge_screen32;
enum { SCREEN_NO = ccs::SCREEN32_NO, SCREEN_EDGE = ccs::SCREEN32_EDGE, SCREEN_UNSURE = ccs::SCREEN32_UNSURE };

__device__ __forceinline__ ScreenParams screen_params(const DevParams &p, double h)
{
    ScreenParams q;
    q.eta = (float)p.eta;
    q.half_eta = (float)(0.5 * p.eta);
    q.eps2 = (float)p.eps2;
    q.G = (float)p.G;
    q.h = (float)h;
    return q;
}

// Edge decision of eq. 20: the certified FP64 screen (and, in mixed
// precision, the FP32 screen before it) in front of the literal formula.
template <bool MIXED>
__device__ __forceinline__ bool edge_decide(double dx, double dy, double dz, double dvx, double dvy, double dvz,
                                            double msum, const DevParams &p, const ScreenParams &q,
                                            const ccs::Screen64 &s64, double h)
{
    if (MIXED) {
        const int sc = edge_screen32(dx, dy, dz, dvx, dvy, dvz, msum, q);
        if (sc != SCREEN_UNSURE) return sc == SCREEN_EDGE;
    }
    const double r2 = ((dx * dx + dy * dy) + dz * dz) + p.eps2;
    const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
    const double rv = (dx * dvx + dy * dvy) + dz * dvz;
    const double mu = p.G * msum;
    const int sc = ccs::screen64(r2, v2, rv, mu, s64);
    if (sc != ccs::SCREEN64_UNSURE) return sc == ccs::SCREEN64_EDGE;
    return edge_pair(dx, dy, dz, dvx, dvy, dvz, msum, p, h);
}

// Screen verdict for one pair (ccs::SCREEN64_NO / _EDGE / _UNSURE): the FP32
// screen in mixed precision, the FP64 screen for what it leaves open.
template <bool MIXED>
__device__ __forceinline__ int edge_screen(double dx, double dy, double dz, double dvx, double dvy, double dvz,
                                           double msum, const DevParams &p, const ScreenParams &q,
                                           const ccs::Screen64 &s64)
{
    static_assert((int)SCREEN_NO == (int)ccs::SCREEN64_NO && (int)SCREEN_EDGE == (int)ccs::SCREEN64_EDGE &&
                      (int)SCREEN_UNSURE == (int)ccs::SCREEN64_UNSURE,
                  "screen verdict codes");
    if (MIXED) {
        const int sc = edge_screen32(dx, dy, dz, dvx, dvy, dvz, msum, q);
        if (sc != SCREEN_UNSURE) return sc;
    }
    const double r2 = ((dx * dx + dy * dy) + dz * dz) + p.eps2;
    const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
    const double rv = (dx * dvx + dy * dvy) + dz * dvz;
    const double mu = p.G * msum;
    return ccs::screen64(r2, v2, rv, mu, s64);
}

// FP32 pair force on an FP64 coordinate difference (mixed kick): adds
// G m_j d / (|d|^2 + eps^2)^(3/2) to a Kahan-compensated FP32 sum.
struct Kahan3 {
    float sx, sy, sz, cx, cy, cz;
};

__device__ __forceinline__ void kahan_add(float &s, float &c, float v)
{
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

__device__ __forceinline__ bool accel_term32(double xi, double yi, double zi, double xj, double yj, double zj,
                                             float gmj, float eps2, Kahan3 &k)
{
    const float dx = (float)(xj - xi), dy = (float)(yj - yi), dz = (float)(zj - zi);
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float f = gmj * (ri * ri * ri);
    kahan_add(k.sx, k.cx, f * dx);
    kahan_add(k.sy, k.cy, f * dy);
    kahan_add(k.sz, k.cz, f * dz);
    return r2 > 0.0f;
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

// The same pair term for the fast kick order, which is compared with the
// sequential FP64 sum to a tolerance rather than bit for bit: 1/r from the
// hardware reciprocal square root (about 2^-23 relative) and two Newton steps
// (about 2^-46, then rounding level), no division; gmj = G m_j.
__device__ __forceinline__ bool accel_term_rsq(double xi, double yi, double zi, double xj, double yj,
                                               double zj, double gmj, double eps2, double &ax, double &ay,
                                               double &az)
{
    const double dx = xj - xi;
    const double dy = yj - yi;
    const double dz = zj - zi;
    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
    double y = __builtin_amdgcn_rsq(r2);
    double e = __builtin_fma(-(r2 * y), y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    e = __builtin_fma(-(r2 * y), y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    const double f = gmj * (y * (y * y));
    ax = __builtin_fma(f, dx, ax);
    ay = __builtin_fma(f, dy, ay);
    az = __builtin_fma(f, dz, az);
    return r2 != 0.0;
}

// The same term behind a mask, for loops without a branch per partner: a
// partner that is off (same component, or the particle itself) contributes a
// zero factor whatever its distance.  A coincident pair that is on gives a
// non-finite sum, which the caller checks once.  One Newton step on the
// hardware reciprocal square root: about 2^-46 relative per pair force,
// against the fast order's bound of 1e-12 of the sum of the pair forces'
// magnitudes per particle.
__device__ __forceinline__ void accel_term_rsq_if(bool on, double xi, double yi, double zi, double xj, double yj,
                                                  double zj, double gmj, double eps2, double &ax, double &ay,
                                                  double &az)
{
    const double dx = xj - xi;
    const double dy = yj - yi;
    const double dz = zj - zi;
    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
    // an off partner sees r2 = 1 and mass 0: a finite zero factor
    const double rs = on ? r2 : 1.0;
    double y = __builtin_amdgcn_rsq(rs);
    const double e = __builtin_fma(-(rs * y), y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    const double f = (on ? gmj : 0.0) * (y * (y * y));
    ax = __builtin_fma(f, dx, ax);
    ay = __builtin_fma(f, dy, ay);
    az = __builtin_fma(f, dz, az);
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
    uint64_t tau, kick, drift, comp, split, kepler;
    int32_t maxd;
};

// E_{h, H_ab} (eq. 10) for a two-particle component: the relative motion by
// the Kepler flow, the centre of mass uniformly.
__device__ inline bool kepler_pair_dev(Body &a, Body &b, double h, double G)
{
    const double M = a.m + b.m;
    const double cx = (a.m * a.x + b.m * b.x) / M, cy = (a.m * a.y + b.m * b.y) / M, cz = (a.m * a.z + b.m * b.z) / M;
    const double ux = (a.m * a.vx + b.m * b.vx) / M, uy = (a.m * a.vy + b.m * b.vy) / M,
                 uz = (a.m * a.vz + b.m * b.vz) / M;
    double rx = b.x - a.x, ry = b.y - a.y, rz = b.z - a.z, vx = b.vx - a.vx, vy = b.vy - a.vy, vz = b.vz - a.vz;
    if (!cck::kepler_flow(G * M, rx, ry, rz, vx, vy, vz, h)) return false;
    const double X = cx + h * ux, Y = cy + h * uy, Z = cz + h * uz;
    const double fa = b.m / M, fb = a.m / M;
    a.x = X - fa * rx; a.y = Y - fa * ry; a.z = Z - fa * rz;
    b.x = X + fb * rx; b.y = Y + fb * ry; b.z = Z + fb * rz;
    a.vx = ux - fa * vx; a.vy = uy - fa * vy; a.vz = uz - fa * vz;
    b.vx = ux + fb * vx; b.vy = uy + fb * vy; b.vz = uz + fb * vz;
    return true;
}

// The FP64 screen's h-independent terms for the current state of a pair
// (differences a - b, as edge_decide forms them).
__device__ __forceinline__ ccs::Screen64Pair pair_screen(const Body &a, const Body &b, double msum,
                                                         const DevParams &p)
{
    const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const double dvx = a.vx - b.vx, dvy = a.vy - b.vy, dvz = a.vz - b.vz;
    const double r2 = ((dx * dx + dy * dy) + dz * dz) + p.eps2;
    const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
    const double rv = (dx * dvx + dy * dvy) + dz * dvz;
    return ccs::screen64_pair(r2, v2, rv, p.G * msum, p.eta);
}

// edge_decide for the walker: in FP64 the screen's verdict at h from the
// terms `sp` kept for the state, the literal formula for what it leaves open.
template <bool MIXED>
__device__ __forceinline__ bool pair_decide(const Body &a, const Body &b, double msum, const ccs::Screen64Pair &sp,
                                            const DevParams &p, double h)
{
    if (MIXED)
        return edge_decide<true>(a.x - b.x, a.y - b.y, a.z - b.z, a.vx - b.vx, a.vy - b.vy, a.vz - b.vz, msum, p,
                                 screen_params(p, h), ccs::screen64_params(p.eta, h), h);
    const int sc = ccs::screen64_at(sp, ccs::screen64_params(p.eta, h));
    if (sc != ccs::SCREEN64_UNSURE) return sc == ccs::SCREEN64_EDGE;
    return edge_pair(a.x - b.x, a.y - b.y, a.z - b.z, a.vx - b.vx, a.vy - b.vy, a.vz - b.vz, msum, p, h);
}

// Returns 0, or EB_DEPTH / EB_BUDGET / EB_NONFINITE (a and b are then partly
// advanced; the caller discards them: a failing global step is restored from
// its snapshot).  With CC_KEPLER (p.kepler), a pair that is a component
// found by a split (`component`) is advanced by the Kepler flow for H; a
// top-level two-particle set is split first, and once its two particles form
// a component each half of it is one Kepler flow of h/2.
//   One walk is a sequence of dependent steps in one lane, so its length is
// set by the instructions per node: the state only changes at a leaf (or a
// Kepler step), so the FP64 screen's h-independent terms are formed once per
// state and reused by the decisions of a descent; the counters are kept per
// walk (decisions, decisions that found an edge, leaves) and added at the end;
// and the levels whose second half has ended are left in one step.
template <bool MIXED>
__device__ inline int evolve_pair(Body &a, Body &b, double H, int32_t depth0, const DevParams &p,
                                  PairCounters &c, bool component = false)
{
    if (p.kepler && component) {
        c.kepler++;
        return kepler_pair_dev(a, b, H, p.G) ? 0 : EB_NONFINITE;
    }
    if (depth0 > p.max_depth) return EB_DEPTH;
    uint64_t second = 0;  // bit l set while level l runs its second half
    uint32_t nd = 0, ne = 0, nl = 0;
    int lvl = 0, maxlvl = 0, rc = 0;
    double h = H;
    const double msum = a.m + b.m;
    ccs::Screen64Pair sp{};
    bool fresh = true;  // the state changed since sp was formed
    for (;;) {
        ++nd;
        if (!MIXED && fresh) {
            sp = pair_screen(a, b, msum, p);
            fresh = false;
        }
        const bool e = pair_decide<MIXED>(a, b, msum, sp, p, h);
        if (e && p.kepler) {
            // the pair is a component at h: its two halves are Kepler flows of h/2
            ++ne;
            if (!kepler_pair_dev(a, b, 0.5 * h, p.G) || !kepler_pair_dev(a, b, 0.5 * h, p.G)) {
                rc = EB_NONFINITE;
                break;
            }
            fresh = true;
        } else if (e) {
            // deeper than the walker can track, or than max_depth
            if (lvl >= 63 || depth0 + lvl + 1 > p.max_depth) {
                rc = EB_DEPTH;
                break;
            }
            ++ne;
            ++lvl;
            maxlvl = max(maxlvl, lvl);
            h = 0.5 * h;
            second &= ~(1ull << lvl);
            continue;
        } else {
            if (++nl > PAIR_LEAF_BUDGET) {
                rc = EB_BUDGET;
                break;
            }
            // leaf: D_{h/2} K_h D_{h/2} on two singletons
            const double hh = 0.5 * h;
            a.x += hh * a.vx; a.y += hh * a.vy; a.z += hh * a.vz;
            b.x += hh * b.vx; b.y += hh * b.vy; b.z += hh * b.vz;
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
            a.x += hh * a.vx; a.y += hh * a.vy; a.z += hh * a.vz;
            b.x += hh * b.vx; b.y += hh * b.vy; b.z += hh * b.vz;
            fresh = true;
        }
        // advance to the next sibling: the levels lvl, lvl-1, ... whose second
        // half has just ended are left, and the deepest level l <= lvl still
        // in its first half starts its second half (the walk ends if none is)
        const uint64_t open = ~second & (((2ull << lvl) - 1ull) & ~1ull);
        if (open == 0) break;
        const int l = 63 - __builtin_clzll(open);
        second = (second & ((2ull << l) - 1ull)) | (1ull << l);
        h = ldexp(H, -l);
        lvl = l;
    }
    c.split += nd;
    c.tau += nd;
    c.comp += ne;
    c.kick += nl;
    c.drift += 4ull * nl;
    if (p.kepler) c.kepler += 2ull * ne;
    if (depth0 + maxlvl > c.maxd) c.maxd = depth0 + maxlvl;
    return rc;
}

}  // namespace ccg
