// cc_kepler.h -- the two-body (Kepler) flow of the CC_KEPLER option on the
// GPU (also built for the host by a test).  The including file supplies the
// CC_KEPLER_FN qualifiers; sqrt, sin, sinh, fmod, fabs and isfinite are the
// platform's double-precision functions.
#pragma once

#ifndef CC_KEPLER_FN
#error "define CC_KEPLER_FN (function qualifiers) before including cc_kepler.h"
#endif

namespace cck {

// ---------------------------------------------------------------------------
// Two-body flow of eq. 10 (eps = 0) in universal variables (Bate, Mueller &
// White 1971): relative position r = q_b - q_a and velocity v over time t
// under mu = G (m_a + m_b).  With sigma = r0.v0 / sqrt(mu) and
// alpha = 2/|r0| - |v0|^2/mu, the universal anomaly x solves
//   F(x) = sigma x^2 c2 + (1 - alpha |r0|) x^3 c3 + |r0| x - sqrt(mu) t = 0,
// c2, c3 the Stumpff functions of z = alpha x^2; F' is the radius and
// F'' = sigma (1 - z c2) + (1 - alpha |r0|) x (1 - z c3).  Here x is found by
// Laguerre's iteration (order 5) inside a bracket of the root; bound orbits
// are first reduced by whole periods.  Then r = f r0 + g v0,
// v = f' r0 + g' v0 (Lagrange coefficients).
// ---------------------------------------------------------------------------
CC_KEPLER_FN void stumpff(double z, double &c2, double &c3)
{
    if (fabs(z) < 1.0) {
        // c2 = (1/2!)(1 - z/(3.4)(1 - z/(5.6)(...))), c3 = (1/3!)(1 - z/(4.5)(1 - z/(6.7)(...)));
        // 14 terms reach 1/30! at |z| = 1, far below the last bit; the
        // nested factors are multiplied by rounded reciprocals (no division)
        double a = 1.0, b = 1.0;
#pragma unroll
        for (int k = 14; k >= 1; --k) {
            a = 1.0 - (z * a) * (1.0 / ((2.0 * k + 1.0) * (2.0 * k + 2.0)));
            b = 1.0 - (z * b) * (1.0 / ((2.0 * k + 2.0) * (2.0 * k + 3.0)));
        }
        c2 = 0.5 * a;
        c3 = b * (1.0 / 6.0);
    } else if (z > 0.0) {
        const double w = sqrt(z);
        const double sh = sin(0.5 * w);
        c2 = (2.0 * sh * sh) / z;
        c3 = (w - sin(w)) / (z * w);
    } else {
        const double w = sqrt(-z);
        const double sh = sinh(0.5 * w);
        c2 = (2.0 * sh * sh) / (-z);
        c3 = (sinh(w) - w) / (-z * w);
    }
}

// Advances (r, v) in place; returns false when |r| = 0 or the input is not finite.
CC_KEPLER_FN bool kepler_flow(double mu, double &rx, double &ry, double &rz, double &vx, double &vy, double &vz,
                                  double t)
{
    const double r0 = sqrt(rx * rx + ry * ry + rz * rz);
    if (!(r0 > 0.0) || !isfinite(r0) || !(mu > 0.0)) return false;
    if (t == 0.0) return true;
    const double smu = sqrt(mu);
    const double v2 = vx * vx + vy * vy + vz * vz;
    const double sigma = (rx * vx + ry * vy + rz * vz) / smu;
    const double alpha = 2.0 / r0 - v2 / mu;
    const double one_ar = 1.0 - alpha * r0;
    if (alpha > 0.0) {
        const double twopi = 6.283185307179586476925286766559;
        const double period = twopi / sqrt(mu * alpha * alpha * alpha);
        t = fmod(t, period);
        if (t < 0.0) t += period;  // a bound orbit: reduced into [0, period)
    }
    const double st = smu * t;
    // F is increasing (F' = r > 0), so every iterate also narrows a bracket
    // [lo, hi] of the root, and a step that leaves it is replaced by
    // bisection.  Bracket: within one period for a bound orbit after the
    // reduction; otherwise from the hyperbolic estimate (Vallado) outwards,
    // never past |x| sqrt(-alpha) = 700 where cosh and sinh would overflow.
    double lo = 0.0, hi = 0.0, x;
    const auto Fx = [&](double xx) {
        double a2, a3;
        stumpff(alpha * xx * xx, a2, a3);
        const double v = ((sigma * xx * xx) * a2 + (one_ar * xx * xx * xx) * a3) + r0 * xx - st;
        return isfinite(v) ? v : (xx > 0.0 ? HUGE_VAL : -HUGE_VAL);
    };
    if (alpha > 0.0) {
        hi = 6.283185307179586476925286766559 / sqrt(alpha);
        x = st * alpha;
    } else {
        double guess = st / r0;
        if (alpha < 0.0) {
            const double a = 1.0 / alpha;
            const double sg = t >= 0.0 ? 1.0 : -1.0;
            const double arg = (-2.0 * mu * alpha * t) / (sigma * smu + sg * sqrt(-mu * a) * (1.0 - r0 * alpha));
            if (arg > 0.0 && isfinite(arg)) guess = sg * sqrt(-a) * log(arg);
        }
        const double cap = alpha < 0.0 ? 700.0 / sqrt(-alpha) : HUGE_VAL;
        double ag = fmin(fabs(guess) > 0.0 ? fabs(guess) : 1.0 / r0, cap);
        for (int k = 0; k < 2100; ++k) {
            const double fv = Fx(t >= 0.0 ? ag : -ag);
            if ((t >= 0.0 ? fv >= 0.0 : fv <= 0.0) || ag >= cap) break;
            ag = fmin(2.0 * ag, cap);
        }
        if (t >= 0.0) hi = ag;
        else lo = -ag;
        x = guess;
    }
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    double c2 = 0.5, c3 = 1.0 / 6.0, z = 0.0;
    for (int it = 0; it < 200; ++it) {
        z = alpha * x * x;
        stumpff(z, c2, c3);
        double F = ((sigma * x * x) * c2 + (one_ar * x * x * x) * c3) + r0 * x - st;
        if (!isfinite(F)) F = x > 0.0 ? HUGE_VAL : -HUGE_VAL;
        if (F > 0.0) hi = x;
        else lo = x;
        const double F1 = (sigma * x) * (1.0 - z * c3) + (one_ar * x * x) * c2 + r0;
        const double F2 = sigma * (1.0 - z * c2) + (one_ar * x) * (1.0 - z * c3);
        const double disc = sqrt(fabs(16.0 * F1 * F1 - 20.0 * F * F2));
        const double den = F1 + (F1 >= 0.0 ? disc : -disc);
        double xn = x - 5.0 * F / den;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        const double dx = xn - x;
        x = xn;
        if (fabs(dx) <= 1e-15 * fabs(x) + 1e-300 || hi - lo <= 4e-16 * fabs(x)) break;
    }
    z = alpha * x * x;
    stumpff(z, c2, c3);
    const double f = 1.0 - (x * x / r0) * c2;
    const double g = t - (x * x * x / smu) * c3;
    const double nx = f * rx + g * vx, ny = f * ry + g * vy, nz = f * rz + g * vz;
    const double rn = sqrt(nx * nx + ny * ny + nz * nz);
    const double fd = (smu / (rn * r0)) * x * (z * c3 - 1.0);
    const double gd = 1.0 - (x * x / rn) * c2;
    const double nvx = fd * rx + gd * vx, nvy = fd * ry + gd * vy, nvz = fd * rz + gd * vz;
    rx = nx; ry = ny; rz = nz;
    vx = nvx; vy = nvy; vz = nvz;
    return isfinite(rn) && rn > 0.0;
}

}  // namespace cck
