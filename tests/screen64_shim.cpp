// Host build of the device FP64 edge screen, for checking on the CPU that every
// decision it takes equals the literal FP64 edge test of the oracle.
#define CC_SCREEN64_FN static inline
// a deliberately coarse reciprocal square root (about 2^-23, like a hardware
// seed): the screen must certify its refined roots by itself
#define CC_SCREEN64_RSQ(x) ((double)(1.0f / __builtin_sqrtf((float)(x))))
#include "../paper_1407_7105_amd/csrc/cc_screen64.h"

#include <stdint.h>

extern "C" void screen64_pairs(const double *x, const double *y, const double *z, const double *vx,
                               const double *vy, const double *vz, const double *m, const int32_t *pi,
                               const int32_t *pj, int64_t npairs, const double *h, double eta, double eps2,
                               double G, int32_t *out)
{
    for (int64_t k = 0; k < npairs; ++k) {
        const int i = pi[k], j = pj[k];
        // the same rounded inputs the device edge test forms
        const double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
        const double dvx = vx[i] - vx[j], dvy = vy[i] - vy[j], dvz = vz[i] - vz[j];
        const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
        const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
        const double rv = (dx * dvx + dy * dvy) + dz * dvz;
        const double mu = G * (m[i] + m[j]);
        const ccs::Screen64 s = ccs::screen64_params(eta, h[k]);
        out[k] = ccs::screen64(r2, v2, rv, mu, s);
    }
}

// Far-pair test: 1 when it certifies "no edge", 0 when it leaves the pair to the screen.
extern "C" void far64_pairs(const double *x, const double *y, const double *z, const double *vx, const double *vy,
                            const double *vz, const double *m, const int32_t *pi, const int32_t *pj, int64_t npairs,
                            const double *h, double eta, double eps2, double G, int32_t *out)
{
    for (int64_t k = 0; k < npairs; ++k) {
        const int i = pi[k], j = pj[k];
        const double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
        const double dvx = vx[i] - vx[j], dvy = vy[i] - vy[j], dvz = vz[i] - vz[j];
        const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
        const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
        const double mu = G * (m[i] + m[j]);
        out[k] = ccs::far64(r2, v2, mu, ccs::far64_params(eta, h[k])) ? 1 : 0;
    }
}

// The sweep's form of the far-pair test: both particles checked against the
// box once, r^2 and |u|^2 by fused multiply-adds, mu = G m_i + G m_j; a pair
// outside the box is left to the screen (0).
extern "C" void far64b_pairs(const double *x, const double *y, const double *z, const double *vx, const double *vy,
                             const double *vz, const double *m, const int32_t *pi, const int32_t *pj, int64_t npairs,
                             const double *h, double eta, double eps2, double G, int32_t *out)
{
    for (int64_t k = 0; k < npairs; ++k) {
        const int i = pi[k], j = pj[k];
        const double gi = G * m[i], gj = G * m[j];
        const ccs::Far64 f = ccs::far64_params(eta, h[k]);
        const bool box = f.on && eps2 <= 0x1p98 && ccs::far64_in_box(x[i], y[i], z[i], vx[i], vy[i], vz[i], gi) &&
                         ccs::far64_in_box(x[j], y[j], z[j], vx[j], vy[j], vz[j], gj);
        out[k] = (box && ccs::far64_boxed(x[i] - x[j], y[i] - y[j], z[i] - z[j], vx[i] - vx[j], vy[i] - vy[j],
                                          vz[i] - vz[j], gi + gj, eps2, f)) ? 1 : 0;
    }
}
