// Host build of the device FP32 edge screen, for checking on the CPU that every
// decision it takes equals the literal FP64 edge test of the oracle.  The
// hardware reciprocal and square root are stood in for by correctly rounded
// ones pushed by up to two units in the last place, the direction drawn from
// the argument's bits: the screen's error budget must absorb that.
#include <math.h>
#include <stdint.h>
#include <string.h>

static inline float push_ulps(float v, float x)
{
    uint32_t b;
    memcpy(&b, &x, sizeof b);
    b ^= b >> 13;
    b *= 0x5bd1e995u;
    b ^= b >> 15;
    const int k = (int)(b % 5u) - 2;  // -2 .. 2 units
    for (int i = 0; i < k; ++i) v = nextafterf(v, INFINITY);
    for (int i = 0; i > k; --i) v = nextafterf(v, -INFINITY);
    return v;
}
static inline float rcp_approx(float x) { return push_ulps(1.0f / x, x); }
static inline float sqrt_approx(float x) { return x > 0.0f ? push_ulps(sqrtf(x), x) : sqrtf(x); }

#define CC_SCREEN32_FN static inline
#define CC_SCREEN32_RCP(x) rcp_approx(x)
#define CC_SCREEN32_SQRT(x) sqrt_approx(x)
#include "../paper_1407_7105_amd/csrc/cc_screen32.h"

extern "C" void screen32_pairs(const double *x, const double *y, const double *z, const double *vx,
                               const double *vy, const double *vz, const double *m, const int32_t *pi,
                               const int32_t *pj, int64_t npairs, const double *h, double eta, double eps2,
                               double G, int32_t *out)
{
    for (int64_t k = 0; k < npairs; ++k) {
        const int i = pi[k], j = pj[k];
        // the same FP64 differences the device edge test forms, and the
        // parameters rounded to FP32 as the device does
        ccs::ScreenParams32 q;
        q.eta = (float)eta;
        q.half_eta = (float)(0.5 * eta);
        q.eps2 = (float)eps2;
        q.G = (float)G;
        q.h = (float)h[k];
        out[k] = ccs::edge_screen32(x[i] - x[j], y[i] - y[j], z[i] - z[j], vx[i] - vx[j], vy[i] - vy[j],
                                    vz[i] - vz[j], m[i] + m[j], q);
    }
}
