// cc_screen32.h -- FP32 screen for the edge test tau(i,j) < h (eq. 20 with
// the symmetrised pair time step of eq. 19), in front of the FP64 screen on
// the mixed-precision path.  Its answer, when it gives one, equals that of the
// literal FP64 evaluation; otherwise SCREEN32_UNSURE.
//
// Host-compilable: the including file defines CC_SCREEN32_FN and, for a host
// build, CC_SCREEN32_RCP / CC_SCREEN32_SQRT (the hardware reciprocal and
// square root on the device).
#pragma once

#ifndef CC_SCREEN32_FN
#define CC_SCREEN32_FN static inline
#endif
#ifndef CC_SCREEN32_RCP
#define CC_SCREEN32_RCP(x) __builtin_amdgcn_rcpf(x)
#endif
#ifndef CC_SCREEN32_SQRT
#define CC_SCREEN32_SQRT(x) __builtin_amdgcn_sqrtf(x)
#endif
// a term is decided only when it clears the threshold by this many times its
// error bound
#ifndef CC_SCREEN32_SLACK
#define CC_SCREEN32_SLACK 2.0f
#endif

namespace ccs {

// ---------------------------------------------------------------------------
// Mixed-precision edge test (same decision as edge_pair, exactly).
//
// The FP64 coordinate differences are rounded to FP32 and tau's two
// symmetrised terms are formed in FP32 with the hardware reciprocal and square
// root, together with a bound on their error relative to the FP64 values of
// edge_pair (u = 2^-24; the reciprocal/root instructions are budgeted at 8u,
// several times their specified accuracy; every other operation at u):
//   r^2, |u|^2:     6u relative        q.u:  6u r|u| absolute
//   t_ff:           26u relative       t_ff': 48u|t_ff'| + 10u t_ff |u|/r
//   t_fb:           36u relative       t_fb': (1+w)(6u + 72u|c|), c = q.u/(r|u|),
//                                             w = mu/(r|u|^2)
//   1 - eta t'/2:   (eta/2) E(t') + 2u (1 + (eta/2)|t'|)
//   eta t / d:      e = 50u + E(d) / (d - E(d))      (when d - E(d) > 0)
// A term is decided when s(1+2e) < h (edge), s(1-2e) > h (no edge from it),
// or d + E(d) <= 0 (no bound); anything else, and any input outside a range in
// which no FP32 intermediate can leave the normal range, returns SCREEN_UNSURE
// and the caller evaluates edge_pair.
// ---------------------------------------------------------------------------
enum { SCREEN32_NO = 0, SCREEN32_EDGE = 1, SCREEN32_UNSURE = 2 };

struct ScreenParams32 {
    float eta, half_eta, eps2, G, h;
};

CC_SCREEN32_FN float frcp(float x) { return CC_SCREEN32_RCP(x); }
CC_SCREEN32_FN float fsqrt(float x) { return CC_SCREEN32_SQRT(x); }

// decided term: 0 = >= h or unbounded, 1 = < h, 2 = unsure
CC_SCREEN32_FN int screen_term(float t, float et, float d, float Ed, float eta, float h)
{
    const float U = 5.9604645e-8f;  // 2^-24
    if (d + Ed <= 0.0f) return 0;    // denominator certainly not positive: no bound
    const float dl = d - Ed;
    if (!(dl > 0.0f)) return 2;
    const float s = eta * t * frcp(d);
    const float e = et + 12.0f * U + Ed * frcp(dl) * 1.0001f;
    if (!(e < 0.05f)) return 2;
    if (s * (1.0f + CC_SCREEN32_SLACK * e) < h) return 1;
    if (s * (1.0f - CC_SCREEN32_SLACK * e) > h) return 0;
    return 2;
}

CC_SCREEN32_FN int edge_screen32(double ddx, double ddy, double ddz, double ddvx, double ddvy,
                                             double ddvz, double msum, const ScreenParams32 &q)
{
    const float U = 5.9604645e-8f;  // 2^-24
    const float x = (float)ddx, y = (float)ddy, z = (float)ddz;
    const float vx = (float)ddvx, vy = (float)ddvy, vz = (float)ddvz;
    const float r2 = __builtin_fmaf(x, x, __builtin_fmaf(y, y, __builtin_fmaf(z, z, q.eps2)));
    const float v2 = __builtin_fmaf(vx, vx, __builtin_fmaf(vy, vy, vz * vz));
    const float rv = __builtin_fmaf(x, vx, __builtin_fmaf(y, vy, z * vz));
    const float mu = q.G * (float)msum;
    // ranges that keep every intermediate below normal FP32 limits
    if (!(r2 > 1e-16f && r2 < 1e16f) || !(mu > 1e-12f && mu < 1e12f) || !(v2 < 1e16f)) return SCREEN32_UNSURE;
    const float r = fsqrt(r2);
    const float tff = fsqrt(r2 * r * frcp(mu));
    const float dtff = ((1.5f * tff) * rv) * frcp(r2);
    const float vmag = fsqrt(v2);
    const float adff = __builtin_fabsf(dtff);
    const float E_dtff = 1.01f * (48.0f * U * adff + 10.0f * U * tff * vmag * frcp(r));
    const float dff = __builtin_fmaf(-q.half_eta, dtff, 1.0f);
    const float E_dff = q.half_eta * E_dtff + 2.0f * U * (1.0f + q.half_eta * adff);
    const int aff = screen_term(tff, 26.0f * U, dff, E_dff, q.eta, q.h);
    if (aff == 1) return SCREEN32_EDGE;
    int afb;
    if (v2 == 0.0f) {
        // no fly-by bound only if the FP64 relative velocity is exactly zero
        if (ddvx != 0.0 || ddvy != 0.0 || ddvz != 0.0) return SCREEN32_UNSURE;
        afb = 0;
    } else {
        if (!(v2 > 1e-16f)) return SCREEN32_UNSURE;
        const float tfb = r * frcp(vmag);
        const float irv = frcp(r * vmag);
        const float c = rv * irv;
        const float w = mu * frcp(r * v2);
        const float dtfb = c * (1.0f + w);
        const float ac = __builtin_fabsf(c);
        const float E_dtfb = 1.01f * (1.0f + w) * (6.0f * U + 72.0f * U * ac);
        const float dfb = __builtin_fmaf(-q.half_eta, dtfb, 1.0f);
        const float E_dfb = q.half_eta * E_dtfb + 2.0f * U * (1.0f + q.half_eta * __builtin_fabsf(dtfb));
        afb = screen_term(tfb, 36.0f * U, dfb, E_dfb, q.eta, q.h);
        if (afb == 1) return SCREEN32_EDGE;
    }
    return (aff == 0 && afb == 0) ? SCREEN32_NO : SCREEN32_UNSURE;
}

}  // namespace ccs
