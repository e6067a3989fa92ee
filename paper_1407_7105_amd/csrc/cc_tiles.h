// cc_tiles.h -- index arithmetic of the all-pairs sweep's triangular tile grid
// (also built for the host by a test).
//
// A set of n particles is cut into T = ceil(n / 64) tiles per side; the sweep
// visits the upper triangle (ti <= tj) of the T x T grid, one tile per
// wavefront, numbered row by row.  The including file supplies the
// CC_TILES_FN qualifiers.
#pragma once

#include <stdint.h>

#ifndef CC_TILES_FN
#error "define CC_TILES_FN (function qualifiers) before including cc_tiles.h"
#endif

namespace cct {

// Tile t (0-based) of the triangle: row ti holds the T - ti tiles
// (ti, ti..T-1), so the rows before ti hold B(ti) = ti T - ti (ti - 1) / 2
// tiles and ti is the largest r with B(r) <= t.  The root of the quadratic
// gives r up to the rounding of its square root; whole steps correct it.
// Constant time: a row-by-row walk would take O(T) steps per tile.
CC_TILES_FN void tri_tile(int T, int t, int &ti, int &tj)
{
    const double b = 2.0 * T + 1.0;
    int64_t r = (int64_t)((b - __builtin_sqrt(b * b - 8.0 * (double)t)) * 0.5);
    if (r < 0) r = 0;
    if (r > T - 1) r = T - 1;
    while (r > 0 && r * T - r * (r - 1) / 2 > t) --r;
    while (r < T - 1 && (r + 1) * T - (r + 1) * r / 2 <= t) ++r;
    ti = (int)r;
    tj = ti + (int)(t - (r * T - r * (r - 1) / 2));
}

// Blocked order of the same triangle, for grids of at least BLOCKED_MIN_T
// tiles per side (smaller sets, up to 32 768 particles, keep their whole
// state in one L2 in any order and take the row-by-row one, whose decode is
// cheaper): the grid is cut into super-tiles of S x S tiles (the last super-row and
// super-column w = T - (U-1) S wide, U = ceil(T / S)), visited row by row in
// the upper triangle of the U x U super-grid, and each super-tile's tiles row
// by row (a diagonal super-tile only its upper triangle).  Consecutive tiles
// then share their 2 S tile rows and columns (S = 16: 2048 particles, 115 KB
// of state), which stay in the L2 of the XCD that runs them.
//   Super-row I < U-1 holds A + (U-2-I) S^2 tiles, A = S (S+1) / 2 + S w, so
// the super-rows before I hold C(I) = I A + S^2 (I (U-2) - I (I-1) / 2)
// tiles; I is the largest r with C(r) <= t (root of the quadratic, corrected
// by whole steps as in tri_tile).
constexpr int SUPER = 16;
constexpr int BLOCKED_MIN_T = 512;

CC_TILES_FN void blocked_tile(int T, int t, int &ti, int &tj)
{
    if (T < BLOCKED_MIN_T) {
        tri_tile(T, t, ti, tj);
        return;
    }
    const int64_t S = SUPER;
    const int64_t U = (T + S - 1) / S;
    const int64_t w = T - (U - 1) * S;
    const int64_t S2 = S * S;
    const int64_t A = S * (S + 1) / 2 + S * w;
    auto C = [&](int64_t r) -> int64_t { return r * A + S2 * (r * (U - 2) - r * (r - 1) / 2); };
    // C(r) = -(S^2/2) r^2 + (A + S^2 (U - 2) + S^2/2) r: the larger root of
    // C(r) = t is beyond the range; the smaller one is the estimate
    const double a = 0.5 * (double)S2, bq = (double)A + (double)S2 * ((double)U - 1.5);
    const double disc = bq * bq - 4.0 * a * (double)t;
    int64_t I = (int64_t)((bq - __builtin_sqrt(disc > 0.0 ? disc : 0.0)) / (2.0 * a));
    if (I < 0) I = 0;
    if (I > U - 1) I = U - 1;
    while (I > 0 && C(I) > t) --I;
    while (I < U - 1 && C(I + 1) <= t) ++I;
    int64_t r = t - C(I);
    const int64_t sI = (I == U - 1) ? w : S;
    const int64_t diag = sI * (sI + 1) / 2;
    if (r < diag) {
        int a0, b0;
        tri_tile((int)sI, (int)r, a0, b0);
        ti = (int)(I * S) + a0;
        tj = (int)(I * S) + b0;
        return;
    }
    r -= diag;
    const int64_t q = r / S2;          // full-width super-tiles before this one
    const int64_t J = I + 1 + q;
    const int64_t rr = r - q * S2;
    const int64_t sJ = (J == U - 1) ? w : S;
    ti = (int)(I * S + rr / sJ);
    tj = (int)(J * S + rr % sJ);
}

}  // namespace cct
