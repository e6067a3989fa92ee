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

}  // namespace cct
