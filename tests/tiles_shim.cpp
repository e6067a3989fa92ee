// Host build of the sweep's tile-index arithmetic, for checking it on the CPU.
#define CC_TILES_FN static inline
#include "../paper_1407_7105_amd/csrc/cc_tiles.h"

#include <stdint.h>

// For every t in [t0, t0 + count): out[2k], out[2k+1] = (ti, tj) of tile t0 + k.
extern "C" void tri_tiles(int T, int64_t t0, int64_t count, int32_t *out)
{
    for (int64_t k = 0; k < count; ++k) {
        int ti, tj;
        cct::tri_tile(T, (int)(t0 + k), ti, tj);
        out[2 * k] = ti;
        out[2 * k + 1] = tj;
    }
}

// The same in the blocked order.
extern "C" void blocked_tiles(int T, int64_t t0, int64_t count, int32_t *out)
{
    for (int64_t k = 0; k < count; ++k) {
        int ti, tj;
        cct::blocked_tile(T, (int)(t0 + k), ti, tj);
        out[2 * k] = ti;
        out[2 * k + 1] = tj;
    }
}
