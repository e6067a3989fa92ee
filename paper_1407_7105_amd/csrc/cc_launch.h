// cc_launch.h -- host-side launchers of the kernels in cc_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "cc_device.h"

namespace ccg {

// Segment list of one grid level, already on the device.
struct GridLevelArgs {
    const Seg *seg;
    const int32_t *chunk_off;  // prefix over ceil(n/256) slot chunks, nseg+1
    const int32_t *tile_off;   // prefix over the sweep's triangular 64x64 tiles, nseg+1
    const int32_t *act_off;    // prefix over n, nseg+1
    int nseg, nchunks, ntiles, nact;
    int32_t epoch;             // marks this visit's not-a-star flags (no clearing between visits)
};

struct ListArgs {
    Seg *pairs;
    Seg *small[4];
    Seg *big;
    int32_t *count;  // [0] pairs, [1..4] small bins, [5] big
    int32_t cap_pairs, cap_small, cap_big;
    int32_t small_max;
    int32_t bin_lim[3];
    int32_t *labp;   // optional permuted-order labels
    uint8_t *singp;  // optional permuted-order singleton flags
    const int32_t *errf;  // error bits, snapshot into count[7]
    const int32_t *notstar;  // not-a-star flags: star segments are counted into count[6]
};

struct SmallArgs {
    const Seg *pairs;      // two-particle components
    const Seg *bin[4];     // other on-chip components by size bin
    const int32_t *count;  // [0] pairs, [1..4] bins
    int32_t cap, cap_pairs;
    int32_t *queue;        // 3 ints, 0 before a launch: workgroup and wavefront queue heads, blocks finished
};

hipError_t launch_validate(const double *x, const double *y, const double *z, const double *vx, const double *vy,
                           const double *vz, const double *m, int64_t n, int32_t *err, hipStream_t st);
hipError_t launch_pair_tau(SoA S, const int32_t *pi, const int32_t *pj, int64_t npairs, double *out, DevParams p,
                           hipStream_t st);
hipError_t launch_drift_mask(SoA S, int64_t n, const uint8_t *mask, double h, hipStream_t st);
hipError_t launch_iota(int32_t *a, int64_t n, hipStream_t st);
hipError_t launch_fill_i32(int32_t *a, int64_t n, int32_t v, hipStream_t st);

// Union-find reset of slots [0, n) (parent[u] = u, cnt[u] = 0).
hipError_t launch_uf_init(int32_t *parent, int32_t *cnt, int n, hipStream_t st);
// screen32: FP32 screen in front of the FP64 one (the template flag MIXED of
// the kernels' edge test); split_tiles: launches of at most this many tiles
// take one block per tile
// (the pairs it evaluates are counted by launch_label)
hipError_t launch_sweep(SoA S, const GridLevelArgs &a, int32_t *notstar, int32_t *parent, DevParams p, double h,
                        bool screen32, int split_tiles, bool star_pass, int32_t *err, hipStream_t st);
// star test of every segment from its first slot (sets notstar for the
// segments that are not fully connected)
hipError_t launch_star(SoA S, const GridLevelArgs &a, int32_t *notstar, DevParams p, double h, bool screen32,
                       uint64_t *stats, uint64_t *fam, hipStream_t st);
// labels and component sizes; with keys/vals the sort keys of the active
// particles, with count the work-list counters cleared
// Labels and component sizes after a sweep; also counts the pairs the sweep
// evaluated (per segment: all of them, unless star_pass skipped a star set)
// into stats and sweep_fam.
hipError_t launch_label(const GridLevelArgs &a, const int32_t *notstar, int32_t *parent, int32_t *label, int32_t *cnt,
                        uint32_t *keys, uint32_t *vals, int32_t *count, int32_t *hold, bool star_pass,
                        uint64_t *stats, uint64_t *sweep_fam, int32_t *err, hipStream_t st);
// HOLD split: merge the non-trivial components of every segment into one set
// F (labels, sort keys and the size of F; hold: 2 ints per segment, prepared
// by launch_label)
hipError_t launch_hold(const GridLevelArgs &a, int32_t *label, int32_t *cnt, uint32_t *keys, int32_t *hold,
                       hipStream_t st);
size_t sort_temp_bytes(int n);
hipError_t launch_sort(void *temp, size_t temp_bytes, const uint32_t *keys_in, uint32_t *keys_out,
                       const uint32_t *vals_in, uint32_t *vals_out, int n, int end_bit, hipStream_t st);
// Between the two working buffers.  forward (inverse == false):
// to[act(k)] <- from[src[k]]; with `lab` (sorted labels), also the entry-order
// singleton flags, with `lists` the component work lists, with drift_hh > 0
// the singletons' drift, with count_kick the pairs the level's tiled kick
// will kick (stats and kick_fam).  Forward resets the union-find of the slots
// (parent and cnt_next) for the next level.  inverse: to[src[k]] <- from[act(k)].
hipError_t launch_permute(SoA from, SoA to, const GridLevelArgs &a, const uint32_t *src, const uint32_t *lab,
                          const int32_t *cnt, uint8_t *sing, const ListArgs *lists, double drift_hh,
                          int32_t *parent, int32_t *cnt_next, uint64_t *kick_fam, bool count_kick, uint64_t *stats,
                          bool inverse, hipStream_t st);
hipError_t launch_drift_seg(SoA W, const GridLevelArgs &a, const uint8_t *sing, double hh, uint64_t *stats,
                            hipStream_t st);
hipError_t launch_kick_seg(SoA W, const GridLevelArgs &a, const int32_t *label, double h, double eps2, double G,
                           int32_t *err, uint64_t *stats, uint64_t *fam, hipStream_t st);
// kick K_h of the level, then the drift D_{h/2} of its singletons (singp)
// Tiled kick of a level (blocks listed by the host, see KickBlock), the group
// sums (KickJob) and the combine that applies the kick with the singletons'
// closing drift.
hipError_t launch_kick_tiles(SoA W, const GridLevelArgs &a, const KickBlock *blk, int nblk, const KickJob *jobs,
                             int njobs, const KickTile *ktile, const int32_t *labp, const uint8_t *singp, double h,
                             double eps2, double G, bool mixed, double *part, int32_t *parent, int32_t *cnt_next,
                             int32_t *err, uint64_t *stats, hipStream_t st);
// cc_kick's sums into separate arrays (mixed: FP32 pair forces, Kahan per tile)
hipError_t launch_kick_all(SoA W, int n, const int32_t *label, double eps2, double G, bool mixed, double *ax,
                           double *ay, double *az, int32_t *err, hipStream_t st);
hipError_t launch_apply_kick(SoA W, int n, const double *ax, const double *ay, const double *az, double h,
                             hipStream_t st);
// One launch for a level's on-chip components: nbp blocks of two-particle
// components (one per thread), nbb blocks of bins 2-3 (one per workgroup,
// cap = largest size), nbw blocks of bins 0-1 (one per wavefront).
// mode: 0 = FP64 slot order, 1 = FP64 ascending index order, 2 = mixed.
size_t items_lds_bytes(int cap);
// sets the kernel's LDS limit (host-side, once per process); launch_items does
// it on first use, a graph capture needs it done before
hipError_t configure_items(int cap, int mode);
hipError_t launch_items(SoA W, const SmallArgs &s, int cap, int mode, int nbp, int nbb, int nbw, double H,
                        DevParams p, int32_t *err, uint64_t *stats, uint64_t *fam, hipStream_t st);
int diag_blocks(int n);

// Static scratch of cc_kick_static (cc_static.hip): 3 x CC_KICK_STATIC_MAX_N
// doubles of acceleration sums, then the error flag.
constexpr size_t STATIC_ACC_BYTES = (size_t)3 * 65536 * sizeof(double);
// With device `dev` current: look up (once per device) the scratch array's
// device address.  cc_create calls it.
hipError_t static_scratch_setup(int dev);
// The scratch address on device `dev` (nullptr if never set up).
void *static_scratch(int dev);
hipError_t launch_diag(SoA S, int n, double eps2, double G, double *part, double *out, hipStream_t st);

}  // namespace ccg
