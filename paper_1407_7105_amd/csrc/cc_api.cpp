// cc_api.cpp -- host runtime and C ABI of the CC integrator (include/cc.h).
//
// cc_evolve keeps a working copy of the state.  One global step runs
// evolve_cc(all, dt) (Fig. 2):
//   * sets larger than the on-chip limit are split by grid-wide kernels
//     (all-pairs sweep with union-find that also takes the star test, labels,
//     a stable sort by label that makes every component contiguous), their
//     sub-components are evolved for h/2 -- two-particle ones by the pair
//     kernel, small ones by the on-chip kernel, large ones by recursing here
//     -- and the level's drift/kick/drift runs between the two halves;
//   * every level restores its entry slot order before it returns, so each
//     set is always visited in ascending particle index and every kick sums
//     its partners in the same order as a sequential i<j sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cc.h"
#include "cc_device.h"
#include "cc_launch.h"

using namespace ccg;

namespace {

constexpr int TPB = 256;
constexpr int DEFAULT_SMALL_MAX = 128;  // the autotuner's choice on the 16 384-body workload
constexpr int kLevels = 64;  // grid recursion levels a context can hold (max_depth <= 60)
#ifndef CC_SIDE_STREAMS
#define CC_SIDE_STREAMS 3
#endif
constexpr int kSide = CC_SIDE_STREAMS;  // side streams for the on-chip launches (with the main one: 4 hardware queues)
constexpr int SWEEP_TILE = 64;  // edge of the all-pairs sweep tiles
constexpr int32_t DEFAULT_SWEEP_SPLIT = 2048;
constexpr int32_t DEFAULT_KICK_GROUPS = 32;

// kernel families for timing
enum Fam { F_SWEEP, F_LABEL, F_SORT, F_PERMUTE, F_DRIFT, F_KICK, F_PAIRS, F_SMALL, F_VALIDATE, F_OTHER, F_N };
const char *fam_name[F_N] = {"sweep", "label", "sort", "permute", "drift",
                             "kick", "pairs", "small", "validate", "other"};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Level {
    size_t cap_n = 0, cap_seg = 0;
    int32_t *label = nullptr;
    uint8_t *sing = nullptr;
    int32_t *labp = nullptr;   // label of the particle at each slot, component-contiguous order
    uint8_t *singp = nullptr;  // singleton flag, component-contiguous order
    uint32_t *src = nullptr;
    Seg *pairs = nullptr;
    Seg *small[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *notstar = nullptr;  // cap_seg: epoch of the visit that found the set not to be a star
    int32_t *hold = nullptr;     // 2 x cap_seg: the HOLD split's label of F and its size per segment
    bool star_hint = false;      // the last visit found a star set: test for stars before sweeping
    // Report block, read back with one copy per visit: count[8] ([0] pairs,
    // [1..4] small bins, [5] big, [6] star segments, [7] error bits) followed
    // by the big list.
    int32_t *rep = nullptr, *h_rep = nullptr;
    int32_t *count = nullptr, *h_count = nullptr;
    Seg *big = nullptr, *h_big = nullptr;
    // Descriptor block, uploaded with one copy per visit: nseg segments
    // followed by 3 arrays of nseg+1 ints (chunk, tile and slot prefixes).
    unsigned char *desc = nullptr, *h_desc = nullptr;
    Seg *seg = nullptr, *h_seg = nullptr;
    int32_t *offs = nullptr, *h_offs = nullptr;
    // Kick list, uploaded once the level's components are known: one
    // KickTile per i tile, the KickBlocks, the KickJobs.  kick_ev marks the end
    // of the last upload from h_kick, which the next visit must not overwrite
    // before.
    unsigned char *kick = nullptr, *h_kick = nullptr;
    size_t cap_kick = 0;  // bytes
    hipEvent_t kick_ev = nullptr;
    bool kick_pending = false;
    int cap_big = 0, cap_small = 0, cap_pairs = 0;
};

struct TimedRec {
    int fam;
    hipEvent_t a, b;
};

}  // namespace

struct cc_ctx {
    int device = 0;
    cc_params params{};
    std::string err;
    hipStream_t st = nullptr;
    // default priority: a level's on-chip components beside the recursion,
    // level k on side[k % kSide] (a deeper level's launch need not queue
    // behind a long launch of a shallower one)
    hipStream_t side[kSide] = {};
    std::vector<hipEvent_t> sync_pool;     // ordering events (no timing)
    std::vector<hipEvent_t> sync_used;
    int cus = 256;
    size_t cap = 0;
    size_t cap_cl = 0;
    // working state
    double *w[7] = {};
    int32_t *orig = nullptr;
    double *snap[6] = {};
    double *tmp[7] = {};
    int32_t *tmp_orig = nullptr;
    uint32_t *keys = nullptr, *keys_out = nullptr, *vals = nullptr;
    void *sort_temp = nullptr;
    size_t sort_bytes = 0;
    int32_t *parent = nullptr, *cnt = nullptr;
    uint64_t *stats = nullptr;
    uint64_t *h_stats = nullptr;
    int32_t *errf = nullptr;
    int32_t *h_err = nullptr;
    int32_t *qhead = nullptr;    // per level: head and blocks finished of the workgroup and the wavefront queues
    int32_t epoch = 0;           // visit counter for the non-star flags
    int32_t sweep_split = DEFAULT_SWEEP_SPLIT;  // sweep launches up to this many tiles: one block per tile
    int32_t kick_groups = DEFAULT_KICK_GROUPS;  // kick launches aim at this many blocks per compute unit
    double *kick_acc = nullptr;  // 3*cap for cc_kick
    double *kick_part = nullptr; // partial accelerations of the tiled kick
    size_t kick_part_cap = 0;    // in kick blocks
    std::vector<int32_t> kick_scratch;  // host scratch of the kick-list builder
    // A level's on-chip launch waiting for its child level's first sweep to
    // be queued (see dispatch_sets)
    struct Deferred {
        bool on = false;
        int k = 0;
        double H = 0.0;
        int n_pairs = 0;
        int n_small[4] = {0, 0, 0, 0};
        hipStream_t sd = nullptr;
        hipEvent_t done = nullptr;
    } deferred;
    double *diag_part = nullptr;
    size_t diag_cap = 0;
    double *diag_out = nullptr, *h_diag = nullptr;
    std::vector<Level> levels;
    // timing
    bool timing = false;
    std::vector<TimedRec> recs;
    std::vector<hipEvent_t> ev_pool;
    double fam_ms[F_N] = {};
    uint64_t fam_launch[F_N] = {};
    uint64_t *fam_work = nullptr;  // device counters [F_N][2] (tau pairs, kick pairs)
};

namespace {

int fail(cc_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(c, e_ == hipErrorOutOfMemory ? CC_ERR_OOM : CC_ERR_DEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                         \
    } while (0)

#define RC(expr)                 \
    do {                         \
        int r_ = (expr);         \
        if (r_ != CC_OK) return r_; \
    } while (0)

DevParams dev_params(const cc_ctx *c)
{
    DevParams p{};
    p.eta = c->params.eta;
    p.eps2 = c->params.eps2;
    p.G = c->params.G;
    p.max_depth = c->params.max_depth;
    p.kepler = c->params.kepler;
    p.hold = c->params.hold;
    return p;
}

// Largest set integrated on chip; 1 in plain mode, where every set of two or
// more bodies takes the grid-wide kernels.
int small_max_of(const cc_params &p) { return p.plain ? 1 : (p.small_max > 0 ? p.small_max : DEFAULT_SMALL_MAX); }
int small_max(const cc_ctx *c) { return small_max_of(c->params); }

bool mixed(const cc_ctx *c) { return c->params.precision == CC_MIXED; }

// The mixed path sums kicks over parallel tiles; EXACT order applies to FP64.
bool exact_order(const cc_ctx *c) { return !mixed(c) && c->params.kick_order == CC_ORDER_EXACT; }

// FP32 screen in front of the FP64 one in the grid-wide sweep
bool screen32(const cc_ctx *c) { return c->params.screen == CC_SCREEN_FP32; }

int check_params(cc_ctx *c, const cc_params *p)
{
    if (!p) return fail(c, CC_ERR_ARG, "params is NULL");
    if (!(p->eta > 0.0) || !(p->eta <= 1.0)) return fail(c, CC_ERR_ARG, "eta must be in (0, 1]");
    if (!(p->eps2 >= 0.0) || !std::isfinite(p->eps2)) return fail(c, CC_ERR_ARG, "eps2 must be finite and >= 0");
    if (!(p->G > 0.0) || !std::isfinite(p->G)) return fail(c, CC_ERR_ARG, "G must be finite and > 0");
    if (p->max_depth < 0 || p->max_depth > 60) return fail(c, CC_ERR_ARG, "max_depth must be in [0, 60]");
    if (p->precision != CC_FP64 && p->precision != CC_MIXED) return fail(c, CC_ERR_ARG, "unknown precision");
    if (p->small_max != 0 && (p->small_max < 3 || p->small_max > 1024))
        return fail(c, CC_ERR_ARG, "small_max must be 0 or in [3, 1024]");
    if (p->kick_order != CC_ORDER_FAST && p->kick_order != CC_ORDER_EXACT)
        return fail(c, CC_ERR_ARG, "unknown kick_order");
    if (p->screen != CC_SCREEN_FP64 && p->screen != CC_SCREEN_FP32) return fail(c, CC_ERR_ARG, "unknown screen");
    if (p->kepler != 0 && p->kepler != 1) return fail(c, CC_ERR_ARG, "kepler must be 0 or 1");
    if (p->kepler && p->eps2 != 0.0)
        return fail(c, CC_ERR_ARG, "the Kepler solution of two-body components needs eps2 == 0");
    if (p->hold != 0 && p->hold != 1) return fail(c, CC_ERR_ARG, "hold must be 0 or 1");
    if (p->hold && p->kepler) return fail(c, CC_ERR_ARG, "the Kepler option belongs to the CC split, not to HOLD");
    if (p->plain != 0 && p->plain != 1) return fail(c, CC_ERR_ARG, "plain must be 0 or 1");
    if (p->plain && p->kepler)
        return fail(c, CC_ERR_ARG, "the Kepler option runs in the on-chip pair walker, which plain mode leaves out");
    return CC_OK;
}

template <class T>
int dalloc(cc_ctx *c, T **p, size_t count)
{
    if (*p) {
        hipFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    HIPCHK(hipMalloc((void **)p, count * sizeof(T)));
    return CC_OK;
}

template <class T>
int halloc(cc_ctx *c, T **p, size_t count)
{
    if (*p) {
        hipHostFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    HIPCHK(hipHostMalloc((void **)p, count * sizeof(T), hipHostMallocDefault));
    return CC_OK;
}

int ensure_capacity(cc_ctx *c, size_t n, size_t ncl)
{
    if (n > (size_t)0x3FFFFFFF) return fail(c, CC_ERR_ARG, "n = %zu exceeds the supported 2^30", n);
    if (n > c->cap) {
        size_t cap = std::max(n, (size_t)1024);
        for (int a = 0; a < 7; ++a) RC(dalloc(c, &c->w[a], cap));
        for (int a = 0; a < 6; ++a) RC(dalloc(c, &c->snap[a], cap));
        for (int a = 0; a < 7; ++a) RC(dalloc(c, &c->tmp[a], cap));
        RC(dalloc(c, &c->orig, cap));
        RC(dalloc(c, &c->tmp_orig, cap));
        RC(dalloc(c, &c->keys, cap));
        RC(dalloc(c, &c->keys_out, cap));
        RC(dalloc(c, &c->vals, cap));
        RC(dalloc(c, &c->parent, cap * PARENT_STRIDE));  // one entry per 128-byte line
        RC(dalloc(c, &c->cnt, 2 * cap));  // component sizes, one array per level parity
        RC(dalloc(c, &c->kick_acc, 3 * cap));
        size_t sb = sort_temp_bytes((int)cap);
        if (c->sort_temp) hipFree(c->sort_temp);
        c->sort_temp = nullptr;
        HIPCHK(hipMalloc(&c->sort_temp, sb ? sb : 1));
        c->sort_bytes = sb;
        c->cap = cap;
        for (auto &lv : c->levels) lv.cap_n = 0;  // reallocate lazily
    }
    if (ncl > c->cap_cl) {
        size_t cl = std::max(ncl, (size_t)1);
        RC(dalloc(c, &c->stats, cl * ST_N));
        RC(halloc(c, &c->h_stats, cl * ST_N));
        c->cap_cl = cl;
    }
    return CC_OK;
}

int ensure_level(cc_ctx *c, int k, size_t nseg)
{
    if (k >= (int)c->levels.size()) return fail(c, CC_ERR_DEPTH, "grid recursion deeper than %d levels", k);
    Level &lv = c->levels[k];
    const size_t n = c->cap;
    if (lv.cap_n < n) {
        const int sm = small_max(c);
        RC(dalloc(c, &lv.label, n));
        RC(dalloc(c, &lv.sing, n));
        RC(dalloc(c, &lv.labp, n));
        RC(dalloc(c, &lv.singp, n));
        RC(dalloc(c, &lv.src, n));
        // top-level clusters of one particle also enter the small lists, so
        // a list can hold up to n items
        lv.cap_pairs = (int)(n / 2 + 1);
        lv.cap_small = (int)(n + 1);
        lv.cap_big = (int)(n / (size_t)(sm + 1) + 1);
        RC(dalloc(c, &lv.pairs, lv.cap_pairs));
        for (int b = 0; b < 4; ++b) RC(dalloc(c, &lv.small[b], lv.cap_small));
        const size_t rep_ints = 8 + (size_t)lv.cap_big * (sizeof(Seg) / sizeof(int32_t));
        RC(dalloc(c, &lv.rep, rep_ints));
        RC(halloc(c, &lv.h_rep, rep_ints));
        lv.count = lv.rep;
        lv.h_count = lv.h_rep;
        lv.big = reinterpret_cast<Seg *>(lv.rep + 8);
        lv.h_big = reinterpret_cast<Seg *>(lv.h_rep + 8);
        lv.cap_n = n;
    }
    if (lv.cap_seg < nseg) {
        const size_t cs = std::max(nseg, (size_t)64);
        RC(dalloc(c, &lv.notstar, cs));
        RC(dalloc(c, &lv.hold, 2 * cs));
        // no stale flag may equal a later visit's epoch
        HIPCHK(hipMemset(lv.notstar, 0, cs * sizeof(int32_t)));
        const size_t bytes = cs * sizeof(Seg) + 3 * (cs + 1) * sizeof(int32_t);
        RC(dalloc(c, &lv.desc, bytes));
        RC(halloc(c, &lv.h_desc, bytes));
        lv.seg = reinterpret_cast<Seg *>(lv.desc);
        lv.h_seg = reinterpret_cast<Seg *>(lv.h_desc);
        lv.cap_seg = cs;
    }
    return CC_OK;
}

// The two working buffers: a level at grid depth k holds its sets in buffer
// k % 2 and makes their components contiguous in the other one (each
// permutation is one out-of-place launch).  Buffer 0 holds the state between
// steps.
SoA work_soa(cc_ctx *c, int parity)
{
    if (parity & 1) return SoA{c->tmp[0], c->tmp[1], c->tmp[2], c->tmp[3], c->tmp[4], c->tmp[5], c->tmp[6], c->tmp_orig};
    return SoA{c->w[0], c->w[1], c->w[2], c->w[3], c->w[4], c->w[5], c->w[6], c->orig};
}

// Component-size counters of grid depth k (two arrays, by parity: a level
// resets the next level's while it still reads its own).
int32_t *cnt_of(cc_ctx *c, int k) { return c->cnt + (size_t)(k & 1) * c->cap; }

SoA user_soa(const cc_state *s)
{
    return SoA{s->x, s->y, s->z, s->vx, s->vy, s->vz, const_cast<double *>(s->m), nullptr};
}

// ---- timing ----
hipEvent_t get_event(cc_ctx *c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Span {
    cc_ctx *c;
    int fam;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Span(cc_ctx *cc, int f, hipStream_t stream = nullptr) : c(cc), fam(f), s(stream ? stream : cc->st)
    {
        if (c->timing) {
            a = get_event(c);
            if (a) hipEventRecord(a, s);
        }
    }
    ~Span()
    {
        if (c->timing && a) {
            hipEvent_t b = get_event(c);
            if (b) {
                hipEventRecord(b, s);
                c->recs.push_back({fam, a, b});
            }
        }
    }
};

// An ordering event (no timing) from the pool; returned to it once both
// streams have been synchronised.
int take_event(cc_ctx *c, hipEvent_t *e)
{
    if (!c->sync_pool.empty()) {
        *e = c->sync_pool.back();
        c->sync_pool.pop_back();
    } else {
        HIPCHK(hipEventCreateWithFlags(e, hipEventDisableTiming));
    }
    c->sync_used.push_back(*e);
    return CC_OK;
}

// An ordering event recorded on `from`; `to` waits for it.
int order_streams(cc_ctx *c, hipStream_t from, hipStream_t to)
{
    hipEvent_t e;
    RC(take_event(c, &e));
    HIPCHK(hipEventRecord(e, from));
    HIPCHK(hipStreamWaitEvent(to, e, 0));
    return CC_OK;
}

// after a full synchronisation of both streams the ordering events are free again
void recycle_sync_events(cc_ctx *c)
{
    for (auto e : c->sync_used) c->sync_pool.push_back(e);
    c->sync_used.clear();
}

void flush_timing(cc_ctx *c)
{
    if (c->recs.empty()) return;
    hipStreamSynchronize(c->st);
    for (auto sd : c->side) hipStreamSynchronize(sd);
    for (auto &r : c->recs) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.a, r.b);
        c->fam_ms[r.fam] += ms;
        c->fam_launch[r.fam]++;
        c->ev_pool.push_back(r.a);
        c->ev_pool.push_back(r.b);
    }
    c->recs.clear();
}

uint64_t *fam_ptr(cc_ctx *c, int f) { return (c->timing && c->fam_work) ? c->fam_work + 2 * f : nullptr; }

// ---- grid-level recursion ----

int sync_read_err(cc_ctx *c)
{
    HIPCHK(hipMemcpyAsync(c->h_err, c->errf, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return CC_OK;
}

int err_code(cc_ctx *c, int bits)
{
    if (bits & EB_MASS) return fail(c, CC_ERR_ARG, "a mass is not finite and positive");
    if (bits & EB_NONFINITE) return fail(c, CC_ERR_NONFINITE, "non-finite state or zero separation in a kick");
    if (bits & EB_DEPTH) return fail(c, CC_ERR_DEPTH, "recursion deeper than max_depth = %d", c->params.max_depth);
    if (bits & EB_CAPACITY) return fail(c, CC_ERR_DEVICE, "internal work-list capacity exceeded");
    if (bits & EB_BUDGET)
        return fail(c, CC_ERR_DEPTH, "a per-launch work budget ran out (halvings of a component, or steps of the "
                                     "union-find)");
    return CC_OK;
}

int32_t next_epoch(cc_ctx *c)
{
    if (++c->epoch <= 0) c->epoch = 1;
    return c->epoch;
}

// The offset arrays follow the nseg segments in the descriptor block.
void place_offsets(Level &lv, int nseg)
{
    lv.offs = reinterpret_cast<int32_t *>(lv.desc + (size_t)nseg * sizeof(Seg));
    lv.h_offs = reinterpret_cast<int32_t *>(lv.h_desc + (size_t)nseg * sizeof(Seg));
}

int upload_desc(cc_ctx *c, Level &lv, int nseg)
{
    const size_t bytes = (size_t)nseg * sizeof(Seg) + 3 * ((size_t)nseg + 1) * sizeof(int32_t);
    HIPCHK(hipMemcpyAsync(lv.desc, lv.h_desc, bytes, hipMemcpyHostToDevice, c->st));
    return CC_OK;
}

// A descriptor block: nseg segments, then the prefixes over 256-slot chunks,
// over the sweep's triangular tiles and over slots (nseg+1 ints each).
struct DescTotals {
    int nchunks, ntiles, nact;
};

size_t desc_bytes(size_t nseg) { return nseg * sizeof(Seg) + 3 * (nseg + 1) * sizeof(int32_t); }

int write_desc(cc_ctx *c, const std::vector<Seg> &segs, unsigned char *host, DescTotals *t)
{
    const size_t nseg = segs.size(), S1 = nseg + 1;
    Seg *sg = reinterpret_cast<Seg *>(host);
    int32_t *chunk = reinterpret_cast<int32_t *>(host + nseg * sizeof(Seg)), *tile = chunk + S1, *act = chunk + 2 * S1;
    chunk[0] = tile[0] = act[0] = 0;
    for (size_t s = 0; s < nseg; ++s) {
        sg[s] = segs[s];
        const int n = segs[s].n;
        const int64_t T = (n + TPB - 1) / TPB;
        const int64_t T64 = (n + SWEEP_TILE - 1) / SWEEP_TILE;
        const int64_t nt = tile[s] + T64 * (T64 + 1) / 2;
        if (nt > INT32_MAX) return fail(c, CC_ERR_ARG, "set of %d particles is too large", n);
        chunk[s + 1] = chunk[s] + (int32_t)T;
        tile[s + 1] = (int32_t)nt;
        act[s + 1] = act[s] + n;
    }
    *t = DescTotals{chunk[nseg], tile[nseg], act[nseg]};
    return CC_OK;
}

GridLevelArgs desc_args(const unsigned char *dev, int nseg, const DescTotals &t, int32_t epoch)
{
    const int32_t *offs = reinterpret_cast<const int32_t *>(dev + (size_t)nseg * sizeof(Seg));
    const size_t S1 = (size_t)nseg + 1;
    return GridLevelArgs{reinterpret_cast<const Seg *>(dev), offs, offs + S1, offs + 2 * S1, nseg, t.nchunks,
                         t.ntiles, t.nact, epoch};
}

// A level's two-particle and small components in one launch.  Queue
// counters are per level: the launch of a level may still run on the side
// stream while a deeper level launches its own.  n_small[b] = items in size
// bin b; the items live in working buffer `parity`.
int run_small_and_pairs(cc_ctx *c, int k, Level &lv, double H, int n_pairs, const int n_small[4], hipStream_t st,
                        int parity)
{
    const int n_block_items = n_small[2] + n_small[3];
    const int n_wave_items = n_small[0] + n_small[1];
    if (n_pairs + n_block_items + n_wave_items == 0) return CC_OK;
    const DevParams p = dev_params(c);
    SoA W = work_soa(c, parity);
    SmallArgs sa{};
    sa.pairs = lv.pairs;
    for (int b = 0; b < 4; ++b) sa.bin[b] = lv.small[b];
    sa.count = lv.count;
    sa.cap = lv.cap_small;
    sa.cap_pairs = lv.cap_pairs;
    sa.queue = c->qhead + 4 * k;
    const int sm = small_max(c);
    const int per_cu = (int)std::min<size_t>(8, std::max<size_t>(1, (160 * 1024) / (items_lds_bytes(sm) + 1024)));
    const int nbp = (n_pairs + TPB - 1) / TPB;
    const int nbb = std::min(n_block_items, c->cus * per_cu);
    const int nbw = std::min((n_wave_items + TPB / 64 - 1) / (TPB / 64), c->cus * per_cu);
    Span s(c, F_SMALL, st);
    HIPCHK(launch_items(W, sa, sm, mixed(c) ? 2 : (exact_order(c) ? 1 : 0), nbp, nbb, nbw, H, p, c->errf, c->stats,
                        fam_ptr(c, F_SMALL), st));
    return CC_OK;
}

int evolve_grid(cc_ctx *c, int k, const std::vector<Seg> &segs, double h,
                const unsigned char *pre_desc = nullptr, const DescTotals *pre_tot = nullptr);
int launch_deferred(cc_ctx *c);

// Kick blocks of one level visit, in the component-contiguous order: every
// 256-slot i tile sees its whole segment, except that a tile lying inside one
// large component leaves that component out (all of its pairs are inside it).
// The j ranges are cut into chunks of cj partners, a multiple of KICK_JW
// chosen so that the launch has about kick_groups blocks per compute unit of
// equal work, wherever in the segments the work lies.  The list (a KickTile
// per i tile, then the blocks) goes up with one copy on the main stream, and
// the partial-acceleration buffer grows to the slot count.  The descriptor
// block of the next level's sets (the large components) follows in the same
// copy; both halves' visits of that level use it.  A tile with more
// than KICK_FANIN blocks is summed in two stages: group sums of KICK_FANIN
// consecutive blocks (KickJobs, slots after the blocks'), then the groups.
int upload_kick_list(cc_ctx *c, Level &lv, const std::vector<Seg> &segs, const std::vector<Seg> &big, int *nblk_out,
                     int *njobs_out, const unsigned char **child_desc, DescTotals *child_tot)
{
    // per i tile, the partners [xlo, xhi) it leaves out (offsets within the
    // segment; empty when xlo == xhi)
    std::vector<int32_t> &tr = c->kick_scratch;
    tr.clear();
    int64_t work = 0;
    size_t bi = 0;  // big is sorted by start; segments come in slot order
    for (const Seg &g : segs) {
        const int T = (g.n + TPB - 1) / TPB;
        for (int I = 0; I < T; ++I) {
            const int lo = g.start + I * TPB, hi = g.start + std::min(g.n, (I + 1) * TPB);
            while (bi < big.size() && big[bi].start + big[bi].n <= lo) ++bi;
            int32_t xlo = 0, xhi = 0;
            if (bi < big.size() && big[bi].start <= lo && hi <= big[bi].start + big[bi].n) {
                xlo = big[bi].start - g.start;
                xhi = big[bi].start + big[bi].n - g.start;
            }
            tr.push_back(xlo);
            tr.push_back(xhi);
            work += (int64_t)(hi - lo) * (g.n - (xhi - xlo));
        }
    }
    const int64_t target = std::max<int64_t>(1, (int64_t)c->kick_groups * c->cus);
    int64_t cj = (work + target * TPB - 1) / (target * TPB);
    cj = std::max<int64_t>(KICK_JW, (cj + KICK_JW - 1) / KICK_JW * KICK_JW);
    const auto nchunk = [cj](int64_t len) { return len > 0 ? (len + cj - 1) / cj : 0; };
    int64_t nblk = 0;
    {
        size_t t = 0;
        for (const Seg &g : segs)
            for (int I = 0; I < (g.n + TPB - 1) / TPB; ++I, ++t) nblk += nchunk(tr[2 * t]) + nchunk(g.n - tr[2 * t + 1]);
    }
    const size_t ntile = tr.size() / 2;
    int64_t njobs = 0;
    {
        size_t t = 0;
        for (const Seg &g : segs)
            for (int I = 0; I < (g.n + TPB - 1) / TPB; ++I, ++t) {
                const int64_t nb = nchunk(tr[2 * t]) + nchunk(g.n - tr[2 * t + 1]);
                if (nb > KICK_FANIN) njobs += (nb + KICK_FANIN - 1) / KICK_FANIN;
            }
    }
    if (nblk + njobs > INT32_MAX) return fail(c, CC_ERR_ARG, "kick list too long");
    const size_t nslot = (size_t)(nblk + njobs);
    const size_t kbytes = ntile * sizeof(KickTile) + (size_t)nblk * sizeof(KickBlock) + (size_t)njobs * sizeof(KickJob);
    // the next level's descriptor block rides along (16-byte aligned)
    const size_t doff = (kbytes + 15) & ~(size_t)15;
    const size_t bytes = doff + (big.empty() ? 0 : desc_bytes(big.size()));
    if (lv.kick_pending) {
        HIPCHK(hipEventSynchronize(lv.kick_ev));
        lv.kick_pending = false;
    }
    if (bytes > lv.cap_kick || nslot > c->kick_part_cap) {
        // buffers still read by queued kicks: let both streams drain first
        HIPCHK(hipStreamSynchronize(c->st));
        for (auto sd : c->side) HIPCHK(hipStreamSynchronize(sd));
        if (bytes > lv.cap_kick) {
            const size_t cap = std::max(bytes, 2 * lv.cap_kick);
            RC(dalloc(c, &lv.kick, cap));
            RC(halloc(c, &lv.h_kick, cap));
            lv.cap_kick = cap;
        }
        if (nslot > c->kick_part_cap) {
            const size_t cap = std::max(nslot, 2 * c->kick_part_cap);
            RC(dalloc(c, &c->kick_part, cap * 3 * TPB));
            c->kick_part_cap = cap;
        }
    }
    if (!lv.kick_ev) HIPCHK(hipEventCreateWithFlags(&lv.kick_ev, hipEventDisableTiming));
    KickTile *kt = reinterpret_cast<KickTile *>(lv.h_kick);
    KickBlock *kb = reinterpret_cast<KickBlock *>(lv.h_kick + ntile * sizeof(KickTile));
    KickJob *kj = reinterpret_cast<KickJob *>(lv.h_kick + ntile * sizeof(KickTile) + (size_t)nblk * sizeof(KickBlock));
    int32_t b = 0, j = 0;
    size_t t = 0;
    for (int s = 0; s < (int)segs.size(); ++s) {
        const Seg &g = segs[s];
        for (int I = 0; I < (g.n + TPB - 1) / TPB; ++I, ++t) {
            const int32_t b0 = b;
            const int32_t ranges[2][2] = {{0, tr[2 * t]}, {tr[2 * t + 1], g.n}};
            for (const auto &r : ranges)
                for (int64_t j0 = r[0]; j0 < r[1]; j0 += cj)
                    kb[b++] = KickBlock{s, I, (int32_t)j0, (int32_t)std::min<int64_t>(cj, r[1] - j0)};
            const int32_t nb = b - b0;
            if (nb <= KICK_FANIN) {
                kt[t] = KickTile{b0, nb};
            } else {
                const int32_t g0 = (int32_t)nblk + j;
                for (int32_t q = 0; q < nb; q += KICK_FANIN) {
                    kj[j] = KickJob{b0 + q, std::min<int32_t>(KICK_FANIN, nb - q), (int32_t)nblk + j, 0};
                    ++j;
                }
                kt[t] = KickTile{g0, (int32_t)nblk + j - g0};
            }
        }
    }
    *child_desc = nullptr;
    if (!big.empty()) {
        RC(write_desc(c, big, lv.h_kick + doff, child_tot));
        *child_desc = lv.kick + doff;
    }
    HIPCHK(hipMemcpyAsync(lv.kick, lv.h_kick, bytes, hipMemcpyHostToDevice, c->st));
    HIPCHK(hipEventRecord(lv.kick_ev, c->st));
    lv.kick_pending = true;
    *nblk_out = (int)nblk;
    *njobs_out = (int)njobs;
    return CC_OK;
}

// Items of one list of independent sets at level depth: route by size.
// The on-chip components of a level and its large components are disjoint
// sets: the former run on the side stream while the host drives the recursion
// into the latter on the main stream; the main stream waits for the side
// stream before the level's own kick.
int dispatch_sets(cc_ctx *c, int k, Level &lv, double H, const std::vector<Seg> &big, int n_pairs,
                  const int n_small[4], const unsigned char *big_desc = nullptr, const DescTotals *big_tot = nullptr)
{
    const bool on_chip = n_pairs + n_small[0] + n_small[1] + n_small[2] + n_small[3] > 0;
    if (!on_chip || big.empty()) {
        RC(run_small_and_pairs(c, k, lv, H, n_pairs, n_small, c->st, k + 1));
        if (!big.empty()) RC(evolve_grid(c, k + 1, big, H, big_desc, big_tot));
        return CC_OK;
    }
    // The launch goes to a side stream once the child level's first sweep is
    // queued on the main stream (launch_deferred, called by evolve_grid after
    // that sweep): started together, its blocks took the compute units'
    // registers while that sweep began, which slowed the sweep, and the
    // launch is not needed before this level's kick, after the whole child
    // recursion.
    hipStream_t sd = c->side[k % kSide];
    auto &d = c->deferred;
    d.on = true;
    d.k = k;
    d.H = H;
    d.n_pairs = n_pairs;
    for (int b = 0; b < 4; ++b) d.n_small[b] = n_small[b];
    d.sd = sd;
    RC(take_event(c, &d.done));
    hipEvent_t done = d.done;
    const int rc = evolve_grid(c, k + 1, big, H, big_desc, big_tot);
    if (c->deferred.on) {
        // the child queued no sweep: launch now, or drop it after an error
        if (rc != CC_OK) c->deferred.on = false;
        else RC(launch_deferred(c));
    }
    RC(rc);
    HIPCHK(hipStreamWaitEvent(c->st, done, 0));
    return CC_OK;
}

// The pending on-chip launch of dispatch_sets, on its side stream after the
// work queued on the main stream so far (the child level's sweep).
int launch_deferred(cc_ctx *c)
{
    auto &d = c->deferred;
    if (!d.on) return CC_OK;
    d.on = false;
    RC(order_streams(c, c->st, d.sd));
    RC(run_small_and_pairs(c, d.k, c->levels[d.k], d.H, d.n_pairs, d.n_small, d.sd, d.k + 1));
    HIPCHK(hipEventRecord(d.done, d.sd));
    return CC_OK;
}

bool trace_on()
{
    static const int on = [] {
        const char *e = std::getenv("CC_TRACE");
        return (e && *e && *e != '0') ? 1 : 0;
    }();
    return on != 0;
}

// pre_desc: the sets' descriptor block already on the device (uploaded by the
// parent level together with its kick list), with its totals.
int evolve_grid(cc_ctx *c, int k, const std::vector<Seg> &segs, double h, const unsigned char *pre_desc,
                const DescTotals *pre_tot)
{
    if (segs.empty()) return CC_OK;
    if (segs[0].depth > c->params.max_depth)
        return fail(c, CC_ERR_DEPTH, "recursion deeper than max_depth = %d", c->params.max_depth);
    const int nseg = (int)segs.size();
    RC(ensure_level(c, k, nseg));
    Level &lv = c->levels[k];
    const DevParams p = dev_params(c);
    SoA W = work_soa(c, k);       // the sets of this level, entry order
    SoA Wp = work_soa(c, k + 1);  // the same slots, component-contiguous

    // segment descriptors and prefix arrays
    GridLevelArgs a{};
    if (pre_desc) {
        a = desc_args(pre_desc, nseg, *pre_tot, next_epoch(c));
    } else {
        DescTotals t{};
        RC(write_desc(c, segs, lv.h_desc, &t));
        RC(upload_desc(c, lv, nseg));
        a = desc_args(lv.desc, nseg, t, next_epoch(c));
    }
    const bool exact = exact_order(c);
    // The star test of Sec. 2.3 runs ahead of the sweep only on levels whose
    // last visit found a star; otherwise the sweep's first tile row takes it.
    const bool star_pass = lv.star_hint;
    if (star_pass) {
        Span s(c, F_SWEEP);
        HIPCHK(launch_star(W, a, lv.notstar, p, h, screen32(c), c->stats, fam_ptr(c, F_SWEEP), c->st));
    }
    {
        Span s(c, F_SWEEP);
        HIPCHK(launch_sweep(W, a, lv.notstar, c->parent, p, h, screen32(c), c->sweep_split, star_pass, c->errf,
                            c->st));
    }
    RC(launch_deferred(c));
    {
        Span s(c, F_LABEL);
        const bool hold = c->params.hold != 0;
        HIPCHK(launch_label(a, lv.notstar, c->parent, lv.label, cnt_of(c, k), c->keys, c->vals, lv.count,
                            hold ? lv.hold : nullptr, star_pass, c->stats, fam_ptr(c, F_SWEEP), c->errf, c->st));
        // HOLD (Sec. 2.1): the non-trivial components of each set become one
        // set F before the sort makes it contiguous
        if (hold) HIPCHK(launch_hold(a, lv.label, cnt_of(c, k), c->keys, lv.hold, c->st));
    }
    int bits = 0;
    {
        int maxslot = 1;
        for (int s = 0; s < nseg; ++s) maxslot = std::max(maxslot, segs[s].start + segs[s].n);
        int end_bit = 1;
        while ((1 << end_bit) < maxslot + 1 && end_bit < 31) end_bit++;
        Span s(c, F_SORT);
        HIPCHK(launch_sort(c->sort_temp, c->sort_bytes, c->keys, c->keys_out, c->vals, lv.src, a.nact, end_bit, c->st));
    }
    ListArgs L{};
    L.pairs = lv.pairs;
    for (int b = 0; b < 4; ++b) L.small[b] = lv.small[b];
    L.big = lv.big;
    L.count = lv.count;
    L.cap_pairs = lv.cap_pairs;
    L.cap_small = lv.cap_small;
    L.cap_big = lv.cap_big;
    L.small_max = small_max(c);
    L.bin_lim[0] = 8;
    L.bin_lim[1] = 32;
    L.bin_lim[2] = 128;
    L.labp = exact ? nullptr : lv.labp;
    L.singp = exact ? nullptr : lv.singp;
    L.errf = c->errf;
    L.notstar = lv.notstar;
    {
        Span s(c, F_PERMUTE);
        // FAST order: the singletons' first drift touches no particle of a
        // component, so it may precede the first-half recursion; it is
        // applied by the permutation itself.
        HIPCHK(launch_permute(W, Wp, a, lv.src, c->keys_out, cnt_of(c, k), lv.sing, &L, exact ? 0.0 : 0.5 * h,
                              c->parent, cnt_of(c, k + 1), fam_ptr(c, F_KICK), !exact, c->stats, false, c->st));
    }
    HIPCHK(hipMemcpyAsync(lv.h_rep, lv.rep, 8 * sizeof(int32_t) + (size_t)lv.cap_big * sizeof(Seg),
                          hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    bits = lv.h_count[7];
    if (bits) return err_code(c, bits);
    const int n_pairs = lv.h_count[0];
    const int n_small[4] = {lv.h_count[1], lv.h_count[2], lv.h_count[3], lv.h_count[4]};
    const int n_big = lv.h_count[5];
    lv.star_hint = lv.h_count[6] > 0;
    if (n_pairs > lv.cap_pairs || lv.h_count[1] > lv.cap_small || lv.h_count[2] > lv.cap_small ||
        lv.h_count[3] > lv.cap_small || lv.h_count[4] > lv.cap_small || n_big > lv.cap_big)
        return fail(c, CC_ERR_DEVICE, "internal work-list capacity exceeded");
    std::vector<Seg> big(lv.h_big, lv.h_big + n_big);
    std::sort(big.begin(), big.end(), [](const Seg &x, const Seg &y) { return x.start < y.start; });
    const bool any_sub = (n_pairs + n_small[0] + n_small[1] + n_small[2] + n_small[3] + n_big) > 0;
    const double H = 0.5 * h;
    if (trace_on()) {
        int nmax = 0;
        for (const Seg &g : segs) nmax = std::max(nmax, g.n);
        std::fprintf(stderr, "cc-trace level=%d nseg=%d nact=%d nmax=%d pairs=%d small=%d/%d/%d/%d big=%d\n", k, nseg,
                     a.nact, nmax, n_pairs, lv.h_count[1], lv.h_count[2], lv.h_count[3], lv.h_count[4], n_big);
    }

    if (!exact) {
        // Component-contiguous order throughout: (the first drift, done by
        // the permutation), the kick list, first half, kick and closing drift
        // of the level, second half, then back to the entry order.
        int nblk = 0, njobs = 0;
        const unsigned char *big_desc = nullptr;
        DescTotals big_tot{};
        RC(upload_kick_list(c, lv, segs, big, &nblk, &njobs, &big_desc, &big_tot));
        const KickTile *ktile = reinterpret_cast<const KickTile *>(lv.kick);
        const KickBlock *kblk = reinterpret_cast<const KickBlock *>(lv.kick + (size_t)a.nchunks * sizeof(KickTile));
        const KickJob *kjob = reinterpret_cast<const KickJob *>(lv.kick + (size_t)a.nchunks * sizeof(KickTile) +
                                                                (size_t)nblk * sizeof(KickBlock));
        if (any_sub) RC(dispatch_sets(c, k, c->levels[k], H, big, n_pairs, n_small, big_desc, &big_tot));
        Level &lv2 = c->levels[k];
        {
            // the kick, then the second drift of the singletons (fused)
            Span s(c, F_KICK);
            HIPCHK(launch_kick_tiles(Wp, a, kblk, nblk, kjob, njobs, ktile, lv2.labp, lv2.singp, h, c->params.eps2,
                                     c->params.G, mixed(c), c->kick_part, c->parent, cnt_of(c, k + 1), c->errf,
                                     c->stats, c->st));
        }
        if (any_sub) RC(dispatch_sets(c, k, c->levels[k], H, big, n_pairs, n_small, big_desc, &big_tot));
        Level &lv3 = c->levels[k];
        Span s(c, F_PERMUTE);
        HIPCHK(launch_permute(Wp, W, a, lv3.src, nullptr, nullptr, nullptr, nullptr, 0.0, nullptr, nullptr, nullptr,
                              false, c->stats, true, c->st));
        return CC_OK;
    }

    // Exact order: the level's drift/kick/drift runs in the entry order, in
    // which every set is ascending in particle index.
    if (any_sub) RC(dispatch_sets(c, k, c->levels[k], H, big, n_pairs, n_small));
    {
        Level &lv2 = c->levels[k];
        Span s(c, F_PERMUTE);
        HIPCHK(launch_permute(Wp, W, a, lv2.src, nullptr, nullptr, nullptr, nullptr, 0.0, nullptr, nullptr, nullptr,
                              false, c->stats, true, c->st));
    }
    {
        Level &lv2 = c->levels[k];
        {
            Span s(c, F_DRIFT);
            HIPCHK(launch_drift_seg(W, a, lv2.sing, H, c->stats, c->st));
        }
        {
            Span s(c, F_KICK);
            HIPCHK(launch_kick_seg(W, a, lv2.label, h, c->params.eps2, c->params.G, c->errf, c->stats,
                                   fam_ptr(c, F_KICK), c->st));
        }
        {
            Span s(c, F_DRIFT);
            HIPCHK(launch_drift_seg(W, a, lv2.sing, H, c->stats, c->st));
        }
    }
    // second half with the same partition
    if (any_sub) {
        {
            Level &lv2 = c->levels[k];
            Span s(c, F_PERMUTE);
            HIPCHK(launch_permute(W, Wp, a, lv2.src, nullptr, nullptr, nullptr, nullptr, 0.0, c->parent,
                                  cnt_of(c, k + 1), nullptr, false, c->stats, false, c->st));
        }
        RC(dispatch_sets(c, k, c->levels[k], H, big, n_pairs, n_small));
        Level &lv2 = c->levels[k];
        Span s(c, F_PERMUTE);
        HIPCHK(launch_permute(Wp, W, a, lv2.src, nullptr, nullptr, nullptr, nullptr, 0.0, nullptr, nullptr, nullptr,
                              false, c->stats, true, c->st));
    }
    return CC_OK;
}

// One global step on a list of top-level sets (clusters), all at depth 0.
// Route the top-level sets (clusters): two-particle and small ones into the
// level-0 work lists (uploaded on the main stream, which is then synchronised:
// the host vectors must outlive the copies), large ones into `big`.
int route_top(cc_ctx *c, const std::vector<Seg> &top, std::vector<Seg> &big, int &n_pairs, int n_small[4])
{
    std::vector<Seg> pairs, small[4];
    const int sm = small_max(c);
    big.clear();
    for (const Seg &g : top) {
        // Clusters of one or two bodies take the grid path (a split, then a
        // two-body component joins the level's pair list like any other):
        // on-chip launches only ever hold sets of three or more at their
        // top.  Two GPU runs with such clusters in the on-chip launch went
        // silent and the cause was not found, so that route stays closed.
        if (g.n < 3) big.push_back(g);
        else if (g.n <= sm) {
            const int b = g.n <= 8 ? 0 : g.n <= 32 ? 1 : g.n <= 128 ? 2 : 3;
            small[b].push_back(g);
        } else big.push_back(g);
    }
    n_pairs = (int)pairs.size();
    for (int b = 0; b < 4; ++b) n_small[b] = (int)small[b].size();
    if (n_pairs + n_small[0] + n_small[1] + n_small[2] + n_small[3] == 0) return CC_OK;
    RC(ensure_level(c, 0, 1));
    Level &lv = c->levels[0];
    lv.h_count[0] = n_pairs;
    for (int b = 0; b < 4; ++b) lv.h_count[1 + b] = n_small[b];
    for (int b = 5; b < 8; ++b) lv.h_count[b] = 0;
    HIPCHK(hipMemcpyAsync(lv.count, lv.h_count, 8 * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
    if (!pairs.empty())
        HIPCHK(hipMemcpyAsync(lv.pairs, pairs.data(), pairs.size() * sizeof(Seg), hipMemcpyHostToDevice, c->st));
    for (int b = 0; b < 4; ++b)
        if (!small[b].empty())
            HIPCHK(hipMemcpyAsync(lv.small[b], small[b].data(), small[b].size() * sizeof(Seg), hipMemcpyHostToDevice,
                                  c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return CC_OK;
}

// One global step on a list of top-level sets (clusters), all at depth 0.
int global_step(cc_ctx *c, const std::vector<Seg> &top, double dt)
{
    std::vector<Seg> big;
    int n_pairs = 0, n_small[4] = {0, 0, 0, 0};
    RC(route_top(c, top, big, n_pairs, n_small));
    if (n_pairs + n_small[0] + n_small[1] + n_small[2] + n_small[3] > 0)
        RC(run_small_and_pairs(c, 0, c->levels[0], dt, n_pairs, n_small, c->st, 0));
    if (!big.empty()) {
        // the union-find of the top level; deeper levels are reset on the way
        int end = 0;
        for (const Seg &g : big) end = std::max(end, g.start + g.n);
        HIPCHK(launch_uf_init(c->parent, cnt_of(c, 0), end, c->st));
        RC(evolve_grid(c, 0, big, dt));
    }
    return CC_OK;
}

// Global steps of sets that are all evolved on chip (an ensemble of small
// clusters): the device work of one step -- error reset, validation,
// snapshot, the on-chip launch, validation, error read-back -- is captured once
// as a HIP graph on the side stream and replayed per step, with one host
// synchronisation per step for the error check.  *done = steps completed;
// *captured = false if the graph could not be built (nothing has run then, and
// the caller takes the steps one launch at a time).
int evolve_on_chip_graph(cc_ctx *c, const std::vector<Seg> &top, int64_t n, int64_t nsteps, double dt,
                         int64_t *done, bool *captured)
{
    *captured = false;
    std::vector<Seg> big;
    int n_pairs = 0, n_small[4] = {0, 0, 0, 0};
    RC(route_top(c, top, big, n_pairs, n_small));  // also orders the caller's copies before the graph
    const int mode = mixed(c) ? 2 : (exact_order(c) ? 1 : 0);
    HIPCHK(configure_items(small_max(c), mode));
    const size_t bytes = (size_t)n * sizeof(double);
    hipStream_t g = c->side[0];
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(g, hipStreamCaptureModeThreadLocal));
    int rc = CC_OK;
    {
        const bool ok = launch_fill_i32(c->errf, 1, 0, g) == hipSuccess &&
                        launch_validate(c->w[0], c->w[1], c->w[2], c->w[3], c->w[4], c->w[5], c->w[6], n, c->errf,
                                        g) == hipSuccess;
        if (!ok) rc = fail(c, CC_ERR_DEVICE, "graph capture of the step prologue failed");
        for (int a = 0; a < 6 && rc == CC_OK; ++a)
            if (hipMemcpyAsync(c->snap[a], c->w[a], bytes, hipMemcpyDeviceToDevice, g) != hipSuccess)
                rc = fail(c, CC_ERR_DEVICE, "graph capture of the snapshot failed");
        if (rc == CC_OK) rc = run_small_and_pairs(c, 0, c->levels[0], dt, n_pairs, n_small, g, 0);
        if (rc == CC_OK &&
            (launch_validate(c->w[0], c->w[1], c->w[2], c->w[3], c->w[4], c->w[5], c->w[6], n, c->errf, g) !=
                 hipSuccess ||
             hipMemcpyAsync(c->h_err, c->errf, sizeof(int32_t), hipMemcpyDeviceToHost, g) != hipSuccess))
            rc = fail(c, CC_ERR_DEVICE, "graph capture of the step epilogue failed");
    }
    const hipError_t ec = hipStreamEndCapture(g, &graph);
    if (rc == CC_OK && ec != hipSuccess) rc = fail(c, CC_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    if (rc == CC_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(c, CC_ERR_DEVICE, "hipGraphInstantiate failed");
    if (rc != CC_OK) {
        if (graph) hipGraphDestroy(graph);
        (void)hipGetLastError();
        c->err.clear();
        return CC_OK;
    }
    *captured = true;
    for (int64_t step = 0; step < nsteps && rc == CC_OK; ++step) {
        if (hipGraphLaunch(exec, g) != hipSuccess || hipStreamSynchronize(g) != hipSuccess) {
            rc = fail(c, CC_ERR_DEVICE, "graph replay failed");
            break;
        }
        if (*c->h_err) {
            rc = err_code(c, *c->h_err);
            for (int a = 0; a < 6; ++a) hipMemcpyAsync(c->w[a], c->snap[a], bytes, hipMemcpyDeviceToDevice, g);
            hipStreamSynchronize(g);
            break;
        }
        *done = step + 1;
    }
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    return rc;
}

int check_state_ptrs(cc_ctx *c, const cc_state *s)
{
    if (!s) return fail(c, CC_ERR_ARG, "state is NULL");
    if (!s->x || !s->y || !s->z || !s->vx || !s->vy || !s->vz || !s->m)
        return fail(c, CC_ERR_ARG, "a state pointer is NULL");
    return CC_OK;
}

int step_count(cc_ctx *c, double dt, double t_end, int64_t *nsteps)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, CC_ERR_ARG, "dt must be finite and > 0");
    if (!(t_end > 0.0) || !std::isfinite(t_end)) return fail(c, CC_ERR_ARG, "t_end must be finite and > 0");
    const double q = t_end / dt;
    if (!(q >= 1.0) || q != std::floor(q) || q > 2147483647.0)
        return fail(c, CC_ERR_ARG, "t_end/dt = %.17g is not a positive integer", q);
    *nsteps = (int64_t)q;
    return CC_OK;
}

int evolve_common(cc_ctx *c, cc_state *s, int64_t n, const int64_t *off, int32_t ncl, double dt, double t_end,
                  cc_stats *out, void *stream)
{
    c->err.clear();
    RC(check_state_ptrs(c, s));
    int64_t nsteps = 0;
    RC(step_count(c, dt, t_end, &nsteps));
    if (n < 1) return fail(c, CC_ERR_ARG, "n must be >= 1");
    std::vector<Seg> top;
    for (int32_t k = 0; k < ncl; ++k) {
        const int64_t a = off[k], b = off[k + 1];
        if (a < 0 || b <= a || b > n) return fail(c, CC_ERR_ARG, "offsets must be strictly increasing in [0, n]");
        top.push_back(Seg{(int32_t)a, (int32_t)(b - a), k, 0});
    }
    HIPCHK(hipSetDevice(c->device));
    c->st = (hipStream_t)stream;
    RC(ensure_capacity(c, (size_t)n, (size_t)ncl));
    HIPCHK(hipMemsetAsync(c->stats, 0, (size_t)ncl * ST_N * sizeof(uint64_t), c->st));
    const size_t bytes = (size_t)n * sizeof(double);
    double *user[7] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, const_cast<double *>(s->m)};
    for (int a = 0; a < 7; ++a) HIPCHK(hipMemcpyAsync(c->w[a], user[a], bytes, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(launch_iota(c->orig, n, c->st));
    int rc = CC_OK;
    int64_t done = 0;
    bool all_on_chip = true;
    for (const Seg &g : top) all_on_chip = all_on_chip && g.n >= 3 && g.n <= small_max(c);
    if (all_on_chip && nsteps >= 2 && !c->timing) {
        bool captured = false;
        rc = evolve_on_chip_graph(c, top, n, nsteps, dt, &done, &captured);
        if (captured || rc != CC_OK) nsteps = 0;  // the loop below has nothing left to do
    }
    for (int64_t step = 0; step < nsteps; ++step) {
        HIPCHK(launch_fill_i32(c->errf, 1, 0, c->st));
        {
            Span sp(c, F_VALIDATE);
            HIPCHK(launch_validate(c->w[0], c->w[1], c->w[2], c->w[3], c->w[4], c->w[5], c->w[6], n, c->errf, c->st));
        }
        for (int a = 0; a < 6; ++a) HIPCHK(hipMemcpyAsync(c->snap[a], c->w[a], bytes, hipMemcpyDeviceToDevice, c->st));
        RC(sync_read_err(c));
        if (*c->h_err) {
            rc = err_code(c, *c->h_err);
            break;
        }
        rc = global_step(c, top, dt);
        if (rc == CC_OK) {
            HIPCHK(launch_validate(c->w[0], c->w[1], c->w[2], c->w[3], c->w[4], c->w[5], c->w[6], n, c->errf, c->st));
            RC(sync_read_err(c));
            if (*c->h_err) rc = err_code(c, *c->h_err);
        }
        if (rc != CC_OK) {
            for (auto sd : c->side) hipStreamSynchronize(sd);
            hipStreamSynchronize(c->st);
            recycle_sync_events(c);
            for (int a = 0; a < 6; ++a)
                hipMemcpyAsync(c->w[a], c->snap[a], bytes, hipMemcpyDeviceToDevice, c->st);
            break;
        }
        done = step + 1;
        if (c->timing) flush_timing(c);
        recycle_sync_events(c);
    }
    // copy the working state back (slots are in entry order = particle order)
    for (int a = 0; a < 6; ++a) HIPCHK(hipMemcpyAsync(user[a], c->w[a], bytes, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->h_stats, c->stats, (size_t)ncl * ST_N * sizeof(uint64_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (c->timing) flush_timing(c);
    if (out) {
        for (int32_t k = 0; k < ncl; ++k) {
            const uint64_t *h = c->h_stats + (size_t)k * ST_N;
            cc_stats &o = out[k];
            o.tau_pairs = h[ST_TAU];
            o.tau_pairs_alg = h[ST_TAU_ALG];
            o.kick_pairs = h[ST_KICK];
            o.drifts = h[ST_DRIFT];
            o.components = h[ST_COMP];
            o.splits = h[ST_SPLIT];
            o.max_depth_seen = (int64_t)h[ST_MAXD];
            o.t_reached = (double)done * dt;
            o.kepler_solves = h[ST_KEPLER];
        }
    }
    return rc;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int cc_create(cc_ctx **out, int32_t hip_device, const cc_params *p)
{
    if (!out) return CC_ERR_ARG;
    *out = nullptr;
    cc_ctx *c = new (std::nothrow) cc_ctx();
    if (!c) return CC_ERR_OOM;
    int rc = check_params(c, p);
    if (rc != CC_OK) {
        delete c;
        return rc;
    }
    c->params = *p;
    c->device = hip_device;
    c->levels.resize(kLevels);  // fixed size: references to levels stay valid during the recursion
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
        delete c;
        return CC_ERR_DEVICE;
    }
    if (hipSetDevice(hip_device) != hipSuccess) {
        delete c;
        return CC_ERR_DEVICE;
    }
    // device address of cc_kick_static's scratch array (once per device)
    if (ccg::static_scratch_setup(hip_device) != hipSuccess) {
        delete c;
        return CC_ERR_DEVICE;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
        c->cus = cus;
    // default priority, no implicit synchronisation with the null stream
    for (auto &sd : c->side)
        if (hipStreamCreateWithFlags(&sd, hipStreamNonBlocking) != hipSuccess) {
            for (auto q : c->side)
                if (q) hipStreamDestroy(q);
            delete c;
            return CC_ERR_DEVICE;
        }
    if (dalloc(c, &c->errf, 1) != CC_OK || halloc(c, &c->h_err, 1) != CC_OK || dalloc(c, &c->qhead, 4 * kLevels) != CC_OK ||
        dalloc(c, &c->diag_out, 16) != CC_OK || halloc(c, &c->h_diag, 16) != CC_OK ||
        dalloc(c, &c->fam_work, 2 * F_N) != CC_OK) {
        cc_destroy(c);
        return CC_ERR_OOM;
    }
    if (hipMemset(c->qhead, 0, 4 * kLevels * sizeof(int32_t)) != hipSuccess) {
        cc_destroy(c);
        return CC_ERR_DEVICE;
    }
    *out = c;
    return CC_OK;
}

void cc_destroy(cc_ctx *c)
{
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    auto F = [](void *p) {
        if (p) hipFree(p);
    };
    auto FH = [](void *p) {
        if (p) hipHostFree(p);
    };
    for (auto *p : c->w) F(p);
    for (auto *p : c->snap) F(p);
    for (auto *p : c->tmp) F(p);
    F(c->orig); F(c->tmp_orig); F(c->keys); F(c->keys_out); F(c->vals); F(c->sort_temp);
    F(c->parent); F(c->cnt); F(c->stats); F(c->errf); F(c->qhead); F(c->kick_acc); F(c->kick_part); F(c->diag_part);
    F(c->diag_out); F(c->fam_work);
    FH(c->h_stats); FH(c->h_err); FH(c->h_diag);
    for (auto &lv : c->levels) {
        F(lv.label); F(lv.sing); F(lv.labp); F(lv.singp); F(lv.src); F(lv.pairs);
        for (auto *p : lv.small) F(p);
        F(lv.rep); F(lv.notstar); F(lv.hold); F(lv.desc); F(lv.kick);
        FH(lv.h_rep); FH(lv.h_desc); FH(lv.h_kick);
        if (lv.kick_ev) hipEventDestroy(lv.kick_ev);
    }
    for (auto &r : c->recs) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : c->ev_pool) hipEventDestroy(e);
    for (auto e : c->sync_pool) hipEventDestroy(e);
    for (auto e : c->sync_used) hipEventDestroy(e);
    for (auto sd : c->side)
        if (sd) hipStreamDestroy(sd);
    delete c;
}

int cc_set_params(cc_ctx *c, const cc_params *p)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    RC(check_params(c, p));
    const bool sm_changed = small_max(c) != small_max_of(*p);
    c->params = *p;
    if (sm_changed)
        for (auto &lv : c->levels) lv.cap_n = 0;
    return CC_OK;
}

const char *cc_last_error(const cc_ctx *c) { return c ? c->err.c_str() : "NULL context"; }

int cc_pair_timesteps(cc_ctx *c, const cc_state *s, int64_t n, const int32_t *pi, const int32_t *pj, int64_t npairs,
                      double *tau_out, void *stream)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    RC(check_state_ptrs(c, s));
    if (n < 1 || npairs < 0) return fail(c, CC_ERR_ARG, "n must be >= 1 and npairs >= 0");
    if (npairs == 0) return CC_OK;
    if (!pi || !pj || !tau_out) return fail(c, CC_ERR_ARG, "pair or output pointer is NULL");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(launch_pair_tau(user_soa(s), pi, pj, npairs, tau_out, dev_params(c), (hipStream_t)stream));
    return CC_OK;
}

int cc_split_labels(cc_ctx *c, const cc_state *s, int64_t n, double h, int32_t *label_out, int64_t *n_nontrivial_out,
                    void *stream)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    RC(check_state_ptrs(c, s));
    if (n < 1) return fail(c, CC_ERR_ARG, "n must be >= 1");
    if (!label_out) return fail(c, CC_ERR_ARG, "label_out is NULL");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(c, CC_ERR_ARG, "h must be finite and > 0");
    HIPCHK(hipSetDevice(c->device));
    c->st = (hipStream_t)stream;
    RC(ensure_capacity(c, (size_t)n, 1));
    RC(ensure_level(c, 0, 1));
    Level &lv = c->levels[0];
    const int T = (int)((n + TPB - 1) / TPB);
    const int64_t T64 = (n + SWEEP_TILE - 1) / SWEEP_TILE;
    if (T64 * (T64 + 1) / 2 > INT32_MAX) return fail(c, CC_ERR_ARG, "n too large");
    const int NT = (int)(T64 * (T64 + 1) / 2);
    lv.h_seg[0] = Seg{0, (int32_t)n, 0, 0};
    place_offsets(lv, 1);
    int32_t *o = lv.h_offs;
    o[0] = 0; o[1] = T; o[2] = 0; o[3] = NT; o[4] = 0; o[5] = (int32_t)n;
    RC(upload_desc(c, lv, 1));
    GridLevelArgs a{lv.seg, lv.offs, lv.offs + 2, lv.offs + 4, 1, T, NT, (int)n, next_epoch(c)};
    HIPCHK(hipMemsetAsync(c->stats, 0, ST_N * sizeof(uint64_t), c->st));
    const DevParams p = dev_params(c);
    SoA S = user_soa(s);
    HIPCHK(launch_uf_init(c->parent, cnt_of(c, 0), (int)n, c->st));
    HIPCHK(hipMemsetAsync(c->errf, 0, sizeof(int32_t), c->st));
    HIPCHK(launch_sweep(S, a, lv.notstar, c->parent, p, h, screen32(c), c->sweep_split, false, c->errf, c->st));
    HIPCHK(launch_label(a, lv.notstar, c->parent, label_out, cnt_of(c, 0), nullptr, nullptr, nullptr, nullptr, false,
                        c->stats, nullptr, c->errf, c->st));
    RC(sync_read_err(c));
    if (*c->h_err) return err_code(c, *c->h_err);
    if (n_nontrivial_out) {
        // roots carry their component size in cnt (zeroed for every slot by the reset)
        std::vector<int32_t> cnt((size_t)n);
        HIPCHK(hipMemcpyAsync(cnt.data(), cnt_of(c, 0), (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        int64_t nt = 0;
        for (int64_t i = 0; i < n; ++i) nt += (cnt[(size_t)i] >= 2);
        *n_nontrivial_out = nt;
    }
    return CC_OK;
}

int cc_kick(cc_ctx *c, cc_state *s, int64_t n, const int32_t *label, double h, void *stream)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    RC(check_state_ptrs(c, s));
    if (n < 1) return fail(c, CC_ERR_ARG, "n must be >= 1");
    if (!std::isfinite(h)) return fail(c, CC_ERR_ARG, "h must be finite");
    HIPCHK(hipSetDevice(c->device));
    c->st = (hipStream_t)stream;
    RC(ensure_capacity(c, (size_t)n, 1));
    SoA S = user_soa(s);
    double *ax = c->kick_acc, *ay = ax + c->cap, *az = ay + c->cap;
    HIPCHK(launch_fill_i32(c->errf, 1, 0, c->st));
    HIPCHK(launch_kick_all(S, (int)n, label, c->params.eps2, c->params.G, mixed(c), ax, ay, az, c->errf, c->st));
    RC(sync_read_err(c));
    if (*c->h_err) return err_code(c, *c->h_err);
    HIPCHK(launch_apply_kick(S, (int)n, ax, ay, az, h, c->st));
    return CC_OK;
}

int cc_kick_static(cc_ctx *c, cc_state *s, int64_t n, const int32_t *label, double h, void *stream)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    RC(check_state_ptrs(c, s));
    if (n < 1) return fail(c, CC_ERR_ARG, "n must be >= 1");
    if (n > CC_KICK_STATIC_MAX_N)
        return fail(c, CC_ERR_ARG, "n = %lld exceeds the static scratch limit of %d particles", (long long)n,
                    CC_KICK_STATIC_MAX_N);
    if (!std::isfinite(h)) return fail(c, CC_ERR_ARG, "h must be finite");
    HIPCHK(hipSetDevice(c->device));
    // the address cc_create looked up for this device (never the array's name)
    unsigned char *base = static_cast<unsigned char *>(ccg::static_scratch(c->device));
    if (!base) return fail(c, CC_ERR_DEVICE, "static scratch of device %d was not set up", c->device);
    double *ax = reinterpret_cast<double *>(base), *ay = ax + n, *az = ay + n;
    int32_t *err = reinterpret_cast<int32_t *>(base + ccg::STATIC_ACC_BYTES);
    hipStream_t st = (hipStream_t)stream;
    SoA S = user_soa(s);
    HIPCHK(launch_fill_i32(err, 1, 0, st));  // the previous call's flag is still there
    HIPCHK(launch_kick_all(S, (int)n, label, c->params.eps2, c->params.G, mixed(c), ax, ay, az, err, st));
    int32_t h_err = 0;
    HIPCHK(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h_err) return err_code(c, h_err);
    HIPCHK(launch_apply_kick(S, (int)n, ax, ay, az, h, st));
    return CC_OK;
}

int cc_drift(cc_ctx *c, cc_state *s, int64_t n, const uint8_t *mask, double h, void *stream)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    RC(check_state_ptrs(c, s));
    if (n < 1) return fail(c, CC_ERR_ARG, "n must be >= 1");
    if (!std::isfinite(h)) return fail(c, CC_ERR_ARG, "h must be finite");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(launch_drift_mask(user_soa(s), n, mask, h, (hipStream_t)stream));
    return CC_OK;
}

int cc_evolve(cc_ctx *c, cc_state *s, int64_t n, double dt, double t_end, cc_stats *out, void *stream)
{
    if (!c) return CC_ERR_ARG;
    const int64_t off[2] = {0, n};
    return evolve_common(c, s, n, off, 1, dt, t_end, out, stream);
}

int cc_autotune(cc_ctx *c, const cc_state *s, int64_t n, double dt, cc_tune *out, void *stream)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    RC(check_state_ptrs(c, s));
    if (n < 1) return fail(c, CC_ERR_ARG, "n must be >= 1");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, CC_ERR_ARG, "dt must be finite and > 0");
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    // trials run on a copy; the caller's state is only read
    double *copy[7] = {};
    const size_t bytes = (size_t)n * sizeof(double);
    const double *src[7] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->m};
    int rc = CC_OK;
    for (int a = 0; a < 7 && rc == CC_OK; ++a)
        if (hipMalloc((void **)&copy[a], bytes) != hipSuccess) rc = fail(c, CC_ERR_OOM, "autotune copy of the state");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == CC_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(c, CC_ERR_DEVICE, "autotune events");
    const cc_params keep = c->params;
    const int32_t keep_split = c->sweep_split, keep_kg = c->kick_groups;
    // (in plain mode nothing runs on chip: the on-chip size limit is not tuned)
    cc_tune best{keep.plain ? keep.small_max : small_max(c), c->sweep_split, c->kick_groups, 1e300, 0};
    // one untimed step (buffers sized for the setting), then the best of two
    auto time_step = [&](double *ms_out) -> int {
        float best_ms = 1e30f;
        for (int trial = 0; trial < 3; ++trial) {
            for (int a = 0; a < 7; ++a)
                if (hipMemcpyAsync(copy[a], src[a], bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
                    return fail(c, CC_ERR_DEVICE, "autotune copy");
            cc_state w{copy[0], copy[1], copy[2], copy[3], copy[4], copy[5], copy[6]};
            hipEventRecord(e0, st);
            RC(cc_evolve(c, &w, n, dt, dt, nullptr, stream));
            hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) return fail(c, CC_ERR_DEVICE, "autotune timing");
            float ms = 0.0f;
            hipEventElapsedTime(&ms, e0, e1);
            if (trial > 0) best_ms = std::min(best_ms, ms);
        }
        *ms_out = best_ms;
        return CC_OK;
    };
    auto apply = [&](const cc_tune &t) -> int {
        cc_params q = keep;
        q.small_max = t.small_max;
        RC(cc_set_params(c, &q));
        c->sweep_split = t.sweep_split_tiles;
        c->kick_groups = t.kick_groups_per_cu;
        return CC_OK;
    };
    // coordinate descent over the three shapes, each from the best so far
    const int32_t sm_cand[] = {64, 128, 256, 512};
    const int32_t split_cand[] = {0, 512, 2048, 8192};
    const int32_t kg_cand[] = {8, 16, 32, 64};
    for (int knob = keep.plain ? 1 : 0; knob < 3 && rc == CC_OK; ++knob) {
        const int32_t *cand = knob == 0 ? sm_cand : knob == 1 ? split_cand : kg_cand;
        cc_tune base = best;
        for (int i = 0; i < 4 && rc == CC_OK; ++i) {
            cc_tune t = base;
            if (knob == 0) t.small_max = cand[i];
            else if (knob == 1) t.sweep_split_tiles = cand[i];
            else t.kick_groups_per_cu = cand[i];
            double ms = 0.0;
            if ((rc = apply(t)) != CC_OK || (rc = time_step(&ms)) != CC_OK) break;
            best.trials++;
            if (ms < best.ms_per_step) {
                const int32_t trials = best.trials;
                best = t;
                best.ms_per_step = ms;
                best.trials = trials;
            }
        }
    }
    for (auto p : copy)
        if (p) hipFree(p);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (rc != CC_OK) {
        const std::string msg = c->err;
        cc_set_params(c, &keep);
        c->sweep_split = keep_split;
        c->kick_groups = keep_kg;
        c->err = msg;
        return rc;
    }
    RC(apply(best));
    if (out) *out = best;
    return CC_OK;
}

int cc_evolve_batch(cc_ctx *c, cc_state *s, const int64_t *offsets, int32_t ncl, double dt, double t_end,
                    cc_stats *out, void *stream)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    if (!offsets || ncl < 1) return fail(c, CC_ERR_ARG, "offsets is NULL or ncl < 1");
    if (offsets[0] != 0) return fail(c, CC_ERR_ARG, "offsets[0] must be 0");
    return evolve_common(c, s, offsets[ncl], offsets, ncl, dt, t_end, out, stream);
}

int cc_diagnostics(cc_ctx *c, const cc_state *s, int64_t n, double *out, void *stream)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    RC(check_state_ptrs(c, s));
    if (n < 1 || !out) return fail(c, CC_ERR_ARG, "n must be >= 1 and out non-NULL");
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const size_t need = (size_t)diag_blocks((int)n) * 24;
    if (need > c->diag_cap) {
        RC(dalloc(c, &c->diag_part, need));
        c->diag_cap = need;
    }
    HIPCHK(launch_diag(user_soa(s), (int)n, c->params.eps2, c->params.G, c->diag_part, c->diag_out, st));
    HIPCHK(hipMemcpyAsync(c->h_diag, c->diag_out, 12 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double *d = c->h_diag;
    out[0] = d[0];
    out[1] = d[1];
    for (int q = 2; q < 8; ++q) out[q] = d[q];
    for (int q = 8; q < 11; ++q) out[q] = d[q] / d[11];
    out[11] = d[11];
    return CC_OK;
}

int cc_timing_enable(cc_ctx *c, int32_t enable)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    HIPCHK(hipSetDevice(c->device));
    flush_timing(c);
    c->timing = enable != 0;
    if (c->timing) {
        for (int f = 0; f < F_N; ++f) {
            c->fam_ms[f] = 0.0;
            c->fam_launch[f] = 0;
        }
        HIPCHK(hipMemset(c->fam_work, 0, 2 * F_N * sizeof(uint64_t)));
    }
    return CC_OK;
}

int cc_timing_report(cc_ctx *c, cc_kernel_time *out, int32_t max)
{
    if (!c) return CC_ERR_ARG;
    c->err.clear();
    HIPCHK(hipSetDevice(c->device));
    flush_timing(c);
    uint64_t w[2 * F_N];
    HIPCHK(hipMemcpy(w, c->fam_work, sizeof w, hipMemcpyDeviceToHost));
    int k = 0;
    for (int f = 0; f < F_N; ++f) {
        if (k < max && out) {
            std::snprintf(out[k].name, sizeof out[k].name, "%s", fam_name[f]);
            out[k].launches = c->fam_launch[f];
            out[k].ms = c->fam_ms[f];
            out[k].tau_pairs = w[2 * f];
            out[k].kick_pairs = w[2 * f + 1];
        }
        k++;
    }
    return k;
}

}  // extern "C"
