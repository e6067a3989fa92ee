// cc_kernels.hip -- gfx950 kernels of the CC integrator.
//
// Grid-level kernels work on a list of segments (each an evolve_cc call on a
// contiguous slot range of the working arrays); the on-chip kernel runs the
// whole recursion of Fig. 2 for a component that fits in one workgroup's LDS;
// the pair kernel runs two-particle components one per lane.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include "cc_device.h"
#include "cc_launch.h"
#define CC_TILES_FN __device__ __forceinline__
#include "cc_tiles.h"

namespace ccg {

constexpr int TPB = 256;  // threads per block everywhere (4 wave64)
constexpr int WAVE = 64;  // wavefront width on gfx950

// Largest s in [0, nseg) with off[s] <= b (off is a prefix-sum array).
__device__ __forceinline__ int find_seg(const int32_t *off, int nseg, int b)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void stat_add(uint64_t *stats, int cluster, int idx, uint64_t v)
{
    if (v) atomicAdd((unsigned long long *)&stats[(size_t)cluster * ST_N + idx], (unsigned long long)v);
}

__device__ __forceinline__ void stat_max(uint64_t *stats, int cluster, int32_t d)
{
    atomicMax((unsigned long long *)&stats[(size_t)cluster * ST_N + ST_MAXD], (unsigned long long)d);
}

// Per-kernel-family algorithmic work (tau pairs, kick pairs) for roofline
// reporting; fam == nullptr when timing is off.
__device__ __forceinline__ void fam_add(uint64_t *fam, int idx, uint64_t v)
{
    if (fam && v) atomicAdd((unsigned long long *)&fam[idx], (unsigned long long)v);
}

// wave64 sum of a uint64
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// wave64 bitwise or of a uint64
__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Inclusive prefix sum over the lanes of a wavefront.
__device__ __forceinline__ int wave_incl_scan_i32(int v)
{
    const int lane = (int)(threadIdx.x & 63);
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Position of the k-th (0-based) set bit of m (k < popcount(m)).
__device__ __forceinline__ int nth_set_bit(uint64_t m, int k)
{
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = m & ((1ull << w) - 1ull);
        const int c = __popcll(low);
        if (k >= c) {
            k -= c;
            m >>= w;
            pos += w;
        } else {
            m = low;
        }
    }
    return pos;
}

// Block-wide sum to thread 0 (TPB threads).
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *sh)
{
    v = wave_sum_u64(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    uint64_t t = 0;
    if (threadIdx.x == 0) t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// Global union-find helpers (parent array in global memory, L1 bypassed,
// one entry per PARENT_STRIDE ints).
// The smaller root always becomes the parent, so a tree's root is its
// smallest slot and the final label is the component's smallest slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t gload(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void gstore(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Parent pointers only ever point to smaller slots, so a walk ends within
// the segment size; the budgets only guard against a corrupted structure and
// set `over` when they run out (the caller reports EB_BUDGET: never a silent
// wrong partition).
__device__ __forceinline__ int32_t *pslot(int32_t *par, int32_t a) { return par + (size_t)a * PARENT_STRIDE; }

__device__ __forceinline__ int32_t gfind(int32_t *par, int32_t a, bool &over)
{
    for (int it = 0; it < FIND_BUDGET; ++it) {
        const int32_t q = gload(pslot(par, a));
        if (q == a) return a;
        const int32_t g = gload(pslot(par, q));
        if (g != q) gstore(pslot(par, a), g);  // path halving: g is an ancestor of a
        a = q;
    }
    over = true;
    return a;
}

__device__ __forceinline__ int32_t gunite(int32_t *par, int32_t a, int32_t b, bool &over)
{
    for (int it = 0; it < UNITE_RETRIES; ++it) {
        a = gfind(par, a, over);
        b = gfind(par, b, over);
        if (a == b) return a;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(pslot(par, b), b, a) == b) return a;
    }
    over = true;
    return a;
}

// Read-only views of the state in the constant address space: wave-uniform
// loads through them become scalar loads into scalar registers.  Only for
// kernels that do not write the arrays they read this way.
typedef __attribute__((address_space(4))) const double CDouble;
typedef __attribute__((address_space(4))) const int32_t CInt;
__device__ __forceinline__ const CDouble *to_const(const double *p) { return (const CDouble *)(p); }
__device__ __forceinline__ const CInt *to_const(const int32_t *p) { return (const CInt *)(p); }

// LDS union-find (same rule: the smaller root becomes the parent)
__device__ __forceinline__ bool bit_of(const uint32_t *w, int p) { return (w[p >> 5] >> (p & 31)) & 1u; }

__device__ __forceinline__ int32_t lload(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lstore(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Find with path halving: every pointer written is an ancestor of the node,
// which keeps the structure valid under concurrent hooking.
__device__ __forceinline__ int32_t lfind(int32_t *par, int32_t a, bool &over)
{
    for (int it = 0; it < LDS_FIND_BUDGET; ++it) {
        const int32_t q = lload(&par[a]);
        if (q == a) return a;
        const int32_t g = lload(&par[q]);
        if (g != q) lstore(&par[a], g);
        a = q;
    }
    over = true;
    return a;
}

// Joins the sets of a and b; returns the root of the joined set (as seen now).
__device__ __forceinline__ int32_t lunite(int32_t *par, int32_t a, int32_t b, bool &over)
{
    for (int it = 0; it < LDS_FIND_BUDGET; ++it) {
        a = lfind(par, a, over);
        b = lfind(par, b, over);
        if (a == b) return a;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&par[b], b, a) == b) return a;
    }
    over = true;
    return a;
}

// ---------------------------------------------------------------------------
// Elementwise kernels
// ---------------------------------------------------------------------------
__global__ void k_validate(const double *__restrict__ x, const double *__restrict__ y,
                           const double *__restrict__ z, const double *__restrict__ vx,
                           const double *__restrict__ vy, const double *__restrict__ vz,
                           const double *__restrict__ m, int64_t n, int32_t *err)
{
    int bits = 0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        if (!(m[i] > 0.0) || !isfinite(m[i])) bits |= EB_MASS;
        if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i]) || !isfinite(vx[i]) || !isfinite(vy[i]) ||
            !isfinite(vz[i]))
            bits |= EB_NONFINITE;
    }
    if (bits) atomicOr(err, bits);
}

__global__ void k_pair_tau(SoA S, const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                           int64_t npairs, double *__restrict__ out, DevParams p)
{
    for (int64_t k = blockIdx.x * (int64_t)TPB + threadIdx.x; k < npairs; k += (int64_t)gridDim.x * TPB) {
        const int32_t i = pi[k], j = pj[k];
        out[k] = tau_pair(S.x[i] - S.x[j], S.y[i] - S.y[j], S.z[i] - S.z[j], S.vx[i] - S.vx[j],
                          S.vy[i] - S.vy[j], S.vz[i] - S.vz[j], S.m[i] + S.m[j], p);
    }
}

__global__ void k_drift_mask(SoA S, int64_t n, const uint8_t *__restrict__ mask, double h)
{
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        if (mask && !mask[i]) continue;
        S.x[i] += h * S.vx[i];
        S.y[i] += h * S.vy[i];
        S.z[i] += h * S.vz[i];
    }
}

__global__ void k_iota(int32_t *a, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
        a[i] = (int32_t)i;
}

__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) a[i] = v;
}

// ---------------------------------------------------------------------------
// Grid-level split.  Segments are described by prefix arrays over slot
// chunks of TPB (chunk_off) and over triangular tile pairs (tile_off).
// ---------------------------------------------------------------------------

// Union-find reset of slots [0, n): parent[u] = u, cnt[u] = 0.  Deeper
// levels are reset by the kernels that precede their visits (the level's
// forward permutation and its kick combine).
__global__ void k_uf_init(int32_t *parent, int32_t *cnt, int n)
{
    for (int u = blockIdx.x * TPB + threadIdx.x; u < n; u += gridDim.x * TPB) {
        *pslot(parent, u) = u;
        cnt[u] = 0;
    }
}

// Star test (Sec. 2.3, the fully connected case) ahead of the sweep: with X
// the segment's first slot, the segment is one component if tau(X,U) < h for
// every other U; notstar[s] is set when some U fails.  Run on levels whose
// previous visit found a star, so that a star costs n-1 pair steps and the
// sweep skips it.
template <bool MIXED>
__global__ __launch_bounds__(TPB) void k_star(SoA S, const Seg *__restrict__ seg,
                                               const int32_t *__restrict__ chunk_off, int nseg,
                                               int32_t *__restrict__ notstar, int32_t epoch, DevParams p, double h,
                                               uint64_t *stats, uint64_t *fam)
{
    __shared__ uint64_t sh[4];
    const int s = find_seg(chunk_off, nseg, blockIdx.x);
    const Seg g = seg[s];
    const int local = (blockIdx.x - chunk_off[s]) * TPB + threadIdx.x;
    const int X = g.start;
    uint64_t ev = 0;
    if (local > 0 && local < g.n) {
        const int u = g.start + local;
        ev = 1;
        if (!edge_decide<MIXED>(S.x[X] - S.x[u], S.y[X] - S.y[u], S.z[X] - S.z[u], S.vx[X] - S.vx[u],
                                S.vy[X] - S.vy[u], S.vz[X] - S.vz[u], S.m[X] + S.m[u], p, screen_params(p, h),
                                ccs::screen64_params(p.eta, h), h))
            notstar[s] = epoch;
    }
    const uint64_t t = block_sum_u64(ev, sh);
    if (threadIdx.x == 0) {
        stat_add(stats, g.cluster, ST_TAU, t);
        fam_add(fam, 0, t);
    }
}

// All-pairs sweep of a segment: for each pair i<j with tau(i,j) < h, merge
// their sets.  Without a star pass ahead of it, the tiles of the first row
// take the star test of Sec. 2.3 themselves (the set is fully connected when
// its first slot X has tau(X,U) < h with every other U): a tile that sees X
// miss one of its partners marks the segment in notstar.  After a star pass
// (star_pass), the tiles of a star segment do nothing.  Work is cut into
// 64x64 tiles (i tile <= j tile), one per wavefront, four per block.  A wavefront stages
// its j tile in LDS, joins edges in a union-find local to the tile over its
// 128 particles (64 when i tile = j tile), skipping an edge whose particles
// already share the global root read at tile start, and finally merges each
// particle whose local root has a different global root into the global
// structure: at most one global union per particle per tile.
constexpr int ST = 64;  // sweep tile edge (one wavefront)

#ifndef SWEEP_WAVES
#define SWEEP_WAVES 7
#endif
#ifndef FAR_UNROLL
#define FAR_UNROLL 4
#endif

// Workgroups of a launch are handed to the eight XCDs in turn (block b to XCD
// b mod 8), and each XCD has its own L2.  The sweep renumbers its blocks so
// that every XCD takes one contiguous share of the tile order: with the
// blocked tile order, consecutive tiles share their particles, which then
// stay in that XCD's L2.  A bijection of [0, nb).
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int q = nb / NXCD, r = nb % NXCD;
    const int x = b % NXCD, k = b / NXCD;
    return x * q + min(x, r) + k;
}

// A partner of the sweep's far-pair loop, with G m for the test's mu.
struct alignas(16) Partner {
    double x, y, z, m, vx, vy, vz, gm;
};

// Launches of up to split_tiles tiles split each tile's partners over JS = 4
// wavefronts so that the partner loops are short (the host's tuned value; a
// split in two for mid-size launches measured slower than none).

// One ST x ST tile of a set's pair triangle per JS wavefronts: wavefront
// jpart of the tile takes the tile's i particles against its ST/JS partners
// (JS = 1 for large launches; JS > 1 shortens the partner loop when a launch
// has few tiles).  The tile's edges are first linked in an LDS union-find over
// its 2 ST particles, then merged into the global structure.
template <bool MIXED, int JS>
__global__ __launch_bounds__(TPB, SWEEP_WAVES) void k_sweep(SoA S, const Seg *__restrict__ seg,
                                                const int32_t *__restrict__ tile_off, int nseg,
                                                int32_t *__restrict__ notstar, int32_t epoch, int star_pass,
                                                int32_t *__restrict__ parent, DevParams p, double h,
                                                int32_t *err)
{
    constexpr int NW = TPB / ST;   // wavefronts per block
    constexpr int TPW = NW / JS;   // tiles per block
    constexpr int JW = ST / JS;    // partners per wavefront
    static_assert(NW % JS == 0, "JS must divide the wavefronts of a block");
    // each wavefront's partners: one 64-byte record per partner, read by all
    // lanes at once (a broadcast) in the far-pair loop
    __shared__ Partner pj[NW][JW];
    // lpar and groot also hold the wavefront's edge and undecided bits during
    // a cooperative stage two (JS = 1: one wavefront per tile)
    __shared__ __align__(16) int32_t lpar[TPW][2 * ST];
    __shared__ __align__(16) int32_t groot[TPW][2 * ST];
    __shared__ uint32_t eflag[TPW][2 * ST / 32];  // slots of the tile that carry an edge
    const int w = threadIdx.x / ST, lane = threadIdx.x % ST;
    const int ts = w / JS, jpart = w % JS;
    // one tile per wavefront: its index, decode and segment are wavefront-
    // uniform and go to the scalar unit
    const int tile = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * TPW + ts);
    const int total = tile_off[nseg];
    int s = 0, ti = 0, tj = 0, T = 0;
    bool active = tile < total;
    if (active) {
        s = find_seg(tile_off, nseg, tile);
        active = !star_pass || notstar[s] == epoch;
    }
    Seg g{0, 0, 0, 0};
    if (active) {
        g = seg[s];
        T = (g.n + ST - 1) / ST;
        cct::blocked_tile(T, tile - tile_off[s], ti, tj);
    }
    const bool diag = (ti == tj);
    const int jn = active ? min(ST, g.n - tj * ST) : 0;
    const int j0w = jpart * JW;                      // first partner of this wavefront within the tile
    const int jnw = max(0, min(JW, jn - j0w));       // partners of this wavefront
    const int il = ti * ST + lane;
    const bool ivalid = active && il < g.n;
    const int i = g.start + (ivalid ? il : 0);
    int32_t *lp = lpar[ts];
    int32_t *gr = groot[ts];
    uint32_t *ef = eflag[ts];
    if (jpart == 0 && lane < 2 * ST / 32) ef[lane] = 0;
    // this wavefront's partners, and whether they and its own particles all
    // lie in the far-pair test's box
    bool inbox = true;
    if (active && lane < jnw) {
        const int j = g.start + tj * ST + j0w + lane;
        Partner q;
        q.x = S.x[j];
        q.y = S.y[j];
        q.z = S.z[j];
        q.m = S.m[j];
        q.vx = S.vx[j];
        q.vy = S.vy[j];
        q.vz = S.vz[j];
        q.gm = p.G * q.m;
        pj[w][lane] = q;
        inbox = ccs::far64_in_box(q.x, q.y, q.z, q.vx, q.vy, q.vz, q.gm);
    }
    double xi = 0.0, yi = 0.0, zi = 0.0, vxi = 0.0, vyi = 0.0, vzi = 0.0, mi = 0.0;
    if (active) {
        xi = S.x[i];
        yi = S.y[i];
        zi = S.z[i];
        vxi = S.vx[i];
        vyi = S.vy[i];
        vzi = S.vz[i];
        mi = S.m[i];
        if (ivalid) inbox &= ccs::far64_in_box(xi, yi, zi, vxi, vyi, vzi, p.G * mi);
    }
    const bool allbox = __all(inbox);
    __syncthreads();
    uint64_t emask = 0;
    if (active) {
        const ScreenParams q = screen_params(p, h);
        const ccs::Screen64 s64 = ccs::screen64_params(p.eta, h);
        const ccs::Far64 f64 = ccs::far64_params(p.eta, h);
        // Decide every pair first (one bit per partner: edge, or left to the
        // literal formula), then resolve the undecided pairs and link the
        // edges.  Stage one, uniform across the wavefront: the far-pair test
        // on r^2, |u|^2 and mu, which settles most pairs of the deep levels;
        // partners are broadcast from LDS, FAR_UNROLL per step.  Each test's
        // verdict stays a wavefront mask (the lanes with an open pair against
        // that partner, scalar registers); only a step that left some pair
        // open moves its bits into the lanes' masks.  Outside the test's box
        // (never for particles of a star cluster) every pair stays open.
        const Partner *P = pj[w];
        const int jnu = __builtin_amdgcn_readfirstlane(jnw);
        uint64_t smask = jnu >= 64 ? ~0ull : ((1ull << jnu) - 1ull);
        if (allbox && f64.on && p.eps2 <= 0x1p98) {
            const double gmi = p.G * mi, eps2 = p.eps2;
            smask = 0;
            int j0 = 0;
            for (; j0 + FAR_UNROLL <= jnu; j0 += FAR_UNROLL) {
                uint64_t open[FAR_UNROLL];
                uint64_t any = 0;
#pragma unroll
                for (int k = 0; k < FAR_UNROLL; ++k) {
                    const Partner r = P[j0 + k];
                    const ccs::Far64Terms t = ccs::far64_boxed_terms(xi - r.x, yi - r.y, zi - r.z, vxi - r.vx,
                                                                     vyi - r.vy, vzi - r.vz, gmi + r.gm, eps2, f64);
                    open[k] = ~(__ballot(t.r2ok) & __ballot(t.ff) & __ballot(t.fb1) &
                                (__ballot(t.fb2) | __ballot(t.still)));
                    any |= open[k];
                }
                if (any) {
#pragma unroll
                    for (int k = 0; k < FAR_UNROLL; ++k) smask |= ((open[k] >> lane) & 1ull) << (j0 + k);
                }
            }
            for (; j0 < jnu; ++j0) {
                const Partner r = P[j0];
                const bool far = ccs::far64_boxed(xi - r.x, yi - r.y, zi - r.z, vxi - r.vx, vyi - r.vy, vzi - r.vz,
                                                  gmi + r.gm, eps2, f64);
                smask |= far ? 0ull : (1ull << j0);
            }
        }
        // partners of this lane: j > i on the diagonal tile, all j otherwise
        const int sh = lane + 1 - j0w;  // first partner bit with j > i
        const uint64_t keep = !ivalid ? 0ull : (!diag || sh <= 0) ? ~0ull : (sh >= 64) ? 0ull : (~0ull << sh);
        smask &= keep;
        // Stage two: the certified screen on the open pairs.  Each lane takes
        // its own, unless a few lanes hold most of them (near the top pivot
        // steps, where many pairs lie close to the threshold): then the
        // wavefront deals them out 64 at a time, each lane screening the k-th
        // open pair of the wavefront for its owner lane, and the verdicts go
        // back to the owners through LDS (this tile's lpar and groot, not yet
        // in use).  Both ways screen the same pairs with the same arguments.
        uint64_t umask = 0;
        const int nopen = __popcll(smask);
        bool coop = false;
        if (JS == 1 && !MIXED) {  // (with the FP32 screen in front, the registers spill)
            const int cmax = wave_max_i32(nopen);
            if (cmax > 4) {
                const int incl = wave_incl_scan_i32(nopen);
                const int total = __shfl(incl, 63, 64);
                const int rounds = (total + 63) / 64;
                coop = cmax > 2 * rounds + 2;  // uniform across the wavefront
                if (coop) {
                    uint64_t *em = reinterpret_cast<uint64_t *>(lp);  // 64 words each
                    uint64_t *um = reinterpret_cast<uint64_t *>(gr);
                    em[lane] = 0;
                    um[lane] = 0;
                    const int excl = incl - nopen;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    for (int base = 0; base < total; base += 64) {
                        const int t = base + lane;
                        // owner: the last lane whose first open pair is at or before t
                        int o = 0;
#pragma unroll
                        for (int stp = 32; stp >= 1; stp >>= 1) {
                            const int ex = __shfl(excl, o + stp, 64);
                            if (o + stp < 64 && ex <= t) o += stp;
                        }
                        const int ko = t - __shfl(excl, o, 64);
                        const uint64_t mo = __shfl(smask, o, 64);
                        if (t < total) {
                            const int jj = nth_set_bit(mo, ko);
                            const int io = g.start + ti * ST + o;
                            const Partner &r = P[jj];
                            const int d = edge_screen<MIXED>(S.x[io] - r.x, S.y[io] - r.y, S.z[io] - r.z,
                                                             S.vx[io] - r.vx, S.vy[io] - r.vy, S.vz[io] - r.vz,
                                                             S.m[io] + r.m, p, q, s64);
                            const uint64_t bit = 1ull << jj;
                            if (d == ccs::SCREEN64_EDGE) atomicOr(&em[o], bit);
                            if (d == ccs::SCREEN64_UNSURE) atomicOr(&um[o], bit);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    emask = em[lane];
                    umask = um[lane];
                    smask = 0;
                }
            }
        }
        // this lane's particle again for stages two and three (a cached
        // load: kept in registers through the cooperative stage two, it spilled)
        const double xs = __builtin_nontemporal_load(&S.x[i]), ys = __builtin_nontemporal_load(&S.y[i]),
                     zs = __builtin_nontemporal_load(&S.z[i]), vxs = __builtin_nontemporal_load(&S.vx[i]),
                     vys = __builtin_nontemporal_load(&S.vy[i]), vzs = __builtin_nontemporal_load(&S.vz[i]),
                     ms = __builtin_nontemporal_load(&S.m[i]);
        while (smask) {
            const int jj = __builtin_ctzll(smask);
            smask &= smask - 1;
            const Partner &r = P[jj];
            const int d = edge_screen<MIXED>(xs - r.x, ys - r.y, zs - r.z, vxs - r.vx, vys - r.vy, vzs - r.vz,
                                             ms + r.m, p, q, s64);
            const uint64_t bit = 1ull << jj;
            emask |= (d == ccs::SCREEN64_EDGE) ? bit : 0ull;
            umask |= (d == ccs::SCREEN64_UNSURE) ? bit : 0ull;
        }
        while (umask) {
            const int jj = __builtin_ctzll(umask);
            umask &= umask - 1;
            const Partner &r = P[jj];
            if (edge_pair(xs - r.x, ys - r.y, zs - r.z, vxs - r.vx, vys - r.vy, vzs - r.vz, ms + r.m, p, h))
                emask |= 1ull << jj;
        }
        if (ti == 0 && lane == 0) {
            // star test: X = the segment's first slot against this wave's partners
            const uint64_t all = keep & (jnw >= 64 ? ~0ull : ((1ull << jnw) - 1ull));
            if (emask != all) notstar[s] = epoch;
        }
        // flag the slots that carry an edge: this lane's particle, and every
        // partner some lane links to
        if (emask) atomicOr(&ef[lane >> 5], 1u << (lane & 31));
        const uint64_t any = wave_or_u64(emask);  // (also orders the LDS reads above before the reset below)
        if (lane == 0 && any) {
            const int base = (diag ? 0 : ST) + j0w;  // slot of partner bit 0 (a multiple of JW)
            atomicOr(&ef[base >> 5], (uint32_t)(any << (base & 31)));
            if (JW > 32) atomicOr(&ef[(base >> 5) + 1], (uint32_t)(any >> 32));
        }
    }
    // the tile-local union-find over its 2 ST slots (after a cooperative
    // stage two, which used this memory)
    if (jpart == 0) {
        lp[lane] = lane;
        gr[lane] = -1;
    }
    if (lane < JW) {
        const int v = ST + j0w + lane;
        lp[v] = v;
        gr[v] = -1;
    }
    __syncthreads();
    // global roots of the flagged slots only: a tile without an edge (most
    // tiles of the deep levels) makes no union-find access at all
    bool over = false;  // a union-find budget ran out
    if (jpart == 0 && ivalid && bit_of(ef, lane)) gr[lane] = gfind(parent, i, over);
    if (lane < jnw && !diag && bit_of(ef, ST + j0w + lane))
        gr[ST + j0w + lane] = gfind(parent, g.start + tj * ST + j0w + lane, over);
    __syncthreads();
    if (emask) {
        const int32_t gi = gr[lane];
        int32_t lr = lane;  // an ancestor of this particle in the local structure
        const int joff = (diag ? 0 : ST) + j0w;
        while (emask) {
            const int jj = __builtin_ctzll(emask);
            emask &= emask - 1;
            const int vj = joff + jj;
            if (gr[vj] != gi) lr = lunite(lp, lr, vj, over);
        }
    }
    __syncthreads();
    // merge the tile's local sets into the global structure
    for (int v = jpart * ST + lane; v < 2 * ST; v += JS * ST) {
        if (gr[v] < 0) continue;
        const int r = lfind(lp, v, over);
        if (r != v && gr[r] != gr[v]) gunite(parent, gr[v], gr[r], over);
    }
    if (over) atomicOr(err, EB_BUDGET);
}

// Labels (smallest slot of the component) and component sizes.  With keys,
// also the sort keys of the active particles (key = label, value = slot: a
// stable sort by label makes every component contiguous, members in slot
// order), and with `count` the level's work-list counters are cleared.
__global__ __launch_bounds__(TPB) void k_label(const Seg *__restrict__ seg, const int32_t *__restrict__ chunk_off,
                                                const int32_t *__restrict__ act_off, int nseg,
                                                const int32_t *__restrict__ notstar, int32_t epoch,
                                                int32_t *__restrict__ parent, int32_t *__restrict__ label,
                                                int32_t *__restrict__ cnt, uint32_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals, int32_t *__restrict__ count,
                                                int32_t *__restrict__ hold, int star_pass, uint64_t *stats,
                                                uint64_t *sweep_fam, int32_t *err)
{
    const int s = find_seg(chunk_off, nseg, blockIdx.x);
    const Seg g = seg[s];
    const int local = (blockIdx.x - chunk_off[s]) * TPB + threadIdx.x;
    const bool ns = notstar[s] == epoch;
    const bool valid = local < g.n;
    if (count && blockIdx.x == 0 && threadIdx.x < 8) count[threadIdx.x] = 0;
    if (hold && local == 0) {
        hold[2 * s] = INT32_MAX;
        hold[2 * s + 1] = 0;
    }
    int32_t l = -1;
    if (valid) {
        const int u = g.start + local;
        bool over = false;
        l = ns ? gfind(parent, u, over) : g.start;
        if (over) atomicOr(err, EB_BUDGET);
        label[u] = l;
        if (keys) {
            const int k = act_off[s] + local;
            keys[k] = (uint32_t)l;
            vals[k] = (uint32_t)u;
        }
    }
    // component sizes: one atomic per distinct label of the wavefront (a
    // large component fills whole wavefronts with one label)
    const int lane = threadIdx.x % WAVE;
    uint64_t pending = __ballot(valid);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int32_t ll = __shfl(l, leader, WAVE);
        const uint64_t same = __ballot(valid && l == ll) & pending;
        if (lane == leader) atomicAdd(&cnt[ll], (int32_t)__popcll(same));
        pending &= ~same;
    }
    if (local == 0) {
        const uint64_t n = (uint64_t)g.n;
        // the HOLD split needs every particle's own time step: all pairs
        stat_add(stats, g.cluster, ST_TAU_ALG, (ns || hold) ? n * (n - 1) / 2 : n - 1);
        // the sweep evaluated every pair of the segment unless a star pass
        // ahead of it found the segment a star (counted here, once per
        // segment, rather than by an atomic per sweep tile)
        const uint64_t swept = (!star_pass || ns) ? n * (n - 1) / 2 : 0;
        stat_add(stats, g.cluster, ST_TAU, swept);
        fam_add(sweep_fam, 0, swept);
        stat_add(stats, g.cluster, ST_SPLIT, 1);
        stat_max(stats, g.cluster, g.depth);
    }
}

// HOLD split (Sec. 2.1, eqs. 11-12): a particle is fast when its own time
// step min_j tau(i,j) is below h, which is exactly when its component at h is
// non-trivial.  Per segment, the smallest fast slot becomes the label of F and
// the fast particles are counted; each component speaks through its root (the
// slot equal to its label), so one atomic per component.
__global__ __launch_bounds__(TPB) void k_hold_fast(const Seg *__restrict__ seg, const int32_t *__restrict__ chunk_off,
                                                    int nseg, const int32_t *__restrict__ label,
                                                    const int32_t *__restrict__ cnt, int32_t *__restrict__ hold)
{
    const int s = find_seg(chunk_off, nseg, blockIdx.x);
    const Seg g = seg[s];
    const int local = (blockIdx.x - chunk_off[s]) * TPB + threadIdx.x;
    if (local >= g.n) return;
    const int u = g.start + local;
    if (label[u] != u) return;
    const int32_t c = cnt[u];
    if (c >= 2) {
        atomicMin(&hold[2 * s], u);
        atomicAdd(&hold[2 * s + 1], c);
    }
}

// Every fast particle takes F's label (entry-order labels and the sort keys);
// F's label slot takes F's size.  The size written there is at least the
// component size it replaces, so concurrent "is fast" tests read the same
// answer either way.
__global__ __launch_bounds__(TPB) void k_hold_relabel(const Seg *__restrict__ seg,
                                                       const int32_t *__restrict__ chunk_off,
                                                       const int32_t *__restrict__ act_off, int nseg,
                                                       int32_t *__restrict__ label, int32_t *cnt,
                                                       uint32_t *__restrict__ keys, const int32_t *__restrict__ hold)
{
    const int s = find_seg(chunk_off, nseg, blockIdx.x);
    const Seg g = seg[s];
    const int local = (blockIdx.x - chunk_off[s]) * TPB + threadIdx.x;
    if (local >= g.n) return;
    const int u = g.start + local;
    const int32_t l = label[u];
    if (__hip_atomic_load(&cnt[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 2) return;
    const int32_t f = hold[2 * s];
    label[u] = f;
    keys[act_off[s] + local] = (uint32_t)f;
    if (u == f) __hip_atomic_store(&cnt[u], hold[2 * s + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Work lists of a level, filled while its components are made contiguous.
struct Lists {
    Seg *pairs;
    Seg *small[4];
    Seg *big;
    int32_t *count;  // [0] pairs, [1..4] small bins, [5] big
    int32_t cap_pairs, cap_small, cap_big;
    int32_t small_max;
    int32_t bin_lim[3];  // upper sizes of bins 0..2 (bin 3 up to small_max)
    int32_t *labp;       // optional: label of the particle now at each slot
    uint8_t *singp;      // optional: singleton flag of the particle now at each slot
    const int32_t *errf; // error bits, copied to count[7] for the host's one read-back
    const int32_t *notstar;  // the level's not-a-star flags: star segments are counted in count[6]
};

// Forward permutation of a level between the two working buffers: the k-th
// active particle in (label, slot) order, from slot src[k] of `from`, goes to
// its segment's k-th slot of `to`, so that every component is contiguous.
// It also resets the union-find of those slots for the next level.  With
// `lab` (the sorted labels) it records the singleton flags in entry order,
// with the lists the component-contiguous labels and singleton flags and the
// level's work lists (pairs, small components by size, big components), and
// with drift_hh > 0 it applies the singletons' drift D_{hh} on the way (the
// same operations as k_drift_seg).  Reads and writes touch different
// buffers: one launch, one block per 256-slot chunk of a segment.
__global__ __launch_bounds__(TPB) void k_permute(SoA from, SoA to, const Seg *__restrict__ seg,
                                                  const int32_t *__restrict__ chunk_off,
                                                  const int32_t *__restrict__ act_off, int nseg,
                                                  const uint32_t *__restrict__ src, const uint32_t *__restrict__ lab,
                                                  const int32_t *__restrict__ cnt, uint8_t *__restrict__ sing, Lists L,
                                                  int with_lists, double drift_hh, int32_t *__restrict__ parent,
                                                  int32_t *__restrict__ cnt_next, uint64_t *kick_fam, int count_kick,
                                                  int32_t epoch, uint64_t *stats)
{
    __shared__ uint64_t sh[4];
    const int s = find_seg(chunk_off, nseg, blockIdx.x);
    const Seg g = seg[s];
    const int local = (blockIdx.x - chunk_off[s]) * TPB + threadIdx.x;
    uint64_t drifted = 0;
    if (local < g.n) {
        const int k = act_off[s] + local;
        const int dst = g.start + local;
        const int u = (int)src[k];
        // union-find reset for the next level's visits (its counters are
        // the other parity's, so no read of cnt here races with the reset)
        if (parent) {
            *pslot(parent, dst) = dst;
            cnt_next[dst] = 0;
        }
        const int32_t l = lab ? (int32_t)lab[k] : -1;
        const bool single = lab && cnt[l] == 1;
        double x = from.x[u], y = from.y[u], z = from.z[u];
        const double vx = from.vx[u], vy = from.vy[u], vz = from.vz[u];
        if (single && drift_hh > 0.0) {
            x += drift_hh * vx;
            y += drift_hh * vy;
            z += drift_hh * vz;
            drifted = 1;
        }
        to.x[dst] = x;
        to.y[dst] = y;
        to.z[dst] = z;
        to.vx[dst] = vx;
        to.vy[dst] = vy;
        to.vz[dst] = vz;
        to.m[dst] = from.m[u];
        to.orig[dst] = from.orig[u];
        if (lab) {
            if (sing) sing[u] = single ? 1 : 0;
            if (with_lists) {
                if (k == 0) L.count[7] = __hip_atomic_load(L.errf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (local == 0 && L.notstar[s] != epoch) atomicAdd(&L.count[6], 1);  // a star segment
                if (count_kick && local == 0) {
                    // the tiled kick's pairs: all of the segment's ...
                    const uint64_t all = (uint64_t)g.n * (uint64_t)(g.n - 1) / 2;
                    stat_add(stats, g.cluster, ST_KICK, all);
                    fam_add(kick_fam, 1, all);
                }
                if (L.labp) {
                    L.labp[dst] = l;
                    L.singp[dst] = single ? 1 : 0;
                }
                const bool first = (local == 0) || ((int32_t)lab[k - 1] != l);
                const int32_t size = cnt[l];
                if (first && size >= 2) {
                    stat_add(stats, g.cluster, ST_COMP, 1);
                    if (count_kick) {
                        // ... less those inside a component (modulo 2^64)
                        const uint64_t in = (uint64_t)size * (uint64_t)(size - 1) / 2;
                        stat_add(stats, g.cluster, ST_KICK, (uint64_t)0 - in);
                        fam_add(kick_fam, 1, (uint64_t)0 - in);
                    }
                    const Seg c = {dst, size, g.cluster, g.depth + 1};
                    if (size == 2 && L.small_max >= 2) {
                        const int i = atomicAdd(&L.count[0], 1);
                        if (i < L.cap_pairs) L.pairs[i] = c;
                    } else if (size <= L.small_max) {
                        const int b = size <= L.bin_lim[0] ? 0 : size <= L.bin_lim[1] ? 1 : size <= L.bin_lim[2] ? 2 : 3;
                        const int i = atomicAdd(&L.count[1 + b], 1);
                        if (i < L.cap_small) L.small[b][i] = c;
                    } else {
                        const int i = atomicAdd(&L.count[5], 1);
                        if (i < L.cap_big) L.big[i] = c;
                    }
                }
            }
        }
    }
    if (drift_hh > 0.0) {  // uniform across the launch
        const uint64_t t = block_sum_u64(drifted, sh);
        if (threadIdx.x == 0) stat_add(stats, g.cluster, ST_DRIFT, t);
    }
}

// Inverse permutation: the k-th slot of its segment in `from` goes back to
// slot src[k] of `to` (entry order).
__global__ void k_unpermute(SoA from, SoA to, const Seg *__restrict__ seg, const int32_t *__restrict__ act_off,
                            int nseg, int nact, const uint32_t *__restrict__ src)
{
    const int k = blockIdx.x * TPB + threadIdx.x;
    if (k >= nact) return;
    const int s = find_seg(act_off, nseg, k);
    const int v = seg[s].start + (k - act_off[s]);
    const int u = (int)src[k];
    to.x[u] = from.x[v];
    to.y[u] = from.y[v];
    to.z[u] = from.z[v];
    to.vx[u] = from.vx[v];
    to.vy[u] = from.vy[v];
    to.vz[u] = from.vz[v];
    to.m[u] = from.m[v];
    to.orig[u] = from.orig[v];
}

// Drift D_{hh} of the segment's singletons (entry order).
__global__ void k_drift_seg(SoA W, const Seg *__restrict__ seg, const int32_t *__restrict__ chunk_off, int nseg,
                            const uint8_t *__restrict__ sing, double hh, uint64_t *stats)
{
    __shared__ uint64_t sh[4];
    const int s = find_seg(chunk_off, nseg, blockIdx.x);
    const Seg g = seg[s];
    const int local = (blockIdx.x - chunk_off[s]) * TPB + threadIdx.x;
    uint64_t c = 0;
    if (local < g.n) {
        const int u = g.start + local;
        if (sing[u]) {
            W.x[u] += hh * W.vx[u];
            W.y[u] += hh * W.vy[u];
            W.z[u] += hh * W.vz[u];
            c = 1;
        }
    }
    const uint64_t t = block_sum_u64(c, sh);
    if (threadIdx.x == 0) stat_add(stats, g.cluster, ST_DRIFT, t);
}

// Kick K_h for all pairs of a segment with different labels (V_R + V_CC +
// V_CR, eq. 30).  Each particle sums its partners in ascending slot order
// (= ascending particle index within the segment), exactly the order in
// which a sequential i<j sweep accumulates both members of every pair.
// label == NULL kicks every pair.
__global__ __launch_bounds__(TPB) void k_kick_seg(SoA W, const Seg *__restrict__ seg,
                                                   const int32_t *__restrict__ chunk_off, int nseg,
                                                   const int32_t *__restrict__ label, double h, double eps2,
                                                   double G, int32_t *err, uint64_t *stats, uint64_t *fam)
{
    __shared__ double jx[TPB], jy[TPB], jz[TPB], jm[TPB];
    __shared__ int32_t jl[TPB];
    __shared__ uint64_t sh[4];
    const int s = find_seg(chunk_off, nseg, blockIdx.x);
    const Seg g = seg[s];
    const int local = (blockIdx.x - chunk_off[s]) * TPB + threadIdx.x;
    const bool valid = local < g.n;
    const int i = g.start + (valid ? local : 0);
    const double xi = W.x[i], yi = W.y[i], zi = W.z[i];
    const int32_t li = label ? label[i] : i;
    double ax = 0.0, ay = 0.0, az = 0.0;
    uint64_t pairs = 0;
    bool ok = true;
    for (int jb = 0; jb < g.n; jb += TPB) {
        const int jn = min(TPB, g.n - jb);
        __syncthreads();
        if (threadIdx.x < jn) {
            const int j = g.start + jb + threadIdx.x;
            jx[threadIdx.x] = W.x[j];
            jy[threadIdx.x] = W.y[j];
            jz[threadIdx.x] = W.z[j];
            jm[threadIdx.x] = W.m[j];
            jl[threadIdx.x] = label ? label[j] : j;
        }
        __syncthreads();
        if (valid) {
            for (int jj = 0; jj < jn; ++jj) {
                const int j = g.start + jb + jj;
                if (jl[jj] == li || j == i) continue;
                ok &= accel_term(xi, yi, zi, jx[jj], jy[jj], jz[jj], jm[jj], eps2, G, ax, ay, az);
                pairs += (j > i);
            }
        }
    }
    if (valid) {
        if (!ok) atomicOr(err, EB_NONFINITE);
        W.vx[i] += h * ax;
        W.vy[i] += h * ay;
        W.vz[i] += h * az;
    }
    const uint64_t t = block_sum_u64(pairs, sh);
    if (threadIdx.x == 0 && stats) {
        stat_add(stats, g.cluster, ST_KICK, t);
        fam_add(fam, 1, t);
    }
}

// Kick K_h in the component-contiguous slot order (labels non-decreasing
// within a segment).  Block b takes the i tile and j range of blk[b]; the
// host leaves out of the ranges of an i tile that lies inside one large
// component that component itself (all of its pairs are inside it), and a j
// tile inside the i tile's own component is skipped whole here.  Each block
// writes its partial accelerations; k_kick_combine adds the blocks of every i
// tile in list order, so the result is deterministic.  The pairs kicked are
// counted by the forward permutation (n(n-1)/2 per segment less s(s-1)/2 per
// component), not here.
// A partner of the tiled kick: position and G m.
struct alignas(16) KickPartner {
    double x, y, z, gm;
};

template <bool MIXED>
__global__ __launch_bounds__(TPB, 8) void k_kick_tiles(SoA W, const Seg *__restrict__ seg,
                                                     const KickBlock *__restrict__ blk,
                                                     const int32_t *__restrict__ labp, double eps2, double G,
                                                     double *__restrict__ part, int32_t *err)
{
    // the block's partners, 256 at a time: one 32-byte record each (G m in
    // FP32 precision for the mixed kick), read by all lanes at once
    __shared__ KickPartner kj[TPB];
    __shared__ int32_t jl[TPB];
    const KickBlock kb = blk[blockIdx.x];
    const Seg g = seg[kb.seg];
    const int I = kb.itile;
    const int jlo = kb.j0, jhi = kb.j0 + kb.nj;
    const int il = I * TPB + threadIdx.x;
    const bool valid = il < g.n;
    const int i = g.start + (valid ? il : 0);
    const double xi = W.x[i], yi = W.y[i], zi = W.z[i];
    const int32_t li = labp[i];
    const int ifirst = g.start + I * TPB, ilast = g.start + min(g.n, (I + 1) * TPB) - 1;
    const int32_t iu = (labp[ifirst] == labp[ilast]) ? labp[ifirst] : -1;
    double ax = 0.0, ay = 0.0, az = 0.0;
    bool ok = true;
    for (int jb = jlo; jb < jhi; jb += TPB) {
        const int jn = min(TPB, jhi - jb);
        const int jfirst = g.start + jb, jlast = g.start + jb + jn - 1;
        if (iu >= 0 && labp[jfirst] == iu && labp[jlast] == iu) continue;  // uniform across the block
        __syncthreads();
        if (threadIdx.x < jn) {
            const int j = g.start + jb + threadIdx.x;
            KickPartner q;
            q.x = W.x[j];
            q.y = W.y[j];
            q.z = W.z[j];
            q.gm = MIXED ? (double)(float)(G * W.m[j]) : G * W.m[j];
            kj[threadIdx.x] = q;
            jl[threadIdx.x] = labp[j];
        }
        __syncthreads();
        const int jnu = __builtin_amdgcn_readfirstlane(jn);
        if (!MIXED) {
            // FP64, no branch per partner; a coincident pair shows as a
            // non-finite sum.  Labels are non-decreasing along a segment, so a
            // chunk whose label range misses the i tile's holds no partner of
            // an own component (nor i itself): no mask at all.  Otherwise
            // partners of the own component add a zero factor.
            const bool disjoint = labp[jlast] < labp[ifirst] || labp[jfirst] > labp[ilast];  // uniform
            int jj = 0;
            if (disjoint) {
                for (; jj + 4 <= jnu; jj += 4) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const KickPartner q = kj[jj + k];
                        accel_term_rsq_if(true, xi, yi, zi, q.x, q.y, q.z, q.gm, eps2, ax, ay, az);
                    }
                }
                for (; jj < jnu; ++jj) {
                    const KickPartner q = kj[jj];
                    accel_term_rsq_if(true, xi, yi, zi, q.x, q.y, q.z, q.gm, eps2, ax, ay, az);
                }
            } else {
                for (; jj + 4 <= jnu; jj += 4) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const KickPartner q = kj[jj + k];
                        accel_term_rsq_if(jl[jj + k] != li, xi, yi, zi, q.x, q.y, q.z, q.gm, eps2, ax, ay, az);
                    }
                }
                for (; jj < jnu; ++jj) {
                    const KickPartner q = kj[jj];
                    accel_term_rsq_if(jl[jj] != li, xi, yi, zi, q.x, q.y, q.z, q.gm, eps2, ax, ay, az);
                }
            }
        } else if (valid) {
            // FP32 forces on FP64 differences, Kahan-compensated within the
            // tile, FP64 across tiles
            Kahan3 k{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const float e2 = (float)eps2;
            for (int jj = 0; jj < jnu; ++jj) {
                if (jl[jj] == li) continue;
                const KickPartner q = kj[jj];
                ok &= accel_term32(xi, yi, zi, q.x, q.y, q.z, (float)q.gm, e2, k);
            }
            ax += (double)k.sx - (double)k.cx;
            ay += (double)k.sy - (double)k.cy;
            az += (double)k.sz - (double)k.cz;
        }
    }
    double *pb = part + (size_t)blockIdx.x * 3 * TPB;
    pb[threadIdx.x] = ax;
    pb[TPB + threadIdx.x] = ay;
    pb[2 * TPB + threadIdx.x] = az;
    if (!MIXED) ok = isfinite(ax) && isfinite(ay) && isfinite(az);
    if (valid && !ok) atomicOr(err, EB_NONFINITE);
}

// Group sums of the two-stage reduction: job b adds its slots in order.
__global__ __launch_bounds__(TPB) void k_kick_reduce(const KickJob *__restrict__ jobs, double *__restrict__ part)
{
    const KickJob jb = jobs[blockIdx.x];
    const double *pb = part + (size_t)jb.src * 3 * TPB;
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll 8
    for (int q = 0; q < jb.n; ++q) {
        ax += pb[(size_t)q * 3 * TPB + threadIdx.x];
        ay += pb[(size_t)q * 3 * TPB + TPB + threadIdx.x];
        az += pb[(size_t)q * 3 * TPB + 2 * TPB + threadIdx.x];
    }
    double *po = part + (size_t)jb.dst * 3 * TPB;
    po[threadIdx.x] = ax;
    po[TPB + threadIdx.x] = ay;
    po[2 * TPB + threadIdx.x] = az;
}

// Adds the partial accelerations of every i in slot order, applies the kick,
// then the drift D_{hh} of the singletons that ends the level's D K D; also
// resets the union-find of the level's slots for the second half.
__global__ __launch_bounds__(TPB) void k_kick_combine(SoA W, const Seg *__restrict__ seg,
                                                       const int32_t *__restrict__ chunk_off,
                                                       const KickTile *__restrict__ ktile, int nseg,
                                                       const double *__restrict__ part, double h,
                                                       const uint8_t *__restrict__ sing, double hh,
                                                       int32_t *__restrict__ parent, int32_t *__restrict__ cnt_next,
                                                       uint64_t *stats)
{
    __shared__ uint64_t sh[4];
    const int s = find_seg(chunk_off, nseg, blockIdx.x);
    const Seg g = seg[s];
    const int I = blockIdx.x - chunk_off[s];
    const int il = I * TPB + threadIdx.x;
    uint64_t drifted = 0;
    if (il < g.n) {
        // union-find reset for the second-half visits of the next level
        *pslot(parent, g.start + il) = g.start + il;
        cnt_next[g.start + il] = 0;
        const KickTile kt = ktile[blockIdx.x];
        const double *pb = part + (size_t)kt.src * 3 * TPB;
        double ax = 0.0, ay = 0.0, az = 0.0;
        // in order; unrolled so that many partial loads are in flight
#pragma unroll 8
        for (int q = 0; q < kt.n; ++q) {
            ax += pb[(size_t)q * 3 * TPB + threadIdx.x];
            ay += pb[(size_t)q * 3 * TPB + TPB + threadIdx.x];
            az += pb[(size_t)q * 3 * TPB + 2 * TPB + threadIdx.x];
        }
        const int u = g.start + il;
        W.vx[u] += h * ax;
        W.vy[u] += h * ay;
        W.vz[u] += h * az;
        if (sing[u]) {
            W.x[u] += hh * W.vx[u];
            W.y[u] += hh * W.vy[u];
            W.z[u] += hh * W.vz[u];
            drifted = 1;
        }
    }
    const uint64_t t = block_sum_u64(drifted, sh);
    if (threadIdx.x == 0) stat_add(stats, g.cluster, ST_DRIFT, t);
}

// Kick used by the cc_kick entry point: same sums, but velocities are written
// to separate output arrays so that a failing call leaves the state untouched.
// MIXED: FP32 pair forces on FP64 differences, Kahan-compensated over each
// 256-partner tile, FP64 across tiles (the mixed-precision kick).
template <bool MIXED>
__global__ __launch_bounds__(TPB) void k_kick_all(SoA W, int n, const int32_t *__restrict__ label, double eps2,
                                                   double G, double *__restrict__ ax_out,
                                                   double *__restrict__ ay_out, double *__restrict__ az_out,
                                                   int32_t *err)
{
    __shared__ double jx[TPB], jy[TPB], jz[TPB], jm[TPB];
    __shared__ int32_t jl[TPB];
    const int i0 = blockIdx.x * TPB + threadIdx.x;
    const bool valid = i0 < n;
    const int i = valid ? i0 : 0;
    const double xi = W.x[i], yi = W.y[i], zi = W.z[i];
    const int32_t li = label ? label[i] : i;
    double ax = 0.0, ay = 0.0, az = 0.0;
    bool ok = true;
    for (int jb = 0; jb < n; jb += TPB) {
        const int jn = min(TPB, n - jb);
        __syncthreads();
        if (threadIdx.x < jn) {
            const int j = jb + threadIdx.x;
            jx[threadIdx.x] = W.x[j];
            jy[threadIdx.x] = W.y[j];
            jz[threadIdx.x] = W.z[j];
            jm[threadIdx.x] = W.m[j];
            jl[threadIdx.x] = label ? label[j] : j;
        }
        __syncthreads();
        if (valid) {
            if (MIXED) {
                Kahan3 k{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                const float e2 = (float)eps2;
                for (int jj = 0; jj < jn; ++jj) {
                    const int j = jb + jj;
                    if (jl[jj] == li || j == i) continue;
                    ok &= accel_term32(xi, yi, zi, jx[jj], jy[jj], jz[jj], (float)(G * jm[jj]), e2, k);
                }
                ax += (double)k.sx - (double)k.cx;
                ay += (double)k.sy - (double)k.cy;
                az += (double)k.sz - (double)k.cz;
            } else {
                for (int jj = 0; jj < jn; ++jj) {
                    const int j = jb + jj;
                    if (jl[jj] == li || j == i) continue;
                    ok &= accel_term(xi, yi, zi, jx[jj], jy[jj], jz[jj], jm[jj], eps2, G, ax, ay, az);
                }
            }
        }
    }
    if (valid) {
        if (!ok) atomicOr(err, EB_NONFINITE);
        ax_out[i] = ax;
        ay_out[i] = ay;
        az_out[i] = az;
    }
}

__global__ void k_apply_kick(SoA W, int n, const double *__restrict__ ax, const double *__restrict__ ay,
                             const double *__restrict__ az, double h)
{
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    W.vx[i] += h * ax[i];
    W.vy[i] += h * ay[i];
    W.vz[i] += h * az[i];
}

// ---------------------------------------------------------------------------
// Two-particle components, one per lane.
// ---------------------------------------------------------------------------
// Two-particle components, one per thread: threads t0, t0 + nt, ... of the
// caller take items t0, t0 + nt, ...  Each thread sums its counters while its
// items stay in one cluster; at the end a wavefront whose threads all hold
// the same cluster adds its sums with one atomic per counter (the statistics
// are a handful of words that every wavefront of the launch would otherwise
// hit once per thread).
__device__ __forceinline__ void pair_counters_flush(uint64_t *stats, uint64_t *fam, int cluster,
                                                    const PairCounters &c)
{
    stat_add(stats, cluster, ST_TAU, c.tau);
    stat_add(stats, cluster, ST_TAU_ALG, c.tau);
    stat_add(stats, cluster, ST_KICK, c.kick);
    stat_add(stats, cluster, ST_DRIFT, c.drift);
    stat_add(stats, cluster, ST_COMP, c.comp);
    stat_add(stats, cluster, ST_SPLIT, c.split);
    stat_add(stats, cluster, ST_KEPLER, c.kepler);
    if (c.maxd >= 0) stat_max(stats, cluster, c.maxd);
    fam_add(fam, 0, c.tau);
    fam_add(fam, 1, c.kick);
}

template <bool MIXED>
__device__ void run_pairs(SoA W, const Seg *__restrict__ items, int n, int t0, int nt, double H, const DevParams &p,
                          int32_t *err, uint64_t *stats, uint64_t *fam)
{
    PairCounters tot{0, 0, 0, 0, 0, 0, -1};
    int cl = -1;  // cluster of the sums in tot
    for (int it = t0; it < n; it += nt) {
        const Seg g = items[it];
        int ia = g.start, ib = g.start + 1;
        if (W.orig[ib] < W.orig[ia]) {
            ia = g.start + 1;
            ib = g.start;
        }
        Body a{W.x[ia], W.y[ia], W.z[ia], W.vx[ia], W.vy[ia], W.vz[ia], W.m[ia]};
        Body b{W.x[ib], W.y[ib], W.z[ib], W.vx[ib], W.vy[ib], W.vz[ib], W.m[ib]};
        PairCounters c{0, 0, 0, 0, 0, 0, -1};
        // a top-level set of two particles (depth 0) is split first; deeper
        // ones are components of a split
        const int e = evolve_pair<MIXED>(a, b, H, g.depth, p, c, g.depth > 0);
        if (e) atomicOr(err, e);
        W.x[ia] = a.x; W.y[ia] = a.y; W.z[ia] = a.z; W.vx[ia] = a.vx; W.vy[ia] = a.vy; W.vz[ia] = a.vz;
        W.x[ib] = b.x; W.y[ib] = b.y; W.z[ib] = b.z; W.vx[ib] = b.vx; W.vy[ib] = b.vy; W.vz[ib] = b.vz;
        if (g.cluster != cl) {
            if (cl >= 0) pair_counters_flush(stats, fam, cl, tot);
            tot = PairCounters{0, 0, 0, 0, 0, 0, -1};
            cl = g.cluster;
        }
        tot.tau += c.tau;
        tot.kick += c.kick;
        tot.drift += c.drift;
        tot.comp += c.comp;
        tot.split += c.split;
        tot.kepler += c.kepler;
        tot.maxd = max(tot.maxd, c.maxd);
    }
    // the wavefront is whole again here
    int cmax = cl;
    for (int o = 32; o > 0; o >>= 1) cmax = max(cmax, __shfl_xor(cmax, o, 64));
    if (__all(cl < 0 || cl == cmax)) {
        if (cmax < 0) return;
        PairCounters w;
        w.tau = wave_sum_u64(tot.tau);
        w.kick = wave_sum_u64(tot.kick);
        w.drift = wave_sum_u64(tot.drift);
        w.comp = wave_sum_u64(tot.comp);
        w.split = wave_sum_u64(tot.split);
        w.kepler = wave_sum_u64(tot.kepler);
        int d = tot.maxd;
        for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o, 64));
        w.maxd = d;
        if ((threadIdx.x & 63) == 0) pair_counters_flush(stats, fam, cmax, w);
    } else if (cl >= 0) {
        pair_counters_flush(stats, fam, cl, tot);
    }
}

// ---------------------------------------------------------------------------
// On-chip recursion for one component per workgroup (3 <= n <= CAP).
//
// The state lives in LDS.  The recursion of Fig. 2 is walked level by level:
// level k holds the list L_k of sets to evolve with h_k = H / 2^k (level 0 is
// the item itself).  Splitting L_k reorders each set so that its components
// are contiguous, and records two bitmasks per level: component starts (cs)
// and membership of a non-trivial component (nt); the non-trivial components
// form L_{k+1}.  Sets of two particles are handed to one lane each and run
// to completion (evolve_pair).  Independent sets of one level are processed
// together, which is exact because they share no particles.
// ---------------------------------------------------------------------------
constexpr int MAXL = 64;
constexpr int SMALL_WAVE_CAP = 32;  // items of bins 0-1 (up to 32 particles) run one per wavefront

template <int CAP>
struct SmallLDS {
    double x[CAP], y[CAP], z[CAP], vx[CAP], vy[CAP], vz[CAP], m[CAP];
    int32_t orig[CAP];
    int32_t par[CAP];
    int32_t cnt[CAP];
    int16_t entry[CAP];
    int16_t segS[CAP];
    int16_t segE[CAP];
    int16_t aux[CAP];
    int16_t cid[CAP];
    uint32_t cs[MAXL][CAP / 32];
    uint32_t nt[MAXL][CAP / 32];
    uint32_t flag[CAP / 32];
    int16_t binlist[CAP / 2];
    uint8_t phase[MAXL];
    uint8_t hasnt[MAXL];
    int32_t wsum[4];
    unsigned long long ctr[8];
    int32_t nbin;
    int32_t hasmain;  // the level being visited holds a set of three or more
    int32_t item;
    int32_t err;
    int32_t maxd;
};

// MODE: 0 = FP64, partners in slot order; 1 = FP64, partners in ascending
// particle index (bit-identical to a sequential sweep); 2 = mixed precision.
template <int CAP, int MODE, int NT>
struct SmallKernel {
    static constexpr bool EXACT = (MODE == 1);
    static constexpr bool MIXED = (MODE == 2);
    static constexpr int E = (CAP + NT - 1) / NT;  // positions per thread
    static constexpr int W = (CAP + 31) / 32;      // mask words
    static_assert(NT == TPB || NT == WAVE, "a team is a workgroup or one wavefront");

    // thread index within the team, and the team's barrier
    static __device__ __forceinline__ int tid() { return (int)(threadIdx.x % NT); }
    static __device__ __forceinline__ void sync()
    {
        if (NT == TPB) {
            __syncthreads();
        } else {
            // one wavefront: order its LDS accesses around a wave-level barrier
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
    }

    // Mask word of level-k segment starts: L_k = non-trivial components of level k-1.
    static __device__ __forceinline__ uint32_t start_word(const SmallLDS<CAP> &L, int k, int wi, int n)
    {
        if (k == 0) return wi == 0 ? 1u : 0u;
        return L.cs[k - 1][wi] & L.nt[k - 1][wi];
    }

    static __device__ __forceinline__ uint32_t end_word(const SmallLDS<CAP> &L, int k, int wi, int n)
    {
        uint32_t w;
        if (k == 0) w = (wi == 0) ? 1u : 0u;
        else w = (L.cs[k - 1][wi] & L.nt[k - 1][wi]) | ~L.nt[k - 1][wi];
        // positions >= n end every segment
        const int lo = wi * 32;
        if (lo + 32 > n) {
            const int keep = n - lo;  // bits below keep are real positions
            const uint32_t beyond = keep <= 0 ? 0xFFFFFFFFu : (keep >= 32 ? 0u : (0xFFFFFFFFu << keep));
            w |= beyond;
        }
        return w;
    }

    // segS/segE for every position of L_k (-1 outside) and the list of
    // two-particle sets.
    static __device__ void enumerate(SmallLDS<CAP> &L, int k, int n, bool collect_bins)
    {
        if (tid() == 0) {
            L.nbin = 0;
            L.hasmain = 0;
        }
        sync();
        for (int p = tid(); p < n; p += NT) {
            const bool inL = (k == 0) || bit_of(L.nt[k - 1], p);
            if (!inL) {
                L.segS[p] = -1;
                continue;
            }
            // previous start
            int wi = p >> 5;
            uint32_t bits = start_word(L, k, wi, n) & (0xFFFFFFFFu >> (31 - (p & 31)));
            while (!bits && wi > 0) bits = start_word(L, k, --wi, n);
            const int s = bits ? wi * 32 + 31 - __clz(bits) : 0;
            // next end strictly after p (a segment start, a position outside L_k, or n)
            int e = n;
            wi = p >> 5;
            const int sh = (p & 31) + 1;
            bits = sh < 32 ? (end_word(L, k, wi, n) & (0xFFFFFFFFu << sh)) : 0u;
            for (;;) {
                if (bits) {
                    e = min(n, wi * 32 + __ffs(bits) - 1);
                    break;
                }
                if (++wi * 32 >= n) break;
                bits = end_word(L, k, wi, n);
            }
            L.segS[p] = (int16_t)s;
            L.segE[p] = (int16_t)e;
            if (p == s && e - s >= 3) L.hasmain = 1;
            if (collect_bins && p == s && e - s == 2) {
                const int i = atomicAdd(&L.nbin, 1);
                L.binlist[i] = (int16_t)s;
            }
        }
        sync();
    }

    static __device__ void count(SmallLDS<CAP> &L, int idx, unsigned long long v)
    {
        if (v) atomicAdd(&L.ctr[idx], v);
    }

    static __device__ void run_binaries(SmallLDS<CAP> &L, double h, int depth, const DevParams &p)
    {
        const int nb = L.nbin;
        PairCounters c{0, 0, 0, 0, 0, 0, -1};
        for (int i = tid(); i < nb; i += NT) {
            int ia = L.binlist[i], ib = ia + 1;
            if (L.orig[ib] < L.orig[ia]) {
                const int t = ia;
                ia = ib;
                ib = t;
            }
            Body a{L.x[ia], L.y[ia], L.z[ia], L.vx[ia], L.vy[ia], L.vz[ia], L.m[ia]};
            Body b{L.x[ib], L.y[ib], L.z[ib], L.vx[ib], L.vy[ib], L.vz[ib], L.m[ib]};
            // every two-particle set below an item's top level is a component
            const int e = evolve_pair<MIXED>(a, b, h, depth, p, c, true);
            if (e) atomicOr(&L.err, e);
            L.x[ia] = a.x; L.y[ia] = a.y; L.z[ia] = a.z; L.vx[ia] = a.vx; L.vy[ia] = a.vy; L.vz[ia] = a.vz;
            L.x[ib] = b.x; L.y[ib] = b.y; L.z[ib] = b.z; L.vx[ib] = b.vx; L.vy[ib] = b.vy; L.vz[ib] = b.vz;
        }
        count(L, ST_TAU, c.tau);
        count(L, ST_TAU_ALG, c.tau);
        count(L, ST_KICK, c.kick);
        count(L, ST_DRIFT, c.drift);
        count(L, ST_COMP, c.comp);
        count(L, ST_SPLIT, c.split);
        count(L, ST_KEPLER, c.kepler);
        if (c.maxd >= 0) atomicMax(&L.maxd, c.maxd);
        sync();
    }

    // Exclusive prefix sum of cnt[0..CAP) into par[].
    static __device__ void scan_cnt(SmallLDS<CAP> &L)
    {
        int v[E];
        int tot = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = tid() * E + e;
            v[e] = q < CAP ? L.cnt[q] : 0;
            tot += v[e];
        }
        int incl = tot;
        const int lane = tid() & 63, w = tid() >> 6;
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) L.wsum[w] = incl;
        sync();
        int before = incl - tot;
        for (int q = 0; q < w; ++q) before += L.wsum[q];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = tid() * E + e;
            if (q < CAP) L.par[q] = before;
            before += v[e];
        }
        sync();
    }

    static __device__ __forceinline__ bool is_main(const SmallLDS<CAP> &L, int p)
    {
        const int s = L.segS[p];
        return s >= 0 && (L.segE[p] - s) >= 3;
    }

    // HOLD split (Sec. 2.1, eqs. 11-12): the particles of a main set that
    // have an edge (the members of its non-trivial components) are fast and
    // form one set F, labelled by its first position.  par[] (free between
    // the union-find and the scan) holds each set's first fast position and
    // aux[] (free until the kick) the fast flags.
    static __device__ void hold_merge(SmallLDS<CAP> &L, int n)
    {
        for (int a = tid(); a < n; a += NT) {
            if (!is_main(L, a)) continue;
            L.aux[a] = L.cnt[L.cid[a]] >= 2 ? 1 : 0;
            if (a == L.segS[a]) L.par[a] = CAP;
        }
        sync();
        for (int a = tid(); a < n; a += NT)
            if (is_main(L, a) && L.aux[a]) atomicMin(&L.par[L.segS[a]], a);
        sync();
        for (int a = tid(); a < n; a += NT) {
            if (!is_main(L, a)) continue;
            if (L.aux[a]) L.cid[a] = (int16_t)L.par[L.segS[a]];
            L.cnt[a] = 0;
        }
        sync();
        for (int a = tid(); a < n; a += NT)
            if (is_main(L, a)) atomicAdd(&L.cnt[L.cid[a]], 1);
        sync();
    }

    // Split every main set of L_k at h (eq. 20) and reorder it by component.
    static __device__ void split(SmallLDS<CAP> &L, int k, int n, double h, const DevParams &p)
    {
        for (int w = tid(); w < W; w += NT) {
            L.flag[w] = 0;
            L.cs[k][w] = 0;
            L.nt[k][w] = 0;
        }
        for (int q = tid(); q < CAP; q += NT) L.cnt[q] = 0;
        sync();
        unsigned long long tau = 0;
        bool over = false;  // an LDS union-find budget ran out
        const ScreenParams sq = screen_params(p, h);
        const ccs::Screen64 s64 = ccs::screen64_params(p.eta, h);
        const ccs::Far64 f64 = ccs::far64_params(p.eta, h);
        // star test from each set's first position X
        for (int q = tid(); q < n; q += NT) {
            if (!is_main(L, q)) continue;
            L.par[q] = q;
            const int X = L.segS[q];
            if (q == X) continue;
            tau++;
            if (!edge_decide<MIXED>(L.x[X] - L.x[q], L.y[X] - L.y[q], L.z[X] - L.z[q], L.vx[X] - L.vx[q],
                                    L.vy[X] - L.vy[q], L.vz[X] - L.vz[q], L.m[X] + L.m[q], p, sq, s64, h))
                atomicOr(&L.flag[X >> 5], 1u << (X & 31));
        }
        sync();
        // all-pairs sweep of the sets that are not stars
        for (int a = tid(); a < n; a += NT) {
            if (!is_main(L, a)) continue;
            const int s = L.segS[a];
            if (!bit_of(L.flag, s)) continue;
            const int e = L.segE[a];
            const double xa = L.x[a], ya = L.y[a], za = L.z[a], vxa = L.vx[a], vya = L.vy[a], vza = L.vz[a],
                         ma = L.m[a];
            for (int b = a + 1; b < e; ++b) {
                const double dx = xa - L.x[b], dy = ya - L.y[b], dz = za - L.z[b];
                const double dvx = vxa - L.vx[b], dvy = vya - L.vy[b], dvz = vza - L.vz[b];
                const double mb = L.m[b];
                const double r2 = ((dx * dx + dy * dy) + dz * dz) + p.eps2;
                const double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
                if (ccs::far64(r2, v2, p.G * (ma + mb), f64)) continue;  // certainly no edge
                if (edge_decide<MIXED>(dx, dy, dz, dvx, dvy, dvz, ma + mb, p, sq, s64, h)) lunite(L.par, a, b, over);
            }
            tau += (unsigned long long)(e - a - 1);
        }
        count(L, ST_TAU, tau);
        sync();
        // labels and sizes
        for (int a = tid(); a < n; a += NT) {
            if (!is_main(L, a)) continue;
            const int s = L.segS[a];
            const int lab = bit_of(L.flag, s) ? lfind(L.par, a, over) : s;
            L.cid[a] = (int16_t)lab;
            atomicAdd(&L.cnt[lab], 1);
        }
        if (over) atomicOr(&L.err, EB_BUDGET);
        sync();
        if (p.hold) hold_merge(L, n);
        scan_cnt(L);
        // destination of every position: components in label order, members
        // in position order
        int dst[E], rk[E], sz[E];
        unsigned long long comps = 0, splits = 0, alg = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int a = tid() + e * NT;
            dst[e] = -1;
            if (a >= n || !is_main(L, a)) continue;
            const int s = L.segS[a];
            const int lab = L.cid[a];
            int r = 0;
            for (int q = lab; q < a; ++q) r += (L.cid[q] == lab);
            const int size = L.cnt[lab];
            dst[e] = s + (L.par[lab] - L.par[s]) + r;
            rk[e] = r;
            sz[e] = size;
            if (a == lab && size >= 2) comps++;
            if (a == s) {
                const unsigned long long m = (unsigned long long)(L.segE[a] - s);
                splits++;
                alg += (bit_of(L.flag, s) || p.hold) ? m * (m - 1) / 2 : m - 1;
            }
        }
        count(L, ST_COMP, comps);
        count(L, ST_SPLIT, splits);
        count(L, ST_TAU_ALG, alg);
        // move
        double rx[E], ry[E], rz[E], rvx[E], rvy[E], rvz[E], rm[E];
        int32_t ro[E];
        int16_t re[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int a = tid() + e * NT;
            if (dst[e] < 0) continue;
            rx[e] = L.x[a]; ry[e] = L.y[a]; rz[e] = L.z[a];
            rvx[e] = L.vx[a]; rvy[e] = L.vy[a]; rvz[e] = L.vz[a]; rm[e] = L.m[a];
            ro[e] = L.orig[a];
            re[e] = L.entry[a];
        }
        sync();
        bool any_nt = false;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int d = dst[e];
            if (d < 0) continue;
            L.x[d] = rx[e]; L.y[d] = ry[e]; L.z[d] = rz[e];
            L.vx[d] = rvx[e]; L.vy[d] = rvy[e]; L.vz[d] = rvz[e]; L.m[d] = rm[e];
            L.orig[d] = ro[e];
            L.entry[d] = re[e];
            if (rk[e] == 0) atomicOr(&L.cs[k][d >> 5], 1u << (d & 31));
            if (sz[e] >= 2) {
                atomicOr(&L.nt[k][d >> 5], 1u << (d & 31));
                any_nt = true;
            }
        }
        if (tid() == 0) L.hasnt[k] = 0;
        sync();
        if (any_nt) L.hasnt[k] = 1;
        sync();
    }

    // Drift R by h/2, kick every pair of a main set in different components by
    // h, drift R by h/2 (eq. 30).  Partners are summed in ascending original
    // index, the order of a sequential i<j sweep over the set.
    static __device__ void kick_drift(SoA /*unused*/, SmallLDS<CAP> &L, int k, int n, double h,
                                      const DevParams &p)
    {
        const double hh = 0.5 * h;
        unsigned long long drifts = 0, kicks = 0;
        bool ok = true;
        for (int a = tid(); a < n; a += NT) {
            if (!is_main(L, a)) continue;
            int wi = a >> 5;
            uint32_t bits = L.cs[k][wi] & (0xFFFFFFFFu >> (31 - (a & 31)));
            while (!bits && wi > 0) bits = L.cs[k][--wi];
            L.cid[a] = (int16_t)(bits ? wi * 32 + 31 - __clz(bits) : L.segS[a]);
            if (!bit_of(L.nt[k], a)) {
                L.x[a] += hh * L.vx[a];
                L.y[a] += hh * L.vy[a];
                L.z[a] += hh * L.vz[a];
                drifts++;
            }
        }
        sync();
        // Partner order: with EXACT, ascending original index (the order of a
        // sequential i<j sweep over the set); otherwise slot order.
        for (int a = tid(); a < n; a += NT) {
            if (!is_main(L, a)) continue;
            const int s = L.segS[a], e = L.segE[a];
            bool multi = false;
            for (int q = s + 1; q < e && !multi; ++q) multi = bit_of(L.cs[k], q);
            if (!multi) {
                L.aux[a] = -1;
                continue;
            }
            if (EXACT) {
                const int oa = L.orig[a];
                int r = 0;
                for (int q = s; q < e; ++q) r += (L.orig[q] < oa);
                L.aux[s + r] = (int16_t)a;
            } else {
                L.aux[a] = (int16_t)a;
            }
        }
        sync();
        for (int a = tid(); a < n; a += NT) {
            if (!is_main(L, a)) continue;
            const int s = L.segS[a], e = L.segE[a];
            if (L.aux[s] < 0) continue;  // a single component: nothing to kick
            const double xa = L.x[a], ya = L.y[a], za = L.z[a];
            const int ca = L.cid[a];
            const int oa = L.orig[a];
            double ax = 0.0, ay = 0.0, az = 0.0;
            if (MIXED) {
                Kahan3 kh{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                const float e2 = (float)p.eps2;
                for (int q = s; q < e; ++q) {
                    if (L.cid[q] == ca) continue;
                    ok &= accel_term32(xa, ya, za, L.x[q], L.y[q], L.z[q], (float)(p.G * L.m[q]), e2, kh);
                    kicks += (L.orig[q] > oa);
                }
                ax = (double)kh.sx - (double)kh.cx;
                ay = (double)kh.sy - (double)kh.cy;
                az = (double)kh.sz - (double)kh.cz;
            } else {
                for (int t = s; t < e; ++t) {
                    const int q = EXACT ? L.aux[t] : t;
                    if (L.cid[q] == ca) continue;
                    if (EXACT)
                        ok &= accel_term(xa, ya, za, L.x[q], L.y[q], L.z[q], L.m[q], p.eps2, p.G, ax, ay, az);
                    else
                        ok &= accel_term_rsq(xa, ya, za, L.x[q], L.y[q], L.z[q], p.G * L.m[q], p.eps2, ax, ay, az);
                    kicks += (L.orig[q] > oa);
                }
            }
            // velocities are not read by the kick, so each thread updates its own
            L.vx[a] += h * ax;
            L.vy[a] += h * ay;
            L.vz[a] += h * az;
        }
        if (!ok) atomicOr(&L.err, EB_NONFINITE);
        sync();
        for (int a = tid(); a < n; a += NT) {
            if (!is_main(L, a)) continue;
            if (!bit_of(L.nt[k], a)) {
                L.x[a] += hh * L.vx[a];
                L.y[a] += hh * L.vy[a];
                L.z[a] += hh * L.vz[a];
                drifts++;
            }
        }
        count(L, ST_DRIFT, drifts);
        count(L, ST_KICK, kicks);
        sync();
    }

    static __device__ void run_item(SoA Wg, SmallLDS<CAP> &L, const Seg g, double H, const DevParams &p,
                                    int32_t *err, uint64_t *stats, uint64_t *fam)
    {
        const int n = g.n;
        for (int a = tid(); a < n; a += NT) {
            const int u = g.start + a;
            L.x[a] = Wg.x[u]; L.y[a] = Wg.y[u]; L.z[a] = Wg.z[u];
            L.vx[a] = Wg.vx[u]; L.vy[a] = Wg.vy[u]; L.vz[a] = Wg.vz[u]; L.m[a] = Wg.m[u];
            L.orig[a] = Wg.orig[u];
            L.entry[a] = (int16_t)a;
        }
        if (tid() < 8) L.ctr[tid()] = 0;
        if (tid() == 0) {
            L.err = 0;
            L.maxd = -1;
            L.phase[0] = 0;
        }
        sync();
        int k = 0;
        double h = H;
        uint64_t visits = 0;
        for (;;) {
            if (++visits > ITEM_VISIT_BUDGET) {
                if (tid() == 0) L.err |= EB_BUDGET;
                sync();
                break;
            }
            int ph = L.phase[k];
            bool descend = false;
            bool fresh = false;
            if (ph == 0) {
                const int depth = g.depth + k;
                enumerate(L, k, n, true);
                // the level is an evolve_cc call of its own unless, with
                // CC_KEPLER, it holds only two-particle components (Kepler
                // solutions, no split)
                const bool splits_here = !p.kepler || L.hasmain;
                if (splits_here && (depth > p.max_depth || k >= MAXL - 1)) {
                    if (tid() == 0) L.err |= EB_DEPTH;
                    sync();
                    break;
                }
                if (splits_here && tid() == 0) atomicMax(&L.maxd, depth);
                run_binaries(L, h, depth, p);
                if (L.err) break;
                split(L, k, n, h, p);
                if (L.hasnt[k]) {
                    descend = true;
                    if (tid() == 0) L.phase[k] = 1;
                } else {
                    ph = 1;
                    fresh = true;
                }
            }
            if (!descend && ph == 1) {
                if (!fresh) enumerate(L, k, n, false);
                kick_drift(Wg, L, k, n, h, p);
                if (L.err) break;
                if (L.hasnt[k]) {
                    descend = true;
                    if (tid() == 0) L.phase[k] = 2;
                }
            }
            if (descend) {
                if (tid() == 0) L.phase[k + 1] = 0;
                sync();
                k++;
                h = 0.5 * h;
                continue;
            }
            // level k finished (both halves, or no components)
            sync();
            if (k == 0) break;
            k--;
            h = 2.0 * h;
        }
        sync();
        if (L.err) {
            if (tid() == 0) atomicOr(err, L.err);
        } else {
            for (int a = tid(); a < n; a += NT) {
                const int u = g.start + L.entry[a];
                Wg.x[u] = L.x[a]; Wg.y[u] = L.y[a]; Wg.z[u] = L.z[a];
                Wg.vx[u] = L.vx[a]; Wg.vy[u] = L.vy[a]; Wg.vz[u] = L.vz[a];
            }
        }
        if (tid() < ST_N && tid() != ST_MAXD) stat_add(stats, g.cluster, tid(), L.ctr[tid()]);
        if (tid() == 0) {
            fam_add(fam, 0, L.ctr[ST_TAU]);
            fam_add(fam, 1, L.ctr[ST_KICK]);
        }
        if (tid() == 0 && L.maxd >= 0) stat_max(stats, g.cluster, L.maxd);
        sync();
    }
};

struct SmallItems {
    const Seg *bin[4];
    const int32_t *count;  // counts of bins 0..3 at count[0..3]; count[-1] = two-particle components
    int32_t cap;           // capacity of each bin list
    int32_t cap_pairs;     // capacity of the two-particle list
};

// A team of NT threads (the workgroup, or one wavefront with its own LDS
// region) takes items of bins [blo, bhi] from a queue, largest sizes first.
template <int CAP, int MODE, int NT>
__device__ void run_team(SoA W, SmallLDS<CAP> &L, const SmallItems &items, int blo, int bhi, int32_t *qhead,
                         double H, const DevParams &p, int32_t *err, uint64_t *stats, uint64_t *fam)
{
    using K = SmallKernel<CAP, MODE, NT>;
    const int tid = K::tid();
    int c[4] = {0, 0, 0, 0};
    for (int b = blo; b <= bhi; ++b) c[b] = min(items.count[b], items.cap);
    const int total = c[0] + c[1] + c[2] + c[3];
    for (;;) {
        if (tid == 0) L.item = atomicAdd(qhead, 1);
        K::sync();
        int it = L.item;
        K::sync();
        if (it >= total) break;
        int b = bhi;
        while (it >= c[b]) {
            it -= c[b];
            b--;
        }
        const Seg g = items.bin[b][it];
        if (g.n == 1) {
            // a lone particle: split gives R = {it}; drift h/2 twice
            if (tid == 0) {
                const int u = g.start;
                const double hh = 0.5 * H;
                for (int r = 0; r < 2; ++r) {
                    W.x[u] += hh * W.vx[u];
                    W.y[u] += hh * W.vy[u];
                    W.z[u] += hh * W.vz[u];
                }
                stat_add(stats, g.cluster, ST_DRIFT, 2);
                stat_add(stats, g.cluster, ST_SPLIT, 1);
                stat_max(stats, g.cluster, g.depth);
            }
            continue;
        }
        K::run_item(W, L, g, H, p, err, stats, fam);
    }
}

// The components of one level that are evolved on chip, in one launch: the
// first nbp blocks take the two-particle components one per thread, the next
// nbb blocks the components of bins 2-3 one per workgroup, the rest the
// components of bins 0-1 one per wavefront.  q[0], q[1] are the heads of the
// workgroup and wavefront queues, q[2] counts finished blocks; all three are
// 0 before a launch and the last block to finish resets them.
template <int CAP, int MODE>
__global__ __launch_bounds__(TPB) void k_items(SoA W, const Seg *__restrict__ pairs, SmallItems items, int nbp,
                                                int nbb, int32_t *q, double H, DevParams p, int32_t *err,
                                                uint64_t *stats, uint64_t *fam)
{
    constexpr bool MIXED = (MODE == 2);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int bid = blockIdx.x;
    if (bid < nbp) {
        const int n = min(items.count[-1], items.cap_pairs);
        run_pairs<MIXED>(W, pairs, n, bid * TPB + threadIdx.x, nbp * TPB, H, p, err, stats, fam);
    } else if (bid < nbp + nbb) {
        SmallLDS<CAP> &L = *reinterpret_cast<SmallLDS<CAP> *>(smem_raw);
        run_team<CAP, MODE, TPB>(W, L, items, 2, 3, &q[0], H, p, err, stats, fam);
    } else {
        SmallLDS<SMALL_WAVE_CAP> &L = reinterpret_cast<SmallLDS<SMALL_WAVE_CAP> *>(smem_raw)[threadIdx.x / WAVE];
        run_team<SMALL_WAVE_CAP, MODE, WAVE>(W, L, items, 0, 1, &q[1], H, p, err, stats, fam);
    }
    // Each team took its final, out-of-range ticket before its block counts out.
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&q[2], 1) == (int)gridDim.x - 1) {
            atomicExch(&q[0], 0);
            atomicExch(&q[1], 0);
            atomicExch(&q[2], 0);
        }
    }
}

// ---------------------------------------------------------------------------
// Diagnostics: per-block Neumaier partials, combined in a fixed order.
// ---------------------------------------------------------------------------
struct NS {
    double s, c;
};

__device__ __forceinline__ void ns_add(NS &a, double v)
{
    const double t = a.s + v;
    if (fabs(a.s) >= fabs(v)) a.c += (a.s - t) + v;
    else a.c += (v - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void ns_merge(NS &a, const NS &b)
{
    ns_add(a, b.s);
    ns_add(a, b.c);
}

constexpr int NDIAG = 12;

__global__ __launch_bounds__(TPB) void k_diag(SoA S, int n, double eps2, double G, double *__restrict__ part)
{
    __shared__ double jx[TPB], jy[TPB], jz[TPB], jm[TPB];
    __shared__ NS red[TPB];
    const int i0 = blockIdx.x * TPB + threadIdx.x;
    const bool valid = i0 < n;
    const int i = valid ? i0 : 0;
    NS acc[NDIAG];
    for (int q = 0; q < NDIAG; ++q) acc[q] = NS{0.0, 0.0};
    const double xi = S.x[i], yi = S.y[i], zi = S.z[i], mi = S.m[i];
    if (valid) {
        const double vx = S.vx[i], vy = S.vy[i], vz = S.vz[i];
        const double v2 = (vx * vx + vy * vy) + vz * vz;
        ns_add(acc[0], 0.5 * mi * v2);
        ns_add(acc[2], mi * vx); ns_add(acc[3], mi * vy); ns_add(acc[4], mi * vz);
        ns_add(acc[5], mi * (yi * vz - zi * vy));
        ns_add(acc[6], mi * (zi * vx - xi * vz));
        ns_add(acc[7], mi * (xi * vy - yi * vx));
        ns_add(acc[8], mi * xi); ns_add(acc[9], mi * yi); ns_add(acc[10], mi * zi);
        ns_add(acc[11], mi);
    }
    const int jstart = blockIdx.x * TPB;  // pairs j > i only
    for (int jb = jstart; jb < n; jb += TPB) {
        const int jn = min(TPB, n - jb);
        __syncthreads();
        if (threadIdx.x < jn) {
            jx[threadIdx.x] = S.x[jb + threadIdx.x];
            jy[threadIdx.x] = S.y[jb + threadIdx.x];
            jz[threadIdx.x] = S.z[jb + threadIdx.x];
            jm[threadIdx.x] = S.m[jb + threadIdx.x];
        }
        __syncthreads();
        if (valid) {
            for (int jj = 0; jj < jn; ++jj) {
                if (jb + jj <= i) continue;
                const double dx = jx[jj] - xi, dy = jy[jj] - yi, dz = jz[jj] - zi;
                const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
                ns_add(acc[1], -G * mi * jm[jj] / sqrt(r2));
            }
        }
    }
    // block reduction in fixed (tree) order, one quantity at a time
    for (int q = 0; q < NDIAG; ++q) {
        __syncthreads();
        red[threadIdx.x] = acc[q];
        __syncthreads();
        for (int st = TPB / 2; st > 0; st >>= 1) {
            if (threadIdx.x < st) ns_merge(red[threadIdx.x], red[threadIdx.x + st]);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[(size_t)blockIdx.x * NDIAG * 2 + 2 * q] = red[0].s;
            part[(size_t)blockIdx.x * NDIAG * 2 + 2 * q + 1] = red[0].c;
        }
    }
}

__global__ void k_diag_final(const double *__restrict__ part, int nblk, double *__restrict__ out)
{
    const int q = threadIdx.x;
    if (q >= NDIAG) return;
    NS a{0.0, 0.0};
    for (int b = 0; b < nblk; ++b) {
        ns_add(a, part[(size_t)b * NDIAG * 2 + 2 * q]);
        ns_add(a, part[(size_t)b * NDIAG * 2 + 2 * q + 1]);
    }
    out[q] = a.s + a.c;
}

// ---------------------------------------------------------------------------
// Host-side launchers (declared in cc_launch.h)
// ---------------------------------------------------------------------------
static inline int nblocks(int64_t n, int cap = 65535 * 16)
{
    int64_t b = (n + TPB - 1) / TPB;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t launch_validate(const double *x, const double *y, const double *z, const double *vx, const double *vy,
                           const double *vz, const double *m, int64_t n, int32_t *err, hipStream_t st)
{
    hipLaunchKernelGGL(k_validate, dim3(nblocks(n, 4096)), dim3(TPB), 0, st, x, y, z, vx, vy, vz, m, n, err);
    return hipGetLastError();
}

hipError_t launch_pair_tau(SoA S, const int32_t *pi, const int32_t *pj, int64_t npairs, double *out, DevParams p,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_pair_tau, dim3(nblocks(npairs, 8192)), dim3(TPB), 0, st, S, pi, pj, npairs, out, p);
    return hipGetLastError();
}

hipError_t launch_drift_mask(SoA S, int64_t n, const uint8_t *mask, double h, hipStream_t st)
{
    hipLaunchKernelGGL(k_drift_mask, dim3(nblocks(n, 4096)), dim3(TPB), 0, st, S, n, mask, h);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t *a, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_iota, dim3(nblocks(n, 4096)), dim3(TPB), 0, st, a, n);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *a, int64_t n, int32_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(n, 4096)), dim3(TPB), 0, st, a, n, v);
    return hipGetLastError();
}

hipError_t launch_uf_init(int32_t *parent, int32_t *cnt, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_uf_init, dim3(nblocks(n, 4096)), dim3(TPB), 0, st, parent, cnt, n);
    return hipGetLastError();
}

hipError_t launch_star(SoA S, const GridLevelArgs &a, int32_t *notstar, DevParams p, double h, bool mixed,
                       uint64_t *stats, uint64_t *fam, hipStream_t st)
{
    if (mixed)
        hipLaunchKernelGGL(k_star<true>, dim3(a.nchunks), dim3(TPB), 0, st, S, a.seg, a.chunk_off, a.nseg, notstar,
                           a.epoch, p, h, stats, fam);
    else
        hipLaunchKernelGGL(k_star<false>, dim3(a.nchunks), dim3(TPB), 0, st, S, a.seg, a.chunk_off, a.nseg, notstar,
                           a.epoch, p, h, stats, fam);
    return hipGetLastError();
}

hipError_t launch_sweep(SoA S, const GridLevelArgs &a, int32_t *notstar, int32_t *parent, DevParams p, double h,
                        bool mixed, int split_tiles, bool star_pass, int32_t *err, hipStream_t st)
{
    if (a.ntiles == 0) return hipSuccess;
    const int js = a.ntiles <= split_tiles ? 4 : 1;
    const int tpb = (TPB / ST) / js;  // tiles per block
    const int nb = (a.ntiles + tpb - 1) / tpb;
#define CC_SWEEP(M, J)                                                                                          \
    hipLaunchKernelGGL((k_sweep<M, J>), dim3(nb), dim3(TPB), 0, st, S, a.seg, a.tile_off, a.nseg, notstar, a.epoch, \
                       star_pass ? 1 : 0, parent, p, h, err)
    if (mixed) {
        if (js == 4) CC_SWEEP(true, 4);
        else if (js == 2) CC_SWEEP(true, 2);
        else CC_SWEEP(true, 1);
    } else {
        if (js == 4) CC_SWEEP(false, 4);
        else if (js == 2) CC_SWEEP(false, 2);
        else CC_SWEEP(false, 1);
    }
#undef CC_SWEEP
    return hipGetLastError();
}

hipError_t launch_label(const GridLevelArgs &a, const int32_t *notstar, int32_t *parent, int32_t *label, int32_t *cnt,
                        uint32_t *keys, uint32_t *vals, int32_t *count, int32_t *hold, bool star_pass,
                        uint64_t *stats, uint64_t *sweep_fam, int32_t *err, hipStream_t st)
{
    hipLaunchKernelGGL(k_label, dim3(a.nchunks), dim3(TPB), 0, st, a.seg, a.chunk_off, a.act_off, a.nseg, notstar,
                       a.epoch, parent, label, cnt, keys, vals, count, hold, star_pass ? 1 : 0, stats, sweep_fam,
                       err);
    return hipGetLastError();
}

hipError_t launch_hold(const GridLevelArgs &a, int32_t *label, int32_t *cnt, uint32_t *keys, int32_t *hold,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_hold_fast, dim3(a.nchunks), dim3(TPB), 0, st, a.seg, a.chunk_off, a.nseg, label, cnt, hold);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hold_relabel, dim3(a.nchunks), dim3(TPB), 0, st, a.seg, a.chunk_off, a.act_off, a.nseg,
                       label, cnt, keys, hold);
    return hipGetLastError();
}

size_t sort_temp_bytes(int n)
{
    size_t bytes = 0;
    (void)rocprim::radix_sort_pairs(nullptr, bytes, (uint32_t *)nullptr, (uint32_t *)nullptr, (uint32_t *)nullptr,
                              (uint32_t *)nullptr, (size_t)n, 0, 32, 0, false);
    return bytes;
}

hipError_t launch_sort(void *temp, size_t temp_bytes, const uint32_t *keys_in, uint32_t *keys_out,
                       const uint32_t *vals_in, uint32_t *vals_out, int n, int end_bit, hipStream_t st)
{
    size_t need = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, need, keys_in, keys_out, vals_in, vals_out, (size_t)n, 0,
                                             end_bit, st, false);
    if (e != hipSuccess) return e;
    if (need > temp_bytes) return hipErrorInvalidValue;
    size_t bytes = temp_bytes;
    return rocprim::radix_sort_pairs(temp, bytes, keys_in, keys_out, vals_in, vals_out, (size_t)n, 0, end_bit, st,
                                     false);
}

hipError_t launch_permute(SoA from, SoA to, const GridLevelArgs &a, const uint32_t *src, const uint32_t *lab,
                          const int32_t *cnt, uint8_t *sing, const ListArgs *lists, double drift_hh,
                          int32_t *parent, int32_t *cnt_next, uint64_t *kick_fam, bool count_kick, uint64_t *stats,
                          bool inverse, hipStream_t st)
{
    const int nb = nblocks(a.nact, 1 << 30);
    if (inverse) {
        hipLaunchKernelGGL(k_unpermute, dim3(nb), dim3(TPB), 0, st, from, to, a.seg, a.act_off, a.nseg, a.nact, src);
        return hipGetLastError();
    }
    Lists L{};
    int with = 0;
    if (lists) {
        with = 1;
        L.pairs = lists->pairs;
        for (int b = 0; b < 4; ++b) L.small[b] = lists->small[b];
        L.big = lists->big;
        L.count = lists->count;
        L.cap_pairs = lists->cap_pairs;
        L.cap_small = lists->cap_small;
        L.cap_big = lists->cap_big;
        L.small_max = lists->small_max;
        for (int b = 0; b < 3; ++b) L.bin_lim[b] = lists->bin_lim[b];
        L.labp = lists->labp;
        L.singp = lists->singp;
        L.errf = lists->errf;
        L.notstar = lists->notstar;
    }
    hipLaunchKernelGGL(k_permute, dim3(a.nchunks), dim3(TPB), 0, st, from, to, a.seg, a.chunk_off, a.act_off, a.nseg,
                       src, lab, cnt, sing, L, with, drift_hh, parent, cnt_next, kick_fam, count_kick ? 1 : 0,
                       a.epoch, stats);
    return hipGetLastError();
}

hipError_t launch_drift_seg(SoA W, const GridLevelArgs &a, const uint8_t *sing, double hh, uint64_t *stats,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_drift_seg, dim3(a.nchunks), dim3(TPB), 0, st, W, a.seg, a.chunk_off, a.nseg, sing, hh,
                       stats);
    return hipGetLastError();
}

hipError_t launch_kick_seg(SoA W, const GridLevelArgs &a, const int32_t *label, double h, double eps2, double G,
                           int32_t *err, uint64_t *stats, uint64_t *fam, hipStream_t st)
{
    hipLaunchKernelGGL(k_kick_seg, dim3(a.nchunks), dim3(TPB), 0, st, W, a.seg, a.chunk_off, a.nseg, label, h, eps2,
                       G, err, stats, fam);
    return hipGetLastError();
}

hipError_t launch_kick_tiles(SoA W, const GridLevelArgs &a, const KickBlock *blk, int nblk, const KickJob *jobs,
                             int njobs, const KickTile *ktile, const int32_t *labp, const uint8_t *singp, double h,
                             double eps2, double G, bool mixed, double *part, int32_t *parent, int32_t *cnt_next,
                             int32_t *err, uint64_t *stats, hipStream_t st)
{
    if (nblk > 0) {
        if (mixed)
            hipLaunchKernelGGL(k_kick_tiles<true>, dim3(nblk), dim3(TPB), 0, st, W, a.seg, blk, labp, eps2, G, part,
                               err);
        else
            hipLaunchKernelGGL(k_kick_tiles<false>, dim3(nblk), dim3(TPB), 0, st, W, a.seg, blk, labp, eps2, G, part,
                               err);
    }
    if (njobs > 0) hipLaunchKernelGGL(k_kick_reduce, dim3(njobs), dim3(TPB), 0, st, jobs, part);
    hipLaunchKernelGGL(k_kick_combine, dim3(a.nchunks), dim3(TPB), 0, st, W, a.seg, a.chunk_off, ktile, a.nseg,
                       (const double *)part, h, singp, 0.5 * h, parent, cnt_next, stats);
    return hipGetLastError();
}

hipError_t launch_kick_all(SoA W, int n, const int32_t *label, double eps2, double G, bool mixed, double *ax,
                           double *ay, double *az, int32_t *err, hipStream_t st)
{
    if (mixed)
        hipLaunchKernelGGL(k_kick_all<true>, dim3(nblocks(n, 1 << 30)), dim3(TPB), 0, st, W, n, label, eps2, G, ax, ay,
                           az, err);
    else
        hipLaunchKernelGGL(k_kick_all<false>, dim3(nblocks(n, 1 << 30)), dim3(TPB), 0, st, W, n, label, eps2, G, ax,
                           ay, az, err);
    return hipGetLastError();
}

hipError_t launch_apply_kick(SoA W, int n, const double *ax, const double *ay, const double *az, double h,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_apply_kick, dim3(nblocks(n, 1 << 30)), dim3(TPB), 0, st, W, n, ax, ay, az, h);
    return hipGetLastError();
}

// LDS limit of k_items<CAP, MODE>, set once per process (before any capture)
template <int CAP, int MODE>
static hipError_t configure_items_cap(size_t lds)
{
    static bool configured = false;
    if (!configured) {
        hipError_t e = hipFuncSetAttribute((const void *)k_items<CAP, MODE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        configured = true;
    }
    return hipSuccess;
}

template <int CAP, int MODE>
static hipError_t launch_items_cap(SoA W, const SmallArgs &s, int nbp, int nbb, int nbw, double H, DevParams p,
                                   int32_t *err, uint64_t *stats, uint64_t *fam, hipStream_t st)
{
    const size_t lds = std::max(sizeof(SmallLDS<CAP>), sizeof(SmallLDS<SMALL_WAVE_CAP>) * (TPB / WAVE));
    {
        hipError_t e = configure_items_cap<CAP, MODE>(lds);
        if (e != hipSuccess) return e;
    }
    SmallItems it{};
    for (int b = 0; b < 4; ++b) it.bin[b] = s.bin[b];
    it.count = s.count + 1;
    it.cap = s.cap;
    it.cap_pairs = s.cap_pairs;
    hipLaunchKernelGGL((k_items<CAP, MODE>), dim3(nbp + nbb + nbw), dim3(TPB), lds, st, W, s.pairs, it, nbp, nbb,
                       s.queue, H, p, err, stats, fam);
    return hipGetLastError();
}

size_t items_lds_bytes(int cap)
{
    const size_t w = sizeof(SmallLDS<SMALL_WAVE_CAP>) * (TPB / WAVE);
    if (cap <= 256) return std::max(sizeof(SmallLDS<256>), w);
    if (cap <= 512) return std::max(sizeof(SmallLDS<512>), w);
    return std::max(sizeof(SmallLDS<1024>), w);
}

hipError_t configure_items(int cap, int mode)
{
#define CC_CONF(C, M) configure_items_cap<C, M>(std::max(sizeof(SmallLDS<C>), sizeof(SmallLDS<SMALL_WAVE_CAP>) * (TPB / WAVE)))
    const int c = cap <= 256 ? 256 : cap <= 512 ? 512 : 1024;
    if (c == 256) return mode == 1 ? CC_CONF(256, 1) : mode == 2 ? CC_CONF(256, 2) : CC_CONF(256, 0);
    if (c == 512) return mode == 1 ? CC_CONF(512, 1) : mode == 2 ? CC_CONF(512, 2) : CC_CONF(512, 0);
    return mode == 1 ? CC_CONF(1024, 1) : mode == 2 ? CC_CONF(1024, 2) : CC_CONF(1024, 0);
#undef CC_CONF
}

hipError_t launch_items(SoA W, const SmallArgs &s, int cap, int mode, int nbp, int nbb, int nbw, double H,
                        DevParams p, int32_t *err, uint64_t *stats, uint64_t *fam, hipStream_t st)
{
    if (nbp + nbb + nbw <= 0) return hipSuccess;
#define CC_ITEMS_CAPS(M)                                                                               \
    if (cap <= 256) return launch_items_cap<256, M>(W, s, nbp, nbb, nbw, H, p, err, stats, fam, st); \
    if (cap <= 512) return launch_items_cap<512, M>(W, s, nbp, nbb, nbw, H, p, err, stats, fam, st); \
    return launch_items_cap<1024, M>(W, s, nbp, nbb, nbw, H, p, err, stats, fam, st);
    if (mode == 1) {
        CC_ITEMS_CAPS(1)
    }
    if (mode == 2) {
        CC_ITEMS_CAPS(2)
    }
    CC_ITEMS_CAPS(0)
#undef CC_ITEMS_CAPS
}

int diag_blocks(int n) { return nblocks(n, 1 << 30); }

hipError_t launch_diag(SoA S, int n, double eps2, double G, double *part, double *out, hipStream_t st)
{
    const int nb = diag_blocks(n);
    hipLaunchKernelGGL(k_diag, dim3(nb), dim3(TPB), 0, st, S, n, eps2, G, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, part, nb, out);
    return hipGetLastError();
}

}  // namespace ccg
