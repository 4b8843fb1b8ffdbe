// Neighbour-search structure: bounding box, Morton keys, LSD radix sort,
// gathers into sorted order, leaf boxes and the 8-ary box tree above them.
//
// The paper builds a balanced KD-tree by median splits with N_LEAF particles
// per leaf and propagates each cell's smoothing-sphere extent box upwards
// (section 4.2).  On the GPU the same role is played by a Morton-order sort
// (one radix sort instead of a recursive median selection, which the paper
// names as its tree-build scaling bottleneck, section 5.2.1) followed by
// leaves of leaf_size consecutive sorted particles; every leaf and node keeps
// the bounding box of its particles and their largest h.
#include "sph_internal.hpp"

#include <algorithm>

namespace sph {

namespace {

constexpr int kBoxThreads = 256;
constexpr int kRsThreads = 256;
// Bits per axis of the Morton key, by set size: at least 64 cells per mean
// particle spacing along an axis (particles sharing a cell keep their input
// order: the sort is stable), rounded up to what a number of 8-bit passes
// holds: 10 bits (4 passes) up to 2^12 particles, 13 (5 passes) up to 2^21,
// else 16 (6 passes).  The sort and the segment rule use the same count.
constexpr int key_bits(int64_t n)
{
    return n <= (int64_t(1) << 12) ? 10 : (n <= (int64_t(1) << 21) ? 13 : 16);
}
static_assert(kRsTile == kRsThreads * kRsItems && kRsTileSmall == kRsThreads * kRsItemsSmall,
              "radix tiles are 256 threads wide");

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kBoxThreads) void k_box_partial(int64_t n, const double *__restrict__ x,
                                                             const double *__restrict__ y,
                                                             const double *__restrict__ z,
                                                             double *__restrict__ part)
{
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        double v[3] = {x[k], y[k], z[k]};
        for (int a = 0; a < 3; a++) { mn[a] = fmin(mn[a], v[a]); mx[a] = fmax(mx[a], v[a]); }
    }
    __shared__ double sh[6][kBoxThreads];
    for (int a = 0; a < 3; a++) { sh[a][threadIdx.x] = mn[a]; sh[3 + a][threadIdx.x] = mx[a]; }
    __syncthreads();
    for (int s = kBoxThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int a = 0; a < 3; a++) {
                sh[a][threadIdx.x] = fmin(sh[a][threadIdx.x], sh[a][threadIdx.x + s]);
                sh[3 + a][threadIdx.x] = fmax(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void k_box_final(int nb, const double *__restrict__ part,
                                                  double *__restrict__ box)
{
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += 64)
        for (int a = 0; a < 3; a++) {
            mn[a] = fmin(mn[a], part[b * 6 + a]);
            mx[a] = fmax(mx[a], part[b * 6 + 3 + a]);
        }
    for (int o = 32; o > 0; o >>= 1)
        for (int a = 0; a < 3; a++) {
            mn[a] = fmin(mn[a], __shfl_xor(mn[a], o));
            mx[a] = fmax(mx[a], __shfl_xor(mx[a], o));
        }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; a++) { box[a] = mn[a]; box[3 + a] = mx[a]; }
}

__device__ inline uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

// Keys in the box stored at `box` (the bounding box a reduction wrote there),
// or, with fb.fixed (periodic sets), in the given box, which the first thread
// also stores at `box` for the kernels after this one (one launch fewer).
struct FixedBox {
    int fixed;
    double lo[3], hi[3];
};

__global__ __launch_bounds__(256) void k_keys(int64_t n, const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z, double *box,
                                              FixedBox fb, int bits,
                                              uint64_t *__restrict__ keys,
                                              uint32_t *__restrict__ vals)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    double b[6];
    for (int a = 0; a < 3; a++) {
        b[a] = fb.fixed ? fb.lo[a] : box[a];
        b[3 + a] = fb.fixed ? fb.hi[a] : box[3 + a];
    }
    if (fb.fixed && k == 0)
        for (int a = 0; a < 6; a++) box[a] = b[a];
    double ext = fmax(fmax(b[3] - b[0], b[4] - b[1]), b[5] - b[2]);
    double cells = (double)(1u << bits);
    double scale = ext > 0.0 ? cells / ext : 0.0;
    double top = cells - 1.0;
    double q[3] = {(x[k] - b[0]) * scale, (y[k] - b[1]) * scale, (z[k] - b[2]) * scale};
    uint64_t key = 0;
    for (int a = 0; a < 3; a++) {
        double c = floor(q[a]);
        c = c < 0.0 ? 0.0 : (c > top ? top : c);
        if (c != c) c = 0.0;   // NaN position: any key; flagged by the density loop
        key |= spread3((uint64_t)c) << a;
    }
    keys[k] = key;
    vals[k] = (uint32_t)k;
}

// ---- LSD radix sort, 8-bit digits ------------------------------------------

// inclusive block-wide sum scan, 256 threads, one value each; sh[255] holds
// the total on return
__device__ inline uint32_t block_scan_256(uint32_t v, uint32_t *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const uint32_t o = t >= d ? sh[t - d] : 0u;
        __syncthreads();
        sh[t] += o;
        __syncthreads();
    }
    return sh[t];
}

template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(int64_t n, const uint64_t *__restrict__ keys,
                                                        int shift, uint32_t *__restrict__ hist,
                                                        int64_t ntiles)
{
    constexpr int64_t TILE = (int64_t)kRsThreads * ITEMS;
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = blockIdx.x * TILE;
    for (int it = 0; it < ITEMS; it++) {
        int64_t k = base + it * kRsThreads + threadIdx.x;
        if (k < n) atomicAdd(&cnt[(keys[k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Per digit (one block each): exclusive scan over the tiles of that digit's
// counts, in place, 256 tiles at a time; the digit's total goes to totals[d].
// The digits' own offsets (a scan of the 256 totals) are formed by every
// scatter block.
__global__ __launch_bounds__(256) void k_rs_digit_scan(uint32_t *__restrict__ hist, int64_t ntiles,
                                                       uint32_t *__restrict__ totals)
{
    __shared__ uint32_t sh[256];
    uint32_t *a = hist + (int64_t)blockIdx.x * ntiles;
    uint32_t run = 0;
    for (int64_t b0 = 0; b0 < ntiles; b0 += 256) {
        const int64_t k = b0 + threadIdx.x;
        const uint32_t v = k < ntiles ? a[k] : 0u;
        const uint32_t incl = block_scan_256(v, sh);
        if (k < ntiles) a[k] = run + incl - v;
        run += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = run;
}

// Stable scatter.  Wave w of the block owns keys [tile + w*64*ITEMS, +64*ITEMS)
// and walks them in ITEMS rounds of 64 in index order; equal digits within a round
// are ranked with 8 ballots, across rounds with per-wave LDS counters, and
// across waves by an exclusive prefix of those counters.  raw = 0: offs holds
// k_rs_digit_scan's per-digit scans over the tiles and totals the digit
// totals; raw = 1 (few tiles): offs holds k_rs_hist's counts as they are and
// each block forms both itself (one thread per digit summing that digit's
// counts over the tiles), which saves the scan's launch.
template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(int64_t n, const uint64_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin,
                                                           uint64_t *__restrict__ kout,
                                                           uint32_t *__restrict__ vout, int shift,
                                                           const uint32_t *__restrict__ offs,
                                                           int64_t ntiles,
                                                           const uint32_t *__restrict__ totals,
                                                           int raw)
{
    __shared__ uint32_t wcnt[kRsThreads / kWave][256];
    __shared__ uint32_t dbase[256];
    __shared__ uint32_t tbase[256];            // first slot of each digit in the tile
    constexpr int TILE = kRsThreads * ITEMS;
    __shared__ uint64_t skey[TILE];            // the tile in digit order
    __shared__ uint32_t sval[TILE];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    for (int k = threadIdx.x; k < (kRsThreads / kWave) * 256; k += kRsThreads)
        (&wcnt[0][0])[k] = 0;
    // this digit's keys in the tiles before this one, and in all tiles
    static_assert(kRsThreads == 256, "one thread per digit");
    uint32_t before_tile, digit_total;
    if (raw) {
        const uint32_t *h = offs + (int64_t)threadIdx.x * ntiles;
        before_tile = 0u;
        digit_total = 0u;
        for (int64_t t = 0; t < ntiles; t++) {
            const uint32_t v = h[t];
            before_tile += t < (int64_t)blockIdx.x ? v : 0u;
            digit_total += v;
        }
    } else {
        before_tile = offs[threadIdx.x * ntiles + blockIdx.x];
        digit_total = totals[threadIdx.x];
    }
    // first position of each digit: exclusive scan of the digit totals
    {
        const uint32_t v = digit_total;
        const uint32_t incl = block_scan_256(v, dbase);
        __syncthreads();
        dbase[threadIdx.x] = incl - v;
    }
    __syncthreads();
    const uint64_t lt = __lanemask_lt();
    const int64_t base = blockIdx.x * (int64_t)TILE + w * (ITEMS * kWave);
    uint64_t key[ITEMS];
    uint32_t val[ITEMS];
    uint32_t rank[ITEMS];
    for (int r = 0; r < ITEMS; r++) {
        int64_t k = base + r * kWave + lane;
        bool valid = k < n;
        key[r] = valid ? kin[k] : 0ull;
        val[r] = valid ? vin[k] : 0u;
        uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        uint64_t mask = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            uint64_t bb = __ballot((d >> b) & 1u);
            mask &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t before = valid ? wcnt[w][d] : 0u;
        uint32_t prior = (uint32_t)__popcll(mask & lt);
        rank[r] = before + prior;
        wave_lds_sync();
        bool leader = valid && prior == 0;
        if (leader) wcnt[w][d] = before + (uint32_t)__popcll(mask);
        wave_lds_sync();
    }
    __syncthreads();
    // per digit (one thread each): the waves' offsets inside the tile's run
    // of that digit, then the run's first slot in the tile
    uint32_t run = 0;
    for (int ww = 0; ww < kRsThreads / kWave; ww++) {
        uint32_t v = wcnt[ww][threadIdx.x];
        wcnt[ww][threadIdx.x] = run;
        run += v;
    }
    {
        const uint32_t incl = block_scan_256(run, tbase);
        __syncthreads();
        tbase[threadIdx.x] = incl - run;
    }
    __syncthreads();
    // stage the tile in digit order (stable: wave, then item, then lane)
    for (int r = 0; r < ITEMS; r++) {
        int64_t k = base + r * kWave + lane;
        if (k < n) {
            uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
            uint32_t lp = tbase[d] + wcnt[w][d] + rank[r];
            skey[lp] = key[r];
            sval[lp] = val[r];
        }
    }
    __syncthreads();
    // slot i of the tile goes to (global start of its digit's run in this tile)
    // + (i - tile start of that run); dbase + offs >= tbase, so no wrap
    dbase[threadIdx.x] += before_tile - tbase[threadIdx.x];
    __syncthreads();
    const int64_t left = n - blockIdx.x * (int64_t)TILE;   // >= 1
    const int tile_n = left < TILE ? (int)left : TILE;
    for (int i = threadIdx.x; i < tile_n; i += kRsThreads) {
        const uint64_t kk = skey[i];
        const uint32_t d = (uint32_t)(kk >> shift) & 255u;
        const uint32_t pos = dbase[d] + (uint32_t)i;
        kout[pos] = kk;
        vout[pos] = sval[i];
    }
}

// ---- gathers ------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_gather(int64_t n, const uint32_t *__restrict__ perm,
                                                GatherList g, int identity)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t src = identity ? k : (int64_t)perm[k];
    copy_listed(g, src, k);
}

__global__ void k_iota(int64_t n, uint32_t *__restrict__ v)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) v[k] = (uint32_t)k;
}

// ---- leaves and tree -------------------------------------------------------------
//
// Leaves are runs of at most G consecutive sorted particles that never cross
// the boundary of a Morton cell about 4 h wide: a new segment starts between
// sorted particles k-1 and k when their keys differ above the level whose
// cell edge is the largest power-of-two fraction of the box not below
// 4 max(h_k-1, h_k).  Without this rule a run of G particles can straddle a
// jump of the Morton curve and get a box as large as the domain.

constexpr int kScanTile = 1024;     // particles per block in the leaf scans
constexpr int kScanThreads = 256;   // 4 particles per thread

__device__ inline bool seg_break(int64_t k, const uint64_t *__restrict__ keys,
                                 const double *__restrict__ h, double ext, int bits)
{
    if (k == 0) return true;
    double hm = fmax(h[k - 1], h[k]);
    int T = 1;
    if (hm > 0.0 && ext > 0.0) {
        double t = floor(log2(ext / (4.0 * hm)));
        T = t < 1.0 ? 1 : (t > (double)bits ? bits : (int)t);
    }
    int sh = 3 * (bits - T);
    return (keys[k - 1] >> sh) != (keys[k] >> sh);
}

// block-wide inclusive scan of one value per thread (max or sum)
template <bool MAX>
__device__ inline uint32_t block_scan(uint32_t v, uint32_t *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        uint32_t o = t >= d ? sh[t - d] : 0u;
        __syncthreads();
        sh[t] = MAX ? (sh[t] > o ? sh[t] : o) : sh[t] + o;
        __syncthreads();
    }
    uint32_t r = sh[t];
    __syncthreads();
    return r;
}

// per tile: break flags and the largest segment start inside the tile
__global__ __launch_bounds__(kScanThreads) void k_seg_tiles(int64_t n, const uint64_t *__restrict__ keys,
                                                            const double *__restrict__ h,
                                                            const double *__restrict__ box,
                                                            int bits, uint32_t *__restrict__ flag,
                                                            uint32_t *__restrict__ tmax)
{
    __shared__ uint32_t sh[kScanThreads];
    const double ext = fmax(fmax(box[3] - box[0], box[4] - box[1]), box[5] - box[2]);
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * 4;
    uint32_t mx = 0;
    for (int e = 0; e < 4; e++) {
        int64_t k = base + e;
        if (k < n) {
            bool b = seg_break(k, keys, h, ext, bits);
            flag[k] = b ? 1u : 0u;
            if (b) mx = (uint32_t)k;
        }
    }
    uint32_t r = block_scan<true>(mx, sh);
    if (threadIdx.x == kScanThreads - 1) tmax[blockIdx.x] = r;
}

// exclusive scan over the tile values, one block (max or sum); copy (when not
// null) receives the values as they were
template <bool MAX>
__global__ __launch_bounds__(1024) void k_scan_tiles(uint32_t *__restrict__ a, int64_t ntile,
                                                     uint32_t *__restrict__ copy)
{
    __shared__ uint32_t sums[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (ntile + 1023) / 1024;
    const int64_t s0 = t * chunk, s1 = s0 + chunk < ntile ? s0 + chunk : ntile;
    uint32_t s = 0;
    for (int64_t k = s0; k < s1; k++) s = MAX ? (a[k] > s ? a[k] : s) : s + a[k];
    sums[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        uint32_t v = t >= d ? sums[t - d] : 0u;
        __syncthreads();
        sums[t] = MAX ? (sums[t] > v ? sums[t] : v) : sums[t] + v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? sums[t - 1] : 0u;
    for (int64_t k = s0; k < s1; k++) {
        uint32_t v = a[k];
        if (copy) copy[k] = v;
        a[k] = run;
        run = MAX ? (v > run ? v : run) : run + v;
    }
}

// per tile: segment start of every particle, leaf-start flags, leaf count
__global__ __launch_bounds__(kScanThreads) void k_seg_apply(int64_t n, int G,
                                                            uint32_t *__restrict__ flag,
                                                            const uint32_t *__restrict__ tmax,
                                                            uint32_t *__restrict__ tcnt)
{
    __shared__ uint32_t sh[kScanThreads];
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * 4;
    uint32_t loc[4];
    uint32_t mx = 0;
    for (int e = 0; e < 4; e++) {
        int64_t k = base + e;
        loc[e] = (k < n && flag[k]) ? (uint32_t)k : 0u;
        mx = loc[e] > mx ? loc[e] : mx;
    }
    uint32_t incl = block_scan<true>(mx, sh);
    uint32_t prev = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0u;
    // sh was overwritten by the scan's final value per thread before return;
    // recompute the exclusive prefix from the inclusive values
    __syncthreads();
    sh[threadIdx.x] = incl;
    __syncthreads();
    prev = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0u;
    uint32_t seg = prev > tmax[blockIdx.x] ? prev : tmax[blockIdx.x];
    uint32_t count = 0;
    for (int e = 0; e < 4; e++) {
        int64_t k = base + e;
        if (k >= n) break;
        if (flag[k]) seg = (uint32_t)k;
        uint32_t ls = ((uint32_t)(k - seg) % (uint32_t)G) == 0u ? 1u : 0u;
        flag[k] = ls;
        count += ls;
    }
    __syncthreads();
    uint32_t tot = block_scan<false>(count, sh);
    if (threadIdx.x == kScanThreads - 1) tcnt[blockIdx.x] = tot;
}

// per tile: leaf index of every particle and the first particle of every leaf
__global__ __launch_bounds__(kScanThreads) void k_leaf_ids(int64_t n, const uint32_t *__restrict__ flag,
                                                           const uint32_t *__restrict__ toff,
                                                           uint32_t *__restrict__ leaf_id,
                                                           uint32_t *__restrict__ lstart)
{
    __shared__ uint32_t sh[kScanThreads];
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * 4;
    uint32_t cnt = 0;
    for (int e = 0; e < 4; e++) {
        int64_t k = base + e;
        if (k < n) cnt += flag[k];
    }
    uint32_t incl = block_scan<false>(cnt, sh);
    uint32_t run = toff[blockIdx.x] + incl - cnt;   // leaf starts before this thread's items
    for (int e = 0; e < 4; e++) {
        int64_t k = base + e;
        if (k >= n) break;
        if (flag[k]) {
            lstart[run] = (uint32_t)k;
            run++;
        }
        leaf_id[k] = run - 1;
        if (k == n - 1) lstart[run] = (uint32_t)n;
    }
}

// tree levels from the leaf count (one thread)
__global__ void k_tree_info(int64_t n, int G, const uint32_t *__restrict__ toff,
                            const uint32_t *__restrict__ tcnt, int64_t ntile,
                            TreeInfo *__restrict__ T)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t L = (int64_t)toff[ntile - 1] + tcnt[ntile - 1];
    T->leaf_size = G;
    T->n = n;
    int64_t cnt = L, off = 0;
    int lev = 0;
    for (; lev < kMaxLevels; lev++) {
        T->off[lev] = off;
        T->cnt[lev] = cnt;
        off += cnt;
        if (cnt <= 1) { lev++; break; }
        cnt = (cnt + 7) / 8;
    }
    T->nlev = lev;
    for (int l = lev; l < kMaxLevels; l++) { T->off[l] = off; T->cnt[l] = 0; }
}

__device__ inline Node merge_children(const Node *__restrict__ child, int64_t c0, int64_t c1)
{
    Node nd;
    for (int a = 0; a < 3; a++) { nd.lo[a] = INFINITY; nd.hi[a] = -INFINITY; }
    nd.hmax = 0.0;
    nd.pad = 0.0;
    for (int64_t c = c0; c < c1; c++) {
        const Node &ch = child[c];
        for (int a = 0; a < 3; a++) { nd.lo[a] = fmin(nd.lo[a], ch.lo[a]); nd.hi[a] = fmax(nd.hi[a], ch.hi[a]); }
        nd.hmax = fmax(nd.hmax, ch.hmax);
    }
    return nd;
}

// Leaf boxes and largest h: 16 lanes per leaf read its (consecutive)
// particles together, then reduce with shuffles inside their 16-lane group.
constexpr int kLeafLanes = 16;

__global__ __launch_bounds__(256) void k_leaves(const TreeInfo *__restrict__ T,
                                                const uint32_t *__restrict__ lstart,
                                                const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z,
                                                const double *__restrict__ h,
                                                Node *__restrict__ nodes)
{
    const int64_t L = T->cnt[0];
    const int q = threadIdx.x % kLeafLanes;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kLeafLanes);
    // the 16 lanes of a group share l, so they take the same trips
    for (int64_t l = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kLeafLanes; l < L; l += stride) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double hm = 0.0;
        for (int64_t k = lstart[l] + q; k < (int64_t)lstart[l + 1]; k += kLeafLanes) {
            const double v[3] = {x[k], y[k], z[k]};
            for (int a = 0; a < 3; a++) { lo[a] = fmin(lo[a], v[a]); hi[a] = fmax(hi[a], v[a]); }
            hm = fmax(hm, h[k]);
        }
        for (int o = kLeafLanes / 2; o > 0; o >>= 1) {
            for (int a = 0; a < 3; a++) {
                lo[a] = fmin(lo[a], __shfl_xor(lo[a], o));
                hi[a] = fmax(hi[a], __shfl_xor(hi[a], o));
            }
            hm = fmax(hm, __shfl_xor(hm, o));
        }
        if (q == 0) {
            Node nd;
            for (int a = 0; a < 3; a++) { nd.lo[a] = lo[a]; nd.hi[a] = hi[a]; }
            nd.hmax = hm;
            nd.pad = 0.0;
            nodes[l] = nd;
        }
    }
}

// largest h of every leaf after the h solve changed h (boxes are unchanged),
// one thread per leaf over its consecutive particles
__global__ __launch_bounds__(256) void k_leaf_hmax(const TreeInfo *__restrict__ T,
                                                   const uint32_t *__restrict__ lstart,
                                                   const double *__restrict__ h,
                                                   Node *__restrict__ nodes)
{
    const int64_t L = T->cnt[0];
    const int q = threadIdx.x % kLeafLanes;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kLeafLanes);
    for (int64_t l = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kLeafLanes; l < L; l += stride) {
        double hm = 0.0;
        for (int64_t k = lstart[l] + q; k < (int64_t)lstart[l + 1]; k += kLeafLanes) hm = fmax(hm, h[k]);
        for (int o = kLeafLanes / 2; o > 0; o >>= 1) hm = fmax(hm, __shfl_xor(hm, o));
        if (q == 0) nodes[l].hmax = hm;
    }
}

constexpr int64_t kSmallLevel = 2048;   // children per level handled by one block
constexpr int kBigLevels = 4;           // levels built grid-wide at most

// level `lev` from level lev-1, grid-wide, when the child level is large
__global__ __launch_bounds__(256) void k_tree_level_big(const TreeInfo *__restrict__ T,
                                                        Node *__restrict__ nodes, int lev)
{
    if (lev >= T->nlev || T->cnt[lev - 1] <= kSmallLevel) return;
    const Node *child = nodes + T->off[lev - 1];
    Node *par = nodes + T->off[lev];
    const int64_t nchild = T->cnt[lev - 1], npar = T->cnt[lev];
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npar;
         p += (int64_t)gridDim.x * blockDim.x) {
        int64_t c1 = 8 * p + 8 < nchild ? 8 * p + 8 : nchild;
        par[p] = merge_children(child, 8 * p, c1);
    }
}

// all remaining (small) levels by one block, level after level
__global__ __launch_bounds__(1024) void k_tree_level_small(const TreeInfo *__restrict__ T,
                                                           Node *__restrict__ nodes)
{
    const int nlev = T->nlev;
    for (int lev = 1; lev < nlev; lev++) {
        if (lev <= kBigLevels && T->cnt[lev - 1] > kSmallLevel) continue;
        const Node *child = nodes + T->off[lev - 1];
        Node *par = nodes + T->off[lev];
        const int64_t nchild = T->cnt[lev - 1], npar = T->cnt[lev];
        for (int64_t p = threadIdx.x; p < npar; p += blockDim.x) {
            int64_t c1 = 8 * p + 8 < nchild ? 8 * p + 8 : nchild;
            par[p] = merge_children(child, 8 * p, c1);
        }
        __syncthreads();
    }
}

// FP32-pair mode: single-precision offsets of each particle from the centre of
// its leaf box.
__global__ __launch_bounds__(256) void k_offsets(int64_t n, const uint32_t *__restrict__ leaf_id,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ y,
                                                 const double *__restrict__ z,
                                                 const Node *__restrict__ leaves,
                                                 float *__restrict__ fx, float *__restrict__ fy,
                                                 float *__restrict__ fz)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const Node &nd = leaves[leaf_id[k]];
    fx[k] = (float)(x[k] - 0.5 * (nd.lo[0] + nd.hi[0]));
    fy[k] = (float)(y[k] - 0.5 * (nd.lo[1] + nd.hi[1]));
    fz[k] = (float)(z[k] - 0.5 * (nd.lo[2] + nd.hi[2]));
}

// Force record of particle k: A_k = P_k / (Omega_k rho_k^2),
// c_k = sqrt(gamma P_k / rho_k), 1/h_k, v_k, m_k, rho_k with
// P_k = (gamma - 1) rho_k u_k.
__global__ __launch_bounds__(256) void k_force_prep(int64_t n, double gamma,
                                                    const double *__restrict__ rho,
                                                    const double *__restrict__ omega,
                                                    const double *__restrict__ u,
                                                    const double *__restrict__ h,
                                                    const double *__restrict__ m,
                                                    const double *__restrict__ vx,
                                                    const double *__restrict__ vy,
                                                    const double *__restrict__ vz,
                                                    ForceRec *__restrict__ rec,
                                                    ForceRec32 *__restrict__ rec32)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double r = rho[k];
    const double P = (gamma - 1.0) * r * u[k];
    ForceRec f;
    f.c = sqrt(gamma * P / r);
    f.hinv = 1.0 / h[k];
    f.vx = vx[k];
    f.vy = vy[k];
    f.vz = vz[k];
    f.m = m[k];
    f.A = P / (omega[k] * r * r);
    f.rho = r;
    rec[k] = f;
    if (rec32) {
        ForceRec32 g;
        g.c = (float)f.c;
        g.hinv = (float)f.hinv;
        g.vx = (float)f.vx;
        g.vy = (float)f.vy;
        g.vz = (float)f.vz;
        g.m = (float)f.m;
        g.A = (float)f.A;
        g.rho = (float)f.rho;
        rec32[k] = g;
    }
}

} // namespace

// nodes of the tree over at most n leaves (every leaf holds >= 1 particle)
int64_t node_count_bound(int64_t n)
{
    int64_t cnt = std::max<int64_t>(n, 1), tot = 0;
    while (true) {
        tot += cnt;
        if (cnt <= 1) break;
        cnt = ceil_div(cnt, 8);
    }
    return tot;
}

static inline unsigned grid_for(int64_t n, int threads)
{
    return (unsigned)((n + threads - 1) / threads);
}

sph_status build_order(sph_ctx *c, int64_t n, const double *x, const double *y, const double *z)
{
    if (n == 0) return SPH_OK;
    const sph_params &p = c->p;
    FixedBox fb{};
    if (p.periodic) {
        // k_keys takes the box by value and stores it for the later kernels
        fb.fixed = 1;
        for (int a = 0; a < 3; a++) { fb.lo[a] = p.box_lo[a]; fb.hi[a] = p.box_hi[a]; }
    } else {
        int nb = (int)std::min<int64_t>(1024, ceil_div(n, kBoxThreads));
        hipLaunchKernelGGL(k_box_partial, dim3(nb), dim3(kBoxThreads), 0, c->stream, n, x, y, z,
                           c->d_part);
        hipLaunchKernelGGL(k_box_final, dim3(1), dim3(64), 0, c->stream, nb, c->d_part, c->d_box);
    }
    const int bits = key_bits(n);
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, x, y, z,
                       c->d_box, fb, bits, c->keys[0], c->vals[0]);
    // small sets: tiles of 1024 keys (more, shorter blocks); up to
    // kRsRawTiles tiles the scatter blocks form the digit offsets from the raw
    // counts themselves (one launch fewer per pass).  A stable sort's result
    // does not depend on the tiling.
    const bool small = rs_use_small(n);
    const int64_t ntiles = small ? rs_small_tiles(n) : ceil_div(n, kRsTile);
    if (256 * ntiles + 256 > c->hist_cap) return fail(c, SPH_ENOMEM, "radix count capacity");
    const int passes = (3 * bits + 7) / 8;
    const int raw = ntiles <= kRsRawTiles ? 1 : 0;
    int cur = 0;
    for (int ps = 0; ps < passes; ps++) {
        int shift = 8 * ps;
        if (small)
            hipLaunchKernelGGL(k_rs_hist<kRsItemsSmall>, dim3((unsigned)ntiles), dim3(kRsThreads), 0,
                               c->stream, n, c->keys[cur], shift, c->hist, ntiles);
        else
            hipLaunchKernelGGL(k_rs_hist<kRsItems>, dim3((unsigned)ntiles), dim3(kRsThreads), 0,
                               c->stream, n, c->keys[cur], shift, c->hist, ntiles);
        if (!raw)
            hipLaunchKernelGGL(k_rs_digit_scan, dim3(256), dim3(256), 0, c->stream, c->hist, ntiles,
                               c->hist + 256 * ntiles);
        if (small)
            hipLaunchKernelGGL(k_rs_scatter<kRsItemsSmall>, dim3((unsigned)ntiles), dim3(kRsThreads),
                               0, c->stream, n, c->keys[cur], c->vals[cur], c->keys[cur ^ 1],
                               c->vals[cur ^ 1], shift, c->hist, ntiles, c->hist + 256 * ntiles, raw);
        else
            hipLaunchKernelGGL(k_rs_scatter<kRsItems>, dim3((unsigned)ntiles), dim3(kRsThreads), 0,
                               c->stream, n, c->keys[cur], c->vals[cur], c->keys[cur ^ 1],
                               c->vals[cur ^ 1], shift, c->hist, ntiles, c->hist + 256 * ntiles, raw);
        cur ^= 1;
    }
    c->perm = c->vals[cur];
    c->skeys = c->keys[cur];
    c->scratch_u32 = (uint32_t *)c->keys[cur ^ 1];
    c->tree_n = -1;
    return hip_check(c, hipGetLastError(), "build_order");
}

sph_status gather(sph_ctx *c, int64_t n, const GatherList &g, bool identity_src_index)
{
    if (n == 0 || g.count == 0) return SPH_OK;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, c->perm, g,
                       identity_src_index ? 1 : 0);
    return hip_check(c, hipGetLastError(), "gather");
}

// nodes above the leaves, merged level by level.  A grid-wide level is
// launched only where its children can outnumber what the one-block kernel
// takes (kSmallLevel): level l has at most ceil(n / 8^(l-1)) children (a leaf
// holds at least one particle), and a launch with fewer would return at once,
// so small sets skip those launches.
static void upper_levels(sph_ctx *c, int64_t n)
{
    int64_t children = n;
    for (int l = 1; l <= kBigLevels; l++) {
        const int64_t parents = ceil_div(children, 8);
        if (children > kSmallLevel)
            hipLaunchKernelGGL(k_tree_level_big, dim3(grid_for(parents, 256)), dim3(256), 0,
                               c->stream, c->d_tree, c->nodes, l);
        children = parents;
    }
    hipLaunchKernelGGL(k_tree_level_small, dim3(1), dim3(1024), 0, c->stream, c->d_tree, c->nodes);
}

sph_status build_tree(sph_ctx *c, int64_t n)
{
    c->tree_n = -1;
    if (n == 0) return SPH_OK;
    const int G = c->p.leaf_size;
    if (!c->skeys || !c->scratch_u32 || !c->lstart || !c->leaf_id || !c->d_tree || !c->nodes)
        return fail(c, SPH_ESTATE, "build_tree: order not built");
    const int64_t ntile = ceil_div(n, kScanTile);
    if (2 * ntile > c->hist_cap) return fail(c, SPH_ENOMEM, "scan tile capacity");
    if (c->node_cap < node_count_bound(n)) return fail(c, SPH_ENOMEM, "node capacity");
    uint32_t *tmax = c->hist, *tcnt = c->hist + ntile;
    uint32_t *flag = c->scratch_u32;
    hipLaunchKernelGGL(k_seg_tiles, dim3((unsigned)ntile), dim3(kScanThreads), 0, c->stream, n,
                       c->skeys, c->s.h, c->d_box, key_bits(n), flag, tmax);
    hipLaunchKernelGGL((k_scan_tiles<true>), dim3(1), dim3(1024), 0, c->stream, tmax, ntile,
                       (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_seg_apply, dim3((unsigned)ntile), dim3(kScanThreads), 0, c->stream, n, G,
                       flag, tmax, tcnt);
    // tcnt -> exclusive offsets in place; the counts themselves go to tmax
    // for the total
    hipLaunchKernelGGL((k_scan_tiles<false>), dim3(1), dim3(1024), 0, c->stream, tcnt, ntile,
                       tmax);
    hipLaunchKernelGGL(k_tree_info, dim3(1), dim3(64), 0, c->stream, n, G, tcnt, tmax, ntile,
                       c->d_tree);
    hipLaunchKernelGGL(k_leaf_ids, dim3((unsigned)ntile), dim3(kScanThreads), 0, c->stream, n,
                       flag, tcnt, c->leaf_id, c->lstart);
    hipLaunchKernelGGL(k_leaves, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, c->d_tree,
                       c->lstart, c->s.x, c->s.y, c->s.z, c->s.h, c->nodes);
    upper_levels(c, n);
    if (c->p.precision == SPH_FP32_PAIR)
        hipLaunchKernelGGL(k_offsets, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n,
                           c->leaf_id, c->s.x, c->s.y, c->s.z, c->nodes, c->s.fx, c->s.fy, c->s.fz);
    sph_status st = hip_check(c, hipGetLastError(), "build_tree");
    if (st == SPH_OK) c->tree_n = n;
    return st;
}

sph_status refresh_hmax(sph_ctx *c, int64_t n)
{
    if (n == 0) return SPH_OK;
    if (c->tree_n != n) return fail(c, SPH_ESTATE, "refresh_hmax: tree not built");
    hipLaunchKernelGGL(k_leaf_hmax, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, c->d_tree,
                       c->lstart, c->s.h, c->nodes);
    upper_levels(c, n);
    return hip_check(c, hipGetLastError(), "refresh_hmax");
}

sph_status force_prep(sph_ctx *c, int64_t n, const double *u_sorted, const double *vx,
                      const double *vy, const double *vz)
{
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_force_prep, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n,
                       c->p.gamma, c->s.rho, c->s.omega, u_sorted, c->s.h, c->s.m, vx, vy, vz,
                       c->s.frec, c->p.precision == SPH_FP32_PAIR ? c->s.frec32 : nullptr);
    return hip_check(c, hipGetLastError(), "force_prep");
}

sph_status iota(sph_ctx *c, int64_t n, uint32_t *v)
{
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, v);
    return hip_check(c, hipGetLastError(), "iota");
}

} // namespace sph
