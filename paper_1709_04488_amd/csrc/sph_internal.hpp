// Internal definitions shared by the HIP translation units of libsph.
// Device code targets gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/sph.h"

namespace sph {

// Smoothing kernels (section 2), W(r, h) = sigma h^-3 f(r/h) with compact
// support R h:
//   M4 cubic spline, R = 2, sigma = 1/pi, in B-spline form
//     f(q) = (2-q)_+^3 / 4 - (1-q)_+^3
//   (1 - 3/2 q^2 + 3/4 q^3 on [0,1), (2-q)^3/4 on [1,2));
//   quintic spline (Morris 1996), R = 3, sigma = 1/(120 pi),
//     f(q) = (3-q)_+^5 - 6 (2-q)_+^5 + 15 (1-q)_+^5.
// list: density-loop candidate-list entries per particle (below).
template <int K>
struct Kern;
template <>
struct Kern<SPH_KERNEL_M4> {
    static constexpr double R = 2.0;
    static constexpr double sigma = 0.31830988618379067154;
    static constexpr int list = 160;
};
template <>
struct Kern<SPH_KERNEL_QUINTIC> {
    static constexpr double R = 3.0;
    static constexpr double sigma = 0.0026525823848649222;
    static constexpr int list = 480;
};
inline double kern_support(int k) { return k == SPH_KERNEL_QUINTIC ? 3.0 : 2.0; }
inline int kern_list(int k)
{
    return k == SPH_KERNEL_QUINTIC ? Kern<SPH_KERNEL_QUINTIC>::list : Kern<SPH_KERNEL_M4>::list;
}

constexpr int kWave = 64;
constexpr int kMaxLevels = 16;   // tree levels above the leaves (8-ary)
constexpr int kFront = 512;      // per-wave LDS capacity of a walk frontier / candidate list
constexpr int kXcds = 8;         // MI355X: 8 XCDs, blocks dispatched round-robin
constexpr int kMaxBatch = 128;   // particle sets per batched pair-kernel launch
constexpr int kArgBytes = 1024;  // device argument block of one pair-kernel launch

// Persistent pair-kernel grid: one wave per block, at most as many blocks as
// the GPU holds at once (256 CUs x 16 waves: the pair kernels run at 4 waves
// per SIMD), at least one block per 8 particles below that, a
// multiple of the XCD count.  Each block owns a slice of the density loop's
// candidate-list scratch, so the cap also bounds that scratch.
constexpr int64_t kMaxPairBlocks = 256 * 16;

// Active-leaf compaction of block time-steps: leaves per block, and the
// per-block counts (one more than the blocks, for the bound of n leaves)
// Radix sort tiles: 4096 keys (256 threads x 16) per block; sets of at most
// kRsRawTiles small tiles of 1024 keys (256 x 4) sort with those instead (four
// times the blocks and a quarter of each block's chain), and up to kRsRawTiles
// tiles the scatter forms the digit offsets from the raw counts.  The counts
// take 256 words per tile plus 256 digit totals.
constexpr int kRsItems = 16, kRsItemsSmall = 4;
constexpr int64_t kRsTile = 256 * kRsItems, kRsTileSmall = 256 * kRsItemsSmall;
constexpr int64_t kRsRawTiles = 64;
constexpr int64_t rs_small_tiles(int64_t n) { return (n + kRsTileSmall - 1) / kRsTileSmall; }
constexpr bool rs_use_small(int64_t n) { return rs_small_tiles(n) <= kRsRawTiles; }
constexpr int64_t hist_words(int64_t cap)
{
    // the larger of the two tilings any n <= cap can use
    const int64_t big = (cap + kRsTile - 1) / kRsTile;
    const int64_t small = rs_small_tiles(cap) < kRsRawTiles ? rs_small_tiles(cap) : kRsRawTiles;
    return 256 * (big > small ? big : small) + 256;
}

constexpr int kActTile = 1024;
constexpr int64_t act_tiles(int64_t cap) { return (cap + kActTile - 1) / kActTile + 1; }
inline unsigned pair_grid(int64_t n)
{
    int64_t blocks = (n + 7) / 8;
    blocks = blocks < kXcds ? kXcds : (blocks > kMaxPairBlocks ? kMaxPairBlocks : blocks);
    blocks = ((blocks + kXcds - 1) / kXcds) * kXcds;
    return (unsigned)blocks;
}

// Density-loop candidate lists: up to Kern<K>::list entries per home
// particle (160 for the M4, whose sphere of radius 2 Rc holds ~90 neighbours
// at eta = 1.2; 480 for the quintic's ~300 within 3 Rc), each an FP64 r^2 and
// an FP64 mass, for the candidates within R Rc, Rc = kCacheGrow h (capped by
// the walk radius), so that Newton steps within that bound reuse them.  A
// block holds the lists of one leaf's G particles.
constexpr double kCacheGrow = 1.15;
inline int64_t cache_bytes(int G, int kernel, int64_t blocks)
{
    return blocks * 2 * (int64_t)kern_list(kernel) * G * (int64_t)sizeof(double);
}

// Tree node: bounding box of the particles below it and their largest h.
// 64 bytes, so one node is half a 128-byte cache line.
struct alignas(64) Node {
    double lo[3];
    double hmax;
    double hi[3];
    double pad;
};

// Tree description, written on the device by the build (the leaf count is
// data dependent) and read by every pair kernel.
struct TreeInfo {
    int32_t nlev;                  // levels including the leaf level (level 0)
    int32_t leaf_size;
    int64_t n;                     // particles
    int64_t off[kMaxLevels];       // first node of each level in the node array
    int64_t cnt[kMaxLevels];       // nodes per level (cnt[0] = leaves)
};
constexpr int kTreeWords = (int)(sizeof(TreeInfo) / 8);

struct Box {
    int32_t periodic;
    double lo[3];
    double len[3];                 // periodic box lengths
    double half[3];                // len / 2
};

// Device status word: [0] flags, [1] h solves not converged, [2] non-finite
// results, [3] periodic 2h >= L/2, [4] walk overflows (slow path taken),
// [5] max Newton-Raphson iterations, [6..7] spare.
enum : int32_t {
    kFlagNotConverged = 1,
    kFlagNonFinite = 2,
    kFlagStencil = 4,
    kFlagLevel = 8,     // block time-steps: a level deeper than the timeline allows
};
constexpr int kStatusWords = 8;

// Device counters of the last evaluation.  [0, 1] are written by the
// conserved-quantity reduction; the density loop zeroes and fills
// [kCntDensFirst, kCntDensFirst + kCntDensWords), the force loop
// [kCntForceFirst, kCntForceFirst + kCntForceWords).
enum : int {
    kCntNngb = 0,            // sum of density neighbour counts
    kCntNforce = 1,          // sum of force neighbour counts
    kCntDensEvals = 2,       // density pairs evaluated, all Newton-Raphson iterations
    kCntNrMax = 3,           // largest Newton-Raphson iteration count of a wave
    kCntDensOverflows = 4,   // density walks that overflowed the LDS frontier
    kCntDensVisits = 5,      // candidate leaves staged by density sweeps
    kCntDensWalks = 6,       // density tree walks
    kCntNrTotal = 7,         // density evaluations summed over particles
    kCntDensTests = 8,       // particle-candidate distance tests, density
    kCntDensBoxes = 9,       // particle-leaf box tests, density
    kCntForceEvals = 10,     // force pairs evaluated
    kCntForceOverflows = 11, // force walks that overflowed the LDS frontier
    kCntForceTests = 12,     // particle-candidate distance tests, force
    kCntForceBoxes = 13,     // particle-leaf box tests, force
    kCntDensListOverflows = 14, // particles whose candidate list outgrew its capacity in a sweep
    kCountWords = 16,
    kCntDensFirst = kCntDensEvals,
    kCntDensWords = kCntDensBoxes - kCntDensEvals + 1,
    kCntForceFirst = kCntForceEvals,
    kCntForceWords = kCntForceBoxes - kCntForceEvals + 1,
};

// What the force loop reads of every neighbour j, in one 64-byte line:
// c_j, 1/h_j, v_j, m_j, A_j = P_j / (Omega_j rho_j^2) and rho_j.
struct alignas(64) ForceRec {
    double c, hinv, vx, vy, vz, m, A, rho;
};

// FP32-pair mode: the same record rounded to single precision (32 bytes), so
// the force loop's pair terms read half the bytes and convert nothing.  The
// home particle's values are rounded the same way, so the (j, i) pair sees
// exactly the values of the (i, j) pair.
struct alignas(32) ForceRec32 {
    float c, hinv, vx, vy, vz, m, A, rho;
};

// Arrays in sorted (Morton) order.  FP32-pair mode adds float offsets from the
// centre of each particle's leaf.
struct Sorted {
    double *x = nullptr, *y = nullptr, *z = nullptr;
    double *vx = nullptr, *vy = nullptr, *vz = nullptr;
    double *m = nullptr, *u = nullptr, *h = nullptr;
    double *rho = nullptr, *omega = nullptr;
    ForceRec *frec = nullptr;                  // force record
    ForceRec32 *frec32 = nullptr;              // its single-precision copy (FP32-pair)
    double *ax = nullptr, *ay = nullptr, *az = nullptr, *du = nullptr;
    double *vsig = nullptr, *dt = nullptr;
    int32_t *nngb = nullptr, *nforce = nullptr;
    uint32_t *id = nullptr;                    // original (caller) index
    // resident-state integration arrays
    double *vpx = nullptr, *vpy = nullptr, *vpz = nullptr, *up = nullptr;
    // artificial-viscosity switches: alpha (state), its predictor and rate
    // (MM97), div v of the previous step (CD10); div v and |curl v| outputs
    double *al = nullptr, *alp = nullptr, *adot = nullptr, *dprev = nullptr;
    double *divv = nullptr, *curlv = nullptr;
    // block time-steps: level, step start and end (ticks), half-step v and u
    // (and alpha under MM97), the active flag and the limiter's neighbour
    // level and wake-up mark of the current sub-step
    int32_t *lev = nullptr;
    int64_t *ts = nullptr, *te = nullptr;
    double *vhx = nullptr, *vhy = nullptr, *vhz = nullptr, *uh = nullptr, *alh = nullptr;
    int32_t *act = nullptr, *lmx = nullptr, *mark = nullptr;
    // FP32-pair mode
    float *fx = nullptr, *fy = nullptr, *fz = nullptr;
};

// Device clock of the block time-steps (one level-0 step = 2^lmax ticks).
struct BlockClock {
    int64_t T;          // current tick within the level-0 step
    int64_t Tn;         // tick of the sub-step in progress
    int64_t full;       // level-0 steps completed
    int64_t nsub;       // sub-steps taken
    int64_t active;     // active particles of the last sub-step
    int64_t updates;    // active particles summed over the sub-steps
    double tick;        // time per tick of the current level-0 step
    double tick_next;   // time per tick of the next one (set at a full sync)
    double time;        // elapsed time
    double dt_max;      // length of the current level-0 step
    double dt_max_next; // of the next one (set at a full sync)
    int64_t pad[5];
};

struct Timer {
    bool on = false;
    double ms[3] = {0, 0, 0};
    int64_t launches[3] = {0, 0, 0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[3];
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
};

} // namespace sph

struct sph_ctx {
    sph_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    size_t budget = 0;
    size_t bytes = 0;
    std::string err;

    // capacity of the per-particle buffers
    int64_t ncap = 0;
    int64_t n = 0;
    std::vector<void *> allocs;          // everything sized by ncap

    // build
    uint64_t *keys[2] = {nullptr, nullptr};
    uint32_t *vals[2] = {nullptr, nullptr};
    uint32_t *hist = nullptr;
    int64_t hist_cap = 0;
    uint32_t *perm = nullptr;            // sorted position -> source index
    double *d_box = nullptr;             // [lo0..2, hi0..2] on device
    double *d_part = nullptr;            // reduction partials
    sph::Node *nodes = nullptr;
    int64_t node_cap = 0;
    sph::TreeInfo *d_tree = nullptr;    // device-resident tree description
    uint32_t *lstart = nullptr;         // leaf -> first sorted particle, [L+1]
    uint32_t *leaf_id = nullptr;        // sorted particle -> leaf
    uint32_t *d_work = nullptr;         // per-XCD claim counters of the pair kernels
    double *cache = nullptr;            // density-loop candidate lists, a slice per pair-kernel block
    int64_t cache_size = 0;             // its bytes (cache_bytes(G, 1) per block at leaf size G)
    void *d_dargs = nullptr;            // device argument block of the density loop
    void *d_fargs = nullptr;            // device argument block of the force loop
    uint64_t *skeys = nullptr;          // sorted keys of the last build
    uint32_t *scratch_u32 = nullptr;    // per-particle scratch (free sort buffer)
    int64_t tree_n = -1;                // n of the tree on the device (-1: none)
    sph::Box box{};

    sph::Sorted s;       // working / resident arrays
    sph::Sorted t;       // alternate buffers for re-sorting the resident state

    // identity of the arrays the current structure was built from
    const double *built_x = nullptr;
    int64_t built_n = -1;
    bool built = false;

    // resident state
    bool resident = false;
    bool res_alpha = false;     // the resident state carries per-particle alpha
    sph::BlockClock *d_clock = nullptr;   // block time-steps (device)
    int32_t *leaf_act = nullptr;     // active particles per leaf of the current sub-step
    // the leaves with an active particle, in leaf order, and their number (on
    // the device): the home leaves of the pair loops in a sub-step; per-tile
    // counts, then offsets, of the compaction that lists them
    uint32_t *act_list = nullptr, *act_tile = nullptr, *act_cnt = nullptr;
    double *d_scal = nullptr;   // [0] dt_next [1] dt_last [2] time [3] KE [4] TE [5..7] P
                                // [8] smallest, [9] largest mass of the last density pass
    // device counters, indexed by the kCnt* constants
    int64_t *d_counts = nullptr;
    double *h_scal = nullptr;   // pinned mirror
    int64_t *h_counts = nullptr;   // pinned mirror of d_counts
    sph::BlockClock *h_clock = nullptr; // pinned mirror of d_clock
    double *dt_used_out = nullptr;
    int64_t steps = 0;

    int32_t *d_status = nullptr;
    int32_t *h_status = nullptr;   // pinned mirror

    // captured pair of resident steps
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    double graph_dt = 0.0;

    sph::Timer timer;
    bool count_tests = false;   // pair loops also count box and candidate tests

    // per-call active set of the pair loops (block time-steps; nullptr: every
    // particle) and the force loop's limiter outputs
    const int32_t *f_act = nullptr;
    bool f_block = false;

    // per-call inputs of the force loop: the sorted per-particle alpha it
    // uses (nullptr: alpha_av for every pair), whether it writes div v and
    // |curl v| (set by the phase functions before forces_prepare)
    const double *f_alpha = nullptr;
    bool f_div = false;

    // this device's copy of the library's static scratch array (the
    // no-allocation entry point); nullptr if its address could not be taken
    void *static_scratch = nullptr;
    std::string static_err;
};

namespace sph {

// ---- host helpers (api.hip) --------------------------------------------------
sph_status fail(sph_ctx *c, sph_status s, const std::string &msg);
sph_status hip_check(sph_ctx *c, hipError_t e, const char *what);
sph_status ensure_capacity(sph_ctx *c, int64_t n);

// ---- build.hip ---------------------------------------------------------------
// Bounding box, keys, sort: fills c->perm (sorted -> source) for n positions.
sph_status build_order(sph_ctx *c, int64_t n, const double *x, const double *y,
                       const double *z);
// Gather `count` arrays through c->perm: dst[k] = src[perm[k]].
struct GatherList {
    int32_t count;
    int32_t kind[32];        // 0: 8-byte word, 1: uint32, 2: float
    const void *src[32];
    void *dst[32];
};
sph_status gather(sph_ctx *c, int64_t n, const GatherList &g, bool identity_src_index);
// Leaf boxes and tree over c->s.{x,y,z,h}; FP32 offsets when requested.
sph_status build_tree(sph_ctx *c, int64_t n);
// leaf and node hmax from the current sorted h (after the h solve), boxes kept
sph_status refresh_hmax(sph_ctx *c, int64_t n);
// Force records from rho, omega, h, m and the given sorted u and velocities.
sph_status force_prep(sph_ctx *c, int64_t n, const double *u_sorted, const double *vx,
                      const double *vy, const double *vz);
sph_status iota(sph_ctx *c, int64_t n, uint32_t *v);
int64_t node_count_bound(int64_t n);

// ---- pairs.hip (dispatch) and pairs.hpp (kernels) -------------------------
sph_status run_density(sph_ctx *c, int64_t n);
sph_status run_forces(sph_ctx *c, int64_t n);
// batched pair loops: prepare writes each set's argument block on its
// stream; launch runs one persistent kernel over cs[0..count) (same stream,
// precision and leaf size)
sph_status density_prepare(sph_ctx *c, int64_t n);
sph_status forces_prepare(sph_ctx *c, int64_t n);
sph_status density_launch(sph_ctx *const *cs, int count, int64_t nmax);
sph_status forces_launch(sph_ctx *const *cs, int count, int64_t nmax);
// meshless finite-volume gradient matrix and gradients over the built tree,
// with h and the number density (c->s.rho) already solved; sorted arrays
sph_status run_mfv(sph_ctx *c, int64_t n, int nf, const double *const *f, double *const *B,
                   double *cond, double *const *grad);
sph_status run_neighbours(sph_ctx *c, int64_t n, int32_t mode, int64_t *counts_sorted,
                          const int64_t *offsets_sorted, int32_t *idx, int64_t cap);

// ---- step.hip ----------------------------------------------------------------
// scatter sorted arrays back to caller order through c->perm
struct ScatterList {
    int32_t count;
    int32_t kind[32];
    const void *src[32];
    void *dst[32];
};
sph_status scatter(sph_ctx *c, int64_t n, const ScatterList &s, const uint32_t *index);

// dst[a][to] = src[a][from] for every array of a Gather/ScatterList, copied as
// bits (8 bytes for kind 0, 4 otherwise).  Up to 16 loads are issued before
// their stores: the lists carry no no-alias guarantee, so a load after a store
// would wait for it, and a one-array-at-a-time loop runs ~10 dependent memory
// round trips per element.
template <class List>
__device__ inline void copy_listed(const List &L, int64_t from, int64_t to)
{
    constexpr int kChunk = 16;
    for (int a0 = 0; a0 < L.count; a0 += kChunk) {
        uint64_t v[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; j++) {
            const int a = a0 + j;
            if (a < L.count)
                v[j] = L.kind[a] == 0 ? ((const uint64_t *)L.src[a])[from]
                                      : (uint64_t)((const uint32_t *)L.src[a])[from];
        }
#pragma unroll
        for (int j = 0; j < kChunk; j++) {
            const int a = a0 + j;
            if (a < L.count) {
                if (L.kind[a] == 0) ((uint64_t *)L.dst[a])[to] = v[j];
                else ((uint32_t *)L.dst[a])[to] = (uint32_t)v[j];
            }
        }
    }
}
sph_status eos_scatter(sph_ctx *c, int64_t n, const uint32_t *index, const double *u_caller,
                       double *P, double *cs);
// scatter plus the equation of state (P, cs may be NULL) from sorted rho, u
sph_status scatter_eos(sph_ctx *c, int64_t n, const ScatterList &s, const uint32_t *index,
                       const double *u_sorted, double *P, double *cs);
sph_status kick_drift(sph_ctx *c, int64_t n, double dt_host);
sph_status closing_kick(sph_ctx *c, int64_t n, double dt_host);
// artificial-viscosity switches on the resident state: MM97 rate adot from
// the predicted alpha and the latest div v; CD10 update of alpha (and
// dprev = div v) with the step length on the device
sph_status av_rate(sph_ctx *c, int64_t n, const double *alpha_now);
sph_status av_cd10(sph_ctx *c, int64_t n, bool first);
sph_status fill(sph_ctx *c, int64_t n, double *v, double value);
// block time-steps on the resident state (step.hip)
sph_status block_next(sph_ctx *c, int64_t n);           // Tn = min te; drift every particle
sph_status block_predict(sph_ctx *c, int64_t n);        // predictors, active set, leaf counts
sph_status block_finish(sph_ctx *c, int64_t n, bool init);  // close, levels, limiter, open, clock
sph_status block_av(sph_ctx *c, int64_t n);             // switches of the active particles
sph_status reduce_dt(sph_ctx *c, int64_t n);
// smallest and largest sorted mass -> d_scal[8], d_scal[9]
sph_status reduce_mass_range(sph_ctx *c, int64_t n);
sph_status reduce_diag(sph_ctx *c, int64_t n);
// zero d_counts[first..first+count) with a kernel (capture-safe, no memset)
sph_status zero_counts(sph_ctx *c, int first, int count);
// zero the per-XCD claim counters of the persistent pair kernels
sph_status zero_work(sph_ctx *c);
// exclusive prefix sum in place over a[0..n], treating a[n] as 0 on input
sph_status scan_offsets(sph_ctx *c, int64_t n, int64_t *a);

// timing
void timer_begin(sph_ctx *c, int which, hipEvent_t *b, hipEvent_t *e);
void timer_end(sph_ctx *c, int which, hipEvent_t b, hipEvent_t e);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

} // namespace sph
