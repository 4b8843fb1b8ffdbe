// Pair loops: density + Newton-Raphson h solve, hydro forces, neighbour
// export, MFV geometry.
//
// Work decomposition (the GPU analogue of the paper's per-leaf-cell neighbour
// gathering, section 4.2, with a leaf as the unit of work as in its OpenMP
// loop, section 5.2.1): one wavefront per home leaf of at most G sorted
// particles, 64/G lanes per particle.  The wave walks the box tree to collect
// the leaves that can hold neighbours of its particles into an LDS list.
// Candidate leaves are then handled 128/G at a time (128 candidate slots):
//   stage  -- one coalesced load per field brings their positions into LDS;
//   test   -- each (home particle, staged leaf) combination is first judged
//             by the distance from the particle to the leaf's box; the
//             passing ones are dealt out over the 64 lanes, which test their
//             candidates and set hit bits in a per-particle 128-bit mask
//             (no pair arithmetic yet);
//   flush  -- each particle's lanes evaluate the pair terms of its hits.
// The test is cheap and runs for every candidate of a passing combination;
// the expensive pair terms run only for hits, with the lanes compacted (a
// wave-wide branch on "any lane hit" would otherwise execute them for almost
// every candidate).  Each output is accumulated by its own lanes in a fixed
// order, so results are deterministic and need no atomics.
//
// This header holds the kernels, templated on the smoothing kernel; it is
// compiled by pairs_m4.hip and pairs_quintic.hip only.
#pragma once

#include "pairs_args.hpp"

#include <algorithm>
#include <type_traits>

namespace sph {
namespace {

// Views of pointers the pair kernels only read.  Through the constant address
// space a load with a wave-uniform address becomes a scalar load into SGPRs
// (the argument blocks, the home leaf's node); through the global address
// space a per-lane load is a plain vector load instead of a flat access, whose
// completion LDS waits would otherwise also have to cover.
template <class T>
__device__ inline const __attribute__((address_space(4))) T *as_const(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}
template <class T>
__device__ inline const __attribute__((address_space(1))) T *as_global(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}
// A whole read-only record, word by word through one of those views.
template <class T>
__device__ inline T load_const(const T *p)
{
    static_assert(sizeof(T) % 4 == 0 && alignof(T) >= 4, "word-sized record");
    T v;
    const auto *src = as_const((const uint32_t *)p);
    uint32_t *dst = (uint32_t *)&v;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); k++) dst[k] = src[k];
    return v;
}
template <class T>
__device__ inline T load_global(const T *p)
{
    static_assert(sizeof(T) % 4 == 0 && alignof(T) >= 4, "word-sized record");
    T v;
    const auto *src = as_global((const uint32_t *)p);
    uint32_t *dst = (uint32_t *)&v;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); k++) dst[k] = src[k];
    return v;
}

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane moves inside a 16-lane DPP row, for butterfly reductions: the
// value of lane l ^ O for O = 1, 2 (quad permutes); for O = 4 and 8 the value
// of the mirrored lane of l's 8- or 16-lane group, which is lane l ^ O's value
// wherever the value is already uniform over groups of O lanes -- as it is at
// that step of a butterfly.  No LDS and no lane-address registers.
template <int O>
__device__ inline int xlane(int v)
{
    static_assert(O == 1 || O == 2 || O == 4 || O == 8, "within one DPP row");
    constexpr int ctrl = O == 1 ? 0xB1 : O == 2 ? 0x4E : O == 4 ? 0x141 : 0x140;
    return __builtin_amdgcn_update_dpp(v, v, ctrl, 0xF, 0xF, false);
}
template <int O>
__device__ inline double xlane(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)xlane<O>((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)xlane<O>((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over each group of K consecutive lanes (K = 1, 2, 4, 8, 16), the same
// bits on every lane of the group (IEEE addition is commutative).
template <int K, class T>
__device__ inline T group_sum(T v)
{
    if constexpr (K >= 2) v += xlane<1>(v);
    if constexpr (K >= 4) v += xlane<2>(v);
    if constexpr (K >= 8) v += xlane<4>(v);
    if constexpr (K >= 16) v += xlane<8>(v);
    return v;
}
template <int K>
__device__ inline double group_max(double v)
{
    if constexpr (K >= 2) v = fmax(v, xlane<1>(v));
    if constexpr (K >= 4) v = fmax(v, xlane<2>(v));
    if constexpr (K >= 8) v = fmax(v, xlane<4>(v));
    if constexpr (K >= 16) v = fmax(v, xlane<8>(v));
    return v;
}

// Wave-wide maxima: each 16-lane row by DPP, then the four rows' values read
// into scalar registers (wave-uniform result).
__device__ inline double wave_max(double v)
{
    v = group_max<16>(v);
    auto row = [&](int l) {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
        const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
        return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    };
    return fmax(fmax(row(0), row(16)), fmax(row(32), row(48)));
}

template <int K>
__device__ inline int group_max_int(int v)
{
    if constexpr (K >= 2) { const int w = xlane<1>(v); v = w > v ? w : v; }
    if constexpr (K >= 4) { const int w = xlane<2>(v); v = w > v ? w : v; }
    if constexpr (K >= 8) { const int w = xlane<4>(v); v = w > v ? w : v; }
    if constexpr (K >= 16) { const int w = xlane<8>(v); v = w > v ? w : v; }
    return v;
}

// Wave-wide sum of small non-negative per-lane counts, wave-uniform.
__device__ inline int64_t wave_sum_int(int v)
{
    v = group_sum<16>(v);
    return (int64_t)__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           (int64_t)__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

__device__ inline int wave_max_int(int v)
{
    int w = xlane<1>(v);
    v = w > v ? w : v;
    w = xlane<2>(v);
    v = w > v ? w : v;
    w = xlane<4>(v);
    v = w > v ? w : v;
    w = xlane<8>(v);
    v = w > v ? w : v;
    const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    const int ab = a > b ? a : b, cd = c > d ? c : d;
    return ab > cd ? ab : cd;
}

// Persistent work loop over the leaves.  Blocks are dispatched round-robin
// over the 8 XCDs, so block b runs on XCD b % 8; each XCD first claims leaves
// from its own contiguous eighth of the leaf range (neighbouring leaves then
// share that XCD's L2), then helps the others.  Claims go through one atomic
// counter per eighth, `claim` consecutive leaves at a time; every leaf is
// processed by exactly one wave, so results do not depend on which wave took
// it.  Atomics on one address serialise (~0.1 us each), so claims are kept
// few: a block's first claim in its own eighth is static (its rank among the
// eighth's blocks; the counter hands out the claims after those), and after
// draining its own eighth a block helps the following eighths in turn and
// stops at the first one it finds exhausted.  Every eighth is still drained
// by its own blocks; a block makes no atomic at start and one failing claim
// on another counter at the end, instead of one on each of them (for a small
// set that finishes early, those tail claims were a large part of the
// launch).
template <class Fn>
__device__ inline void for_each_home_leaf(int64_t L, uint32_t *__restrict__ work, int claim,
                                          Fn fn)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t per = (L + kXcds - 1) / kXcds;
    const int x0 = (int)(blockIdx.x % kXcds);
    const uint32_t rank = blockIdx.x / kXcds;          // among the blocks of eighth x0
    const uint32_t nstatic = gridDim.x / kXcds;        // static first claims per eighth
    for (int r = 0; r < kXcds; r++) {
        const int x = (x0 + r) % kXcds;
        const int64_t beg = x * per;
        const int64_t end = beg + per < L ? beg + per : L;
        if (beg >= end) continue;
        bool got = false;
        for (int k = 0;; k++) {
            uint32_t c = rank;
            if (r > 0 || k > 0 || rank >= nstatic) {   // (a grid not a multiple of 8)
                if (lane == 0) c = nstatic + atomicAdd(&work[x], 1u);
                // wave-uniform from here on (scalar registers): the leaf's
                // argument block, node and particle range are then loaded once
                // per wave
                c = (uint32_t)__builtin_amdgcn_readlane((int)c, 0);
            }
            const int64_t leaf0 = beg + (int64_t)c * claim;
            if (leaf0 >= end) break;
            got = true;
            const int64_t leaf1 = leaf0 + claim < end ? leaf0 + claim : end;
            for (int64_t leaf = leaf0; leaf < leaf1; leaf++) fn(leaf);
        }
        if (r > 0 && !got) break;   // a helped eighth was already exhausted
    }
}

// Status of a wave's particles: when any lane raises `cond`, set `flag` in
// status[0] and add the number of such lanes to status[word], one atomic
// each per wave (a set whose particles all fail then costs one atomic per
// leaf, not one per particle).  Called by every lane of the wave.
__device__ inline void report(int32_t *status, bool cond, int32_t flag, int word)
{
    const int cnt = (int)__popcll(__ballot(cond));
    if (cnt && (threadIdx.x & (kWave - 1)) == 0) {
        atomicOr(&status[0], flag);
        atomicAdd(&status[word], cnt);
    }
}

// Copy the device tree description into LDS once per block.
__device__ inline void load_tree(const TreeInfo *__restrict__ src, TreeInfo &dst)
{
    const auto *s = as_global((const int64_t *)src);
    int64_t *d = (int64_t *)&dst;
    for (int k = threadIdx.x; k < kTreeWords; k += blockDim.x) d[k] = s[k];
    __syncthreads();
}

// Squared gap between box [lo, hi] and node box (0 if they overlap), with the
// periodic images of the node when the box is periodic.
__device__ inline double box_gap2(const double lo[3], const double hi[3], const Node &nd,
                                  const Box &bx)
{
    double s = 0.0;
    for (int a = 0; a < 3; a++) {
        double g = fmax(fmax(nd.lo[a] - hi[a], lo[a] - nd.hi[a]), 0.0);
        if (bx.periodic) {
            double L = bx.len[a];
            double g1 = fmax(fmax(nd.lo[a] + L - hi[a], lo[a] - (nd.hi[a] + L)), 0.0);
            double g2 = fmax(fmax(nd.lo[a] - L - hi[a], lo[a] - (nd.hi[a] - L)), 0.0);
            g = fmin(g, fmin(g1, g2));
        }
        s += g * g;
    }
    return s;
}

// r_ij^2 exactly as (dx*dx + dy*dy) + dz*dz, each operation rounded on its
// own, so neighbour predicates agree bit for bit with any other evaluation
// written the same way.
__device__ inline double exact_r2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    return (a + b) + c;
}

// a*b + c*d with both products rounded before the sum and no fused
// multiply-add, so swapping (a, b) with (c, d) gives the same bits: keeps the
// pair force of (i, j) the exact negative of that of (j, i).
template <class T>
__device__ inline T sym_dot2(T a, T b, T c, T d)
{
#pragma clang fp contract(off)
    T p = a * b;
    T q = c * d;
    return p + q;
}

// Kernel gradients of a pair and their sum, each product rounded before the
// sum: keeps 0.5 (G_i + G_j) identical for (i, j) and (j, i).
template <class T>
__device__ inline void sym_grads(T gfi, T dfi, T gfj, T dfj, T &gi, T &gj, T &gsum)
{
#pragma clang fp contract(off)
    gi = gfi * dfi;
    gj = gfj * dfj;
    gsum = gi + gj;
}

__device__ inline double min_image(double d, double L, double half)
{
    if (d > half) d -= L;
    else if (d < -half) d += L;
    return d;
}

__device__ inline float min_image_f(float d, float L, float half)
{
    if (d > half) d -= L;
    else if (d < -half) d += L;
    return d;
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton-Raphson
// steps on 1/y^2 - x (each squares the relative error), to about 1 ulp in
// eight operations instead of a correctly rounded square root and division.
__device__ inline double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const double r = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, r, y);
    }
    return y;
}

// 1/sqrt(x) for x > 0 with one Newton-Raphson step on the hardware estimate:
// the estimate's relative error is squared once, to well below 1e-13 -- the
// density sums need q = r/h to far better than their 1e-10 parity bound, not
// to the last bit.
__device__ inline double rsqrt_nr1(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double r = fma(-x * y, y, 1.0);
    return fma(0.5 * y, r, y);
}

// 1/x for x > 0: the hardware estimate refined by two Newton-Raphson steps
// on 1/y - x, to about 1 ulp.
__device__ inline double rcp_nr(double x)
{
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const double e = fma(-x, y, 1.0);
        y = fma(y, e, y);
    }
    return y;
}

// Kernel shapes f(q) and f'(q), branch-free in B-spline form:
// M4: f = a^3/4 - b^3, f' = 3 b^2 - 3/4 a^2 with a = (2-q)_+, b = (1-q)_+;
// quintic: f = a^5 - 6 b^5 + 15 c^5, f' = -5 a^4 + 30 b^4 - 75 c^4 with
// a = (3-q)_+, b = (2-q)_+, c = (1-q)_+.
template <int K, class T>
__device__ inline void kern(T qq, T &f, T &df)
{
    if constexpr (K == SPH_KERNEL_QUINTIC) {
        const T a = fmax(T(3) - qq, T(0));
        const T b = fmax(T(2) - qq, T(0));
        const T c = fmax(T(1) - qq, T(0));
        const T a2 = a * a, b2 = b * b, c2 = c * c;
        const T a4 = a2 * a2, b4 = b2 * b2, c4 = c2 * c2;
        f = a4 * a - T(6) * (b4 * b) + T(15) * (c4 * c);
        df = T(30) * b4 - T(5) * a4 - T(75) * c4;
    } else {
        const T a = fmax(T(2) - qq, T(0));
        const T b = fmax(T(1) - qq, T(0));
        const T a2 = a * a, b2 = b * b;
        f = T(0.25) * a2 * a - b2 * b;
        df = T(3) * b2 - T(0.75) * a2;
    }
}

// ---------------------------------------------------------------------------
// Tree walk
// ---------------------------------------------------------------------------
// The walk's result stays in `list`; the second frontier buffer a walk needs
// is lent by the caller (the pair loops lend their staging slots, which hold
// nothing while a walk runs).
struct WalkBuf {
    uint32_t list[kFront];
    uint32_t tmp[kWave];
};

// Breadth-first walk of the 8-ary tree, 64 child tests per step.  Result: n
// nodes of level `lev` in `list` that pass the test.  Normally lev = 0 (the
// candidate leaves).  If expanding a level would overflow the LDS frontier,
// the walk stops there and returns that level's nodes; the caller then tests
// the leaves under each of them directly (bounded extra work instead of a
// scan of every leaf).
struct WalkResult {
    int n;
    int lev;
    const uint32_t *list;
};

// Leaves the walk's result in wb.list, copying it there from the spare
// buffer when the last expansion wrote it there.
__device__ inline WalkResult walk_result(WalkBuf &wb, const uint32_t *cur, int n, int lev)
{
    if (cur != wb.list) {
        const int lane = threadIdx.x & (kWave - 1);
        for (int t = lane; t < n; t += kWave) wb.list[t] = cur[t];
        wave_lds_sync();
    }
    return WalkResult{n, lev, wb.list};
}

// spare: kFront entries of LDS the walk may overwrite
template <class Test>
__device__ WalkResult walk(const TreeInfo &T, const Node *nodes, Test test, WalkBuf &wb,
                           uint32_t *spare)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t lt = __lanemask_lt();
    uint32_t *cur = wb.list, *nxt = spare;
    const int top = T.nlev - 1;
    if (lane == 0) cur[0] = 0;
    wave_lds_sync();
    if (top == 0) {
        bool pass = lane == 0 && test(nodes[0]);
        return WalkResult{__ballot(pass) ? 1 : 0, 0, cur};
    }
    int ncur = 1;
    for (int lev = top; lev > 0; lev--) {
        const Node *cl = nodes + T.off[lev - 1];
        const int64_t nchild = T.cnt[lev - 1];
        const int total = ncur * 8;
        int nout = 0;
        for (int b = 0; b < total; b += kWave) {
            int t = b + lane;
            bool valid = t < total;
            int64_t node = valid ? (int64_t)cur[t >> 3] * 8 + (t & 7) : 0;
            valid = valid && node < nchild;
            bool pass = valid && test(load_global(cl + node));
            uint64_t mask = __ballot(pass);
            int pos = nout + (int)__popcll(mask & lt);
            if (pass && pos < kFront) nxt[pos] = (uint32_t)node;
            nout += (int)__popcll(mask);
        }
        wave_lds_sync();
        if (nout > kFront) return walk_result(wb, cur, ncur, lev);
        uint32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
        ncur = nout;
        if (ncur == 0) break;
    }
    return walk_result(wb, cur, ncur, 0);
}

// Visit the candidate leaves in groups of at most `depth` (<= NL, the LDS
// tile): fn(leaves, count) with a wave-uniform count.  After a truncated walk
// the leaves under each returned node are tested 64 at a time and the
// passing ones grouped.
template <int NL, class Test, class Fn>
__device__ int64_t for_each_leaf_group(const TreeInfo &T, const Node *nodes, const WalkResult &wr,
                                       Test test, WalkBuf &wb, Fn fn, int depth = NL)
{
    const int D = depth >= 1 && depth <= NL ? depth : NL;
    if (wr.lev == 0) {
        for (int t0 = 0; t0 < wr.n; t0 += D) fn(wr.list + t0, wr.n - t0 < D ? wr.n - t0 : D);
        return wr.n;
    }
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t lt = __lanemask_lt();
    const int64_t L = T.cnt[0];
    int64_t span = 1;
    for (int l = 0; l < wr.lev; l++) span *= 8;
    int64_t tested = 0;
    for (int k = 0; k < wr.n; k++) {
        const int64_t b0 = (int64_t)wr.list[k] * span;
        const int64_t b1 = b0 + span < L ? b0 + span : L;
        for (int64_t b = b0; b < b1; b += kWave) {
            const int64_t c = b + lane;
            const bool pass = c < b1 && test(load_global(nodes + c));
            const uint64_t mask = __ballot(pass);
            if (pass) wb.tmp[__popcll(mask & lt)] = (uint32_t)c;
            wave_lds_sync();
            const int cnt = (int)__popcll(mask);
            for (int t0 = 0; t0 < cnt; t0 += D) fn(wb.tmp + t0, cnt - t0 < D ? cnt - t0 : D);
            wave_lds_sync();
            tested += b1 - b < kWave ? b1 - b : kWave;
        }
    }
    return tested;
}

// Per candidate leaf: the periodic shift that the minimum image gives every
// pair (i in home, j in the leaf) closer than `reach`, when that shift is
// unique (both boxes small against the period); otherwise the pair loop
// applies the minimum image pair by pair.
struct Shift {
    double s[3];
    bool per_pair;
};

__device__ inline Shift leaf_shift(const Node &home, const Node &cand, const Box &bx, double reach)
{
    Shift sh{{0.0, 0.0, 0.0}, false};
    if (!bx.periodic) return sh;
    for (int a = 0; a < 3; a++) {
        double dc = 0.5 * (home.lo[a] + home.hi[a]) - 0.5 * (cand.lo[a] + cand.hi[a]);
        sh.s[a] = dc > bx.half[a] ? -bx.len[a] : (dc < -bx.half[a] ? bx.len[a] : 0.0);
        double span = reach + 0.5 * ((home.hi[a] - home.lo[a]) + (cand.hi[a] - cand.lo[a]));
        if (!(span < 0.49 * bx.len[a])) sh.per_pair = true;
    }
    return sh;
}

// ---------------------------------------------------------------------------
// Staging and the compacted candidate tests shared by the pair loops
// ---------------------------------------------------------------------------
// A wave holds the G home particles of one leaf, LPP = 64 / G lanes each.
// Candidate leaves are staged NL = 128 / G at a time (128 candidate slots).
// For every (home particle, staged leaf) combination the wave first measures
// the distance from the particle to the leaf's box; only combinations that can
// hold a pair are expanded, four candidate tests per lane, dealt out densely
// over the 64 lanes.  Hits are bits of a per-particle mask over the 128 slots
// (set with an LDS atomic OR, so the result does not depend on lane timing);
// the flush walks each particle's mask in ascending slot order, its set bits
// shared round-robin by the particle's own lanes.

constexpr int kSlots = 2 * kWave;   // candidate slots per staged group
constexpr int kTestsPerLane = 4;    // candidate tests per lane per combination

// Per-slot candidate data: FP64 positions, or in FP32-pair mode the
// single-precision offsets from the leaf centres; w is the mass (density; not
// staged when all masses are equal) or the squared gather reach (R h)^2
// (forces).
struct SlotsFP64 {
    double x[kSlots], y[kSlots], z[kSlots], w[kSlots];
};
struct SlotsFP32 {
    double w[kSlots];
    float fx[kSlots], fy[kSlots], fz[kSlots];
};
static_assert(sizeof(SlotsFP32) >= kFront * sizeof(uint32_t) &&
                  sizeof(SlotsFP64) >= kFront * sizeof(uint32_t),
              "the staging slots double as the walk's spare frontier buffer");

template <int G, int PREC>
struct Stage {
    static constexpr int NL = kSlots / G;
    union {
        std::conditional_t<PREC == SPH_FP64, SlotsFP64, SlotsFP32> c;
        uint32_t walk_spare[kFront];   // lent to walks, which run between groups
    };
    uint32_t j[kSlots];
    // per staged leaf
    double lo[NL][3], hi[NL][3];
    double sx[NL], sy[NL], sz[NL];   // shift added to x_i - x_j (per-leaf periodic image)
    double hmax[NL];
    float ox[NL], oy[NL], oz[NL];    // FP32-pair: leaf-centre offset (with the shift)
    int32_t jn[NL];
    int32_t per_pair[NL];            // minimum image pair by pair instead of a shift
    // per home particle
    double hx[G], hy[G], hz[G];
    float hfx[G], hfy[G], hfz[G];
    double thr[G];                   // record threshold on r^2 (< 0: particle takes no part)
    uint64_t mask[G][2];             // hits over the 128 slots
    uint8_t combo[kSlots];           // compacted (particle, leaf) combinations
};

// Stage `count` (<= NL) candidate leaves; lane l fills slots l and l + 64,
// slot s holding particle s % G of staged leaf s / G.  REACH2: w holds h and
// the slot keeps the squared gather reach (R h)^2 of kernel K instead.
template <int G, int PREC, int K, bool REACH2 = false, bool MAYBE_NO_W = false>
__device__ inline void stage_group(Stage<G, PREC> &S, const uint32_t *leaves, int count,
                                   const uint32_t *__restrict__ lstart, const Node *__restrict__ nodes,
                                   const Node &home, const Box &bx, double hcov,
                                   const double *__restrict__ x, const double *__restrict__ y,
                                   const double *__restrict__ z, const double *__restrict__ w,
                                   const float *__restrict__ fx, const float *__restrict__ fy,
                                   const float *__restrict__ fz)
{
    constexpr int NL = Stage<G, PREC>::NL;
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int half = 0; half < 2; half++) {
        const int s = lane + half * kWave;
        const int k = s / G, slot = s % G;
        if (k < count) {
            const uint32_t c = leaves[k];
            const int64_t j0 = as_global(lstart)[c];
            const int jn = (int)(as_global(lstart)[c + 1] - j0);
            if (slot < jn) {
                const int64_t j = j0 + slot;
                if (!MAYBE_NO_W || w) {   // MAYBE_NO_W: w == nullptr, the caller reads no w
                    const double wv = as_global(w)[j];
                    S.c.w[s] = REACH2 ? (Kern<K>::R * wv) * (Kern<K>::R * wv) : wv;
                }
                if constexpr (PREC == SPH_FP64) {
                    S.c.x[s] = as_global(x)[j];
                    S.c.y[s] = as_global(y)[j];
                    S.c.z[s] = as_global(z)[j];
                } else {
                    S.c.fx[s] = as_global(fx)[j];
                    S.c.fy[s] = as_global(fy)[j];
                    S.c.fz[s] = as_global(fz)[j];
                }
                S.j[s] = (uint32_t)j;
            }
            if (slot == 0) {
                const Node cand = load_global(nodes + c);
                // hcov < 0: symmetric force criterion, reach R max(h over both leaves)
                const Shift sh = leaf_shift(
                    home, cand, bx, Kern<K>::R * (hcov < 0.0 ? fmax(home.hmax, cand.hmax) : hcov));
                for (int a = 0; a < 3; a++) {
                    S.lo[k][a] = cand.lo[a];
                    S.hi[k][a] = cand.hi[a];
                }
                S.hmax[k] = cand.hmax;
                S.sx[k] = sh.s[0];
                S.sy[k] = sh.s[1];
                S.sz[k] = sh.s[2];
                S.per_pair[k] = sh.per_pair ? 1 : 0;
                S.jn[k] = jn;
                if (PREC == SPH_FP32_PAIR) {
                    S.ox[k] = (float)((0.5 * (home.lo[0] + home.hi[0]) - 0.5 * (cand.lo[0] + cand.hi[0])) +
                                      (sh.per_pair ? 0.0 : sh.s[0]));
                    S.oy[k] = (float)((0.5 * (home.lo[1] + home.hi[1]) - 0.5 * (cand.lo[1] + cand.hi[1])) +
                                      (sh.per_pair ? 0.0 : sh.s[1]));
                    S.oz[k] = (float)((0.5 * (home.lo[2] + home.hi[2]) - 0.5 * (cand.lo[2] + cand.hi[2])) +
                                      (sh.per_pair ? 0.0 : sh.s[2]));
                }
            }
        } else if (slot == 0 && k < NL) {
            S.jn[k] = 0;
        }
    }
    wave_lds_sync();
}

// Separation x_i - x_j of a home particle (given by value) and staged slot s;
// the same expression serves every test and flush, so they see identical bits.
// PP = false: no staged leaf needs the pair-by-pair minimum image (the
// caller has checked), which drops that branch.
template <int G, int PREC, bool PP = true>
__device__ inline void separation(const Stage<G, PREC> &S, const Box &bx, double hx, double hy,
                                  double hz, float hfx, float hfy, float hfz, int s, double &dx,
                                  double &dy, double &dz, double &r2)
{
    const int k = s / G;
    if constexpr (PREC == SPH_FP64) {
        dx = hx - S.c.x[s];
        dy = hy - S.c.y[s];
        dz = hz - S.c.z[s];
        if (PP && S.per_pair[k]) {
            dx = min_image(dx, bx.len[0], bx.half[0]);
            dy = min_image(dy, bx.len[1], bx.half[1]);
            dz = min_image(dz, bx.len[2], bx.half[2]);
        } else {
            dx += S.sx[k];
            dy += S.sy[k];
            dz += S.sz[k];
        }
        r2 = exact_r2(dx, dy, dz);
    } else {
        float fdx = (hfx - S.c.fx[s]) + S.ox[k];
        float fdy = (hfy - S.c.fy[s]) + S.oy[k];
        float fdz = (hfz - S.c.fz[s]) + S.oz[k];
        if (PP && S.per_pair[k]) {
            fdx = min_image_f(fdx, (float)bx.len[0], (float)bx.half[0]);
            fdy = min_image_f(fdy, (float)bx.len[1], (float)bx.half[1]);
            fdz = min_image_f(fdz, (float)bx.len[2], (float)bx.half[2]);
        }
        dx = fdx;
        dy = fdy;
        dz = fdz;
        r2 = (double)(fdx * fdx + fdy * fdy + fdz * fdz);
    }
}

// r_ij^2 for a superset filter (the caller's threshold carries a relative
// slack far above rounding): in FP64 without pair-by-pair images the leaf's
// shift joins the home position first, which the compiler shares between the
// tests of one (particle, leaf) combination; otherwise the exact separation.
template <int G, int PREC, bool PP>
__device__ inline double filter_r2(const Stage<G, PREC> &S, const Box &bx, int p, int s)
{
    if constexpr (PREC == SPH_FP64 && !PP) {
        const int k = s / G;
        const double dx = (S.hx[p] + S.sx[k]) - S.c.x[s];
        const double dy = (S.hy[p] + S.sy[k]) - S.c.y[s];
        const double dz = (S.hz[p] + S.sz[k]) - S.c.z[s];
        return dx * dx + dy * dy + dz * dz;
    } else {
        double dx, dy, dz, r2;
        separation<G, PREC, PP>(S, bx, S.hx[p], S.hy[p], S.hz[p], S.hfx[p], S.hfy[p], S.hfz[p], s,
                                dx, dy, dz, r2);
        return r2;
    }
}

// Squared distance from home particle p to staged leaf k's box in the frame of
// the separation; 0 for a per-pair leaf (every candidate is then tested).
template <int G, int PREC>
__device__ inline double box_dist2(const Stage<G, PREC> &S, int p, int k)
{
    const double c[3] = {S.hx[p] + S.sx[k], S.hy[p] + S.sy[k], S.hz[p] + S.sz[k]};
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        // the gap below lo or above hi, 0 inside (at most one is positive)
        const double d = fmax(fmax(S.lo[k][a] - c[a], c[a] - S.hi[k][a]), 0.0);
        d2 += d * d;
    }
    return S.per_pair[k] ? 0.0 : d2;
}

// The relative slack of the box test: it must accept every combination whose
// candidates the record test can accept (rounding of the two differently
// formed distances; FP32-pair separations carry single-precision error).
template <int PREC>
__device__ constexpr double box_slack() { return PREC == SPH_FP64 ? 1.0 + 1e-6 : 1.0 + 1e-4; }

// Hit masks of one staged group: bit s of S.mask[p] set iff rec(p, s, pp), with
// rec evaluated only where relevant(p, k) holds for the slot's leaf k; pp is
// std::true_type when some staged leaf needs the pair-by-pair minimum image,
// std::false_type otherwise (for separation's PP parameter).
template <int G, int PREC, class Relevant, class Record>
__device__ inline bool group_tests(Stage<G, PREC> &S, int count, Relevant relevant, Record rec,
                                   bool diag, int64_t &boxes, int64_t &tests)
{
    constexpr int NL = Stage<G, PREC>::NL;
    constexpr int LPC = G / kTestsPerLane;   // lanes per combination
    constexpr int CPR = kWave / LPC;         // combinations per round
    static_assert(G * NL == kSlots && LPC * kTestsPerLane == G, "combination layout");
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t lt = __lanemask_lt();
    // combination c = p * NL + k; this lane judges c = lane and c = lane + 64
    bool r0, r1;
    {
        const int p = lane / NL, k = lane % NL;
        r0 = k < count && relevant(p, k);
    }
    {
        const int c = lane + kWave;
        const int p = c / NL, k = c % NL;
        r1 = k < count && relevant(p, k);
    }
    const uint64_t m0 = __ballot(r0), m1 = __ballot(r1);
    const int n0 = (int)__popcll(m0);
    if (r0) S.combo[__popcll(m0 & lt)] = (uint8_t)lane;
    if (r1) S.combo[n0 + (int)__popcll(m1 & lt)] = (uint8_t)(lane + kWave);
    const int C = n0 + (int)__popcll(m1);
    // diagnostics (when asked for), wave-uniform: every judged combination is
    // a box test, and a passing one tests each particle of its leaf (7-bit
    // count per lane)
    if (diag) {
        boxes += (int64_t)count * G;
        const int mine = (r0 ? S.jn[lane % NL] : 0) + (r1 ? S.jn[(lane + kWave) % NL] : 0);
        for (int b = 0; b < 7; b++) tests += (int64_t)__popcll(__ballot((mine >> b) & 1)) << b;
    }
    wave_lds_sync();
    const int u = lane % LPC;
    // combinations of one round start their tests at different slots, which
    // spreads their LDS reads over the banks
    const int rot = lane / LPC;
    // every test runs (slots past the leaf's end read stale but in-bounds
    // LDS) and its slot predicate masks the result: no branch per test
    auto rounds = [&](auto pp_possible) {
        for (int b = 0; b < C; b += CPR) {
            const int idx = b + lane / LPC;
            if (idx < C) {
                const int c = S.combo[idx];
                const int p = c / NL, k = c % NL;
                const int jn = S.jn[k];
                uint64_t bits = 0;
#pragma unroll
                for (int t = 0; t < kTestsPerLane; t++) {
                    const int slot = u + LPC * ((t + rot) % kTestsPerLane);
                    const int s = k * G + slot;
                    const bool hit = (slot < jn) & rec(p, s, pp_possible);
                    bits |= (uint64_t)hit << (s & 63);
                }
                if (bits)
                    atomicOr((unsigned long long *)&S.mask[p][(k * G) >> 6], (unsigned long long)bits);
            }
        }
    };
    const bool any_pp = __ballot(lane < count && S.per_pair[lane < NL ? lane : 0]) != 0ull;
    if (any_pp)
        rounds(std::true_type{});
    else
        rounds(std::false_type{});
    wave_lds_sync();
    return any_pp;
}

// As for_my_bits, but this lane's bits two at a time: fn(sa, sb) with sb < 0
// when sa is its last, so the caller can issue both pairs' loads before
// using either.
// Clear the lowest set bit of the 128-bit mask (w0, w1), without a branch.
__device__ inline void pop_low(uint64_t &w0, uint64_t &w1)
{
    const bool lo = w0 != 0;
    const uint64_t a = w0 & (w0 - 1), b = w1 & (w1 - 1);
    w0 = lo ? a : w0;
    w1 = lo ? w1 : b;
}

template <int LPP, class Fn>
__device__ inline int for_my_bit_pairs(uint64_t w0, uint64_t w1, int e0, Fn fn)
{
    const int n = (int)__popcll(w0) + (int)__popcll(w1);
    auto pop = [&]() { pop_low(w0, w1); };
    auto low = [&]() { return w0 ? (int)__builtin_ctzll(w0) : 64 + (int)__builtin_ctzll(w1); };
    for (int t = 0; t < e0; t++) pop();
    for (int e = e0; e < n; e += 2 * LPP) {
        const int sa = low();
        for (int t = 0; t < LPP; t++) pop();
        int sb = -1;
        if (e + LPP < n) {
            sb = low();
            for (int t = 0; t < LPP; t++) pop();
        }
        fn(sa, sb);
    }
    return n;
}

// The set bits of a 128-bit mask in ascending order, shared round-robin by
// the LPP lanes of a particle: this lane takes the bits of rank e = e0,
// e0 + LPP, ... (0 <= e0 < LPP) and calls fn(slot, e).  Returns the number of
// set bits.
template <int LPP, class Fn>
__device__ inline int for_my_bits(uint64_t w0, uint64_t w1, int e0, Fn fn)
{
    const int n = (int)__popcll(w0) + (int)__popcll(w1);
    for (int t = 0; t < e0; t++) pop_low(w0, w1);
    for (int e = e0; e < n; e += LPP) {
        const int s = w0 ? (int)__builtin_ctzll(w0) : 64 + (int)__builtin_ctzll(w1);
        fn(s, e);
#pragma unroll
        for (int t = 0; t < LPP; t++) pop_low(w0, w1);
    }
    return n;
}

// ---------------------------------------------------------------------------
// Batches: one launch evaluates many independent particle sets.  Every
// request has its own argument block in device memory; a wave claims a
// global leaf index over the concatenation of the requests' leaves and maps
// it back to (request, leaf) through an LDS prefix of the leaf counts.  The
// work done for a leaf depends on its own request only, so a set gives the
// same bits alone and inside any mix.
// ---------------------------------------------------------------------------
// Waves per SIMD the pair kernels are built for (<= 128 VGPRs, <= 10 KB of
// LDS per wave).  Measured on MI355X: occupancy decides these latency-bound
// loops; each step from 2 to 4 waves per SIMD pays for the register spills it
// costs.
template <int PREC>
constexpr int pair_waves_per_simd() { return 4; }


template <class Args>
__device__ inline void batch_prefix(const Batch<Args> &B, uint32_t *pre)
{
    // the host keeps the total leaf count (<= total particles) below 2^32
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        pre[0] = 0;
        for (int r = 0; r < B.nreq; r++) {
            const uint32_t *lc = B.req[r]->leaf_count;
            acc += lc ? *lc : (uint32_t)B.req[r]->tree->cnt[0];
            pre[r + 1] = acc;
        }
    }
    __syncthreads();
}

// request holding global leaf g: largest r with pre[r] <= g
__device__ inline int find_req(const uint32_t *pre, int nreq, int64_t g)
{
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)pre[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Density loop + h solve
// ---------------------------------------------------------------------------

template <int G, int PREC, int K>
__global__ __launch_bounds__(kWave, pair_waves_per_simd<PREC>()) void k_density(Batch<DensArgs> B)
{
    constexpr int LPP = kWave / G;   // lanes per home particle
    constexpr int NL = kSlots / G;   // candidate leaves staged per group
    constexpr int KP = Kern<K>::list;
    constexpr double RK = Kern<K>::R, SIG = Kern<K>::sigma;
    constexpr int ROWS = KP / LPP;   // cache rows of 64 entries
    __shared__ WalkBuf wb;
    __shared__ TreeInfo T;
    __shared__ Stage<G, PREC> S;
    __shared__ uint32_t pre[kMaxBatch + 1];
    // Per home particle, the Newton iteration's bracket and the results of its
    // latest evaluation.  Every lane of a particle computes the same values;
    // kept in registers they were spilled to scratch and reloaded at every
    // step (the loop is register-bound at 4 waves per SIMD), so they live in
    // LDS where the per-wave budget (10 KB at 16 waves per CU) has room: FP64
    // up to G = 16 and FP32-pair.  Each lane of the particle writes the same
    // value and reads its own wave's writes (LDS operations of a wave are
    // performed in order).
    constexpr bool NR_LDS = PREC == SPH_FP32_PAIR || G <= 16;
    __shared__ double nr_mem[NR_LDS ? 5 * G : 1];
    batch_prefix(B, pre);
    const int lane = threadIdx.x;
    const int p = lane / LPP, q = lane % LPP;
    double *const nr_lo = nr_mem + (NR_LDS ? 0 * G + p : 0);
    double *const nr_hi = nr_mem + (NR_LDS ? 1 * G + p : 0);
    double *const nr_h = nr_mem + (NR_LDS ? 2 * G + p : 0);
    double *const nr_rho = nr_mem + (NR_LDS ? 3 * G + p : 0);
    double *const nr_om = nr_mem + (NR_LDS ? 4 * G + p : 0);
    // Candidate lists of this block: for every home particle up to KP entries
    // (r^2, and m unless all masses are equal) of the candidates within R Rc
    // of it, in the order a sweep meets them.  Entry e of particle p sits in
    // row e / LPP, column p LPP + e % LPP, and lane (p, q) owns the entries
    // e = q (mod LPP) both when a sweep writes them and when later Newton
    // steps read them back, summing them in the same order: a step from the
    // list gives the bits of a sweep.  The particle itself is marked (mass or,
    // with equal masses, r^2 = 0 stored negated) to keep it out of the count.
    // FP32-pair forms every r^2 in single precision, so its list holds them
    // as floats (half the bytes, the same values); FP64 lists hold doubles.
    using ListR2 = std::conditional_t<PREC == SPH_FP64, double, float>;
    double *const cslice = B.cache + (size_t)blockIdx.x * (2 * ROWS * kWave);
    ListR2 *const cr2 = reinterpret_cast<ListR2 *>(cslice);
    double *const cm = cslice + ROWS * kWave;
    int64_t evals = 0, walks = 0, visits = 0, overflows = 0, nr_total = 0, tests = 0, boxes = 0;
    int64_t list_over = 0;
    int iter_max = 0;
    int cur = -1;
    const __attribute__((address_space(4))) DensArgs *Ap = nullptr;
    // per-request diagnostics, flushed when the wave moves to another request
    auto flush_counts = [&]() {
        if (lane == 0 && cur >= 0) {
            auto add = [&](int k, int64_t v) {
                if (v) atomicAdd((unsigned long long *)&Ap->counts[k], (unsigned long long)v);
            };
            add(kCntDensEvals, evals);
            atomicMax((unsigned long long *)&Ap->counts[kCntNrMax], (unsigned long long)iter_max);
            add(kCntDensOverflows, overflows);
            add(kCntDensVisits, visits);
            add(kCntDensWalks, walks);
            add(kCntNrTotal, nr_total);
            add(kCntDensTests, tests);
            add(kCntDensBoxes, boxes);
            add(kCntDensListOverflows, list_over);
        }
        evals = walks = visits = overflows = nr_total = tests = boxes = list_over = 0;
        iter_max = 0;
    };
    for_each_home_leaf(pre[B.nreq], B.work, B.claim, [&](int64_t gleaf) {
        // the request and its argument block are wave-uniform (scalar registers)
        const int r = __builtin_amdgcn_readfirstlane(find_req(pre, B.nreq, gleaf));
        if (r != cur) {
            flush_counts();
            cur = r;
            Ap = as_const(B.req[r]);
            load_tree(Ap->tree, T);
        }
        const auto &A = *Ap;
        const int64_t li = gleaf - (int64_t)__builtin_amdgcn_readfirstlane(pre[r]);
        const int64_t leaf = A.leaf_list ? (int64_t)as_const(A.leaf_list)[li] : li;
        if (A.leaf_act && as_const(A.leaf_act)[leaf] == 0) return;   // no active particle
        const Box bx = load_const(&B.req[r]->box);
        const int64_t first = as_const(A.lstart)[leaf];
        const int nhome = (int)(as_const(A.lstart)[leaf + 1] - first);
        const int64_t i = first + p;
        const bool active = p < nhome && (!A.active || as_global(A.active)[i] != 0);
        const int64_t ii = active ? i : first;
        const double hx = as_global(A.x)[ii], hy = as_global(A.y)[ii], hz = as_global(A.z)[ii];
        float hfx = 0.f, hfy = 0.f, hfz = 0.f;
        if (PREC == SPH_FP32_PAIR) {
            hfx = as_global(A.fx)[ii];
            hfy = as_global(A.fy)[ii];
            hfz = as_global(A.fz)[ii];
        }
        const double mi = as_global(A.m)[ii];
        const double mu = as_const(A.mrange)[0];
        const bool equal_m = mu == as_const(A.mrange)[1];
        const Node home = load_const(A.nodes + leaf);
        double h = as_global((const double *)A.h)[ii];
        double lo_b = 0.0, hi_b = INFINITY;          // registers unless NR_LDS
        bool conv = !active;
        double h_out = h, rho_out = 0.0, om_out = 1.0;
        if constexpr (NR_LDS) {
            *nr_lo = 0.0;
            *nr_hi = INFINITY;
            *nr_h = h;
            *nr_rho = 0.0;
            *nr_om = 1.0;
        }
        int n_out = 0;
        if (q == 0) {
            S.hx[p] = hx;
            S.hy[p] = hy;
            S.hz[p] = hz;
            S.hfx[p] = hfx;
            S.hfy[p] = hfy;
            S.hfz[p] = hfz;
            S.mask[p][0] = 0;
            S.mask[p][1] = 0;
        }

        double hcov = A.walk_margin * wave_max(active ? h : 0.0);
        auto make_test = [&](double hc) {
            const double R = RK * hc * (1.0 + 1e-10);
            const double R2 = R * R;
            return [&bx, &home, R2](const Node &nd) { return box_gap2(home.lo, home.hi, nd, bx) < R2; };
        };
        // the walk and the staging are chains of dependent loads: the wave
        // issues them at raised priority, ahead of waves in their arithmetic
        // (measured: the force loop 1 % faster, the density loop unchanged)
        __builtin_amdgcn_s_setprio(2);
        WalkResult wr = walk(T, A.nodes, make_test(hcov), wb, S.walk_spare);
        __builtin_amdgcn_s_setprio(0);
        walks++;
        if (wr.lev) overflows++;
        int iter = 0;
        int evals_leaf = 0;   // this lane's density pairs evaluated for this leaf
        // list state of this particle: `cached` = the list holds every
        // candidate within R Rc (count <= KP); valid while h <= Rc
        bool cached = false;
        double Rc = 0.0;
        int count = 0;
        for (;;) {
            double s0 = 0.0, s2 = 0.0;
            int cnt = 0;
            const double hinv = 1.0 / h;
            const double h2x4 = (RK * h) * (RK * h);
            const float h2x4f = (float)h2x4;
            // pair terms of one list entry (r^2, and the mass when masses differ).
            // Branch-free: an entry outside R h adds 0 * f (+0 or -0, which leave
            // the sums' bits unchanged) and no count; the lanes of a wave almost
            // never agree on skipping, so a branch would save no work.  The
            // particle itself is an entry (r^2 = 0) and is counted here; the
            // count drops it after the reduction.
            auto accumulate = [&](double r2, double mw) {
                const bool in = PREC == SPH_FP64 ? r2 < h2x4 : (float)r2 < h2x4f;
                const double mj = in ? (equal_m ? mu : mw) : 0.0;
                if (PREC == SPH_FP64) {
                    double f, df;
                    // r = r^2 / sqrt(r^2) without a branch (r^2 = 0 gives
                    // 0 * finite = 0; the 1e-300 leaves any r^2 above 1e-284
                    // unchanged); one refinement of the hardware estimate
                    const double qq = (r2 * rsqrt_nr1(r2 + 1e-300)) * hinv;
                    kern<K>(qq, f, df);
                    s0 += mj * f;
                    s2 += mj * (qq * df);
                } else {
                    float f, df;
                    const float qq = sqrtf((float)r2) * (float)hinv;
                    kern<K>(qq, f, df);
                    s0 += mj * (double)f;
                    s2 += mj * (double)(qq * df);
                }
                cnt += in ? 1 : 0;
            };
            if (__ballot(!conv && !cached) != 0ull) {
                // sweep: every particle still iterating takes its pair terms from
                // the candidates directly and rebuilds its list around its
                // current h (the first KP entries; a longer list is not kept)
                double rc2 = -1.0;
                if (!conv) {
                    Rc = fmin(kCacheGrow * h, hcov);
                    rc2 = (RK * Rc) * (RK * Rc) * (1.0 + 1e-6);
                }
                if (q == 0) S.thr[p] = rc2;
                wave_lds_sync();
                int base = 0;
                auto group = [&](const uint32_t *leaves, int ng) {
                    // FP32-pair stages no mass when all masses are equal (measured
                    // faster; the FP64 loop is faster staging it anyway)
                    constexpr bool skip_m = PREC == SPH_FP32_PAIR;
                    __builtin_amdgcn_s_setprio(2);
                    stage_group<G, PREC, K, false, skip_m>(S, leaves, ng, A.lstart, A.nodes, home, bx,
                                                        hcov, A.x, A.y, A.z,
                                                        skip_m && equal_m ? nullptr : A.m, A.fx,
                                                        A.fy, A.fz);
                    __builtin_amdgcn_s_setprio(0);
                    const bool any_pp = group_tests<G, PREC>(
                        S, ng,
                        [&](int pp, int k) {
                            const double thr = S.thr[pp];
                            return thr >= 0.0 && box_dist2(S, pp, k) <= thr * box_slack<PREC>();
                        },
                        [&](int pp, int sl, auto ppc) {
                            return filter_r2<G, PREC, decltype(ppc)::value>(S, bx, pp, sl) < S.thr[pp];
                        },
                        A.count_tests != 0, boxes, tests);
                    const uint64_t w0 = S.mask[p][0], w1 = S.mask[p][1];
                    // list position base + e belongs to lane (base + e) % LPP
                    const int e0 = (q - base % LPP + LPP) % LPP;
                    auto flush = [&](auto ppc) {
                        return for_my_bits<LPP>(w0, w1, e0, [&](int sl, int e) {
                            const int pos = base + e;
                            double dx, dy, dz, r2;
                            // FP64: the home position from LDS (fewer long-lived
                            // registers; measured faster), FP32-pair: the offsets
                            // held in registers (measured faster there)
                            separation<G, PREC, decltype(ppc)::value>(
                                S, bx, PREC == SPH_FP64 ? S.hx[p] : hx, PREC == SPH_FP64 ? S.hy[p] : hy,
                                PREC == SPH_FP64 ? S.hz[p] : hz, hfx, hfy, hfz, sl, dx, dy, dz, r2);
                            // (with equal masses mw is not used, and FP32-pair
                            // does not stage it)
                            double mw = 0.0;
                            if (PREC == SPH_FP64 || !equal_m) mw = S.c.w[sl];
                            if (pos < KP) {
                                const int at = (pos / LPP) * kWave + lane;
                                cr2[at] = (ListR2)r2;
                                if (!equal_m) cm[at] = mw;
                            }
                            accumulate(r2, mw);
                        });
                    };
                    const int n = any_pp ? flush(std::true_type{}) : flush(std::false_type{});
                    base += n;
                    if (q == 0) {
                        S.mask[p][0] = 0;
                        S.mask[p][1] = 0;
                    }
                    wave_lds_sync();
                };
                visits += for_each_leaf_group<NL>(T, A.nodes, wr, make_test(hcov), wb, group,
                                                  B.stage);
                count = base;
                cached = !conv && count <= KP;
                list_over += (int64_t)__popcll(__ballot(!conv && q == 0 && count > KP));
            } else {
                // every particle still iterating has a complete list and h <= Rc:
                // the entries inside R h, in list order, are the hits of a sweep
                // (rows <= ROWS: a cached list has at most KP entries.)  Rows past
                // this lane's entries pass r^2 = (R h)^2, which adds nothing
                // Rows are read kRowBatch at a time, every load issued before the
                // first sum (ROWS is a multiple of kRowBatch, so the rows read past
                // `rows` stay inside the block's slice; they count as not mine)
                constexpr int kRowBatch = 4;
                static_assert(ROWS % kRowBatch == 0, "list rows come in whole batches");
                const int rows = wave_max_int(conv ? 0 : (count + LPP - 1) / LPP);
                const ListR2 *__restrict__ lr2 = cr2 + lane;
                const double *__restrict__ lm = cm + lane;
                const int lim = conv ? 0 : count;   // entries of this particle still iterating
                for (int r0 = 0; r0 < rows; r0 += kRowBatch) {
                    double r2b[kRowBatch], mwb[kRowBatch];
#pragma unroll
                    for (int b = 0; b < kRowBatch; b++) {
                        r2b[b] = (double)lr2[(r0 + b) * kWave];
                        mwb[b] = equal_m ? 0.0 : lm[(r0 + b) * kWave];
                    }
#pragma unroll
                    for (int b = 0; b < kRowBatch; b++) {
                        const bool mine = (r0 + b) * LPP + q < lim;
                        accumulate(mine ? r2b[b] : h2x4, mwb[b]);
                    }
                }
            }
            // one evaluation for every particle still iterating (uniform)
            nr_total += (int64_t)__popcll(__ballot(!conv && q == 0));
            s0 = group_sum<LPP>(s0);
            s2 = group_sum<LPP>(s2);
            cnt = group_sum<LPP>(cnt) - 1;   // without the particle itself
            if (!conv && q == 0) evals_leaf += cnt;
            if (!conv) {
                // the root of g(h) = h^3 rho(h) - eta^3 m = sigma sum m f - eta^3 m
                // (non-decreasing in h) is the h of the h-rho relation.  Newton runs
                // on the equivalent F(h) = h - eta (m / rho(h))^(1/3), which is
                // exactly linear where rho does not vary over the kernel and so
                // converges in fewer steps than Newton on the cubic g; F has the
                // sign of g, and F'(h) = 1 - (h*/h)(1 - Omega) with h* = h - F
                const double g = SIG * s0 - A.eta3 * mi;
                const double hs = h * cbrt(A.eta3 * mi / (SIG * s0));
                const double om = -s2 / (3.0 * s0);
                const double fp = 1.0 - (hs * hinv) * (1.0 - om);
                if constexpr (NR_LDS) {
                    *nr_h = h;
                    *nr_rho = SIG * s0 * hinv * hinv * hinv;
                    *nr_om = om;
                } else {
                    h_out = h;
                    rho_out = SIG * s0 * hinv * hinv * hinv;
                    om_out = om;
                }
                n_out = cnt;
                // the Newton step decides convergence before any safeguard: h and rho
                // are final once the step would change h by at most h_rtol h and rho
                // (d ln rho / d ln h = 3 (Omega - 1)) by at most h_rtol rho, down to
                // a zero step at the root
                const double step = fp > 0.0 ? (h - hs) / fp : INFINITY;
                const double sens = fmax(1.0, 3.0 * fabs(om - 1.0));
                if (g == 0.0 || fabs(step) * sens <= A.h_rtol * h) {
                    conv = true;
                } else {
                    double lo = NR_LDS ? *nr_lo : lo_b, hi = NR_LDS ? *nr_hi : hi_b;
                    if (g < 0.0) lo = fmax(lo, h); else hi = fmin(hi, h);
                    double hn = fp > 0.0 ? h - step : (g < 0.0 ? 2.0 * h : 0.5 * h);
                    hn = fmin(fmax(hn, 0.5 * h), 2.0 * h);
                    // outside the bracket of known signs: bisect it
                    if (!(hn > lo && hn < hi)) hn = hi < INFINITY ? 0.5 * (lo + hi) : 2.0 * h;
                    if (!(hn == hn)) conv = true;
                    else h = hn;
                    if constexpr (NR_LDS) {
                        *nr_lo = lo;
                        *nr_hi = hi;
                    } else {
                        lo_b = lo;
                        hi_b = hi;
                    }
                }
            }
            if (cached && !(h <= Rc)) cached = false;
            iter++;
            if (__ballot(!conv) == 0ull || iter >= A.max_iter) break;
            const double hmx = wave_max(conv ? 0.0 : h);
            if (hmx > hcov) {
                hcov = A.walk_margin * hmx;
                __builtin_amdgcn_s_setprio(2);
                wr = walk(T, A.nodes, make_test(hcov), wb, S.walk_spare);
                __builtin_amdgcn_s_setprio(0);
                walks++;
                if (wr.lev) overflows++;
            }
        }
        bool bad = false, slow = false, wide = false;
        if constexpr (NR_LDS) {
            h_out = *nr_h;
            rho_out = *nr_rho;
            om_out = *nr_om;
        }
        if (active && q == 0) {
            A.h[i] = h_out;
            A.rho[i] = rho_out;
            A.omega[i] = om_out;
            A.nngb[i] = n_out;
            bad = !isfinite(h_out) || !isfinite(rho_out) || !isfinite(om_out) || !(rho_out > 0.0);
            slow = !bad && !conv;
            if (bx.periodic) {
                const double Lmin = fmin(fmin(bx.len[0], bx.len[1]), bx.len[2]);
                wide = !(2.0 * RK * h_out < Lmin);
            }
        }
        report(A.status, bad, kFlagNonFinite, 2);
        report(A.status, slow, kFlagNotConverged, 1);
        report(A.status, wide, kFlagStencil, 3);
        iter_max = iter > iter_max ? iter : iter_max;
        evals += wave_sum_int(evals_leaf);
        wave_lds_sync();   // the home table is rewritten for the next leaf
    });
    flush_counts();
}

// ---------------------------------------------------------------------------
// Force loop
// ---------------------------------------------------------------------------

// AC: the launch carries artificial conductivity (some set of the batch has
// alpha_AC > 0; a set with alpha_AC = 0 then adds exact zeros).
// SW: the launch carries per-particle alpha or the velocity divergence and
// curl (the artificial-viscosity switches); a set without them uses alpha_AV
// for every pair as the plain variant does.
template <int G, int PREC, bool AC, bool SW, int K>
__global__ __launch_bounds__(kWave, pair_waves_per_simd<PREC>()) void k_forces(Batch<ForceArgs> B)
{
    constexpr int LPP = kWave / G;
    constexpr int NL = kSlots / G;
    __shared__ WalkBuf wb;
    __shared__ TreeInfo T;
    __shared__ Stage<G, PREC> S;
    __shared__ uint32_t pre[kMaxBatch + 1];
    batch_prefix(B, pre);
    const int lane = threadIdx.x;
    const int p = lane / LPP, q = lane % LPP;
    int64_t pairs_total = 0, overflows = 0, tests = 0, boxes = 0;
    int cur = -1;
    const __attribute__((address_space(4))) ForceArgs *Fp = nullptr;
    auto flush_counts = [&]() {
        if (lane == 0 && cur >= 0) {
            auto add = [&](int k, int64_t v) {
                if (v) atomicAdd((unsigned long long *)&Fp->counts[k], (unsigned long long)v);
            };
            add(kCntForceEvals, pairs_total);
            add(kCntForceOverflows, overflows);
            add(kCntForceTests, tests);
            add(kCntForceBoxes, boxes);
        }
        pairs_total = overflows = tests = boxes = 0;
    };
    for_each_home_leaf(pre[B.nreq], B.work, B.claim, [&](int64_t gleaf) {
        const int r = __builtin_amdgcn_readfirstlane(find_req(pre, B.nreq, gleaf));
        if (r != cur) {
            flush_counts();
            cur = r;
            Fp = as_const(B.req[r]);
            load_tree(Fp->tree, T);
        }
        const auto &F = *Fp;
        const int64_t li = gleaf - (int64_t)__builtin_amdgcn_readfirstlane(pre[r]);
        const int64_t leaf = F.leaf_list ? (int64_t)as_const(F.leaf_list)[li] : li;
        if (F.leaf_act && as_const(F.leaf_act)[leaf] == 0) return;   // no active particle
        const Box bx = load_const(&B.req[r]->box);
        const double alpha = F.alpha, beta = F.beta;
        const double *const alpha_p = SW ? F.alpha_p : nullptr;
        const double alpha_ac = AC ? F.alpha_ac : 0.0, u_per_c2 = AC ? F.u_per_c2 : 0.0;
        const double inv_gamma = AC ? F.inv_gamma : 0.0;
        const bool ac_price = AC && F.ac_price != 0;
        const int64_t first = as_const(F.lstart)[leaf];
        const int nhome = (int)(as_const(F.lstart)[leaf + 1] - first);
        const int64_t i = first + p;
        const bool active = p < nhome && (!F.active || as_global(F.active)[i] != 0);
        const int64_t ii = p < nhome ? i : first;
        const double hx = as_global(F.x)[ii], hy = as_global(F.y)[ii], hz = as_global(F.z)[ii];
        float hfx = 0.f, hfy = 0.f, hfz = 0.f;
        if (PREC == SPH_FP32_PAIR) {
            hfx = as_global(F.fx)[ii];
            hfy = as_global(F.fy)[ii];
            hfz = as_global(F.fz)[ii];
        }
        const ForceRec ri = load_global(F.rec + ii);
        const double vxi = ri.vx, vyi = ri.vy, vzi = ri.vz;
        const double hi = as_global(F.h)[ii], hinvi = ri.hinv;
        const double rhoi = ri.rho, Ai = ri.A, ci = ri.c;
        const double alpha_i = (SW && alpha_p) ? as_global(alpha_p)[ii] : alpha;
        constexpr double RK = Kern<K>::R, SIG = Kern<K>::sigma;
        const double hi2x4 = (RK * hi) * (RK * hi);
        const double gfi = SIG * (hinvi * hinvi) * (hinvi * hinvi);
        const float hinvif = (float)hinvi;
        const float gfif = (float)SIG * (hinvif * hinvif) * (hinvif * hinvif);
        // FP32-pair: the home particle's values as its single-precision record holds them
        const float vxif = (float)vxi, vyif = (float)vyi, vzif = (float)vzi;
        const float Aif = (float)Ai, cif = (float)ci, rhoif = (float)rhoi;
        const Node home = load_const(F.nodes + leaf);
        if (q == 0) {
            S.hx[p] = hx;
            S.hy[p] = hy;
            S.hz[p] = hz;
            S.hfx[p] = hfx;
            S.hfy[p] = hfy;
            S.hfz[p] = hfz;
            S.thr[p] = active ? hi2x4 : -1.0;
            S.mask[p][0] = 0;
            S.mask[p][1] = 0;
        }
        // symmetric criterion: a node can hold force neighbours of the home leaf
        // if its box is closer than 2 max(h over home, h over node)
        auto test = [&bx, &home](const Node &nd) {
            const double R = RK * fmax(home.hmax, nd.hmax) * (1.0 + 1e-10);
            return box_gap2(home.lo, home.hi, nd, bx) < R * R;
        };
        // walk and staging at raised priority, as in the density loop
        __builtin_amdgcn_s_setprio(2);
        const WalkResult wr = walk(T, F.nodes, test, wb, S.walk_spare);
        __builtin_amdgcn_s_setprio(0);
        if (wr.lev) overflows++;

        double axi = 0.0, ayi = 0.0, azi = 0.0, dui = 0.0, vs_max = -INFINITY;
        double dvs = 0.0, cxs = 0.0, cys = 0.0, czs = 0.0;   // div v, curl v sums (SW)
        int cnt = 0, selfs = 0;
        int lmx_l = 0;                                       // block time-steps
        const int lev_i = F.lev ? as_global(F.lev)[ii] : 0;
        auto group = [&](const uint32_t *leaves, int ng) {
            __builtin_amdgcn_s_setprio(2);
            stage_group<G, PREC, K, true>(S, leaves, ng, F.lstart, F.nodes, home, bx, -1.0, F.x, F.y, F.z,
                                       F.h, F.fx, F.fy, F.fz);
            __builtin_amdgcn_s_setprio(0);
            group_tests<G, PREC>(
                S, ng,
                [&](int pp, int k) {
                    const double thr = S.thr[pp];
                    const double hk = RK * S.hmax[k];
                    return thr >= 0.0 && box_dist2(S, pp, k) <= fmax(thr, hk * hk) * box_slack<PREC>();
                },
                [&](int pp, int sl, auto ppc) {
                    double dx, dy, dz, r2;
                    separation<G, PREC, decltype(ppc)::value>(S, bx, S.hx[pp], S.hy[pp], S.hz[pp],
                                                              S.hfx[pp], S.hfy[pp], S.hfz[pp], sl, dx,
                                                              dy, dz, r2);
                    // the particle itself passes too; the flush drops it
                    const double thr = S.thr[pp];
                    const double hj2x4 = S.c.w[sl];
                    if (PREC == SPH_FP64) return r2 < thr || r2 < hj2x4;
                    return (float)r2 < (float)thr || (float)r2 < (float)hj2x4;
                },
                F.count_tests != 0, boxes, tests);
            const uint64_t w0 = S.mask[p][0], w1 = S.mask[p][1];
            // the record of a neighbour that the pair terms read (one line)
            // FP32-pair: the neighbours' single-precision records (32 bytes)
            using JData = std::conditional_t<PREC == SPH_FP64, ForceRec, ForceRec32>;
            auto load_j = [&](int sl) {
                if constexpr (PREC == SPH_FP64) return load_global(F.rec + S.j[sl]);
                else return load_global(F.rec32 + S.j[sl]);
            };
            auto pair_terms = [&](int sl, const JData &d) {
                double dx, dy, dz, r2;
                // FP64: home position from LDS, as in the density flush
                separation<G, PREC>(S, bx, PREC == SPH_FP64 ? S.hx[p] : hx,
                                    PREC == SPH_FP64 ? S.hy[p] : hy, PREC == SPH_FP64 ? S.hz[p] : hz,
                                    hfx, hfy, hfz, sl, dx, dy, dz, r2);
                const double cj = d.c;
                if (r2 == 0.0) {
                    vs_max = fmax(vs_max, PREC == SPH_FP64 ? ci + cj : (double)(cif + (float)cj));
                    return;
                }
                // the pair's viscosity strength: (alpha_i + alpha_j)/2 with
                // per-particle values, alpha_AV otherwise
                const double aij = (SW && alpha_p) ? 0.5 * (alpha_i + as_global(alpha_p)[S.j[sl]])
                                                   : alpha;
                if constexpr (PREC == SPH_FP64) {
                    const double rinv = rsqrt_nr(r2);
                    const double rr = r2 * rinv;
                    const double ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
                    const double hinvj = d.hinv;
                    const double gfj = SIG * (hinvj * hinvj) * (hinvj * hinvj);
                    double fi, dfi, fj, dfj;
                    kern<K>(rr * hinvi, fi, dfi);
                    kern<K>(rr * hinvj, fj, dfj);
                    double gi, gj, gsum;
                    sym_grads(gfi, dfi, gfj, dfj, gi, gj, gsum);
                    const double w = ((vxi - d.vx) * ex + (vyi - d.vy) * ey) + (vzi - d.vz) * ez;
                    const double mj = d.m;
                    double cvec = -mj * sym_dot2(Ai, gi, d.A, gj);
                    double cdu = Ai * mj * gi * w;
                    const double wneg = fmin(w, 0.0);
                    const double vs = (ci + cj) - beta * wneg;
                    vs_max = fmax(vs_max, vs);
                    const double rbinv = rcp_nr(0.5 * (rhoi + d.rho));
                    const double visc = (mj * rbinv) * aij * vs * wneg;
                    const double gbar = 0.5 * gsum;
                    cvec += visc * gbar;
                    cdu -= visc * 0.5 * wneg * gbar;
                    if constexpr (AC) {
                        // u and P of both particles from their sound speeds
                        const double c2i = ci * ci, c2j = cj * cj;
                        const double vc = ac_price
                            ? sqrt(fabs(rhoi * c2i - d.rho * c2j) * inv_gamma * rbinv)
                            : fabs(w);
                        cdu += (mj * rbinv) * alpha_ac * vc * ((c2i - c2j) * u_per_c2) * gbar;
                    }
                    axi += cvec * ex;
                    ayi += cvec * ey;
                    azi += cvec * ez;
                    dui += cdu;
                    if constexpr (SW) {
                        // v_ij . G_i = w gi and v_ij x G_i = gi (v_ij x rhat)
                        const double vxij = vxi - d.vx, vyij = vyi - d.vy, vzij = vzi - d.vz;
                        dvs += mj * w * gi;
                        cxs += mj * gi * (vyij * ez - vzij * ey);
                        cys += mj * gi * (vzij * ex - vxij * ez);
                        czs += mj * gi * (vxij * ey - vyij * ex);
                    }
                } else {
                    const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
                    // hardware reciprocal square root and reciprocal (1 ulp each),
                    // functions of symmetric operands, so (j, i) sees the same values
                    const float rinv = __builtin_amdgcn_rsqf((float)r2);
                    const float rr = (float)r2 * rinv;
                    const float ex = fdx * rinv, ey = fdy * rinv, ez = fdz * rinv;
                    const float hinvj = d.hinv;
                    // own and other kernel factors formed by the same float
                    // expression, so the (j, i) pair sees exactly the values of
                    // the (i, j) pair
                    const float gfjf = (float)SIG * (hinvj * hinvj) * (hinvj * hinvj);
                    float fi, dfi, fj, dfj;
                    kern<K>(rr * hinvif, fi, dfi);
                    kern<K>(rr * hinvj, fj, dfj);
                    float gi, gj, gsum;
                    sym_grads(gfif, dfi, gfjf, dfj, gi, gj, gsum);
                    const float w = ((vxif - d.vx) * ex + (vyif - d.vy) * ey) + (vzif - d.vz) * ez;
                    const float mj = d.m;
                    const float cjf = d.c;
                    float cvec = -mj * sym_dot2(Aif, gi, d.A, gj);
                    float cdu = Aif * mj * gi * w;
                    const float wneg = fminf(w, 0.0f);
                    const float vs = (cif + cjf) - (float)beta * wneg;
                    vs_max = fmax(vs_max, (double)vs);
                    const float rbinv = __builtin_amdgcn_rcpf(0.5f * (rhoif + d.rho));
                    const float visc = (mj * rbinv) * (float)aij * vs * wneg;
                    const float gbar = 0.5f * gsum;
                    cvec += visc * gbar;
                    cdu -= visc * 0.5f * wneg * gbar;
                    if constexpr (AC) {
                        // differences of u and P formed in double precision from
                        // the single-precision values both sides of the pair see
                        const double c2i = (double)cif * cif, c2j = (double)cjf * cjf;
                        const float du_ij = (float)((c2i - c2j) * u_per_c2);
                        const float vc =
                            ac_price
                                ? sqrtf((float)(fabs((double)rhoif * c2i - (double)d.rho * c2j) *
                                                inv_gamma) * rbinv)
                                : fabsf(w);
                        cdu += (mj * rbinv) * (float)alpha_ac * vc * du_ij * gbar;
                    }
                    axi += (double)(cvec * ex);
                    ayi += (double)(cvec * ey);
                    azi += (double)(cvec * ez);
                    dui += (double)cdu;
                    if constexpr (SW) {
                        const float vxij = vxif - d.vx, vyij = vyif - d.vy, vzij = vzif - d.vz;
                        dvs += (double)(mj * w * gi);
                        cxs += (double)(mj * gi * (vyij * ez - vzij * ey));
                        cys += (double)(mj * gi * (vzij * ex - vxij * ez));
                        czs += (double)(mj * gi * (vxij * ey - vyij * ex));
                    }
                }
            };
            // the particle's hits of this group (same count on all its lanes).
            // FP32-pair: two at a time, both neighbours' records requested
            // before either is used (measured faster; at the FP64 register
            // budget the second record costs more than it hides)
            // the particle itself is among the hits of its own leaf: it takes
            // no pair terms and is not counted
            const uint32_t self = (uint32_t)i;
            // block time-steps: the deepest neighbour level, and inactive
            // neighbours more than lim levels shallower marked to wake up
            auto limiter = [&](uint32_t j) {
                if (!F.lev) return;
                const int lj = as_global(F.lev)[j];
                lmx_l = lj > lmx_l ? lj : lmx_l;
                if (lj < lev_i - F.lim && as_global(F.active)[j] == 0) atomicMax(&F.mark[j], lev_i);
            };
            if (PREC == SPH_FP32_PAIR) {
                cnt += for_my_bit_pairs<LPP>(w0, w1, q, [&](int sa, int sb) {
                    const JData da = load_j(sa);
                    JData db = da;
                    if (sb >= 0) db = load_j(sb);
                    if (S.j[sa] != self) { limiter(S.j[sa]); pair_terms(sa, da); } else selfs++;
                    if (sb >= 0) {
                        if (S.j[sb] != self) { limiter(S.j[sb]); pair_terms(sb, db); } else selfs++;
                    }
                });
            } else {
                cnt += for_my_bits<LPP>(w0, w1, q, [&](int sl, int) {
                    if (S.j[sl] != self) { limiter(S.j[sl]); pair_terms(sl, load_j(sl)); } else selfs++;
                });
            }
            if (q == 0) {
                S.mask[p][0] = 0;
                S.mask[p][1] = 0;
            }
            wave_lds_sync();
        };
        for_each_leaf_group<NL>(T, F.nodes, wr, test, wb, group, B.stage);
        axi = group_sum<LPP>(axi);
        ayi = group_sum<LPP>(ayi);
        azi = group_sum<LPP>(azi);
        dui = group_sum<LPP>(dui);
        vs_max = group_max<LPP>(vs_max);
        selfs = group_sum<LPP>(selfs);
        cnt -= selfs;
        if (F.lev) lmx_l = group_max_int<LPP>(lmx_l);
        if constexpr (SW) {
            dvs = group_sum<LPP>(dvs);
            cxs = group_sum<LPP>(cxs);
            cys = group_sum<LPP>(cys);
            czs = group_sum<LPP>(czs);
        }
        bool bad = false;
        if (active && q == 0) {
            const double vsig = cnt > 0 ? vs_max : 2.0 * ci;
            F.ax[i] = axi;
            F.ay[i] = ayi;
            F.az[i] = azi;
            F.du[i] = dui;
            F.vsig[i] = vsig;
            F.dt[i] = F.ccfl * hi / vsig;
            F.nforce[i] = cnt;
            if (F.lmx) F.lmx[i] = lmx_l;
            if (SW && F.divv) {
                const double orho = as_global(F.omega)[i] * rhoi;
                F.divv[i] = -dvs / orho;
                F.curlv[i] = sqrt((cxs * cxs + cys * cys) + czs * czs) / orho;
            }
            bad = !isfinite(axi) || !isfinite(ayi) || !isfinite(azi) || !isfinite(dui) ||
                  !isfinite(vsig);
        }
        report(F.status, bad, kFlagNonFinite, 2);
        pairs_total += wave_sum_int((q == 0 && active) ? cnt : 0);
        wave_lds_sync();   // the home table is rewritten for the next leaf
    });
    flush_counts();
}

// ---------------------------------------------------------------------------
// Neighbour export (tests): counts, then lists in original indices
// ---------------------------------------------------------------------------

template <int G, int K>
__global__ __launch_bounds__(kWave) void k_neighbours(NgbArgs N, int pass)
{
    constexpr double RK = Kern<K>::R;
    constexpr int LPP = kWave / G;
    constexpr int PER = G / LPP;
    __shared__ WalkBuf wb;
    __shared__ uint32_t spare[kFront];
    __shared__ TreeInfo T;
    load_tree(N.tree, T);
    const int lane = threadIdx.x;
    const int p = lane / LPP, q = lane % LPP;
    const Box &bx = N.box;
    const int32_t mode = N.mode;
    int64_t overflows = 0;
    for_each_home_leaf(T.cnt[0], N.work, 1, [&](int64_t leaf) {
        const int64_t first = N.lstart[leaf];
        const int nhome = (int)(N.lstart[leaf + 1] - first);
        const int64_t i = first + p;
        const bool active = p < nhome;
        const int64_t ii = active ? i : first;
        const double xi = N.x[ii], yi = N.y[ii], zi = N.z[ii], hi = N.h[ii];
        const double hi2x4 = (RK * hi) * (RK * hi);
        const Node home = N.nodes[leaf];
        auto test = [&bx, &home, mode](const Node &nd) {
            const double hh = mode == 0 ? home.hmax : fmax(home.hmax, nd.hmax);
            const double R = RK * hh * (1.0 + 1e-10);
            return box_gap2(home.lo, home.hi, nd, bx) < R * R;
        };
        const WalkResult wr = walk(T, N.nodes, test, wb, spare);
        if (wr.lev) overflows++;
        // two sweeps in pass 2: count this lane's hits, then write them
        int64_t mine = 0, base = 0;
        for (int sweep = 0; sweep < (pass == 1 ? 1 : 2); sweep++) {
            int64_t k = 0;
            auto group = [&](const uint32_t *leaves, int count) {
                for (int g = 0; g < count; g++) {
                    const int64_t c = leaves[g];
                    const Node cand = N.nodes[c];
                    const Shift sh = leaf_shift(
                        home, cand, bx, RK * (mode == 0 ? home.hmax : fmax(home.hmax, cand.hmax)));
                    const int64_t j0 = N.lstart[c];
                    const int jn = (int)(N.lstart[c + 1] - j0);
#pragma unroll
                    for (int t = 0; t < PER; t++) {
                        const int jj = q + LPP * t;
                        if (jj >= jn) continue;
                        const int64_t j = j0 + jj;
                        double dx = xi - N.x[j], dy = yi - N.y[j], dz = zi - N.z[j];
                        if (sh.per_pair) {
                            dx = min_image(dx, bx.len[0], bx.half[0]);
                            dy = min_image(dy, bx.len[1], bx.half[1]);
                            dz = min_image(dz, bx.len[2], bx.half[2]);
                        } else {
                            dx += sh.s[0];
                            dy += sh.s[1];
                            dz += sh.s[2];
                        }
                        const double r2 = exact_r2(dx, dy, dz);
                        bool in = r2 < hi2x4;
                        if (mode == 1) {
                            const double hj = N.h[j];
                            in = in || r2 < (RK * hj) * (RK * hj);
                        }
                        if (in && j != i && active) {
                            if (sweep == 1) {
                                const int64_t pos = base + k;
                                if (pos < N.cap) N.idx[pos] = (int32_t)N.id[j];
                            }
                            k++;
                        }
                    }
                }
            };
            for_each_leaf_group<kWave>(T, N.nodes, wr, test, wb, group);
            if (sweep == 0) {
                mine = k;
                // exclusive prefix over the LPP lanes of this particle
                int64_t incl = mine;
#pragma unroll
                for (int o = 1; o < LPP; o <<= 1) {
                    int64_t v = (int64_t)__shfl_up((long long)incl, o, LPP);
                    if (q >= o) incl += v;
                }
                const int64_t total = (int64_t)__shfl((long long)incl, (p * LPP) + LPP - 1);
                if (pass == 1) {
                    if (active && q == 0) N.counts[i] = total;
                } else {
                    base = active ? N.offsets[N.id[i]] + (incl - mine) : 0;
                }
            }
        }
    });
    if (lane == 0 && overflows) atomicAdd(&N.status[4], (int)overflows);
}

// ---------------------------------------------------------------------------
// Meshless finite-volume geometry (section 2.2): for each particle, over its
// neighbours j with r_ij < R h_i (h solved on the number density), with
// d = r_j - r_i and psi_j = W(r_ij, h_i) / n_i:
//   E  = sum_j d d^T psi_j                    (EQN:MFVEMATRIX), B = E^-1
//   g  = sum_j (f_j - f_i) d psi_j,  grad f = B g   (EQN:MFVGRADIENT with
//        EQN:MFVPSI: B is constant over the sum and comes out of it)
//   gs = sum_j (f_j - f_i) grad_i W(r_ij, h_i), the SPH gradient n_i^-1 gs
//        used when cond(E) = |E|_F |B|_F / 3 exceeds 100.
// One wave per home leaf, LPP lanes per particle taking every LPP-th slot
// of each candidate leaf, sums reduced over the particle's lanes.  The
// candidate leaves are staged in LDS 64 slots at a time (positions, fields,
// per-leaf shift), so each candidate is loaded once per wave rather than by
// every home particle.  The sums of the SPH fallback are taken in a second
// pass over the same pairs, only in waves where some particle's E is
// ill-conditioned (rare), so the first pass holds fewer live sums.  Measured
// on the C1 geometry call: 15.0 ms for one pass from global memory
// (unbounded, 2 waves per SIMD), 13.1 ms with the two passes at 4 waves,
// 10.6 ms staged (11.5 ms staged at 3 waves).
// ---------------------------------------------------------------------------

template <int G, int K>
__global__ __launch_bounds__(kWave, 4) void k_mfv(MfvArgs M)
{
    constexpr double RK = Kern<K>::R;
    constexpr int LPP = kWave / G;
    // candidates staged in LDS one slot per lane (MNL leaves at a time): each
    // is loaded once per wave instead of once per home particle
    constexpr int MS = kWave, MNL = MS / G;
    __shared__ WalkBuf wb;
    __shared__ uint32_t spare[kFront];
    __shared__ TreeInfo T;
    __shared__ double st_x[MS], st_y[MS], st_z[MS], st_f[kMfvFields][MS];
    __shared__ double st_s[MNL][3];
    __shared__ int32_t st_pp[MNL], st_jn[MNL];
    load_tree(M.tree, T);
    const int lane = threadIdx.x;
    const int p = lane / LPP, q = lane % LPP;
    const Box &bx = M.box;
    const int nf = M.nf;
    int64_t overflows = 0;
    for_each_home_leaf(T.cnt[0], M.work, 1, [&](int64_t leaf) {
        const int64_t first = M.lstart[leaf];
        const int nhome = (int)(M.lstart[leaf + 1] - first);
        const int64_t i = first + p;
        const bool active = p < nhome;
        const int64_t ii = active ? i : first;
        const double xi = M.x[ii], yi = M.y[ii], zi = M.z[ii], hi = M.h[ii];
        const double hinv = 1.0 / hi, ninv = 1.0 / M.ndens[ii];
        const double hi2x4 = (RK * hi) * (RK * hi);
        const double wf = Kern<K>::sigma * hinv * hinv * hinv;
        double fi[kMfvFields];
#pragma unroll
        for (int k = 0; k < kMfvFields; k++) fi[k] = k < nf ? M.f[k][ii] : 0.0;
        const Node home = M.nodes[leaf];
        auto test = [&bx, &home](const Node &nd) {
            const double R = RK * home.hmax * (1.0 + 1e-10);
            return box_gap2(home.lo, home.hi, nd, bx) < R * R;
        };
        const WalkResult wr = walk(T, M.nodes, test, wb, spare);
        if (wr.lev) overflows++;
        // The pairs (i, j) with 0 < r_ij < R h_i, candidate leaf by candidate
        // leaf, each leaf's slots q, q + LPP, ... on lane q of the particle:
        // fn(d, psi, gw, s) with d = r_j - r_i, psi = psi_j(r_i),
        // gw = -(dW/dr) / r (grad_i W = gw d) and s the staged slot of j.
        // Every use visits them in the same order.
        auto for_pairs = [&](auto fn) {
            auto group = [&](const uint32_t *leaves, int count) {
                {
                    const int k = lane / G, slot = lane % G;
                    if (k < count) {
                        const uint32_t c = leaves[k];
                        const int64_t j0 = M.lstart[c];
                        const int jn = (int)(M.lstart[c + 1] - j0);
                        if (slot < jn) {
                            const int64_t j = j0 + slot;
                            st_x[lane] = M.x[j];
                            st_y[lane] = M.y[j];
                            st_z[lane] = M.z[j];
#pragma unroll
                            for (int f = 0; f < kMfvFields; f++)
                                if (f < nf) st_f[f][lane] = M.f[f][j];
                        }
                        if (slot == 0) {
                            const Shift sh = leaf_shift(home, M.nodes[c], bx, RK * home.hmax);
                            for (int a = 0; a < 3; a++) st_s[k][a] = sh.s[a];
                            st_pp[k] = sh.per_pair ? 1 : 0;
                            st_jn[k] = jn;
                        }
                    }
                }
                wave_lds_sync();
#pragma unroll 1
                for (int t = 0; t < MS / LPP; t++) {
                    const int s = q + LPP * t;
                    const int k = s / G;
                    if (k >= count || s % G >= st_jn[k]) continue;
                    double dx = xi - st_x[s], dy = yi - st_y[s], dz = zi - st_z[s];
                    if (st_pp[k]) {
                        dx = min_image(dx, bx.len[0], bx.half[0]);
                        dy = min_image(dy, bx.len[1], bx.half[1]);
                        dz = min_image(dz, bx.len[2], bx.half[2]);
                    } else {
                        dx += st_s[k][0];
                        dy += st_s[k][1];
                        dz += st_s[k][2];
                    }
                    const double r2 = exact_r2(dx, dy, dz);
                    if (!(active && r2 < hi2x4 && r2 > 0.0)) continue;
                    const double d[3] = {-dx, -dy, -dz};   // r_j - r_i
                    const double r = sqrt(r2);
                    double fk, dfk;
                    kern<K>(r * hinv, fk, dfk);
                    const double psi = wf * fk * ninv;
                    // grad_i W = dW/dr (r_i - r_j) / r = -(dW/dr / r) d
                    const double gw = -(wf * hinv * dfk) / r;
                    fn(d, psi, gw, s);
                }
                wave_lds_sync();   // the slots are restaged for the next group
            };
            for_each_leaf_group<MNL>(T, M.nodes, wr, test, wb, group);
        };
        // first pass: E and the least-squares sums
        double E[6] = {0, 0, 0, 0, 0, 0};
        double g[3 * kMfvFields];
#pragma unroll
        for (int k = 0; k < 3 * kMfvFields; k++) g[k] = 0.0;
        for_pairs([&](const double *d, double psi, double gw, int sl) {
            E[0] += d[0] * d[0] * psi;
            E[1] += d[0] * d[1] * psi;
            E[2] += d[0] * d[2] * psi;
            E[3] += d[1] * d[1] * psi;
            E[4] += d[1] * d[2] * psi;
            E[5] += d[2] * d[2] * psi;
#pragma unroll
            for (int k = 0; k < kMfvFields; k++) {
                if (k >= nf) break;
                const double df = st_f[k][sl] - fi[k];
#pragma unroll
                for (int a = 0; a < 3; a++) g[3 * k + a] += df * d[a] * psi;
            }
        });
#pragma unroll
        for (int k = 0; k < 6; k++) E[k] = group_sum<LPP>(E[k]);
#pragma unroll
        for (int k = 0; k < 3 * kMfvFields; k++) g[k] = group_sum<LPP>(g[k]);
        // B = E^-1 of the symmetric E by cofactors, and the condition number
        const double c00 = E[3] * E[5] - E[4] * E[4];
        const double c01 = E[2] * E[4] - E[1] * E[5];
        const double c02 = E[1] * E[4] - E[2] * E[3];
        const double c11 = E[0] * E[5] - E[2] * E[2];
        const double c12 = E[1] * E[2] - E[0] * E[4];
        const double c22 = E[0] * E[3] - E[1] * E[1];
        const double det = E[0] * c00 + E[1] * c01 + E[2] * c02;
        const double id = 1.0 / det;
        const double B[6] = {c00 * id, c01 * id, c02 * id, c11 * id, c12 * id, c22 * id};
        auto frob2 = [](const double *s) {
            return (s[0] * s[0] + s[3] * s[3] + s[5] * s[5]) +
                   2.0 * (s[1] * s[1] + s[2] * s[2] + s[4] * s[4]);
        };
        const bool inv_ok = det != 0.0 && isfinite(det);
        const double cn = inv_ok ? sqrt(frob2(E)) * sqrt(frob2(B)) / 3.0 : INFINITY;
        const bool sph = !(cn <= 100.0);
        // second pass, only in a wave where some particle's E is ill-conditioned
        // (rare): the sums of the SPH estimate, in the order of the first pass
        double gs[3 * kMfvFields];
#pragma unroll
        for (int k = 0; k < 3 * kMfvFields; k++) gs[k] = 0.0;
        if (__ballot(active && sph) != 0ull) {
            for_pairs([&](const double *d, double psi, double gw, int sl) {
#pragma unroll
                for (int k = 0; k < kMfvFields; k++) {
                    if (k >= nf) break;
                    const double df = st_f[k][sl] - fi[k];
#pragma unroll
                    for (int a = 0; a < 3; a++) gs[3 * k + a] += df * gw * d[a];
                }
            });
#pragma unroll
            for (int k = 0; k < 3 * kMfvFields; k++) gs[k] = group_sum<LPP>(gs[k]);
        }
        if (active && q == 0) {
#pragma unroll
            for (int k = 0; k < 6; k++)
                if (M.B[k]) M.B[k][i] = inv_ok ? B[k] : NAN;
            if (M.cond) M.cond[i] = cn;
            for (int k = 0; k < nf; k++) {
                const double *gk = g + 3 * k;
                double out[3];
                if (!sph) {
                    out[0] = B[0] * gk[0] + B[1] * gk[1] + B[2] * gk[2];
                    out[1] = B[1] * gk[0] + B[3] * gk[1] + B[4] * gk[2];
                    out[2] = B[2] * gk[0] + B[4] * gk[1] + B[5] * gk[2];
                } else {
                    for (int a = 0; a < 3; a++) out[a] = gs[3 * k + a] * ninv;
                }
                for (int a = 0; a < 3; a++)
                    if (M.grad[3 * k + a]) M.grad[3 * k + a][i] = out[a];
            }
        }
    });
    if (lane == 0 && overflows) atomicAdd(&M.status[4], (int)overflows);
}

} // namespace

// ---------------------------------------------------------------------------
// Launches (instantiated per smoothing kernel by pairs_m4.hip and
// pairs_quintic.hip)
// ---------------------------------------------------------------------------
template <int K>
void launch_density(hipStream_t st, int G, int prec, unsigned grid, const Batch<DensArgs> &B)
{
    auto go = [&](auto g) {
        constexpr int GG = decltype(g)::value;
        if (prec == SPH_FP32_PAIR)
            hipLaunchKernelGGL((k_density<GG, SPH_FP32_PAIR, K>), dim3(grid), dim3(kWave), 0, st, B);
        else
            hipLaunchKernelGGL((k_density<GG, SPH_FP64, K>), dim3(grid), dim3(kWave), 0, st, B);
    };
    switch (G) {
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 32: go(std::integral_constant<int, 32>{}); break;
    default: go(std::integral_constant<int, 16>{}); break;
    }
}

template <int K>
void launch_forces(hipStream_t st, int G, int prec, bool ac, bool sw, unsigned grid,
                   const Batch<ForceArgs> &B)
{
    auto go = [&](auto g) {
        constexpr int GG = decltype(g)::value;
        auto variant = [&](auto pr, auto with_ac, auto with_sw) {
            hipLaunchKernelGGL((k_forces<GG, decltype(pr)::value, decltype(with_ac)::value,
                                         decltype(with_sw)::value, K>),
                               dim3(grid), dim3(kWave), 0, st, B);
        };
        using F32 = std::integral_constant<int, SPH_FP32_PAIR>;
        using F64 = std::integral_constant<int, SPH_FP64>;
        using T = std::true_type;
        using N = std::false_type;
        if (prec == SPH_FP32_PAIR) {
            if (sw) { if (ac) variant(F32{}, T{}, T{}); else variant(F32{}, N{}, T{}); }
            else if (ac) variant(F32{}, T{}, N{});
            else variant(F32{}, N{}, N{});
        } else {
            if (sw) { if (ac) variant(F64{}, T{}, T{}); else variant(F64{}, N{}, T{}); }
            else if (ac) variant(F64{}, T{}, N{});
            else variant(F64{}, N{}, N{});
        }
    };
    switch (G) {
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 32: go(std::integral_constant<int, 32>{}); break;
    default: go(std::integral_constant<int, 16>{}); break;
    }
}

template <int K>
void launch_neighbours(hipStream_t st, int G, unsigned grid, const NgbArgs &a, int pass)
{
    switch (G) {
    case 8: hipLaunchKernelGGL((k_neighbours<8, K>), dim3(grid), dim3(kWave), 0, st, a, pass); break;
    case 32: hipLaunchKernelGGL((k_neighbours<32, K>), dim3(grid), dim3(kWave), 0, st, a, pass); break;
    default: hipLaunchKernelGGL((k_neighbours<16, K>), dim3(grid), dim3(kWave), 0, st, a, pass); break;
    }
}

template <int K>
void launch_mfv(hipStream_t st, int G, unsigned grid, const MfvArgs &a)
{
    switch (G) {
    case 8: hipLaunchKernelGGL((k_mfv<8, K>), dim3(grid), dim3(kWave), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_mfv<32, K>), dim3(grid), dim3(kWave), 0, st, a); break;
    default: hipLaunchKernelGGL((k_mfv<16, K>), dim3(grid), dim3(kWave), 0, st, a); break;
    }
}

} // namespace sph
