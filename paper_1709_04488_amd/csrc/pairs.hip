// Pair-loop dispatch: argument blocks written on the device, batched
// persistent launches of the pair kernels (pairs.hpp, built per smoothing
// kernel by pairs_m4.hip and pairs_quintic.hip), the neighbour export's list
// sort.
#include "pairs_args.hpp"

#include <algorithm>
#include <type_traits>

#define TRY_(expr)                     \
    do {                               \
        sph_status st_ = (expr);       \
        if (st_ != SPH_OK) return st_; \
    } while (0)

namespace sph {
namespace {

// ascending order within each list (insertion sort; lists are ~60 long)
__global__ __launch_bounds__(256) void k_sort_lists(int64_t n, const int64_t *__restrict__ off,
                                                    int32_t *__restrict__ idx, int64_t cap)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t a = off[i], b = off[i + 1];
    if (b > cap) return;
    for (int64_t k = a + 1; k < b; k++) {
        int32_t v = idx[k];
        int64_t m = k - 1;
        while (m >= a && idx[m] > v) { idx[m + 1] = idx[m]; m--; }
        idx[m + 1] = v;
    }
}

template <class Args>
inline void fill_common(sph_ctx *c, int64_t n, Args &a)
{
    a.n = n;
    a.tree = c->d_tree;
    a.lstart = c->lstart;
    a.work = c->d_work;
    a.box = c->box;
    a.nodes = c->nodes;
}

} // namespace

// ---- argument blocks and batched launches ---------------------------------

namespace {

// A set's pair-loop prologue in one launch: its argument block, its counters
// of that loop and its claim counters zeroed.  Stream order puts it after the
// set's previous pair loop and before the next launch that reads them (a
// batched launch claims through its first set's counters).
template <class Args>
__global__ void k_prologue(Args a, Args *dst, int64_t *__restrict__ counts, int first, int nwords,
                           int first2, int nwords2, uint32_t *__restrict__ work)
{
    const int t = threadIdx.x;
    if (t == 0) *dst = a;
    if (t < nwords) counts[first + t] = 0;
    if (t < nwords2) counts[first2 + t] = 0;
    if (t < kXcds) work[t] = 0u;
}

static_assert(sizeof(DensArgs) <= kArgBytes, "density argument block too large");
static_assert(sizeof(ForceArgs) <= kArgBytes, "force argument block too large");
static_assert(kCntDensWords <= 64 && kCntForceWords <= 64, "prologue zeroes one word per lane");

} // namespace

sph_status density_prepare(sph_ctx *c, int64_t n)
{
    DensArgs a{};
    fill_common(c, n, a);
    a.x = c->s.x; a.y = c->s.y; a.z = c->s.z; a.m = c->s.m;
    a.fx = c->s.fx; a.fy = c->s.fy; a.fz = c->s.fz;
    a.h = c->s.h; a.rho = c->s.rho; a.omega = c->s.omega; a.nngb = c->s.nngb;
    a.status = c->d_status;
    a.counts = c->d_counts;
    a.mrange = c->d_scal + 8;
    a.count_tests = c->count_tests ? 1 : 0;
    a.eta3 = c->p.eta * c->p.eta * c->p.eta;
    // FP32-pair mode: the density sum carries single-precision pair terms
    // (relative noise ~1e-7), so the Newton step cannot settle below a few
    // 1e-7; its stop tolerance is floored at 2e-6.
    a.h_rtol = c->p.precision == SPH_FP32_PAIR ? std::max(c->p.h_rtol, 2e-6) : c->p.h_rtol;
    a.walk_margin = 1.1;
    a.max_iter = c->p.h_max_iter;
    a.active = c->f_act;
    a.leaf_act = c->f_act ? c->leaf_act : nullptr;
    a.leaf_list = c->f_act ? c->act_list : nullptr;
    a.leaf_count = c->f_act ? c->act_cnt : nullptr;
    const void *req[] = {a.nodes, a.x, a.y, a.z, a.m, a.h, a.rho, a.omega, a.nngb, a.status,
                         a.counts, a.tree, a.lstart, a.work, c->d_dargs};
    for (const void *q : req)
        if (!q) return fail(c, SPH_EINVAL, "density: internal buffer not allocated");
    if (c->p.precision == SPH_FP32_PAIR && (!a.fx || !a.fy || !a.fz))
        return fail(c, SPH_EINVAL, "density: offsets not allocated");
    if (c->tree_n != n || n <= 0) return fail(c, SPH_ESTATE, "density: tree not built");
    TRY_(reduce_mass_range(c, n));
    hipLaunchKernelGGL(k_prologue<DensArgs>, dim3(1), dim3(64), 0, c->stream, a,
                       (DensArgs *)c->d_dargs, c->d_counts, (int)kCntDensFirst, (int)kCntDensWords,
                       (int)kCntDensListOverflows, 1, c->d_work);
    return hip_check(c, hipGetLastError(), "density arguments");
}

sph_status forces_prepare(sph_ctx *c, int64_t n)
{
    ForceArgs a{};
    fill_common(c, n, a);
    a.x = c->s.x; a.y = c->s.y; a.z = c->s.z;
    a.h = c->s.h;
    a.rec = c->s.frec;
    a.rec32 = c->p.precision == SPH_FP32_PAIR ? c->s.frec32 : nullptr;
    a.fx = c->s.fx; a.fy = c->s.fy; a.fz = c->s.fz;
    a.ax = c->s.ax; a.ay = c->s.ay; a.az = c->s.az; a.du = c->s.du;
    a.vsig = c->s.vsig; a.dt = c->s.dt; a.nforce = c->s.nforce;
    a.status = c->d_status;
    a.counts = c->d_counts;
    a.alpha = c->p.alpha_av; a.beta = c->p.beta_av; a.ccfl = c->p.c_cfl;
    a.alpha_ac = c->p.alpha_ac;
    a.u_per_c2 = 1.0 / (c->p.gamma * (c->p.gamma - 1.0));
    a.inv_gamma = 1.0 / c->p.gamma;
    a.ac_price = c->p.ac_signal == SPH_AC_PRICE ? 1 : 0;
    a.alpha_p = c->f_alpha;
    a.omega = c->s.omega;
    a.active = c->f_act;
    a.leaf_act = c->f_act ? c->leaf_act : nullptr;
    a.leaf_list = c->f_act ? c->act_list : nullptr;
    a.leaf_count = c->f_act ? c->act_cnt : nullptr;
    if (c->f_block) {
        a.lev = c->s.lev;
        a.lmx = c->s.lmx;
        a.mark = c->s.mark;
        a.lim = c->p.block_lim;
    }
    a.divv = c->f_div ? c->s.divv : nullptr;
    a.curlv = c->f_div ? c->s.curlv : nullptr;
    a.count_tests = c->count_tests ? 1 : 0;
    const void *req[] = {a.nodes, a.x, a.y, a.z, a.h, a.rec, a.ax, a.ay, a.az, a.du, a.vsig,
                         a.dt, a.nforce, a.status, a.counts, a.tree, a.lstart, a.work,
                         c->d_fargs};
    for (const void *q : req)
        if (!q) return fail(c, SPH_EINVAL, "forces: internal buffer not allocated");
    if (c->p.precision == SPH_FP32_PAIR && (!a.fx || !a.fy || !a.fz || !a.rec32))
        return fail(c, SPH_EINVAL, "forces: offsets not allocated");
    if (c->tree_n != n || n <= 0) return fail(c, SPH_ESTATE, "forces: tree not built");
    hipLaunchKernelGGL(k_prologue<ForceArgs>, dim3(1), dim3(64), 0, c->stream, a,
                       (ForceArgs *)c->d_fargs, c->d_counts, (int)kCntForceFirst,
                       (int)kCntForceWords, 0, 0, c->d_work);
    return hip_check(c, hipGetLastError(), "force arguments");
}

// One persistent launch over the prepared sets cs[0..count) (same stream,
// same precision, leaf size, smoothing kernel and launch shape, count <=
// kMaxBatch).
sph_status density_launch(sph_ctx *const *cs, int count, int64_t nmax)
{
    if (count <= 0) return SPH_OK;
    sph_ctx *c = cs[0];
    if (count > kMaxBatch) return fail(c, SPH_EINVAL, "batch larger than kMaxBatch");
    Batch<DensArgs> B{};
    B.nreq = count;
    B.claim = c->p.claim_leaves > 0 ? c->p.claim_leaves : 1;
    B.stage = c->p.stage_leaves;
    B.work = c->d_work;
    int64_t leaves_bound = 0;
    for (int r = 0; r < count; r++) {
        B.req[r] = (const DensArgs *)cs[r]->d_dargs;
        leaves_bound += cs[r]->n;
    }
    if (leaves_bound > (int64_t)0xFFFFFFFFll)
        return fail(c, SPH_EINVAL, "a batch holds more than 2^32 - 1 particles");
    (void)nmax;
    unsigned grid = pair_grid(leaves_bound);
    // the candidate lists of the set whose scratch serves the most blocks at
    // this leaf size; the grid never exceeds it
    const sph_ctx *owner = nullptr;
    for (int r = 0; r < count; r++)
        if (cs[r]->cache && (!owner || cs[r]->cache_size > owner->cache_size)) owner = cs[r];
    const int64_t blocks =
        owner ? owner->cache_size / cache_bytes(c->p.leaf_size, c->p.kernel, 1) : 0;
    if (blocks < kXcds) return fail(c, SPH_ESTATE, "density: no candidate-list scratch");
    B.cache = owner->cache;
    if ((int64_t)grid > blocks) grid = (unsigned)(blocks / kXcds * kXcds);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    timer_begin(c, 0, &e0, &e1);
    if (c->p.kernel == SPH_KERNEL_QUINTIC)
        launch_density<SPH_KERNEL_QUINTIC>(c->stream, c->p.leaf_size, c->p.precision, grid, B);
    else
        launch_density<SPH_KERNEL_M4>(c->stream, c->p.leaf_size, c->p.precision, grid, B);
    timer_end(c, 0, e0, e1);
    return hip_check(c, hipGetLastError(), "density kernel");
}

sph_status forces_launch(sph_ctx *const *cs, int count, int64_t nmax)
{
    if (count <= 0) return SPH_OK;
    sph_ctx *c = cs[0];
    if (count > kMaxBatch) return fail(c, SPH_EINVAL, "batch larger than kMaxBatch");
    Batch<ForceArgs> B{};
    B.nreq = count;
    B.claim = c->p.claim_leaves > 0 ? c->p.claim_leaves : 1;
    B.stage = c->p.stage_leaves;
    B.work = c->d_work;
    int64_t leaves_bound = 0;
    for (int r = 0; r < count; r++) {
        B.req[r] = (const ForceArgs *)cs[r]->d_fargs;
        leaves_bound += cs[r]->n;
    }
    if (leaves_bound > (int64_t)0xFFFFFFFFll)
        return fail(c, SPH_EINVAL, "a batch holds more than 2^32 - 1 particles");
    (void)nmax;
    const unsigned grid = pair_grid(leaves_bound);
    bool ac = false, sw = false;
    for (int r = 0; r < count; r++) {
        ac = ac || cs[r]->p.alpha_ac != 0.0;
        sw = sw || cs[r]->f_alpha != nullptr || cs[r]->f_div;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    timer_begin(c, 1, &e0, &e1);
    if (c->p.kernel == SPH_KERNEL_QUINTIC)
        launch_forces<SPH_KERNEL_QUINTIC>(c->stream, c->p.leaf_size, c->p.precision, ac, sw, grid, B);
    else
        launch_forces<SPH_KERNEL_M4>(c->stream, c->p.leaf_size, c->p.precision, ac, sw, grid, B);
    timer_end(c, 1, e0, e1);
    return hip_check(c, hipGetLastError(), "force kernel");
}

sph_status run_density(sph_ctx *c, int64_t n)
{
    if (n == 0) return SPH_OK;
    TRY_(density_prepare(c, n));
    return density_launch(&c, 1, n);
}

sph_status run_forces(sph_ctx *c, int64_t n)
{
    if (n == 0) return SPH_OK;
    TRY_(forces_prepare(c, n));
    return forces_launch(&c, 1, n);
}

sph_status run_mfv(sph_ctx *c, int64_t n, int nf, const double *const *f, double *const *B,
                   double *cond, double *const *grad)
{
    if (n == 0) return SPH_OK;
    if (nf < 0 || nf > kMfvFields) return fail(c, SPH_EINVAL, "mfv: at most 4 fields");
    MfvArgs a{};
    fill_common(c, n, a);
    a.x = c->s.x; a.y = c->s.y; a.z = c->s.z; a.h = c->s.h; a.ndens = c->s.rho;
    a.nf = nf;
    for (int k = 0; k < nf; k++) a.f[k] = f[k];
    for (int k = 0; k < 6; k++) a.B[k] = B[k];
    a.cond = cond;
    for (int k = 0; k < 3 * nf; k++) a.grad[k] = grad[k];
    a.status = c->d_status;
    if (c->tree_n != n) return fail(c, SPH_ESTATE, "mfv: tree not built");
    TRY_(zero_work(c));
    const unsigned grid = pair_grid(n);
    if (c->p.kernel == SPH_KERNEL_QUINTIC)
        launch_mfv<SPH_KERNEL_QUINTIC>(c->stream, c->p.leaf_size, grid, a);
    else
        launch_mfv<SPH_KERNEL_M4>(c->stream, c->p.leaf_size, grid, a);
    return hip_check(c, hipGetLastError(), "mfv kernel");
}

sph_status run_neighbours(sph_ctx *c, int64_t n, int32_t mode, int64_t *counts_sorted,
                          const int64_t *offsets, int32_t *idx, int64_t cap)
{
    if (n == 0) return SPH_OK;
    NgbArgs a{};
    fill_common(c, n, a);
    a.x = c->s.x; a.y = c->s.y; a.z = c->s.z; a.h = c->s.h;
    a.id = c->s.id;
    a.mode = mode;
    a.counts = counts_sorted;
    a.offsets = offsets;
    a.idx = idx;
    a.cap = cap;
    a.status = c->d_status;
    {
        const void *req[] = {a.nodes, a.x, a.y, a.z, a.h, a.id, a.status, a.tree, a.lstart, a.work};
        for (const void *q : req)
            if (!q) return fail(c, SPH_EINVAL, "neighbours: internal buffer not allocated");
        if (!offsets && !counts_sorted) return fail(c, SPH_EINVAL, "neighbours: no counts");
        if (offsets && cap > 0 && !idx) return fail(c, SPH_EINVAL, "neighbours: no idx");
        if (c->tree_n != n) return fail(c, SPH_ESTATE, "neighbours: tree not built");
    }
    const unsigned grid = pair_grid(n);
    const int pass = offsets ? 2 : 1;
    {
        sph_status zs = zero_work(c);
        if (zs != SPH_OK) return zs;
    }
    if (c->p.kernel == SPH_KERNEL_QUINTIC)
        launch_neighbours<SPH_KERNEL_QUINTIC>(c->stream, c->p.leaf_size, grid, a, pass);
    else
        launch_neighbours<SPH_KERNEL_M4>(c->stream, c->p.leaf_size, grid, a, pass);
    if (pass == 2)
        hipLaunchKernelGGL(k_sort_lists, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream,
                           n, offsets, idx, cap);
    return hip_check(c, hipGetLastError(), "neighbour kernel");
}

} // namespace sph
