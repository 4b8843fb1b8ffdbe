// C ABI of libsph: context lifetime, memory plan, argument checks and the
// order in which each entry point enqueues the kernels.
#include "sph_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>

namespace sph {

sph_status fail(sph_ctx *c, sph_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

sph_status hip_check(sph_ctx *c, hipError_t e, const char *what)
{
    if (e == hipSuccess) return SPH_OK;
    return fail(c, SPH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

// per-particle device bytes of everything sized by the capacity
constexpr int64_t bytes_per_particle()
{
    int64_t b = 0;
    b += 2 * 8 + 2 * 4;        // sort keys / values, ping-pong
    b += 17 * 8 + 2 * 4 + 4;   // s: doubles, nngb/nforce, id
    b += (int64_t)sizeof(ForceRec);   // s: force records
    b += (int64_t)sizeof(ForceRec32); // s: their single-precision copies
    b += 4 * 8;                // s: predictor arrays
    b += 6 * 8;                // s: viscosity switches (alpha, predictor, rate, div v of
                               //    the last step, div v, |curl v|)
    b += 3 * 4;                // s: fp32 offsets
    b += 16 * 8 + 4;           // t: re-sort buffers
    b += 2 * 4;                // leaf starts, leaf of each particle
    b += 4 + 2 * 8 + 5 * 8 + 3 * 4;   // s: block time-steps (level, step ticks, half-step v, u,
                                      //    alpha, active flag, limiter level and mark)
    b += 8 * 8 + 4 + 2 * 8;    // t: block re-sort (a, du, rho, Omega, dt, vsig, level, ticks)
    b += 4;                    // active particles per leaf
    b += 4;                    // active leaves (the list; the tile counts are counted apart)
    return b;
}


sph_status check_params(sph_ctx *c, const sph_params *p)
{
    if (!p) return fail(c, SPH_EINVAL, "params is NULL");
    if (!(p->eta > 0.0) || !(p->gamma > 1.0) || !(p->alpha_av >= 0.0) || !(p->beta_av >= 0.0) ||
        !(p->c_cfl > 0.0) || !(p->h_rtol > 0.0) || p->h_max_iter < 1)
        return fail(c, SPH_EINVAL, "invalid method parameter");
    if (p->precision != SPH_FP64 && p->precision != SPH_FP32_PAIR)
        return fail(c, SPH_EINVAL, "precision must be SPH_FP64 or SPH_FP32_PAIR");
    if (p->leaf_size != 8 && p->leaf_size != 16 && p->leaf_size != 32)
        return fail(c, SPH_EINVAL, "leaf_size must be 8, 16 or 32");
    if (!(p->alpha_ac >= 0.0) || !std::isfinite(p->alpha_ac))
        return fail(c, SPH_EINVAL, "alpha_ac must be finite and >= 0");
    if (p->ac_signal != SPH_AC_WADSLEY && p->ac_signal != SPH_AC_PRICE)
        return fail(c, SPH_EINVAL, "ac_signal must be SPH_AC_WADSLEY or SPH_AC_PRICE");
    if (p->kernel != SPH_KERNEL_M4 && p->kernel != SPH_KERNEL_QUINTIC)
        return fail(c, SPH_EINVAL, "kernel must be SPH_KERNEL_M4 or SPH_KERNEL_QUINTIC");
    if (p->stage_leaves < 0 || p->stage_leaves > 2 * kWave / p->leaf_size)
        return fail(c, SPH_EINVAL, "stage_leaves must be 0..128/leaf_size");
    if (p->claim_leaves < 0 || p->claim_leaves > 64)
        return fail(c, SPH_EINVAL, "claim_leaves must be 0..64");
    if (p->block_lmax < 0 || p->block_lmax > 40 || p->block_lim < 0)
        return fail(c, SPH_EINVAL, "need 0 <= block_lmax <= 40 and block_lim >= 0");
    if (p->av_switch != SPH_AV_NONE && p->av_switch != SPH_AV_MM97 && p->av_switch != SPH_AV_CD10)
        return fail(c, SPH_EINVAL, "av_switch must be SPH_AV_NONE, SPH_AV_MM97 or SPH_AV_CD10");
    if (!(p->alpha_min >= 0.0) || !(p->alpha_max >= p->alpha_min) || !std::isfinite(p->alpha_max) ||
        !(p->av_ell >= 0.0) || !std::isfinite(p->av_ell))
        return fail(c, SPH_EINVAL, "need 0 <= alpha_min <= alpha_max (finite) and av_ell >= 0");
    if (p->periodic)
        for (int a = 0; a < 3; a++)
            if (!(p->box_hi[a] > p->box_lo[a]) || !std::isfinite(p->box_hi[a] - p->box_lo[a]))
                return fail(c, SPH_EINVAL, "periodic box must have box_hi > box_lo");
    return SPH_OK;
}

void set_box(sph_ctx *c)
{
    Box &b = c->box;
    b.periodic = c->p.periodic ? 1 : 0;
    for (int a = 0; a < 3; a++) {
        b.lo[a] = c->p.box_lo[a];
        b.len[a] = c->p.box_hi[a] - c->p.box_lo[a];
        b.half[a] = 0.5 * b.len[a];
    }
}

// release the captured step graph, if any
void drop_graph(sph_ctx *c)
{
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

void free_all(sph_ctx *c)
{
    // a captured graph refers to the buffers about to be freed
    drop_graph(c);
    for (void *ptr : c->allocs) (void)hipFree(ptr);
    c->allocs.clear();
    if (c->cache) (void)hipFree(c->cache);
    c->nodes = nullptr;
    c->hist = nullptr;
    c->cache = nullptr;
    c->cache_size = 0;
    c->ncap = 0;
    c->node_cap = 0;
    c->hist_cap = 0;
    c->s = Sorted{};
    c->t = Sorted{};
    c->keys[0] = c->keys[1] = nullptr;
    c->vals[0] = c->vals[1] = nullptr;
    c->perm = nullptr;
    c->skeys = nullptr;
    c->scratch_u32 = nullptr;
    c->lstart = nullptr;
    c->leaf_id = nullptr;
    c->tree_n = -1;
    c->bytes = 4096;   // fixed buffers (status, scalars, box, partials, tree info)
    c->built = false;
    c->resident = false;
}

template <class T>
sph_status alloc(sph_ctx *c, T **ptr, int64_t count)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, SPH_ENOMEM, "hipMalloc failed");
    }
    c->allocs.push_back(p);
    c->bytes += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    *ptr = (T *)p;
    return SPH_OK;
}

} // namespace

// The density loop's candidate-list scratch: enough bytes for the pair grid
// of the current capacity at the current leaf size.  It only grows, so a
// context that alternates between leaf sizes (the autotuner may change it per
// request) does not reallocate.
static sph_status ensure_cache(sph_ctx *c)
{
    const int64_t bytes = cache_bytes(c->p.leaf_size, c->p.kernel, pair_grid(c->ncap));
    if (c->cache && c->cache_size >= bytes) return SPH_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "hipStreamSynchronize");
    if (c->cache) {
        // a captured graph refers to the scratch about to be freed
        drop_graph(c);
        (void)hipFree(c->cache);
        c->bytes -= (size_t)c->cache_size;
        c->cache = nullptr;
        c->cache_size = 0;
    }
    if (c->budget && c->bytes + (size_t)bytes > c->budget)
        return fail(c, SPH_EBUDGET, "candidate-list scratch of " + std::to_string(bytes) +
                                        " bytes exceeds the HBM budget");
    e = hipMalloc((void **)&c->cache, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->cache = nullptr;
        return fail(c, SPH_ENOMEM, "hipMalloc failed (candidate lists)");
    }
    c->bytes += (size_t)bytes;
    c->cache_size = bytes;
    return SPH_OK;
}

// Every buffer sized by the particle capacity, in one list shared by the
// allocating path (one hipMalloc per buffer) and the no-allocation entry point
// (slices of a static device array): take(&ptr, count) provides count
// elements for ptr.  The density loop's candidate lists are not in the list
// (the allocating path sizes them by leaf size, ensure_cache).
template <class Take>
sph_status lay_out(sph_ctx *c, int64_t cap, Take take)
{
    sph_status s = SPH_OK;
    Sorted &S = c->s, &T = c->t;
#define A_(ptr, cnt) if (s == SPH_OK) s = take(&(ptr), (cnt))
    A_(c->keys[0], cap); A_(c->keys[1], cap);
    A_(c->vals[0], cap); A_(c->vals[1], cap);
    double **sd[] = {&S.x, &S.y, &S.z, &S.vx, &S.vy, &S.vz, &S.m, &S.u, &S.h, &S.rho, &S.omega,
                     &S.ax, &S.ay, &S.az, &S.du, &S.vsig, &S.dt,
                     &S.vpx, &S.vpy, &S.vpz, &S.up,
                     &S.al, &S.alp, &S.adot, &S.dprev, &S.divv, &S.curlv,
                     &T.x, &T.y, &T.z, &T.vx, &T.vy, &T.vz, &T.m, &T.u, &T.h,
                     &T.vpx, &T.vpy, &T.vpz, &T.up, &T.al, &T.alp, &T.dprev};
    for (double **pp : sd) A_(*pp, cap);
    A_(S.frec, cap);
    A_(S.frec32, cap);
    A_(S.nngb, cap); A_(S.nforce, cap);
    A_(S.id, cap); A_(T.id, cap);
    A_(S.fx, cap); A_(S.fy, cap); A_(S.fz, cap);
    A_(c->lstart, cap + 1); A_(c->leaf_id, cap);
    double **bd[] = {&S.vhx, &S.vhy, &S.vhz, &S.uh, &S.alh, &T.ax, &T.ay, &T.az, &T.du, &T.rho,
                     &T.omega, &T.dt, &T.vsig};
    for (double **pp : bd) A_(*pp, cap);
    A_(S.lev, cap); A_(T.lev, cap);
    A_(S.ts, cap); A_(S.te, cap); A_(T.ts, cap); A_(T.te, cap);
    A_(S.act, cap); A_(S.lmx, cap); A_(S.mark, cap);
    A_(c->leaf_act, cap);
    A_(c->act_list, cap);
    A_(c->act_tile, act_tiles(cap));
    A_(c->act_cnt, 1);
    A_(c->nodes, node_count_bound(cap));
    A_(c->hist, hist_words(cap));
#undef A_
    if (s != SPH_OK) return s;
    c->node_cap = node_count_bound(cap);
    c->hist_cap = hist_words(cap);
    c->ncap = cap;
    return SPH_OK;
}

sph_status ensure_capacity(sph_ctx *c, int64_t n)
{
    if (n > (int64_t)0xFFFFFFF0ll) return fail(c, SPH_EINVAL, "n exceeds 2^32 - 16");
    if (n <= c->ncap && node_count_bound(n) <= c->node_cap) return ensure_cache(c);
    int64_t cap = std::max<int64_t>(n, 1024);
    int64_t need = bytes_per_particle() * cap + node_count_bound(cap) * (int64_t)sizeof(Node) +
                   4 * hist_words(cap) + 4096 +
                   cache_bytes(c->p.leaf_size, c->p.kernel, pair_grid(cap));
    if (c->budget && (size_t)need > c->budget)
        return fail(c, SPH_EBUDGET, "working set of " + std::to_string(need) +
                                        " bytes exceeds the HBM budget of " +
                                        std::to_string(c->budget));
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "hipStreamSynchronize");
    bool was_resident = c->resident;
    free_all(c);
    if (was_resident) return fail(c, SPH_ESTATE, "resident state lost on reallocation");
    sph_status s = lay_out(c, cap, [c](auto **ptr, int64_t count) { return alloc(c, ptr, count); });
    if (s != SPH_OK) { free_all(c); return s; }
    return ensure_cache(c);
}

void timer_begin(sph_ctx *c, int which, hipEvent_t *b, hipEvent_t *e)
{
    *b = *e = nullptr;
    if (!c->timer.on) return;
    auto &pool = c->timer.pool;
    if (pool.empty()) {
        hipEvent_t x, y;
        if (hipEventCreate(&x) != hipSuccess) return;
        if (hipEventCreate(&y) != hipSuccess) { (void)hipEventDestroy(x); return; }
        pool.push_back({x, y});
    }
    auto pr = pool.back();
    pool.pop_back();
    *b = pr.first;
    *e = pr.second;
    (void)which;
    (void)hipEventRecord(*b, c->stream);
}

void timer_end(sph_ctx *c, int which, hipEvent_t b, hipEvent_t e)
{
    if (!b) return;
    (void)hipEventRecord(e, c->stream);
    c->timer.pending[which].push_back({b, e});
}

} // namespace sph

using namespace sph;

namespace {

sph_status check_ps(sph_ctx *c, const sph_particles *ps)
{
    if (!c) return SPH_EINVAL;
    if (!ps) return fail(c, SPH_EINVAL, "particles is NULL");
    if (ps->n < 0) return fail(c, SPH_EINVAL, "n < 0");
    return SPH_OK;
}

#define REQ(ptr, name)                                                          \
    do {                                                                        \
        if (ps->n > 0 && !(ptr)) return fail(c, SPH_EINVAL, name " is NULL");  \
    } while (0)

#define TRY(expr)                        \
    do {                                 \
        sph_status st_ = (expr);         \
        if (st_ != SPH_OK) return st_;   \
    } while (0)

sph_status build_from(sph_ctx *c, const sph_particles *ps, bool with_m)
{
    const int64_t n = ps->n;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    timer_begin(c, 2, &e0, &e1);
    TRY(build_order(c, n, ps->x, ps->y, ps->z));
    GatherList g{};
    const void *src[] = {ps->x, ps->y, ps->z, ps->h, ps->m};
    void *dst[] = {c->s.x, c->s.y, c->s.z, c->s.h, c->s.m};
    g.count = with_m ? 5 : 4;
    for (int a = 0; a < g.count; a++) { g.kind[a] = 0; g.src[a] = src[a]; g.dst[a] = dst[a]; }
    TRY(gather(c, n, g, false));
    TRY(build_tree(c, n));
    timer_end(c, 2, e0, e1);
    c->built = true;
    c->built_x = ps->x;
    c->built_n = n;
    return SPH_OK;
}

} // namespace

// ---- phases shared by the single and the batched entry points --------------

namespace {

sph_status density_pre(sph_ctx *c, const sph_particles *ps)
{
    TRY(check_ps(c, ps));
    REQ(ps->x, "x"); REQ(ps->y, "y"); REQ(ps->z, "z"); REQ(ps->m, "m"); REQ(ps->h, "h");
    REQ(ps->rho, "rho"); REQ(ps->omega, "omega");
    if ((ps->pressure || ps->cs)) REQ(ps->u, "u");
    c->resident = false;
    const int64_t n = ps->n;
    TRY(ensure_capacity(c, n));
    c->n = n;
    if (n == 0) return SPH_OK;
    TRY(build_from(c, ps, true));
    return density_prepare(c, n);
}

sph_status density_post(sph_ctx *c, const sph_particles *ps)
{
    const int64_t n = ps->n;
    if (n == 0) return SPH_OK;
    ScatterList sl{};
    const void *src[] = {c->s.h, c->s.rho, c->s.omega, c->s.nngb};
    void *dst[] = {ps->h, ps->rho, ps->omega, ps->nngb};
    int kinds[] = {0, 0, 0, 1};
    for (int a = 0; a < 4; a++) {
        if (!dst[a]) continue;
        sl.kind[sl.count] = kinds[a];
        sl.src[sl.count] = src[a];
        sl.dst[sl.count] = dst[a];
        sl.count++;
    }
    TRY(scatter(c, n, sl, c->perm));
    return eos_scatter(c, n, c->perm, ps->u, ps->pressure, ps->cs);
}

sph_status forces_pre(sph_ctx *c, const sph_particles *ps)
{
    TRY(check_ps(c, ps));
    REQ(ps->x, "x"); REQ(ps->y, "y"); REQ(ps->z, "z");
    REQ(ps->vx, "vx"); REQ(ps->vy, "vy"); REQ(ps->vz, "vz");
    REQ(ps->m, "m"); REQ(ps->u, "u"); REQ(ps->h, "h"); REQ(ps->rho, "rho"); REQ(ps->omega, "omega");
    REQ(ps->ax, "ax"); REQ(ps->ay, "ay"); REQ(ps->az, "az"); REQ(ps->dudt, "dudt");
    REQ(ps->vsig, "vsig"); REQ(ps->dt, "dt");
    const int64_t n = ps->n;
    // the sort order of the last build is reused for the same arrays; the
    // positions are gathered again, so the tree always matches them
    bool reuse = c->built && !c->resident && c->built_x == ps->x && c->built_n == n;
    c->resident = false;
    TRY(ensure_capacity(c, n));
    c->n = n;
    if (n == 0) return SPH_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!reuse) {
        TRY(build_order(c, n, ps->x, ps->y, ps->z));
        c->built = true;
        c->built_x = ps->x;
        c->built_n = n;
    }
    timer_begin(c, 2, &e0, &e1);
    GatherList g{};
    const void *src[] = {ps->x, ps->y, ps->z, ps->m, ps->h, ps->rho, ps->omega, ps->u,
                         ps->vx, ps->vy, ps->vz, ps->alpha};
    void *dst[] = {c->s.x, c->s.y, c->s.z, c->s.m, c->s.h, c->s.rho, c->s.omega, c->s.u,
                   c->s.vx, c->s.vy, c->s.vz, c->s.al};
    g.count = ps->alpha ? 12 : 11;
    for (int a = 0; a < g.count; a++) { g.kind[a] = 0; g.src[a] = src[a]; g.dst[a] = dst[a]; }
    TRY(gather(c, n, g, false));
    c->f_alpha = ps->alpha ? c->s.al : nullptr;
    c->f_div = ps->divv || ps->curlv;
    TRY(build_tree(c, n));
    timer_end(c, 2, e0, e1);
    TRY(force_prep(c, n, c->s.u, c->s.vx, c->s.vy, c->s.vz));
    return forces_prepare(c, n);
}

sph_status forces_post(sph_ctx *c, const sph_particles *ps)
{
    const int64_t n = ps->n;
    if (n == 0) return SPH_OK;
    ScatterList sl{};
    const void *ss[] = {c->s.ax, c->s.ay, c->s.az, c->s.du, c->s.vsig, c->s.dt, c->s.nforce,
                        c->s.divv, c->s.curlv};
    void *sd[] = {ps->ax, ps->ay, ps->az, ps->dudt, ps->vsig, ps->dt, ps->nforce, ps->divv,
                  ps->curlv};
    int kinds[] = {0, 0, 0, 0, 0, 0, 1, 0, 0};
    for (int a = 0; a < 9; a++) {
        if (!sd[a]) continue;
        sl.kind[sl.count] = kinds[a];
        sl.src[sl.count] = ss[a];
        sl.dst[sl.count] = sd[a];
        sl.count++;
    }
    TRY(scatter(c, n, sl, c->perm));
    TRY(reduce_dt(c, n));
    return reduce_diag(c, n);
}

// resident state, first half of a step: kicks, drift, re-sort, tree, density arguments
sph_status step_pre(sph_ctx *c, double dt)
{
    if (!c->resident) return fail(c, SPH_ESTATE, "sph_step needs sph_upload_state first");
    if (!std::isfinite(dt)) return fail(c, SPH_EINVAL, "dt is not finite");
    const int64_t n = c->n;
    TRY(kick_drift(c, n, dt));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    timer_begin(c, 2, &e0, &e1);
    TRY(build_order(c, n, c->s.x, c->s.y, c->s.z));
    GatherList g{};
    Sorted &S = c->s, &T = c->t;
    double **sa[] = {&S.x, &S.y, &S.z, &S.vx, &S.vy, &S.vz, &S.m, &S.u, &S.h,
                     &S.vpx, &S.vpy, &S.vpz, &S.up, &S.al, &S.alp, &S.dprev};
    double **ta[] = {&T.x, &T.y, &T.z, &T.vx, &T.vy, &T.vz, &T.m, &T.u, &T.h,
                     &T.vpx, &T.vpy, &T.vpz, &T.up, &T.al, &T.alp, &T.dprev};
    // the switch state moves with the particles: alpha, its predictor (MM97),
    // div v of the last step (CD10)
    const int nd = !c->res_alpha ? 13 : (c->p.av_switch == SPH_AV_MM97 ? 15
                                         : (c->p.av_switch == SPH_AV_CD10 ? 16 : 14));
    for (int a = 0; a < nd; a++) { g.kind[a] = 0; g.src[a] = *sa[a]; g.dst[a] = *ta[a]; }
    g.kind[nd] = 1; g.src[nd] = S.id; g.dst[nd] = T.id;
    g.count = nd + 1;
    TRY(gather(c, n, g, false));
    for (int a = 0; a < nd; a++) std::swap(*sa[a], *ta[a]);
    std::swap(S.id, T.id);
    TRY(build_tree(c, n));
    timer_end(c, 2, e0, e1);
    return density_prepare(c, n);
}

// the per-particle alpha the resident force loop uses: the predictor under
// MM97, the alpha of the start of the step under CD10 (or a constant one
// given at upload)
void resident_force_inputs(sph_ctx *c)
{
    c->f_alpha = !c->res_alpha ? nullptr : (c->p.av_switch == SPH_AV_MM97 ? c->s.alp : c->s.al);
    c->f_div = c->p.av_switch != SPH_AV_NONE;
}

sph_status step_mid(sph_ctx *c)
{
    const int64_t n = c->n;
    resident_force_inputs(c);
    // the force walk needs the boxes' largest h after the h solve
    TRY(refresh_hmax(c, n));
    TRY(force_prep(c, n, c->s.up, c->s.vpx, c->s.vpy, c->s.vpz));
    return forces_prepare(c, n);
}

sph_status step_post(sph_ctx *c, double dt, double *dt_used)
{
    const int64_t n = c->n;
    // viscosity switches from this step's forces: the MM97 rate (for the
    // closing kick), the CD10 update
    TRY(av_rate(c, n, c->s.alp));
    TRY(av_cd10(c, n, false));
    TRY(closing_kick(c, n, dt));
    TRY(reduce_dt(c, n));
    TRY(reduce_diag(c, n));
    c->steps++;
    c->dt_used_out = dt_used;
    return SPH_OK;
}

// Run the pair launches of a batch: group the sets by (precision, leaf size,
// smoothing kernel, launch shape) and launch each group in chunks of
// kMaxBatch.
template <class Launch>
sph_status launch_groups(sph_ctx *const *cs, int count, Launch launch)
{
    std::vector<sph_ctx *> grp;
    std::vector<bool> done((size_t)count, false);
    for (int a = 0; a < count; a++) {
        if (done[a] || cs[a]->n == 0) continue;
        grp.clear();
        for (int b = a; b < count; b++) {
            if (done[b] || cs[b]->n == 0) continue;
            if (cs[b]->p.precision == cs[a]->p.precision && cs[b]->p.leaf_size == cs[a]->p.leaf_size &&
                cs[b]->p.kernel == cs[a]->p.kernel &&
                cs[b]->p.stage_leaves == cs[a]->p.stage_leaves &&
                cs[b]->p.claim_leaves == cs[a]->p.claim_leaves) {
                grp.push_back(cs[b]);
                done[b] = true;
            }
        }
        for (size_t k = 0; k < grp.size(); k += kMaxBatch) {
            int cnt = (int)std::min<size_t>(kMaxBatch, grp.size() - k);
            TRY(launch(grp.data() + k, cnt));
        }
    }
    return SPH_OK;
}

sph_status check_batch(sph_ctx *const *cs, int32_t count)
{
    if (!cs || count < 0) return SPH_EINVAL;
    for (int r = 0; r < count; r++)
        if (!cs[r]) return SPH_EINVAL;
    for (int r = 1; r < count; r++) {
        if (cs[r]->stream != cs[0]->stream || cs[r]->device != cs[0]->device)
            return fail(cs[r], SPH_EINVAL, "batched contexts must share one device and one stream");
        for (int q = 0; q < r; q++)
            if (cs[q] == cs[r]) return fail(cs[r], SPH_EINVAL, "a context appears twice in a batch");
    }
    return SPH_OK;
}

// sph_evaluate in phases shared with the batched call: sort, gather and
// tree, density arguments / leaf hmax, force records and force arguments /
// scatter of every output.
sph_status evaluate_pre(sph_ctx *c, const sph_particles *ps, bool laid_out = false)
{
    TRY(check_ps(c, ps));
    REQ(ps->x, "x"); REQ(ps->y, "y"); REQ(ps->z, "z");
    REQ(ps->vx, "vx"); REQ(ps->vy, "vy"); REQ(ps->vz, "vz");
    REQ(ps->m, "m"); REQ(ps->u, "u"); REQ(ps->h, "h"); REQ(ps->rho, "rho"); REQ(ps->omega, "omega");
    REQ(ps->ax, "ax"); REQ(ps->ay, "ay"); REQ(ps->az, "az"); REQ(ps->dudt, "dudt");
    REQ(ps->vsig, "vsig"); REQ(ps->dt, "dt");
    c->resident = false;
    const int64_t n = ps->n;
    if (!laid_out) TRY(ensure_capacity(c, n));
    c->n = n;
    if (n == 0) return SPH_OK;
    // one sort and one gather of every input; the sorted set stays on the
    // device from the density loop to the force loop
    hipEvent_t e0 = nullptr, e1 = nullptr;
    timer_begin(c, 2, &e0, &e1);
    TRY(build_order(c, n, ps->x, ps->y, ps->z));
    GatherList g{};
    const void *src[] = {ps->x, ps->y, ps->z, ps->h, ps->m, ps->u, ps->vx, ps->vy, ps->vz,
                         ps->alpha};
    void *dst[] = {c->s.x, c->s.y, c->s.z, c->s.h, c->s.m, c->s.u, c->s.vx, c->s.vy, c->s.vz,
                   c->s.al};
    g.count = ps->alpha ? 10 : 9;
    for (int a = 0; a < g.count; a++) { g.kind[a] = 0; g.src[a] = src[a]; g.dst[a] = dst[a]; }
    TRY(gather(c, n, g, false));
    c->f_alpha = ps->alpha ? c->s.al : nullptr;
    c->f_div = ps->divv || ps->curlv;
    TRY(build_tree(c, n));
    timer_end(c, 2, e0, e1);
    c->built = true;
    c->built_x = ps->x;
    c->built_n = n;
    return density_prepare(c, n);
}

sph_status evaluate_mid(sph_ctx *c)
{
    const int64_t n = c->n;
    if (n == 0) return SPH_OK;
    // the force walk needs the boxes' largest h after the h solve
    TRY(refresh_hmax(c, n));
    TRY(force_prep(c, n, c->s.u, c->s.vx, c->s.vy, c->s.vz));
    return forces_prepare(c, n);
}

sph_status evaluate_post(sph_ctx *c, const sph_particles *ps)
{
    const int64_t n = ps->n;
    if (n == 0) return SPH_OK;
    // every output in one pass over the permutation, the equation of state
    // from the sorted rho and u (the same values sph_density scatters)
    ScatterList sl{};
    const void *src[] = {c->s.h, c->s.rho, c->s.omega, c->s.nngb, c->s.ax, c->s.ay, c->s.az,
                         c->s.du, c->s.vsig, c->s.dt, c->s.nforce, c->s.divv, c->s.curlv};
    void *dst[] = {ps->h, ps->rho, ps->omega, ps->nngb, ps->ax, ps->ay, ps->az, ps->dudt,
                   ps->vsig, ps->dt, ps->nforce, ps->divv, ps->curlv};
    const int kinds[] = {0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 1, 0, 0};
    for (int a = 0; a < 13; a++) {
        if (!dst[a]) continue;
        sl.kind[sl.count] = kinds[a];
        sl.src[sl.count] = src[a];
        sl.dst[sl.count] = dst[a];
        sl.count++;
    }
    TRY(scatter_eos(c, n, sl, c->perm, c->s.u, ps->pressure, ps->cs));
    TRY(reduce_dt(c, n));
    return reduce_diag(c, n);
}


// ---- the no-allocation entry point ---------------------------------------------
//
// sph_evaluate_noalloc runs sph_evaluate with every capacity-sized buffer
// (sort keys, sorted copies, tree, candidate lists) carved out of one static
// device array instead of the context's own allocations, so the call makes no
// device allocation, free or stream synchronisation.  The array holds the
// buffers of kStaticMaxN particles; the pair kernels' persistent grid is
// capped by the candidate-list slices that fit (kStaticListBlocks at leaf
// size 32 with the M4 kernel; more at smaller leaves, a third as many with
// the quintic's longer lists).  Every call on one device shares that
// device's copy: calls that overlap on a device race.
constexpr int64_t kStaticMaxN = 32768;
constexpr int64_t kStaticListBlocks = 256;

constexpr int64_t static_node_bound(int64_t n)
{
    int64_t cnt = n < 1 ? 1 : n, tot = 0;
    for (;;) {
        tot += cnt;
        if (cnt <= 1) break;
        cnt = (cnt + 7) / 8;
    }
    return tot;
}
// the static array: every buffer of lay_out at capacity kStaticMaxN (256-byte
// aligned slices: 96 buffers at most), and the candidate lists
constexpr int64_t kStaticBytes =
    kStaticMaxN * bytes_per_particle() + static_node_bound(kStaticMaxN) * (int64_t)sizeof(Node) +
    4 * hist_words(kStaticMaxN) + 4 * (act_tiles(kStaticMaxN) + 1) + 96 * 256 +
    kStaticListBlocks * 2 * (int64_t)Kern<SPH_KERNEL_M4>::list * 32 * (int64_t)sizeof(double);

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];
static hipError_t g_scratch_err[64];
static bool g_scratch_done[64];

// The device address of this device's copy of `scratch`, taken once per device
// with that device current (host code never uses the array's name itself).
void init_static_scratch(sph_ctx *c)
{
    c->static_scratch = nullptr;
    if (c->device < 0 || c->device >= 64) {
        c->static_err = "device index out of range for the static scratch table";
        return;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[c->device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_err[c->device] = e;
        g_scratch_ptr[c->device] = e == hipSuccess ? ptr : nullptr;
        if (e != hipSuccess) (void)hipGetLastError();
        g_scratch_done[c->device] = true;
    }
    c->static_scratch = g_scratch_ptr[c->device];
    if (!c->static_scratch)
        c->static_err = std::string("hipGetSymbolAddress(scratch): ") +
                        hipGetErrorString(g_scratch_err[c->device]);
}

// The capacity-sized buffers of a context, saved around a call that points
// them into the static array.
struct SavedBuffers {
    uint64_t *keys[2];
    uint32_t *vals[2];
    uint32_t *hist;
    int64_t hist_cap;
    uint32_t *perm;
    Node *nodes;
    int64_t node_cap;
    uint32_t *lstart, *leaf_id;
    double *cache;
    int64_t cache_size;
    uint64_t *skeys;
    uint32_t *scratch_u32;
    int64_t tree_n, ncap;
    Sorted s, t;
};

SavedBuffers save_buffers(const sph_ctx *c)
{
    return SavedBuffers{{c->keys[0], c->keys[1]}, {c->vals[0], c->vals[1]}, c->hist, c->hist_cap,
                        c->perm, c->nodes, c->node_cap, c->lstart, c->leaf_id, c->cache,
                        c->cache_size, c->skeys, c->scratch_u32, c->tree_n, c->ncap, c->s, c->t};
}

void restore_buffers(sph_ctx *c, const SavedBuffers &b)
{
    c->keys[0] = b.keys[0]; c->keys[1] = b.keys[1];
    c->vals[0] = b.vals[0]; c->vals[1] = b.vals[1];
    c->hist = b.hist; c->hist_cap = b.hist_cap;
    c->perm = b.perm;
    c->nodes = b.nodes; c->node_cap = b.node_cap;
    c->lstart = b.lstart; c->leaf_id = b.leaf_id;
    c->cache = b.cache; c->cache_size = b.cache_size;
    c->skeys = b.skeys; c->scratch_u32 = b.scratch_u32;
    c->tree_n = b.tree_n; c->ncap = b.ncap;
    c->s = b.s; c->t = b.t;
}

// Point every capacity-sized buffer of c into [base, base + kStaticBytes).
sph_status carve_static(sph_ctx *c, unsigned char *base)
{
    int64_t used = 0;
    auto take_bytes = [&](int64_t bytes) -> unsigned char * {
        const int64_t at = (used + 255) & ~(int64_t)255;
        if (at + bytes > kStaticBytes) return nullptr;
        used = at + bytes;
        return base + at;
    };
    sph_status s = lay_out(c, kStaticMaxN, [&](auto **ptr, int64_t count) {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*ptr)>>;
        unsigned char *q = take_bytes(std::max<int64_t>(count, 1) * (int64_t)sizeof(T));
        if (!q) return fail(c, SPH_ENOMEM, "static scratch layout overflow");
        *ptr = (T *)q;
        return SPH_OK;
    });
    if (s != SPH_OK) return s;
    // the candidate lists take the rest, whole per-block slices at this leaf size
    const int64_t at = (used + 255) & ~(int64_t)255;
    const int64_t per = cache_bytes(c->p.leaf_size, c->p.kernel, 1);
    const int64_t blocks = std::min<int64_t>((kStaticBytes - at) / per, kMaxPairBlocks) / kXcds * kXcds;
    if (blocks < kXcds) return fail(c, SPH_ENOMEM, "static scratch holds no candidate lists");
    c->cache = (double *)(base + at);
    c->cache_size = blocks * per;
    return SPH_OK;
}

} // namespace

extern "C" {

void sph_default_params(sph_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eta = 1.2;
    p->gamma = 5.0 / 3.0;
    p->alpha_av = 1.0;
    p->beta_av = 2.0;
    p->c_cfl = 0.2;
    p->h_rtol = 1e-12;
    p->h_max_iter = 50;
    p->periodic = 1;
    for (int a = 0; a < 3; a++) { p->box_lo[a] = 0.0; p->box_hi[a] = 1.0; }
    p->precision = SPH_FP64;
    p->leaf_size = 16;
    p->alpha_ac = 0.0;
    p->ac_signal = SPH_AC_WADSLEY;
    p->av_switch = SPH_AV_NONE;
    p->alpha_min = 0.1;
    p->alpha_max = 1.0;
    p->av_ell = 0.0;
    p->block_lmax = 0;
    p->block_lim = 2;
}

sph_status sph_create(sph_ctx **out, const sph_params *p, void *hip_stream, size_t budget)
{
    if (!out) return SPH_EINVAL;
    *out = nullptr;
    sph_ctx *c = new (std::nothrow) sph_ctx();
    if (!c) return SPH_ENOMEM;
    sph_status s = check_params(c, p);
    if (s != SPH_OK) { delete c; return s; }
    c->p = *p;
    set_box(c);
    c->stream = (hipStream_t)hip_stream;
    c->budget = budget;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return SPH_EDEVICE; }
    init_static_scratch(c);
    bool ok = hipMalloc((void **)&c->d_status, sizeof(int32_t) * kStatusWords) == hipSuccess &&
              hipMalloc((void **)&c->d_scal, sizeof(double) * 16) == hipSuccess &&
              hipMalloc((void **)&c->d_counts, sizeof(int64_t) * kCountWords) == hipSuccess &&
              hipMalloc((void **)&c->d_box, sizeof(double) * 8) == hipSuccess &&
              hipMalloc((void **)&c->d_part, sizeof(double) * 1024 * 8) == hipSuccess &&
              hipMalloc((void **)&c->d_tree, sizeof(TreeInfo)) == hipSuccess &&
              hipMalloc((void **)&c->d_work, sizeof(uint32_t) * 64) == hipSuccess &&
              hipMalloc(&c->d_dargs, kArgBytes) == hipSuccess &&
              hipMalloc(&c->d_fargs, kArgBytes) == hipSuccess &&
              hipMalloc((void **)&c->d_clock, sizeof(BlockClock)) == hipSuccess &&
              hipHostMalloc((void **)&c->h_status, sizeof(int32_t) * kStatusWords) == hipSuccess &&
              hipHostMalloc((void **)&c->h_scal, sizeof(double) * 16) == hipSuccess &&
              hipHostMalloc((void **)&c->h_counts, sizeof(int64_t) * kCountWords) == hipSuccess &&
              hipHostMalloc((void **)&c->h_clock, sizeof(BlockClock)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        sph_destroy(c);
        return SPH_ENOMEM;
    }
    c->bytes = 4096;
    // every operation of a context goes to its own stream: a null-stream
    // memset is not ordered with a non-blocking stream and could land in the
    // middle of the first calls' work
    ok = hipMemsetAsync(c->d_status, 0, sizeof(int32_t) * kStatusWords, c->stream) == hipSuccess &&
         hipMemsetAsync(c->d_scal, 0, sizeof(double) * 16, c->stream) == hipSuccess &&
         hipMemsetAsync(c->d_counts, 0, sizeof(int64_t) * kCountWords, c->stream) == hipSuccess &&
         hipMemsetAsync(c->d_clock, 0, sizeof(BlockClock), c->stream) == hipSuccess &&
         hipStreamSynchronize(c->stream) == hipSuccess;
    if (!ok) { sph_destroy(c); return SPH_EDEVICE; }
    *out = c;
    return SPH_OK;
}

sph_status sph_destroy(sph_ctx *c)
{
    if (!c) return SPH_OK;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    for (int w = 0; w < 3; w++)
        for (auto &pr : c->timer.pending[w]) c->timer.pool.push_back(pr);
    for (auto &pr : c->timer.pool) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    if (c->d_status) (void)hipFree(c->d_status);
    if (c->d_scal) (void)hipFree(c->d_scal);
    if (c->d_counts) (void)hipFree(c->d_counts);
    if (c->d_box) (void)hipFree(c->d_box);
    if (c->d_part) (void)hipFree(c->d_part);
    if (c->d_tree) (void)hipFree(c->d_tree);
    if (c->d_work) (void)hipFree(c->d_work);
    if (c->d_dargs) (void)hipFree(c->d_dargs);
    if (c->d_fargs) (void)hipFree(c->d_fargs);
    if (c->d_clock) (void)hipFree(c->d_clock);
    if (c->h_status) (void)hipHostFree(c->h_status);
    if (c->h_scal) (void)hipHostFree(c->h_scal);
    if (c->h_counts) (void)hipHostFree(c->h_counts);
    if (c->h_clock) (void)hipHostFree(c->h_clock);
    delete c;
    return SPH_OK;
}

sph_status sph_set_stream(sph_ctx *c, void *hip_stream)
{
    if (!c) return SPH_EINVAL;
    // the context's buffers may still be in use on the old stream
    TRY(hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    c->stream = (hipStream_t)hip_stream;
    return SPH_OK;
}

sph_status sph_set_params(sph_ctx *c, const sph_params *p)
{
    if (!c) return SPH_EINVAL;
    TRY(check_params(c, p));
    if (c->graph_exec || c->graph) {
        // captured steps carry the old parameters (argument blocks and kernel
        // variants): let any replay in flight finish, then drop them
        TRY(hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
        drop_graph(c);
    }
    c->p = *p;
    set_box(c);
    // the buffers are sized by the particle capacity alone (the node bound
    // holds for any leaf size; the candidate lists grow on next use if the
    // new leaf size or kernel needs more), so nothing is reallocated here
    c->built = false;
    return SPH_OK;
}

sph_status sph_build_cells(sph_ctx *c, const sph_particles *ps)
{
    TRY(check_ps(c, ps));
    REQ(ps->x, "x"); REQ(ps->y, "y"); REQ(ps->z, "z"); REQ(ps->h, "h");
    c->resident = false;
    TRY(ensure_capacity(c, ps->n));
    c->n = ps->n;
    return build_from(c, ps, ps->m != nullptr);
}

sph_status sph_density(sph_ctx *c, sph_particles *ps)
{
    TRY(density_pre(c, ps));
    if (ps->n == 0) return SPH_OK;
    TRY(density_launch(&c, 1, ps->n));
    return density_post(c, ps);
}

sph_status sph_forces(sph_ctx *c, sph_particles *ps)
{
    TRY(forces_pre(c, ps));
    if (ps->n == 0) return SPH_OK;
    TRY(forces_launch(&c, 1, ps->n));
    return forces_post(c, ps);
}

sph_status sph_evaluate(sph_ctx *c, sph_particles *ps)
{
    TRY(evaluate_pre(c, ps));
    if (ps->n == 0) return SPH_OK;
    TRY(density_launch(&c, 1, ps->n));
    TRY(evaluate_mid(c));
    TRY(forces_launch(&c, 1, ps->n));
    return evaluate_post(c, ps);
}

sph_status sph_evaluate_noalloc(sph_ctx *c, sph_particles *ps)
{
    TRY(check_ps(c, ps));
    if (ps->n > kStaticMaxN)
        return fail(c, SPH_ECAP, "sph_evaluate_noalloc: n = " + std::to_string(ps->n) +
                                     " exceeds its maximum of " + std::to_string(kStaticMaxN));
    if (!c->static_scratch) return fail(c, SPH_EDEVICE, "static scratch: " + c->static_err);
    const SavedBuffers saved = save_buffers(c);
    const bool timing = c->timer.on;
    c->timer.on = false;   // event creation is not allowed here
    sph_status s = carve_static(c, (unsigned char *)c->static_scratch);
    if (s == SPH_OK) s = evaluate_pre(c, ps, true);
    if (s == SPH_OK && ps->n > 0) {
        s = density_launch(&c, 1, ps->n);
        if (s == SPH_OK) s = evaluate_mid(c);
        if (s == SPH_OK) s = forces_launch(&c, 1, ps->n);
        if (s == SPH_OK) s = evaluate_post(c, ps);
    }
    // the context's own buffers are back; the structure built in the static
    // array is not theirs, and (as after sph_evaluate) no state is resident
    restore_buffers(c, saved);
    c->built = false;
    c->resident = false;
    c->timer.on = timing;
    return s;
}

int64_t sph_noalloc_max_n(void) { return kStaticMaxN; }

sph_status sph_batch_evaluate(sph_ctx *const *cs, sph_particles *const *ps, int32_t count)
{
    TRY(check_batch(cs, count));
    if (count > 0 && !ps) return fail(cs[0], SPH_EINVAL, "particles is NULL");
    for (int r = 0; r < count; r++) TRY(evaluate_pre(cs[r], ps[r]));
    TRY(launch_groups(cs, count, [](sph_ctx *const *g, int k) { return density_launch(g, k, 0); }));
    for (int r = 0; r < count; r++) TRY(evaluate_mid(cs[r]));
    TRY(launch_groups(cs, count, [](sph_ctx *const *g, int k) { return forces_launch(g, k, 0); }));
    for (int r = 0; r < count; r++) TRY(evaluate_post(cs[r], ps[r]));
    return SPH_OK;
}

sph_status sph_batch_density(sph_ctx *const *cs, sph_particles *const *ps, int32_t count)
{
    TRY(check_batch(cs, count));
    if (count > 0 && !ps) return fail(cs[0], SPH_EINVAL, "particles is NULL");
    for (int r = 0; r < count; r++) TRY(density_pre(cs[r], ps[r]));
    TRY(launch_groups(cs, count, [](sph_ctx *const *g, int k) { return density_launch(g, k, 0); }));
    for (int r = 0; r < count; r++) TRY(density_post(cs[r], ps[r]));
    return SPH_OK;
}

sph_status sph_batch_forces(sph_ctx *const *cs, sph_particles *const *ps, int32_t count)
{
    TRY(check_batch(cs, count));
    if (count > 0 && !ps) return fail(cs[0], SPH_EINVAL, "particles is NULL");
    for (int r = 0; r < count; r++) TRY(forces_pre(cs[r], ps[r]));
    TRY(launch_groups(cs, count, [](sph_ctx *const *g, int k) { return forces_launch(g, k, 0); }));
    for (int r = 0; r < count; r++) TRY(forces_post(cs[r], ps[r]));
    return SPH_OK;
}

sph_status sph_batch_step(sph_ctx *const *cs, int32_t count, double dt)
{
    TRY(check_batch(cs, count));
    for (int r = 0; r < count; r++)
        if (cs[r]->p.block_lmax > 0)
            return fail(cs[r], SPH_ESTATE, "block time-steps advance with sph_substep");
    for (int r = 0; r < count; r++) TRY(step_pre(cs[r], dt));
    TRY(launch_groups(cs, count, [](sph_ctx *const *g, int k) { return density_launch(g, k, 0); }));
    for (int r = 0; r < count; r++) TRY(step_mid(cs[r]));
    TRY(launch_groups(cs, count, [](sph_ctx *const *g, int k) { return forces_launch(g, k, 0); }));
    for (int r = 0; r < count; r++) TRY(step_post(cs[r], dt, nullptr));
    return SPH_OK;
}

sph_status sph_upload_state(sph_ctx *c, const sph_particles *ps)
{
    TRY(check_ps(c, ps));
    REQ(ps->x, "x"); REQ(ps->y, "y"); REQ(ps->z, "z");
    REQ(ps->vx, "vx"); REQ(ps->vy, "vy"); REQ(ps->vz, "vz");
    REQ(ps->m, "m"); REQ(ps->u, "u"); REQ(ps->h, "h");
    const int64_t n = ps->n;
    c->resident = false;
    TRY(ensure_capacity(c, n));
    c->n = n;
    if (n == 0) return fail(c, SPH_EINVAL, "resident state needs n > 0");
    drop_graph(c);
    TRY(build_order(c, n, ps->x, ps->y, ps->z));
    GatherList g{};
    const void *src[] = {ps->x, ps->y, ps->z, ps->vx, ps->vy, ps->vz, ps->m, ps->u, ps->h,
                         ps->alpha};
    void *dst[] = {c->s.x, c->s.y, c->s.z, c->s.vx, c->s.vy, c->s.vz, c->s.m, c->s.u, c->s.h,
                   c->s.al};
    g.count = ps->alpha ? 10 : 9;
    for (int a = 0; a < g.count; a++) { g.kind[a] = 0; g.src[a] = src[a]; g.dst[a] = dst[a]; }
    TRY(gather(c, n, g, false));
    c->res_alpha = ps->alpha != nullptr || c->p.av_switch != SPH_AV_NONE;
    if (c->res_alpha && !ps->alpha) TRY(fill(c, n, c->s.al, c->p.alpha_av));
    TRY(hip_check(c, hipMemcpyAsync(c->s.id, c->perm, sizeof(uint32_t) * (size_t)n,
                                    hipMemcpyDeviceToDevice, c->stream), "copy ids"));
    TRY(build_tree(c, n));
    TRY(run_density(c, n));
    TRY(refresh_hmax(c, n));
    TRY(force_prep(c, n, c->s.u, c->s.vx, c->s.vy, c->s.vz));
    // the initial forces see the uploaded alpha
    c->f_alpha = c->res_alpha ? c->s.al : nullptr;
    c->f_div = c->p.av_switch != SPH_AV_NONE;
    TRY(run_forces(c, n));
    TRY(av_rate(c, n, c->s.al));
    TRY(av_cd10(c, n, true));
    // block time-steps: first levels, steps and opening kicks
    if (c->p.block_lmax > 0) TRY(block_finish(c, n, true));
    TRY(reduce_dt(c, n));
    TRY(hip_check(c, hipMemsetAsync(c->d_scal + 1, 0, sizeof(double) * 2, c->stream), "reset time"));
    TRY(reduce_diag(c, n));
    c->built = false;
    c->resident = true;
    c->steps = 0;
    return SPH_OK;
}

sph_status sph_step(sph_ctx *c, double dt, double *dt_used)
{
    if (!c) return SPH_EINVAL;
    if (c->p.block_lmax > 0) return fail(c, SPH_ESTATE, "block time-steps advance with sph_substep");
    TRY(step_pre(c, dt));
    TRY(density_launch(&c, 1, c->n));
    TRY(step_mid(c));
    TRY(forces_launch(&c, 1, c->n));
    return step_post(c, dt, dt_used);
}

// Block sub-step in three phases around the two pair launches (so that a
// batch can launch the pair loops of many sets together).
// First: the next tick at which steps end, drift, re-sort, tree, predictors,
// the active set, the density arguments.  The block flags stay set until
// substep_mid (or clear_block_flags on an error in between).
static sph_status substep_pre(sph_ctx *c)
{
    if (!c->resident) return fail(c, SPH_ESTATE, "sph_substep needs sph_upload_state first");
    if (c->p.block_lmax <= 0) return fail(c, SPH_ESTATE, "the context has no block time-steps");
    const int64_t n = c->n;
    Sorted &S = c->s, &T = c->t;
    // next tick at which steps end; every particle drifts to it
    TRY(block_next(c, n));
    // re-sort: everything that persists per particle moves with it
    hipEvent_t e0 = nullptr, e1 = nullptr;
    timer_begin(c, 2, &e0, &e1);
    TRY(build_order(c, n, S.x, S.y, S.z));
    GatherList g{};
    double **sa[] = {&S.x, &S.y, &S.z, &S.vx, &S.vy, &S.vz, &S.m, &S.u, &S.h, &S.vhx, &S.vhy,
                     &S.vhz, &S.uh, &S.ax, &S.ay, &S.az, &S.du, &S.rho, &S.omega, &S.dt, &S.vsig};
    double **ta[] = {&T.x, &T.y, &T.z, &T.vx, &T.vy, &T.vz, &T.m, &T.u, &T.h, &T.vpx, &T.vpy,
                     &T.vpz, &T.up, &T.ax, &T.ay, &T.az, &T.du, &T.rho, &T.omega, &T.dt, &T.vsig};
    const int nd = 21;
    for (int a = 0; a < nd; a++) { g.kind[a] = 0; g.src[a] = *sa[a]; g.dst[a] = *ta[a]; }
    int k = nd;
    g.kind[k] = 1; g.src[k] = S.id; g.dst[k] = T.id; k++;
    g.kind[k] = 1; g.src[k] = S.lev; g.dst[k] = T.lev; k++;
    g.kind[k] = 0; g.src[k] = S.ts; g.dst[k] = T.ts; k++;
    g.kind[k] = 0; g.src[k] = S.te; g.dst[k] = T.te; k++;
    // per-particle alpha and the switch state, through the re-sort buffers
    // the global step uses for them (the predicted alpha is recomputed every
    // sub-step, so its buffer takes the half-step alpha; MM97 keeps no div v
    // of the last step, so that buffer takes the rate)
    const int sw = c->p.av_switch;
    double **xa[3], **xb[3];
    int nx = 0;
    if (c->res_alpha) { xa[nx] = &S.al; xb[nx++] = &T.al; }
    if (sw == SPH_AV_MM97) {
        xa[nx] = &S.alh; xb[nx++] = &T.alp;
        xa[nx] = &S.adot; xb[nx++] = &T.dprev;
    }
    if (sw == SPH_AV_CD10) { xa[nx] = &S.dprev; xb[nx++] = &T.dprev; }
    for (int a = 0; a < nx; a++) { g.kind[k] = 0; g.src[k] = *xa[a]; g.dst[k] = *xb[a]; k++; }
    g.count = k;
    TRY(gather(c, n, g, false));
    for (int a = 0; a < nd; a++) std::swap(*sa[a], *ta[a]);
    for (int a = 0; a < nx; a++) std::swap(*xa[a], *xb[a]);
    std::swap(S.id, T.id);
    std::swap(S.lev, T.lev);
    std::swap(S.ts, T.ts);
    std::swap(S.te, T.te);
    TRY(build_tree(c, n));
    timer_end(c, 2, e0, e1);
    // predictors, the active set and its count per leaf
    TRY(block_predict(c, n));
    c->f_act = S.act;
    c->f_block = true;
    // the forces see every particle's predicted alpha (MM97) or its current
    // one (CD10, or a constant per-particle alpha given at upload)
    resident_force_inputs(c);
    return density_prepare(c, n);
}

static void clear_block_flags(sph_ctx *c)
{
    c->f_act = nullptr;
    c->f_block = false;
}

// Second: after the density loop, the force arguments of the active set.
static sph_status substep_mid(sph_ctx *c)
{
    const int64_t n = c->n;
    Sorted &S = c->s;
    sph_status st = refresh_hmax(c, n);
    if (st == SPH_OK) st = force_prep(c, n, S.up, S.vpx, S.vpy, S.vpz);
    if (st == SPH_OK) st = forces_prepare(c, n);
    clear_block_flags(c);
    return st;
}

// Third: after the force loop, the switches of the active particles, then
// closing kicks, levels, limiter, opening kicks, clock.
static sph_status substep_post(sph_ctx *c)
{
    const int64_t n = c->n;
    TRY(block_av(c, n));
    TRY(block_finish(c, n, false));
    TRY(reduce_diag(c, n));
    c->steps++;
    return SPH_OK;
}

sph_status sph_substep(sph_ctx *c)
{
    if (!c) return SPH_EINVAL;
    sph_status st = substep_pre(c);
    if (st == SPH_OK) st = density_launch(&c, 1, c->n);
    if (st != SPH_OK) {
        clear_block_flags(c);
        return st;
    }
    TRY(substep_mid(c));
    TRY(forces_launch(&c, 1, c->n));
    return substep_post(c);
}

sph_status sph_batch_substep(sph_ctx *const *cs, int32_t count)
{
    TRY(check_batch(cs, count));
    // every context is checked before any is advanced
    for (int r = 0; r < count; r++) {
        if (!cs[r]->resident) return fail(cs[r], SPH_ESTATE, "sph_substep needs sph_upload_state first");
        if (cs[r]->p.block_lmax <= 0)
            return fail(cs[r], SPH_ESTATE, "the context has no block time-steps");
    }
    sph_status st = SPH_OK;
    for (int r = 0; r < count && st == SPH_OK; r++) st = substep_pre(cs[r]);
    if (st == SPH_OK)
        st = launch_groups(cs, count,
                           [](sph_ctx *const *g, int k) { return density_launch(g, k, 0); });
    if (st != SPH_OK) {
        for (int r = 0; r < count; r++) clear_block_flags(cs[r]);
        return st;
    }
    for (int r = 0; r < count && st == SPH_OK; r++) st = substep_mid(cs[r]);
    for (int r = 0; r < count; r++) clear_block_flags(cs[r]);
    TRY(st);
    TRY(launch_groups(cs, count, [](sph_ctx *const *g, int k) { return forces_launch(g, k, 0); }));
    for (int r = 0; r < count; r++) TRY(substep_post(cs[r]));
    return SPH_OK;
}

sph_status sph_capture_steps(sph_ctx *c, double dt)
{
    if (!c) return SPH_EINVAL;
    if (!c->resident) return fail(c, SPH_ESTATE, "capture needs a resident state");
    if (c->p.block_lmax > 0) return fail(c, SPH_ESTATE, "no graph capture of block time-steps");
    if (!c->stream) return fail(c, SPH_EINVAL, "capture needs a non-null stream");
    if (!std::isfinite(dt)) return fail(c, SPH_EINVAL, "dt is not finite");
    drop_graph(c);
    const bool timing = c->timer.on;
    c->timer.on = false;   // no event records inside the graph
    TRY(hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    TRY(hip_check(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal),
                  "hipStreamBeginCapture"));
    const int64_t steps0 = c->steps;
    sph_status st = SPH_OK;
    // two steps: the re-sort alternates between two buffer sets, so after an
    // even number of steps every array is back where the graph expects it
    for (int k = 0; k < 2 && st == SPH_OK; k++) {
        st = step_pre(c, dt);
        if (st == SPH_OK) st = density_launch(&c, 1, c->n);
        if (st == SPH_OK) st = step_mid(c);
        if (st == SPH_OK) st = forces_launch(&c, 1, c->n);
        if (st == SPH_OK) st = step_post(c, dt, nullptr);
    }
    c->steps = steps0;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->timer.on = timing;
    if (st != SPH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_check(c, e, "hipStreamEndCapture");
    c->graph = g;
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(c);
        return hip_check(c, e, "hipGraphInstantiate");
    }
    // move the graph's set-up onto the device now rather than at the first replay
    e = hipGraphUpload(c->graph_exec, c->stream);
    if (e != hipSuccess) {
        drop_graph(c);
        return hip_check(c, e, "hipGraphUpload");
    }
    c->graph_dt = dt;
    return SPH_OK;
}

sph_status sph_replay_steps(sph_ctx *c)
{
    if (!c) return SPH_EINVAL;
    if (!c->graph_exec || !c->resident) return fail(c, SPH_ESTATE, "no captured steps");
    TRY(hip_check(c, hipGraphLaunch(c->graph_exec, c->stream), "hipGraphLaunch"));
    c->steps += 2;
    return SPH_OK;
}

sph_status sph_download_state(sph_ctx *c, sph_particles *ps)
{
    TRY(check_ps(c, ps));
    if (!c->resident) return fail(c, SPH_ESTATE, "no resident state");
    if (ps->n != c->n) return fail(c, SPH_EINVAL, "n differs from the resident state");
    REQ(ps->x, "x"); REQ(ps->y, "y"); REQ(ps->z, "z");
    REQ(ps->vx, "vx"); REQ(ps->vy, "vy"); REQ(ps->vz, "vz"); REQ(ps->u, "u"); REQ(ps->h, "h");
    const int64_t n = c->n;
    ScatterList sl{};
    const void *src[] = {c->s.x, c->s.y, c->s.z, c->s.vx, c->s.vy, c->s.vz, c->s.u, c->s.h,
                         c->s.rho, c->s.omega, c->s.ax, c->s.ay, c->s.az, c->s.du, c->s.vsig,
                         c->s.dt, c->s.nngb, c->s.nforce, c->s.al, c->s.divv, c->s.curlv,
                         c->s.lev};
    void *dst[] = {(void *)ps->x, (void *)ps->y, (void *)ps->z, (void *)ps->vx, (void *)ps->vy,
                   (void *)ps->vz, (void *)ps->u, ps->h, ps->rho, ps->omega, ps->ax, ps->ay,
                   ps->az, ps->dudt, ps->vsig, ps->dt, ps->nngb, ps->nforce,
                   c->res_alpha ? ps->alpha : nullptr,
                   c->p.av_switch != SPH_AV_NONE ? ps->divv : nullptr,
                   c->p.av_switch != SPH_AV_NONE ? ps->curlv : nullptr,
                   c->p.block_lmax > 0 ? ps->level : nullptr};
    for (int a = 0; a < 22; a++) {
        if (!dst[a]) continue;
        sl.kind[sl.count] = (a == 16 || a == 17 || a == 21) ? 1 : 0;
        sl.src[sl.count] = src[a];
        sl.dst[sl.count] = dst[a];
        sl.count++;
    }
    TRY(scatter(c, n, sl, c->s.id));
    TRY(eos_scatter(c, n, c->s.id, ps->u, ps->pressure, ps->cs));
    return SPH_OK;
}

sph_status sph_state_info(sph_ctx *c, sph_state_stats *info)
{
    if (!c || !info) return SPH_EINVAL;
    if (c->n <= 0) return fail(c, SPH_ESTATE, "nothing evaluated yet");
    // scalars, counters and the block clock in pinned mirrors, one wait
    const bool block = c->p.block_lmax > 0 && c->resident;
    TRY(hip_check(c, hipMemcpyAsync(c->h_scal, c->d_scal, sizeof(double) * 8,
                                    hipMemcpyDeviceToHost, c->stream), "copy scalars"));
    TRY(hip_check(c, hipMemcpyAsync(c->h_counts, c->d_counts, sizeof(int64_t) * kCountWords,
                                    hipMemcpyDeviceToHost, c->stream), "copy counts"));
    if (block)
        TRY(hip_check(c, hipMemcpyAsync(c->h_clock, c->d_clock, sizeof(BlockClock),
                                        hipMemcpyDeviceToHost, c->stream), "copy block clock"));
    TRY(hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    const int64_t *counts = c->h_counts;
    std::memset(info, 0, sizeof(*info));
    info->dt_next = c->h_scal[0];
    info->dt_last = c->h_scal[1];
    info->time = c->h_scal[2];
    info->kinetic = c->h_scal[3];
    info->thermal = c->h_scal[4];
    for (int a = 0; a < 3; a++) info->momentum[a] = c->h_scal[5 + a];
    info->steps = c->steps;
    info->n_dens_pairs = counts[kCntNngb];
    info->n_force_pairs = counts[kCntNforce];
    info->dens_pair_evals = counts[kCntDensEvals];
    info->force_pair_evals = counts[kCntForceEvals];
    info->nr_iter_max = (int32_t)counts[kCntNrMax];
    info->walk_overflows = (int32_t)(counts[kCntDensOverflows] + counts[kCntForceOverflows]);
    info->dens_leaf_visits = counts[kCntDensVisits];
    info->dens_walks = counts[kCntDensWalks];
    info->nr_iter_total = counts[kCntNrTotal];
    info->dens_candidate_tests = counts[kCntDensTests];
    info->dens_box_tests = counts[kCntDensBoxes];
    info->force_candidate_tests = counts[kCntForceTests];
    info->force_box_tests = counts[kCntForceBoxes];
    info->density_walk_overflows = (int32_t)counts[kCntDensOverflows];
    info->force_walk_overflows = (int32_t)counts[kCntForceOverflows];
    info->dens_list_overflows = counts[kCntDensListOverflows];
    if (block) {
        const BlockClock clk = *c->h_clock;
        info->block_full_steps = clk.full;
        info->block_substeps = clk.nsub;
        info->block_active = clk.active;
        info->block_updates = clk.updates;
        info->block_time = clk.time;
        info->block_dt_max = clk.dt_max;
        info->block_synchronised = clk.T == 0 ? 1 : 0;
    }
    return SPH_OK;
}

sph_status sph_neighbours(sph_ctx *c, const sph_particles *ps, int32_t mode, int64_t *offsets,
                          int32_t *idx, int64_t cap)
{
    TRY(check_ps(c, ps));
    REQ(ps->x, "x"); REQ(ps->y, "y"); REQ(ps->z, "z"); REQ(ps->h, "h");
    if (!offsets) return fail(c, SPH_EINVAL, "offsets is NULL");
    if (mode != 0 && mode != 1) return fail(c, SPH_EINVAL, "mode must be 0 or 1");
    if (cap < 0 || (cap > 0 && !idx)) return fail(c, SPH_EINVAL, "bad idx / cap");
    const int64_t n = ps->n;
    c->resident = false;
    TRY(ensure_capacity(c, n));
    c->n = n;
    if (n == 0) {
        TRY(hip_check(c, hipMemsetAsync(offsets, 0, sizeof(int64_t), c->stream), "offsets"));
        return hip_check(c, hipStreamSynchronize(c->stream), "sync");
    }
    TRY(build_from(c, ps, false));
    TRY(hip_check(c, hipMemcpyAsync(c->s.id, c->perm, sizeof(uint32_t) * (size_t)n,
                                    hipMemcpyDeviceToDevice, c->stream), "copy ids"));
    int64_t *counts_sorted = (int64_t *)c->s.ax;   // scratch
    TRY(run_neighbours(c, n, mode, counts_sorted, nullptr, nullptr, 0));
    ScatterList sl{};
    sl.count = 1;
    sl.kind[0] = 0;   // 8-byte copy
    sl.src[0] = counts_sorted;
    sl.dst[0] = offsets;
    TRY(scatter(c, n, sl, c->perm));
    TRY(scan_offsets(c, n, offsets));
    int64_t total = 0;
    TRY(hip_check(c, hipStreamSynchronize(c->stream), "sync"));
    TRY(hip_check(c, hipMemcpyAsync(&total, offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                                    c->stream), "copy total"));
    TRY(hip_check(c, hipStreamSynchronize(c->stream), "sync"));
    if (total > cap) return fail(c, SPH_ECAP, "neighbour lists need " + std::to_string(total) +
                                                  " entries, cap is " + std::to_string(cap));
    TRY(run_neighbours(c, n, mode, counts_sorted, offsets, idx, cap));
    return hip_check(c, hipStreamSynchronize(c->stream), "sync");
}

sph_status sph_mfv_gradients(sph_ctx *c, sph_mfv_set *s)
{
    if (!c) return SPH_EINVAL;
    if (!s) return fail(c, SPH_EINVAL, "set is NULL");
    if (s->n < 0) return fail(c, SPH_EINVAL, "n < 0");
    if (s->nfields < 0 || s->nfields > 4) return fail(c, SPH_EINVAL, "nfields must be 0..4");
    const int64_t n = s->n;
    if (n > 0) {
        if (!s->x || !s->y || !s->z || !s->h) return fail(c, SPH_EINVAL, "x, y, z and h are required");
        for (int k = 0; k < s->nfields; k++)
            if (!s->f[k]) return fail(c, SPH_EINVAL, "a field is NULL");
    }
    c->resident = false;
    TRY(ensure_capacity(c, n));
    c->n = n;
    if (n == 0) return SPH_OK;
    Sorted &S = c->s, &T = c->t;
    // sorted homes of the fields (the re-sort buffers are free outside a
    // resident state) and of the outputs (the force-loop outputs are free)
    double *fs[4] = {T.vx, T.vy, T.vz, T.u};
    double *Bs[6] = {S.ax, S.ay, S.az, S.du, S.vsig, S.dt};
    double *gs[12] = {S.vpx, S.vpy, S.vpz, S.up, S.al, S.alp, S.adot, S.dprev, S.curlv,
                      T.x, T.y, T.z};
    double *conds = S.divv;
    TRY(build_order(c, n, s->x, s->y, s->z));
    GatherList g{};
    const void *src[] = {s->x, s->y, s->z, s->h};
    void *dst[] = {S.x, S.y, S.z, S.h};
    for (int a = 0; a < 4; a++) { g.kind[a] = 0; g.src[a] = src[a]; g.dst[a] = dst[a]; }
    g.count = 4;
    for (int k = 0; k < s->nfields; k++) {
        g.kind[g.count] = 0;
        g.src[g.count] = s->f[k];
        g.dst[g.count] = fs[k];
        g.count++;
    }
    TRY(gather(c, n, g, false));
    // number density: the density solve with unit masses (h^3 n = eta^3)
    TRY(fill(c, n, S.m, 1.0));
    TRY(build_tree(c, n));
    c->built = false;
    TRY(run_density(c, n));
    TRY(refresh_hmax(c, n));
    double *Bo[6], *go[12];
    for (int k = 0; k < 6; k++) Bo[k] = s->B[k] ? Bs[k] : nullptr;
    for (int k = 0; k < 12; k++) go[k] = (k < 3 * s->nfields && s->grad[k]) ? gs[k] : nullptr;
    TRY(run_mfv(c, n, s->nfields, fs, Bo, s->cond ? conds : nullptr, go));
    ScatterList sl{};
    auto add = [&](const void *from, void *to, int kind) {
        if (!to) return;
        sl.kind[sl.count] = kind;
        sl.src[sl.count] = from;
        sl.dst[sl.count] = to;
        sl.count++;
    };
    add(S.h, s->h, 0);
    add(S.rho, s->ndens, 0);
    add(S.nngb, s->nngb, 1);
    for (int k = 0; k < 6; k++) add(Bs[k], s->B[k], 0);
    add(conds, s->cond, 0);
    TRY(scatter(c, n, sl, c->perm));
    if (s->nfields > 0) {
        ScatterList sg{};
        for (int k = 0; k < 3 * s->nfields; k++) {
            if (!s->grad[k]) continue;
            sg.kind[sg.count] = 0;
            sg.src[sg.count] = gs[k];
            sg.dst[sg.count] = s->grad[k];
            sg.count++;
        }
        if (sg.count) TRY(scatter(c, n, sg, c->perm));
    }
    return SPH_OK;
}

sph_status sph_sync(sph_ctx *c)
{
    if (!c) return SPH_EINVAL;
    // the status copy is ordered after the enqueued work: one wait covers both
    hipError_t e = hipMemcpyAsync(c->h_status, c->d_status, sizeof(int32_t) * kStatusWords,
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && c->dt_used_out && c->resident)
        e = hipMemcpyAsync(c->h_scal + 1, c->d_scal + 1, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "read status");
    if (c->dt_used_out && c->resident) *c->dt_used_out = c->h_scal[1];
    c->dt_used_out = nullptr;
    int32_t st[kStatusWords];
    std::memcpy(st, c->h_status, sizeof(st));
    if (st[0] != 0 || st[4] != 0 || st[5] != 0) {
        e = hipMemsetAsync(c->d_status, 0, sizeof(int32_t) * kStatusWords, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_check(c, e, "clear status");
    }
    if (st[0] & kFlagNonFinite)
        return fail(c, SPH_ENONFINITE, std::to_string(st[2]) + " particles with non-finite results");
    if (st[0] & kFlagStencil)
        return fail(c, SPH_ESTENCIL, std::to_string(st[3]) +
                                         " particles with 2h >= L/2 in the periodic box");
    if (st[0] & kFlagNotConverged)
        return fail(c, SPH_ENOTCONVERGED, std::to_string(st[1]) +
                                              " smoothing lengths did not converge");
    if (st[0] & kFlagLevel)
        return fail(c, SPH_ELEVEL, "a particle needs a time-step level deeper than block_lmax");
    c->err.clear();
    return SPH_OK;
}

const char *sph_last_error(const sph_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

size_t sph_device_bytes(const sph_ctx *c) { return c ? c->bytes : 0; }

size_t sph_plan_bytes(const sph_params *p, int64_t n)
{
    if (!p || n < 0) return 0;
    const int64_t cap = std::max<int64_t>(n, 1024);
    return (size_t)(bytes_per_particle() * cap + node_count_bound(cap) * (int64_t)sizeof(Node) +
                    4 * hist_words(cap) + 4096 + 3 * kArgBytes +
                    cache_bytes(p->leaf_size, p->kernel, pair_grid(cap)));
}

sph_status sph_enable_kernel_timing(sph_ctx *c, int32_t enable)
{
    if (!c) return SPH_EINVAL;
    if (enable & ~3) return fail(c, SPH_EINVAL, "enable takes bits 0 and 1 only");
    c->timer.on = (enable & 1) != 0;
    c->count_tests = (enable & 2) != 0;
    return SPH_OK;
}

sph_status sph_kernel_times(sph_ctx *c, int32_t which, double *ms, int64_t *launches)
{
    if (!c || which < 0 || which > 2) return SPH_EINVAL;
    TRY(hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
    for (int w = 0; w < 3; w++) {
        for (auto &pr : c->timer.pending[w]) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) {
                c->timer.ms[w] += t;
                c->timer.launches[w]++;
            }
            c->timer.pool.push_back(pr);
        }
        c->timer.pending[w].clear();
    }
    if (ms) *ms = c->timer.ms[which];
    if (launches) *launches = c->timer.launches[which];
    if (!ms && !launches) { c->timer.ms[which] = 0; c->timer.launches[which] = 0; }
    return SPH_OK;
}

} // extern "C"
