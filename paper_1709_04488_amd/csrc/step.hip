// Elementwise and reduction kernels: scatter back to caller order, equation
// of state on output, kick-drift-kick leapfrog (eqs. EQN:LFKDK1, EQN:LFKDK2),
// global CFL step min_i dt_i (eq. EQN:SPH_DT) and conserved-quantity sums.
// All are HBM-bound streams over SoA arrays.
#include "sph_internal.hpp"

namespace sph {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;
constexpr int kRedVals = 8;

__global__ __launch_bounds__(256) void k_scatter(int64_t n, const uint32_t *__restrict__ index,
                                                 ScatterList s)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t dst = index[k];
    copy_listed(s, k, dst);
}

__global__ __launch_bounds__(256) void k_eos_scatter(int64_t n, double gamma,
                                                     const uint32_t *__restrict__ index,
                                                     const double *__restrict__ rho,
                                                     const double *__restrict__ u_caller,
                                                     double *__restrict__ P, double *__restrict__ cs)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t d = index[k];
    double Pk = (gamma - 1.0) * rho[k] * u_caller[d];
    if (P) P[d] = Pk;
    if (cs) cs[d] = sqrt(gamma * Pk / rho[k]);
}

// k_scatter and, where P or cs is given, the equation of state of k_eos_scatter
// from the sorted rho and u, in one pass over the permutation.
__global__ __launch_bounds__(256) void k_scatter_eos(int64_t n, const uint32_t *__restrict__ index,
                                                     ScatterList s, double gamma,
                                                     const double *__restrict__ rho,
                                                     const double *__restrict__ u_sorted,
                                                     double *__restrict__ P, double *__restrict__ cs)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t dst = index[k];
    copy_listed(s, k, dst);
    if (P || cs) {
        double Pk = (gamma - 1.0) * rho[k] * u_sorted[k];
        if (P) P[dst] = Pk;
        if (cs) cs[dst] = sqrt(gamma * Pk / rho[k]);
    }
}

struct KdkArgs {
    int64_t n;
    Box box;
    double dt_host;
    double *scal;   // [0] dt_next, [1] dt_last, [2] time
    double *x, *y, *z, *vx, *vy, *vz, *u;
    const double *ax, *ay, *az, *du;
    double *vpx, *vpy, *vpz, *up;
    // MM97 switch (nullptr otherwise): alpha kicked like u, its predictor
    double *al, *alp;
    const double *adot;
};

__device__ inline double wrap(double q, double lo, double L)
{
    if (q >= lo + L) q -= L;
    else if (q < lo) q += L;
    return q;
}

// v_1/2 = v + a dt/2, u_1/2 = u + du dt/2, x += v_1/2 dt (wrapped),
// predictor v* = v_1/2 + a dt/2, u* = u_1/2 + du dt/2.
__global__ __launch_bounds__(256) void k_kick_drift(KdkArgs K)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const double dt = K.dt_host > 0.0 ? K.dt_host : K.scal[0];
    if (k == 0) {
        K.scal[1] = dt;
        K.scal[2] += dt;
    }
    if (k >= K.n) return;
    const double hd = 0.5 * dt;
    double vh[3] = {K.vx[k] + hd * K.ax[k], K.vy[k] + hd * K.ay[k], K.vz[k] + hd * K.az[k]};
    double uh = K.u[k] + hd * K.du[k];
    double *pos[3] = {K.x, K.y, K.z};
    for (int a = 0; a < 3; a++) {
        double q = pos[a][k] + dt * vh[a];
        if (K.box.periodic) q = wrap(q, K.box.lo[a], K.box.len[a]);
        pos[a][k] = q;
    }
    K.vx[k] = vh[0]; K.vy[k] = vh[1]; K.vz[k] = vh[2];
    K.u[k] = uh;
    K.vpx[k] = vh[0] + hd * K.ax[k];
    K.vpy[k] = vh[1] + hd * K.ay[k];
    K.vpz[k] = vh[2] + hd * K.az[k];
    K.up[k] = uh + hd * K.du[k];
    if (K.al) {
        const double ah = K.al[k] + hd * K.adot[k];
        K.al[k] = ah;
        K.alp[k] = ah + hd * K.adot[k];
    }
}

// v = v_1/2 + a' dt/2, u = u_1/2 + du' dt/2 with the dt of the opening kick.
__global__ __launch_bounds__(256) void k_closing_kick(KdkArgs K)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= K.n) return;
    const double hd = 0.5 * K.scal[1];
    K.vx[k] += hd * K.ax[k];
    K.vy[k] += hd * K.ay[k];
    K.vz[k] += hd * K.az[k];
    K.u[k] += hd * K.du[k];
    if (K.al) K.al[k] += hd * K.adot[k];
}

__global__ __launch_bounds__(256) void k_fill(int64_t n, double *__restrict__ v, double value)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) v[k] = value;
}

// Morris & Monaghan 1997 rate of alpha from the alpha the forces used, their
// div v, and c and h of the same evaluation (c from the force record):
//   d alpha/dt = -(alpha - alpha_min) ell c / h + max(-div v, 0) (alpha_max - alpha)
__device__ inline double mm97_rate(double a, double d, double c, double h, double amin,
                                   double amax, double ell)
{
    const double decay = -(a - amin) * ell * c / h;
    const double src = d < 0.0 ? -d * (amax - a) : 0.0;
    return decay + src;
}

// Cullen & Dehnen 2010: alpha after a step of length dt from div v now (d)
// and at the previous evaluation (dp), |curl v|, v_sig, c and h
__device__ inline double cd10_alpha(double a, double dt, double d, double dp, double curl,
                                    double vs, double c, double hk, double amin, double amax,
                                    double ell)
{
    const double rate = (d - dp) / dt;
    const double ad = fabs(d);
    const double xi = ad / (ad + curl + 1e-4 * c / hk);
    const double A = rate < 0.0 ? -xi * rate : 0.0;
    const double h2A = hk * hk * A;
    double aloc = amax * h2A / (vs * vs + h2A);
    if (aloc < amin) aloc = amin;
    return a < aloc ? aloc : aloc + (a - aloc) * exp(-dt * 2.0 * ell * vs / hk);
}

__global__ __launch_bounds__(256) void k_av_mm97(int64_t n, double amin, double amax, double ell,
                                                 const double *__restrict__ alpha,
                                                 const double *__restrict__ divv,
                                                 const ForceRec *__restrict__ rec,
                                                 const double *__restrict__ h,
                                                 double *__restrict__ adot)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    adot[k] = mm97_rate(alpha[k], divv[k], rec[k].c, h[k], amin, amax, ell);
}

// Cullen & Dehnen 2010 update of alpha after the forces at the end of a step
// (length scal[1]); first = true at upload only sets dprev.
__global__ __launch_bounds__(256) void k_av_cd10(int64_t n, double amin, double amax, double ell,
                                                 const double *__restrict__ scal, bool first,
                                                 double *__restrict__ alpha,
                                                 const double *__restrict__ divv,
                                                 double *__restrict__ dprev,
                                                 const double *__restrict__ curlv,
                                                 const double *__restrict__ vsig,
                                                 const ForceRec *__restrict__ rec,
                                                 const double *__restrict__ h)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double d = divv[k];
    if (!first)
        alpha[k] = cd10_alpha(alpha[k], scal[1], d, dprev[k], curlv[k], vsig[k], rec[k].c, h[k],
                              amin, amax, ell);
    dprev[k] = d;
}

// min over dt_i -> scal[0]
__global__ __launch_bounds__(kRedThreads) void k_min_partial(int64_t n, const double *__restrict__ v,
                                                             double *__restrict__ part)
{
    double mn = INFINITY;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        mn = fmin(mn, v[k]);
    __shared__ double sh[kRedThreads];
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_min_final(int nb, const double *__restrict__ part,
                                                           double *__restrict__ out)
{
    __shared__ double sh[kRedThreads];
    double mn = INFINITY;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) mn = fmin(mn, part[b]);
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// smallest and largest mass -> out[0], out[1] (equal masses let the density
// loop keep only r^2 in its candidate lists)
__global__ __launch_bounds__(kRedThreads) void k_mrange_partial(int64_t n, const double *__restrict__ m,
                                                                double *__restrict__ part)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        lo = fmin(lo, m[k]);
        hi = fmax(hi, m[k]);
    }
    __shared__ double sl[kRedThreads], sh[kRedThreads];
    sl[threadIdx.x] = lo;
    sh[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + s]);
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sl[0];
        part[2 * blockIdx.x + 1] = sh[0];
    }
}

__global__ __launch_bounds__(kRedThreads) void k_mrange_final(int nb, const double *__restrict__ part,
                                                              double *__restrict__ out)
{
    __shared__ double sl[kRedThreads], sh[kRedThreads];
    double lo = INFINITY, hi = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) {
        lo = fmin(lo, part[2 * b]);
        hi = fmax(hi, part[2 * b + 1]);
    }
    sl[threadIdx.x] = lo;
    sh[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + s]);
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sl[0];
        out[1] = sh[0];
    }
}

// Sums in a fixed order (grid-stride per thread, fixed tree per block, fixed
// order over blocks), so they are reproducible bit for bit.
//   [0] 1/2 m v^2  [1] m u  [2..4] m v  [5] sum nngb  [6] sum nforce
__global__ __launch_bounds__(kRedThreads) void k_diag_partial(int64_t n, const double *__restrict__ m,
                                                              const double *__restrict__ vx,
                                                              const double *__restrict__ vy,
                                                              const double *__restrict__ vz,
                                                              const double *__restrict__ u,
                                                              const int32_t *__restrict__ nngb,
                                                              const int32_t *__restrict__ nforce,
                                                              double *__restrict__ part)
{
    double acc[kRedVals] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        double mk = m[k];
        acc[0] += 0.5 * mk * ((vx[k] * vx[k] + vy[k] * vy[k]) + vz[k] * vz[k]);
        acc[1] += mk * u[k];
        acc[2] += mk * vx[k];
        acc[3] += mk * vy[k];
        acc[4] += mk * vz[k];
        acc[5] += (double)nngb[k];
        acc[6] += (double)nforce[k];
    }
    __shared__ double sh[kRedVals][kRedThreads];
    for (int a = 0; a < kRedVals; a++) sh[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < kRedVals; a++) sh[a][threadIdx.x] += sh[a][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kRedVals) part[blockIdx.x * kRedVals + threadIdx.x] = sh[threadIdx.x][0];
}

// fixed order: thread t sums the partials b = t (mod 256) in order, then a
// fixed tree over the 256 threads
__global__ __launch_bounds__(kRedThreads) void k_diag_final(int nb, const double *__restrict__ part,
                                                            double *__restrict__ scal,
                                                            int64_t *__restrict__ counts)
{
    __shared__ double sh[kRedVals][kRedThreads];
    double acc[kRedVals];
    for (int v = 0; v < kRedVals; v++) acc[v] = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRedThreads)
        for (int v = 0; v < kRedVals; v++) acc[v] += part[b * kRedVals + v];
    for (int v = 0; v < kRedVals; v++) sh[v][threadIdx.x] = acc[v];
    __syncthreads();
    for (int st = kRedThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int v = 0; v < kRedVals; v++) sh[v][threadIdx.x] += sh[v][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 5) scal[3 + threadIdx.x] = sh[threadIdx.x][0];
    else if (threadIdx.x < 7) counts[threadIdx.x - 5] = (int64_t)sh[threadIdx.x][0];
}

__global__ __launch_bounds__(1024) void k_scan_offsets(int64_t n, int64_t *__restrict__ a)
{
    __shared__ int64_t sums[1024];
    const int t = threadIdx.x;
    const int64_t total = n + 1;
    const int64_t chunk = (total + 1023) / 1024;
    const int64_t s0 = t * chunk, s1 = s0 + chunk < total ? s0 + chunk : total;
    int64_t s = 0;
    for (int64_t k = s0; k < s1; k++) s += k < n ? a[k] : 0;
    sums[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t v = t >= d ? sums[t - d] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    int64_t run = sums[t] - s;
    for (int64_t k = s0; k < s1; k++) {
        int64_t v = k < n ? a[k] : 0;
        a[k] = run;
        run += v;
    }
}

__global__ void k_zero_counts(int64_t *__restrict__ c, int first, int count)
{
    if ((int)threadIdx.x < count) c[first + threadIdx.x] = 0;
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

KdkArgs kdk_args(sph_ctx *c, int64_t n, double dt_host)
{
    KdkArgs K{};
    K.n = n;
    K.box = c->box;
    K.dt_host = dt_host;
    K.scal = c->d_scal;
    K.x = c->s.x; K.y = c->s.y; K.z = c->s.z;
    K.vx = c->s.vx; K.vy = c->s.vy; K.vz = c->s.vz; K.u = c->s.u;
    K.ax = c->s.ax; K.ay = c->s.ay; K.az = c->s.az; K.du = c->s.du;
    K.vpx = c->s.vpx; K.vpy = c->s.vpy; K.vpz = c->s.vpz; K.up = c->s.up;
    if (c->p.av_switch == SPH_AV_MM97) {
        K.al = c->s.al;
        K.alp = c->s.alp;
        K.adot = c->s.adot;
    }
    return K;
}

double av_ell(const sph_params &p)
{
    if (p.av_ell > 0.0) return p.av_ell;
    return p.av_switch == SPH_AV_MM97 ? 0.1 : 0.05;
}

} // namespace

sph_status scatter(sph_ctx *c, int64_t n, const ScatterList &s, const uint32_t *index)
{
    if (n == 0 || s.count == 0) return SPH_OK;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, index, s);
    return hip_check(c, hipGetLastError(), "scatter");
}

sph_status scatter_eos(sph_ctx *c, int64_t n, const ScatterList &s, const uint32_t *index,
                       const double *u_sorted, double *P, double *cs)
{
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_scatter_eos, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, index, s,
                       c->p.gamma, c->s.rho, u_sorted, P, cs);
    return hip_check(c, hipGetLastError(), "scatter_eos");
}

sph_status eos_scatter(sph_ctx *c, int64_t n, const uint32_t *index, const double *u_caller,
                       double *P, double *cs)
{
    if (n == 0 || (!P && !cs)) return SPH_OK;
    hipLaunchKernelGGL(k_eos_scatter, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n,
                       c->p.gamma, index, c->s.rho, u_caller, P, cs);
    return hip_check(c, hipGetLastError(), "eos_scatter");
}

sph_status kick_drift(sph_ctx *c, int64_t n, double dt_host)
{
    KdkArgs K = kdk_args(c, n, dt_host);
    hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(n > 0 ? n : 1, 256)), dim3(256), 0, c->stream, K);
    return hip_check(c, hipGetLastError(), "kick_drift");
}

// ---- block time-steps (section 2.1.4) and the limiter (section 2.1.5) -----
//
// The integer timeline and the rules are those of the oracle: a level-0 step
// of dt_max holds P0 = 2^lmax ticks; a particle on level l steps 2^(lmax-l)
// ticks; dt_max = min dt 2^k (k the largest keeping it <= max dt) at every
// full synchronisation.  Every decision below is integer arithmetic or an
// exact power-of-two comparison of the CFL steps, so it is taken exactly
// as the oracle takes it from the same steps.
namespace {

struct BlockArgs {
    int64_t n;
    Box box;
    int32_t lmax, lim;
    BlockClock *clk;
    int32_t *status;
    double *x, *y, *z;
    double *vx, *vy, *vz, *u;       // velocities, u at each particle's last synchronisation
    double *vhx, *vhy, *vhz, *uh;   // after the opening kick
    double *vpx, *vpy, *vpz, *up;   // predicted to the end of the sub-step
    const double *ax, *ay, *az, *du, *dt;
    // MM97 (else null): alpha at the last synchronisation, after the opening
    // kick, predicted, and its rate
    double *al, *alh, *alp, *adot;
    int32_t *lev;
    int64_t *ts, *te;
    int32_t *act, *lmx, *mark;
    const uint32_t *lstart;
    const TreeInfo *tree;
    int32_t *leaf_act;
    int64_t *part;                  // reduction partials
};

// smallest level l <= lmax with dt_max 2^-l <= dt, or -1 (exact comparisons)
__device__ inline int block_level_of(double dt, double dtmax, int lmax)
{
    int l = 0;
    while (l < lmax && ldexp(dtmax, -l) > dt) l++;
    return ldexp(dtmax, -l) > dt ? -1 : l;
}

// Tn = min_i te_i (two stages)
__global__ __launch_bounds__(kRedThreads) void k_block_tn_partial(BlockArgs B)
{
    int64_t mn = INT64_MAX;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < B.n;
         k += (int64_t)gridDim.x * blockDim.x)
        mn = B.te[k] < mn ? B.te[k] : mn;
    __shared__ int64_t sh[kRedThreads];
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s && sh[threadIdx.x + s] < sh[threadIdx.x])
            sh[threadIdx.x] = sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) B.part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_block_tn_final(BlockArgs B, int nb)
{
    __shared__ int64_t sh[kRedThreads];
    int64_t mn = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) mn = B.part[b] < mn ? B.part[b] : mn;
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s && sh[threadIdx.x + s] < sh[threadIdx.x])
            sh[threadIdx.x] = sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        B.clk->Tn = sh[0];
        B.clk->active = 0;
    }
}

// every particle drifts with its half-step velocity to the end of the sub-step
__global__ __launch_bounds__(256) void k_block_drift(BlockArgs B)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= B.n) return;
    const double dlt = (double)(B.clk->Tn - B.clk->T) * B.clk->tick;
    double *pos[3] = {B.x, B.y, B.z};
    const double vel[3] = {B.vhx[k], B.vhy[k], B.vhz[k]};
    for (int a = 0; a < 3; a++) {
        double q = pos[a][k] + dlt * vel[a];
        if (B.box.periodic) {
            if (q >= B.box.lo[a] + B.box.len[a]) q -= B.box.len[a];
            else if (q < B.box.lo[a]) q += B.box.len[a];
        }
        pos[a][k] = q;
    }
}

// predictors at the end of the sub-step, the active set, limiter scratch
__global__ __launch_bounds__(256) void k_block_predict(BlockArgs B)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= B.n) return;
    const int64_t Tn = B.clk->Tn;
    const double dm = ((double)Tn - 0.5 * (double)(B.ts[k] + B.te[k])) * B.clk->tick;
    B.vpx[k] = B.vhx[k] + B.ax[k] * dm;
    B.vpy[k] = B.vhy[k] + B.ay[k] * dm;
    B.vpz[k] = B.vhz[k] + B.az[k] * dm;
    B.up[k] = B.uh[k] + B.du[k] * dm;
    if (B.alh) B.alp[k] = B.alh[k] + B.adot[k] * dm;
    B.act[k] = B.te[k] == Tn ? 1 : 0;
    B.lmx[k] = 0;
    B.mark[k] = -1;
}

// active particles per leaf (the pair loops skip leaves without any)
__global__ __launch_bounds__(256) void k_leaf_active(BlockArgs B)
{
    const int64_t L = B.tree->cnt[0];
    int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int cnt = 0;
    if (l < L)
        for (uint32_t i = B.lstart[l]; i < B.lstart[l + 1]; i++) cnt += B.act[i];
    if (l < L) B.leaf_act[l] = cnt;
    // the clock's count of active particles
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd((unsigned long long *)&B.clk->active,
                                                  (unsigned long long)cnt);
}

// The leaves with an active particle, in leaf order: a count per tile of
// kActTile leaves, one block turning the counts into offsets (and the total),
// then every tile writing its active leaves at its offset, ranked by ballots
// within the waves and by the waves' counts across the block.
__global__ __launch_bounds__(256) void k_act_count(BlockArgs B, uint32_t *__restrict__ tile)
{
    const int64_t L = B.tree->cnt[0];
    const int64_t base = blockIdx.x * (int64_t)kActTile;
    int c = 0;
    for (int k = threadIdx.x; k < kActTile; k += 256) {
        const int64_t l = base + k;
        c += (l < L && B.leaf_act[l] != 0) ? 1 : 0;
    }
    __shared__ int part[4];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) tile[blockIdx.x] = (uint32_t)(part[0] + part[1] + part[2] + part[3]);
}

__global__ __launch_bounds__(1024) void k_act_scan(BlockArgs B, uint32_t *__restrict__ tile,
                                                    uint32_t *__restrict__ total)
{
    const int64_t L = B.tree->cnt[0];
    const int64_t tiles = (L + kActTile - 1) / kActTile;
    __shared__ uint32_t sh[1024];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < tiles; b0 += 1024) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t v = b < tiles ? tile[b] : 0u;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const uint32_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (b < tiles) tile[b] = carry + sh[threadIdx.x] - v;   // exclusive offset
        carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void k_act_scatter(BlockArgs B, const uint32_t *__restrict__ tile,
                                                     uint32_t *__restrict__ list)
{
    const int64_t L = B.tree->cnt[0];
    const int64_t base = blockIdx.x * (int64_t)kActTile;
    if (base >= L) return;   // the whole block: no tile of the tree's leaves
    __shared__ uint32_t wsum[4];
    uint32_t off = tile[blockIdx.x];
    for (int r = 0; r < kActTile / 256; r++) {
        const int64_t l = base + r * 256 + threadIdx.x;
        const bool a = l < L && B.leaf_act[l] != 0;
        const uint64_t m = __ballot(a);
        const int w = threadIdx.x >> 6;
        const uint32_t rank = (uint32_t)__popcll(m & __lanemask_lt());
        if ((threadIdx.x & 63) == 0) wsum[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0;
        for (int k = 0; k < w; k++) before += wsum[k];
        if (a) list[off + before + rank] = (uint32_t)l;
        const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
        off += tot;
    }
}

// closing kick of the active particles with their new accelerations
__global__ __launch_bounds__(256) void k_block_close(BlockArgs B)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= B.n || !B.act[k]) return;
    const double hs = 0.5 * (double)(B.te[k] - B.ts[k]) * B.clk->tick;
    B.vx[k] = B.vhx[k] + B.ax[k] * hs;
    B.vy[k] = B.vhy[k] + B.ay[k] * hs;
    B.vz[k] = B.vhz[k] + B.az[k] * hs;
    B.u[k] = B.uh[k] + B.du[k] * hs;
    if (B.alh) B.al[k] = B.alh[k] + B.adot[k] * hs;
}

// range of the CFL steps (every particle is active at a full synchronisation)
__global__ __launch_bounds__(kRedThreads) void k_block_dt_partial(BlockArgs B)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < B.n;
         k += (int64_t)gridDim.x * blockDim.x) {
        lo = fmin(lo, B.dt[k]);
        hi = fmax(hi, B.dt[k]);
    }
    __shared__ double sl[kRedThreads], sh[kRedThreads];
    sl[threadIdx.x] = lo;
    sh[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + s]);
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *pd = (double *)B.part;
        pd[2 * blockIdx.x] = sl[0];
        pd[2 * blockIdx.x + 1] = sh[0];
    }
}

// at a full synchronisation (or at the start): dt_max = min dt 2^k, k the
// largest integer keeping it <= max dt, and its tick length
__global__ __launch_bounds__(kRedThreads) void k_block_dt_final(BlockArgs B, int nb, bool init)
{
    __shared__ double sl[kRedThreads], sh[kRedThreads];
    const double *pd = (const double *)B.part;
    double lo = INFINITY, hi = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) {
        lo = fmin(lo, pd[2 * b]);
        hi = fmax(hi, pd[2 * b + 1]);
    }
    sl[threadIdx.x] = lo;
    sh[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + s]);
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t P0 = (int64_t)1 << B.lmax;
        if (init || B.clk->Tn == P0) {
            int k = 0;
            while (k < 1000 && ldexp(sl[0], k + 1) <= sh[0]) k++;
            const double dtm = ldexp(sl[0], k);
            B.clk->dt_max_next = dtm;
            B.clk->tick_next = dtm / (double)P0;
        }
    }
}

// new levels and steps of the active particles (fresh at a full
// synchronisation, else deeper at once or one shallower when synchronised;
// never shallower than the deepest neighbour minus lim), reactive wake-up of
// marked inactive particles, opening kicks of the active particles
__global__ __launch_bounds__(256) void k_block_levels(BlockArgs B, bool init)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= B.n) return;
    const int64_t P0 = (int64_t)1 << B.lmax;
    const int64_t Tn = init ? 0 : B.clk->Tn;
    const bool full = init || Tn == P0;
    const int lim = B.lim;
    if (init || B.act[k]) {
        const double dtm = full ? B.clk->dt_max_next : B.clk->dt_max;
        int l = block_level_of(B.dt[k], dtm, B.lmax);
        bool bad = l < 0;
        int64_t nl;
        if (full) {
            nl = l;
            if (!init && nl < (int64_t)B.lmx[k] - lim) nl = (int64_t)B.lmx[k] - lim;
        } else {
            const int64_t cur = B.lev[k];
            if (l > cur) nl = l;
            else if (l < cur && Tn % (P0 >> (cur - 1)) == 0) nl = cur - 1;
            else nl = cur;
            if (nl < (int64_t)B.lmx[k] - lim) nl = (int64_t)B.lmx[k] - lim;
        }
        if (bad || nl > B.lmax) {
            atomicOr(&B.status[0], kFlagLevel);
            nl = B.lmax;
        }
        const int64_t t0 = full ? 0 : Tn;
        B.lev[k] = (int32_t)nl;
        B.ts[k] = t0;
        B.te[k] = t0 + (P0 >> nl);
        const double hs = 0.5 * (double)(P0 >> nl) * (full ? B.clk->tick_next : B.clk->tick);
        B.vhx[k] = B.vx[k] + B.ax[k] * hs;
        B.vhy[k] = B.vy[k] + B.ay[k] * hs;
        B.vhz[k] = B.vz[k] + B.az[k] * hs;
        B.uh[k] = B.u[k] + B.du[k] * hs;
        if (B.alh) B.alh[k] = B.al[k] + B.adot[k] * hs;
    } else if (!full && B.mark[k] >= 0 && B.lev[k] < B.mark[k] - lim) {
        int64_t nl = B.mark[k] - lim;
        if (nl > B.lmax) {
            atomicOr(&B.status[0], kFlagLevel);
            nl = B.lmax;
        }
        const int64_t st = P0 >> nl;
        const int64_t tn = (Tn / st + 1) * st;
        const double cut = 0.5 * (double)((B.te[k] - B.ts[k]) - (tn - B.ts[k])) * B.clk->tick;
        B.vhx[k] -= B.ax[k] * cut;
        B.vhy[k] -= B.ay[k] * cut;
        B.vhz[k] -= B.az[k] * cut;
        B.uh[k] -= B.du[k] * cut;
        if (B.alh) B.alh[k] -= B.adot[k] * cut;
        B.lev[k] = (int32_t)nl;
        B.te[k] = tn;
    }
}

// the clock moves to the end of the sub-step (one thread)
__global__ void k_block_advance(BlockArgs B, bool init)
{
    BlockClock &C = *B.clk;
    const int64_t P0 = (int64_t)1 << B.lmax;
    if (init) {
        C.T = 0;
        C.full = 0;
        C.nsub = 0;
        C.updates = 0;
        C.time = 0.0;
        C.tick = C.tick_next;
        C.dt_max = C.dt_max_next;
        return;
    }
    C.time += (double)(C.Tn - C.T) * C.tick;
    C.nsub += 1;
    C.updates += C.active;
    if (C.Tn == P0) {
        C.full += 1;
        C.T = 0;
        C.tick = C.tick_next;
        C.dt_max = C.dt_max_next;
    } else {
        C.T = C.Tn;
    }
}

// The switches of the particles active in this sub-step, from its forces:
// the MM97 rate from the predicted alpha the forces used; the CD10 update
// over the step that ends now, (t_end - t_start) ticks, from div v now and at
// the particle's previous evaluation.
struct BlockAv {
    int sw;
    double amin, amax, ell;
    double *al, *adot, *dprev;
    const double *alp, *divv, *curlv, *vsig, *h;
    const ForceRec *rec;
};

__global__ __launch_bounds__(256) void k_block_av(BlockArgs B, BlockAv V)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= B.n || !B.act[k]) return;
    const double d = V.divv[k];
    if (V.sw == SPH_AV_MM97) {
        V.adot[k] = mm97_rate(V.alp[k], d, V.rec[k].c, V.h[k], V.amin, V.amax, V.ell);
    } else {
        const double dt = (double)(B.te[k] - B.ts[k]) * B.clk->tick;
        V.al[k] = cd10_alpha(V.al[k], dt, d, V.dprev[k], V.curlv[k], V.vsig[k], V.rec[k].c,
                             V.h[k], V.amin, V.amax, V.ell);
        V.dprev[k] = d;
    }
}

BlockArgs block_args(sph_ctx *c, int64_t n)
{
    BlockArgs B{};
    B.n = n;
    B.box = c->box;
    B.lmax = c->p.block_lmax;
    B.lim = c->p.block_lim;
    B.clk = c->d_clock;
    B.status = c->d_status;
    Sorted &S = c->s;
    B.x = S.x; B.y = S.y; B.z = S.z;
    B.vx = S.vx; B.vy = S.vy; B.vz = S.vz; B.u = S.u;
    B.vhx = S.vhx; B.vhy = S.vhy; B.vhz = S.vhz; B.uh = S.uh;
    B.vpx = S.vpx; B.vpy = S.vpy; B.vpz = S.vpz; B.up = S.up;
    B.ax = S.ax; B.ay = S.ay; B.az = S.az; B.du = S.du; B.dt = S.dt;
    B.lev = S.lev; B.ts = S.ts; B.te = S.te;
    B.act = S.act; B.lmx = S.lmx; B.mark = S.mark;
    if (c->p.av_switch == SPH_AV_MM97) {
        B.al = S.al; B.alh = S.alh; B.alp = S.alp; B.adot = S.adot;
    }
    B.lstart = c->lstart;
    B.tree = c->d_tree;
    B.leaf_act = c->leaf_act;
    B.part = (int64_t *)c->d_part;
    return B;
}

} // namespace

sph_status block_next(sph_ctx *c, int64_t n)
{
    BlockArgs B = block_args(c, n);
    const int nb = (int)std::min<int64_t>(kRedBlocks / 2, (n + kRedThreads - 1) / kRedThreads);
    hipLaunchKernelGGL(k_block_tn_partial, dim3(nb), dim3(kRedThreads), 0, c->stream, B);
    hipLaunchKernelGGL(k_block_tn_final, dim3(1), dim3(kRedThreads), 0, c->stream, B, nb);
    hipLaunchKernelGGL(k_block_drift, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, B);
    return hip_check(c, hipGetLastError(), "block_next");
}

sph_status block_predict(sph_ctx *c, int64_t n)
{
    BlockArgs B = block_args(c, n);
    hipLaunchKernelGGL(k_block_predict, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, B);
    // leaves: at most n
    hipLaunchKernelGGL(k_leaf_active, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, B);
    // the pair loops' home leaves: those with an active particle
    const unsigned tiles = (unsigned)((n + kActTile - 1) / kActTile);
    hipLaunchKernelGGL(k_act_count, dim3(tiles), dim3(256), 0, c->stream, B, c->act_tile);
    hipLaunchKernelGGL(k_act_scan, dim3(1), dim3(1024), 0, c->stream, B, c->act_tile, c->act_cnt);
    hipLaunchKernelGGL(k_act_scatter, dim3(tiles), dim3(256), 0, c->stream, B, c->act_tile,
                       c->act_list);
    return hip_check(c, hipGetLastError(), "block_predict");
}

sph_status block_finish(sph_ctx *c, int64_t n, bool init)
{
    BlockArgs B = block_args(c, n);
    const unsigned g = grid_for(n, 256);
    if (!init) hipLaunchKernelGGL(k_block_close, dim3(g), dim3(256), 0, c->stream, B);
    const int nb = (int)std::min<int64_t>(kRedBlocks / 2, (n + kRedThreads - 1) / kRedThreads);
    hipLaunchKernelGGL(k_block_dt_partial, dim3(nb), dim3(kRedThreads), 0, c->stream, B);
    hipLaunchKernelGGL(k_block_dt_final, dim3(1), dim3(kRedThreads), 0, c->stream, B, nb, init);
    hipLaunchKernelGGL(k_block_levels, dim3(g), dim3(256), 0, c->stream, B, init);
    hipLaunchKernelGGL(k_block_advance, dim3(1), dim3(1), 0, c->stream, B, init);
    return hip_check(c, hipGetLastError(), "block_finish");
}

sph_status block_av(sph_ctx *c, int64_t n)
{
    const int sw = c->p.av_switch;
    if (n == 0 || (sw != SPH_AV_MM97 && sw != SPH_AV_CD10)) return SPH_OK;
    BlockArgs B = block_args(c, n);
    Sorted &S = c->s;
    BlockAv V{sw, c->p.alpha_min, c->p.alpha_max, av_ell(c->p), S.al, S.adot, S.dprev,
              S.alp, S.divv, S.curlv, S.vsig, S.h, S.frec};
    hipLaunchKernelGGL(k_block_av, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, B, V);
    return hip_check(c, hipGetLastError(), "block_av");
}

sph_status fill(sph_ctx *c, int64_t n, double *v, double value)
{
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, v, value);
    return hip_check(c, hipGetLastError(), "fill");
}

sph_status av_rate(sph_ctx *c, int64_t n, const double *alpha_now)
{
    if (n == 0 || c->p.av_switch != SPH_AV_MM97) return SPH_OK;
    hipLaunchKernelGGL(k_av_mm97, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n,
                       c->p.alpha_min, c->p.alpha_max, av_ell(c->p), alpha_now, c->s.divv,
                       c->s.frec, c->s.h, c->s.adot);
    return hip_check(c, hipGetLastError(), "av_rate");
}

sph_status av_cd10(sph_ctx *c, int64_t n, bool first)
{
    if (n == 0 || c->p.av_switch != SPH_AV_CD10) return SPH_OK;
    hipLaunchKernelGGL(k_av_cd10, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n,
                       c->p.alpha_min, c->p.alpha_max, av_ell(c->p), c->d_scal, first, c->s.al,
                       c->s.divv, c->s.dprev, c->s.curlv, c->s.vsig, c->s.frec, c->s.h);
    return hip_check(c, hipGetLastError(), "av_cd10");
}

sph_status closing_kick(sph_ctx *c, int64_t n, double dt_host)
{
    if (n == 0) return SPH_OK;
    KdkArgs K = kdk_args(c, n, dt_host);
    hipLaunchKernelGGL(k_closing_kick, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, K);
    return hip_check(c, hipGetLastError(), "closing_kick");
}

sph_status reduce_mass_range(sph_ctx *c, int64_t n)
{
    if (n == 0) return SPH_OK;
    const int nb = (int)std::min<int64_t>(kRedBlocks / 2, (n + kRedThreads - 1) / kRedThreads);
    hipLaunchKernelGGL(k_mrange_partial, dim3(nb), dim3(kRedThreads), 0, c->stream, n, c->s.m,
                       c->d_part);
    hipLaunchKernelGGL(k_mrange_final, dim3(1), dim3(kRedThreads), 0, c->stream, nb, c->d_part,
                       c->d_scal + 8);
    return hip_check(c, hipGetLastError(), "reduce_mass_range");
}

sph_status reduce_dt(sph_ctx *c, int64_t n)
{
    if (n == 0) return SPH_OK;
    int nb = (int)std::min<int64_t>(kRedBlocks, (n + kRedThreads - 1) / kRedThreads);
    hipLaunchKernelGGL(k_min_partial, dim3(nb), dim3(kRedThreads), 0, c->stream, n, c->s.dt,
                       c->d_part);
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kRedThreads), 0, c->stream, nb, c->d_part,
                       c->d_scal);
    return hip_check(c, hipGetLastError(), "reduce_dt");
}

__global__ void k_zero_work(uint32_t *__restrict__ w)
{
    if (threadIdx.x < kXcds) w[threadIdx.x] = 0u;
}

sph_status zero_work(sph_ctx *c)
{
    hipLaunchKernelGGL(k_zero_work, dim3(1), dim3(64), 0, c->stream, c->d_work);
    return hip_check(c, hipGetLastError(), "zero_work");
}

sph_status zero_counts(sph_ctx *c, int first, int count)
{
    hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, c->stream, c->d_counts, first, count);
    return hip_check(c, hipGetLastError(), "zero_counts");
}

sph_status scan_offsets(sph_ctx *c, int64_t n, int64_t *a)
{
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, c->stream, n, a);
    return hip_check(c, hipGetLastError(), "scan_offsets");
}

sph_status reduce_diag(sph_ctx *c, int64_t n)
{
    if (n == 0) return SPH_OK;
    int nb = (int)std::min<int64_t>(kRedBlocks, (n + kRedThreads - 1) / kRedThreads);
    hipLaunchKernelGGL(k_diag_partial, dim3(nb), dim3(kRedThreads), 0, c->stream, n, c->s.m,
                       c->s.vx, c->s.vy, c->s.vz, c->s.u, c->s.nngb, c->s.nforce, c->d_part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kRedThreads), 0, c->stream, nb, c->d_part,
                       c->d_scal, c->d_counts);
    return hip_check(c, hipGetLastError(), "reduce_diag");
}

} // namespace sph
