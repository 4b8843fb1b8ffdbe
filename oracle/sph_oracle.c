/*
 * Brute-force FP64 reference ("oracle") for the grad-h SPH density and force
 * loops and the kick-drift-kick leapfrog step of the GANDALF paper
 * (Hubber, Rosotti & Booth 2017, arXiv:1709.04488, section 2.1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file.  It exists so that tests, the smoke check and the
 * benchmark's CPU baseline can compare the HIP path against a plain, slow,
 * obviously correct computation.  It shares no code, header, table or
 * constant generator with the HIP path.
 *
 * Every sum runs over all particles j = 1..N in index order, with no cells,
 * no trees and no reordering.  The only shortcut is exact: once a bracket
 * [h_lo, h_hi] on the smoothing length is known, particles with
 * r_ij >= R h_hi are dropped from the list used by the bisection, because the
 * kernel vanishes identically beyond R h (compact support, R = 2 for the M4
 * and 3 for the quintic spline, section 2); adding those zero terms would not
 * change a single bit.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no FMA
 * contraction, so every product and sum is rounded as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENOROOT -4   /* no smoothing length satisfies the h-rho relation */
#define ORC_EBOX -5      /* periodic: the root needs R h >= L/2 */
#define ORC_ECAP -8      /* neighbour export: caller's capacity too small */

typedef struct {
    double eta;      /* h = eta (m/rho)^(1/3), eq. EQN:HRHO */
    double gamma;    /* ideal-gas ratio of specific heats, P = (gamma-1) rho u */
    double alpha;    /* alpha_AV, eq. EQN:MON97ARTVISC */
    double beta;     /* beta_AV (= 2 alpha_AV in the paper) */
    double ccfl;     /* C_CFL, eq. EQN:SPH_DT */
    int32_t periodic;
    int32_t ac_signal; /* conductivity signal speed: 0 Wadsley 2008, 1 Price 2008 */
    double lo[3], hi[3];
    double alpha_ac; /* alpha_AC, eq. EQN:MON97ENERGYDISS (0: no conductivity) */
    /* artificial-viscosity switch named in section 2.1.1: 0 none (alpha_AV for
     * every pair), 1 Morris & Monaghan 1997, 2 Cullen & Dehnen 2010 */
    int32_t av_switch;
    int32_t pad_;
    double alpha_min, alpha_max; /* floor and ceiling of the per-particle alpha */
    double av_ell;   /* decay constant: tau = h/(ell c) (MM97), h/(2 ell v_sig) (CD10) */
    int32_t kernel;  /* 0: M4 cubic spline (R = 2), 1: quintic spline (R = 3) */
    int32_t pad2_;
} orc_params;

/* ---------------------------------------------------------------------------
 * M4 cubic spline (Monaghan & Lattanzio 1985), compact support 2h, 3D
 * normalisation sigma = 1/pi.  The paper names this kernel with R = 2
 * (section 2) and defers the formula to Hubber et al. 2011, appendix A.
 *   f(q) = 1 - 3/2 q^2 + 3/4 q^3     0 <= q < 1
 *        = 1/4 (2 - q)^3             1 <= q < 2
 *        = 0                          q >= 2
 *   W(r,h) = sigma h^-3 f(r/h)
 * ------------------------------------------------------------------------- */
static const double ORC_SIGMA = 0.31830988618379067154; /* 1/pi */

double orc_f(double q)
{
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    if (q < 2.0) { double t = 2.0 - q; return 0.25 * t * t * t; }
    return 0.0;
}

/* df/dq */
double orc_df(double q)
{
    if (q < 1.0) return -3.0 * q + 2.25 * q * q;
    if (q < 2.0) { double t = 2.0 - q; return -0.75 * t * t; }
    return 0.0;
}

double orc_W(double r, double h)
{
    return ORC_SIGMA / (h * h * h) * orc_f(r / h);
}

/* dW/dr: the kernel gradient is grad_i W(r_ij, h) = orc_dWdr(r, h) * rhat_ij */
double orc_dWdr(double r, double h)
{
    return ORC_SIGMA / (h * h * h * h) * orc_df(r / h);
}

/* dW/dh = -sigma h^-4 (3 f(q) + q f'(q)) */
double orc_dWdh(double r, double h)
{
    double q = r / h;
    return -ORC_SIGMA / (h * h * h * h) * (3.0 * orc_f(q) + q * orc_df(q));
}

/* ---------------------------------------------------------------------------
 * Quintic spline (Morris 1996), compact support 3h, the paper's second
 * kernel (section 2).  In B-spline form with a = (3-q)_+, b = (2-q)_+,
 * c = (1-q)_+:
 *   f(q)  = a^5 - 6 b^5 + 15 c^5
 *   f'(q) = -5 a^4 + 30 b^4 - 75 c^4
 * and 3D normalisation sigma = 1/(120 pi) (4 pi sigma int_0^3 f q^2 dq = 1).
 * ------------------------------------------------------------------------- */
static const double ORC_SIGMA_Q = 0.0026525823848649222; /* 1/(120 pi) */

double orc_quintic_f(double q)
{
    double a = q < 3.0 ? 3.0 - q : 0.0, b = q < 2.0 ? 2.0 - q : 0.0, c = q < 1.0 ? 1.0 - q : 0.0;
    double a2 = a * a, b2 = b * b, c2 = c * c;
    return a2 * a2 * a - 6.0 * (b2 * b2 * b) + 15.0 * (c2 * c2 * c);
}

double orc_quintic_df(double q)
{
    double a = q < 3.0 ? 3.0 - q : 0.0, b = q < 2.0 ? 2.0 - q : 0.0, c = q < 1.0 ? 1.0 - q : 0.0;
    double a2 = a * a, b2 = b * b, c2 = c * c;
    return -5.0 * (a2 * a2) + 30.0 * (b2 * b2) - 75.0 * (c2 * c2);
}

/* the kernel of the parameters: support R (in units of h), shape, 3D norm */
static inline double supp(const orc_params *p) { return p->kernel == 1 ? 3.0 : 2.0; }
static inline double kf(const orc_params *p, double q)
{
    return p->kernel == 1 ? orc_quintic_f(q) : orc_f(q);
}
static inline double kdf(const orc_params *p, double q)
{
    return p->kernel == 1 ? orc_quintic_df(q) : orc_df(q);
}
static inline double ksig(const orc_params *p) { return p->kernel == 1 ? ORC_SIGMA_Q : ORC_SIGMA; }
static inline double kW(const orc_params *p, double r, double h)
{
    return ksig(p) / (h * h * h) * kf(p, r / h);
}
static inline double kdWdr(const orc_params *p, double r, double h)
{
    return ksig(p) / (h * h * h * h) * kdf(p, r / h);
}
static inline double kdWdh(const orc_params *p, double r, double h)
{
    double q = r / h;
    return -ksig(p) / (h * h * h * h) * (3.0 * kf(p, q) + q * kdf(p, q));
}

/* ---------------------------------------------------------------------------
 * Pair separation r_i - r_j.  Periodic boxes use the minimum image, one axis
 * at a time: shift by one box length when the separation exceeds half of it.
 * This is equivalent to the paper's periodic ghost copies (section 4.3) as
 * long as 2h < L/2, which the density solve enforces.
 * ------------------------------------------------------------------------- */
static inline double sep(double a, double b, int periodic, double L)
{
    double d = a - b;
    if (periodic) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

static inline double pair_r2(const orc_params *p, const double *x, const double *y,
                             const double *z, int64_t i, int64_t j,
                             double *dx, double *dy, double *dz)
{
    double Lx = p->hi[0] - p->lo[0], Ly = p->hi[1] - p->lo[1], Lz = p->hi[2] - p->lo[2];
    *dx = sep(x[i], x[j], p->periodic, Lx);
    *dy = sep(y[i], y[j], p->periodic, Ly);
    *dz = sep(z[i], z[j], p->periodic, Lz);
    return (*dx * *dx + *dy * *dy) + *dz * *dz;
}

static double min_box_len(const orc_params *p)
{
    double L = p->hi[0] - p->lo[0];
    for (int k = 1; k < 3; k++) if (p->hi[k] - p->lo[k] < L) L = p->hi[k] - p->lo[k];
    return L;
}

/* ---------------------------------------------------------------------------
 * Density and smoothing length (eqs. EQN:SPHRHO, EQN:HRHO, EQN:OMEGA).
 *
 * rho_i(h) = sum_j m_j W(r_ij, h) (self term included: the sum runs over
 * j = 1..N).  The h-rho relation h^3 rho_i(h) = eta^3 m_i is solved as the
 * root of   g(h) = sigma sum_j m_j f(r_ij/h) - eta^3 m_i,
 * which equals h^3 rho_i(h) - eta^3 m_i.  g is non-decreasing in h (f is
 * non-increasing in q) and g(0+) = (sigma - eta^3) m_i < 0, so the root is
 * unique whenever it exists.  It is found by bracketing (doubling/halving
 * the guess) and plain bisection down to a few ulp.  This is deliberately a
 * different root finder from the Newton-Raphson iteration of the HIP path:
 * the answer is defined by the relation, not by the iteration.
 *
 * Omega_i = 1 - (dh/drho) sum_j m_j dW/dh with dh/drho = -h/(3 rho) from
 * EQN:HRHO, i.e. Omega_i = 1 + h rho'_i / (3 rho_i).
 * ------------------------------------------------------------------------- */
typedef struct { double r; double m; } orc_nb;

static double g_full(const orc_params *p, int64_t n, const double *x, const double *y,
                     const double *z, const double *m, int64_t i, double h)
{
    double s = 0.0, h2x4 = (supp(p) * h) * (supp(p) * h);
    for (int64_t j = 0; j < n; j++) {
        double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
        if (r2 < h2x4) s += m[j] * kf(p, sqrt(r2) / h);
    }
    return ksig(p) * s - p->eta * p->eta * p->eta * m[i];
}

static double g_list(const orc_params *p, const orc_nb *nb, int64_t k, double mi, double h)
{
    double s = 0.0;
    for (int64_t a = 0; a < k; a++) s += nb[a].m * kf(p, nb[a].r / h);
    return ksig(p) * s - p->eta * p->eta * p->eta * mi;
}

/* Solve for one particle; fills h, rho, rho' (= sum m dW/dh), omega, nngb. */
static int solve_one(const orc_params *p, int64_t n, const double *x, const double *y,
                     const double *z, const double *m, int64_t i, double hguess,
                     orc_nb *nb, double *h_out, double *rho_out, double *drho_out,
                     double *omega_out, int32_t *nngb_out)
{
    if (!(hguess > 0.0) || !isfinite(hguess)) return ORC_EINVAL;
    double lo, hi;
    double gh = g_full(p, n, x, y, z, m, i, hguess);
    if (gh < 0.0) {
        lo = hguess; hi = 2.0 * hguess;
        int it = 0;
        while (g_full(p, n, x, y, z, m, i, hi) < 0.0) {
            lo = hi; hi *= 2.0;
            if (++it > 80) return ORC_ENOROOT;
            if (p->periodic && 2.0 * supp(p) * lo >= min_box_len(p)) return ORC_EBOX;
        }
    } else {
        hi = hguess; lo = 0.5 * hguess;
        int it = 0;
        while (g_full(p, n, x, y, z, m, i, lo) >= 0.0) {
            hi = lo; lo *= 0.5;
            if (++it > 1100) return ORC_ENOROOT;
        }
    }
    /* Exact pruning: only j with r_ij < 2 hi can contribute for h <= hi. */
    int64_t k = 0;
    double lim = (supp(p) * hi) * (supp(p) * hi);
    for (int64_t j = 0; j < n; j++) {
        double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
        if (r2 < lim) { nb[k].r = sqrt(r2); nb[k].m = m[j]; k++; }
    }
    for (int it = 0; it < 400; it++) {
        double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        if (hi - lo <= 4.0 * (nextafter(hi, INFINITY) - hi)) break;
        if (g_list(p, nb, k, m[i], mid) < 0.0) lo = mid; else hi = mid;
    }
    double h = lo + 0.5 * (hi - lo);
    if (p->periodic && 2.0 * supp(p) * h >= min_box_len(p)) return ORC_EBOX;

    double rho = 0.0, drho = 0.0;
    int32_t cnt = 0;
    double h2x4 = (supp(p) * h) * (supp(p) * h);
    for (int64_t j = 0; j < n; j++) {
        double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
        if (r2 < h2x4) {
            double r = sqrt(r2);
            rho += m[j] * kW(p, r, h);
            drho += m[j] * kdWdh(p, r, h);
            if (j != i) cnt++;
        }
    }
    *h_out = h;
    *rho_out = rho;
    *drho_out = drho;
    *omega_out = 1.0 + h * drho / (3.0 * rho);
    *nngb_out = cnt;
    return ORC_OK;
}

/*
 * Density loop for the selected particles (sel == NULL: all n).  Output k
 * belongs to particle sel[k].  h_guess is indexed by particle.
 */
int orc_density(const orc_params *p, int64_t n, const double *x, const double *y,
                const double *z, const double *m, const double *h_guess,
                int64_t nsel, const int64_t *sel, double *h, double *rho,
                double *drhodh, double *omega, int32_t *nngb)
{
    if (n < 0 || nsel < 0) return ORC_EINVAL;
    if (sel == NULL) nsel = n;
    int status = ORC_OK;
#pragma omp parallel
    {
        orc_nb *nb = (orc_nb *)malloc(sizeof(orc_nb) * (size_t)(n > 0 ? n : 1));
        if (!nb) {
#pragma omp atomic write
            status = ORC_ENOMEM;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nsel; k++) {
            if (!nb) continue;
            int64_t i = sel ? sel[k] : k;
            int rc = solve_one(p, n, x, y, z, m, i, h_guess[i], nb, &h[k], &rho[k],
                               &drhodh[k], &omega[k], &nngb[k]);
            if (rc != ORC_OK) {
#pragma omp critical
                { if (status == ORC_OK) status = rc; }
            }
        }
        free(nb);
    }
    return status;
}

/* rho_i and rho'_i = sum_j m_j dW/dh at a given h_i (no h-rho solve), and
 * the density-neighbour count.  Used to check the solve from outside. */
int orc_rho_at(const orc_params *p, int64_t n, const double *x, const double *y,
               const double *z, const double *m, int64_t nsel, const int64_t *sel,
               const double *hsel, double *rho, double *drhodh, int32_t *nngb)
{
    if (n < 0 || nsel < 0) return ORC_EINVAL;
    if (sel == NULL) nsel = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nsel; k++) {
        int64_t i = sel ? sel[k] : k;
        double h = hsel[k], r0 = 0.0, r1 = 0.0;
        int32_t cnt = 0;
        double h2x4 = (supp(p) * h) * (supp(p) * h);
        for (int64_t j = 0; j < n; j++) {
            double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
            if (r2 < h2x4) {
                double r = sqrt(r2);
                r0 += m[j] * kW(p, r, h);
                r1 += m[j] * kdWdh(p, r, h);
                if (j != i) cnt++;
            }
        }
        rho[k] = r0;
        drhodh[k] = r1;
        nngb[k] = cnt;
    }
    return ORC_OK;
}

/* Ideal-gas equation of state: P = (gamma-1) rho u (section 2.1.1) and the
 * adiabatic sound speed c = sqrt(gamma P / rho). */
void orc_eos(int64_t n, double gamma, const double *rho, const double *u,
             double *P, double *c)
{
    for (int64_t i = 0; i < n; i++) {
        P[i] = (gamma - 1.0) * rho[i] * u[i];
        c[i] = sqrt(gamma * P[i] / rho[i]);
    }
}

/* ---------------------------------------------------------------------------
 * Force loop (eqs. EQN:GRADHMOMEQN, EQN:GRADHENEQN, EQN:MON97ARTVISC,
 * EQN:MON97ENERGYDISS) and the signal speed / CFL step (eq. EQN:SPH_DT and
 * the v_sig definition beside it).
 *
 * For every j != i with r_ij < 2 max(h_i, h_j) (both W(h_i) and W(h_j)
 * appear in the momentum equation):
 *   G_i = dW/dr(r_ij, h_i) rhat_ij,  G_j = dW/dr(r_ij, h_j) rhat_ij
 *   A_i = P_i / (Omega_i rho_i^2)
 *   a_i    += -m_j (A_i G_i + A_j G_j)
 *   du_i   +=  A_i m_j v_ij . G_i
 *   w       =  v_ij . rhat_ij
 *   vs      =  c_i + c_j - beta min(0, w)
 *   vsig_i  =  max(vsig_i, vs)
 *   if w < 0 (mu_ij = w):
 *     rhobar = (rho_i + rho_j)/2,  Gbar = (G_i + G_j)/2
 *     a_i  +=  (m_j / rhobar) alpha vs w Gbar
 *     du_i += -(m_j / rhobar) alpha vs w^2/2 rhat_ij . Gbar
 *   artificial conductivity (second sum of eq. EQN:MON97ENERGYDISS, every
 *   pair, whatever the sign of w):
 *     v'  =  |w|                           (Wadsley 2008, ac_signal = 0)
 *         =  sqrt(|P_i - P_j| / rhobar)    (Price 2008, ac_signal = 1)
 *     du_i += (m_j / rhobar) alpha_AC v' (u_i - u_j) rhat_ij . Gbar
 *   (rhat_ij . Gbar is the mean of the two dW/dr, <= 0, so heat flows from
 *   the hotter particle to the colder one)
 * Per-particle viscosity strengths (alpha != NULL, the AV switches): alpha_AV
 * of the pair is (alpha_i + alpha_j)/2; beta_AV stays the global value.
 * Velocity divergence and curl (outputs divv, curlv, may be NULL), the SPH
 * estimates consistent with the grad-h density (eq. EQN:OMEGA):
 *   divv_i = -1/(Omega_i rho_i) sum_{r_ij < 2 h_i} m_j v_ij . G_i
 *   curlv_i = |1/(Omega_i rho_i) sum_{r_ij < 2 h_i} m_j v_ij x G_i|
 * (G_i vanishes beyond 2 h_i, so they run over the density neighbours).
 * Coincident pairs (r_ij = 0) add nothing to a or du and enter vsig with
 * w = 0.  With no neighbour at all vsig_i = 2 c_i (the self-pair value).
 * dt_i = C_CFL h_i / vsig_i.
 * scale_a[i] = sum_j |pair term of a_i|, scale_u[i] = sum_j |pair term of du_i|
 * (used to judge a_i ~ 0 results that arise by cancellation).
 * ------------------------------------------------------------------------- */
int orc_forces(const orc_params *p, int64_t n, const double *x, const double *y,
               const double *z, const double *vx, const double *vy, const double *vz,
               const double *m, const double *u, const double *h, const double *rho,
               const double *omega, int64_t nsel, const int64_t *sel,
               double *ax, double *ay, double *az, double *dudt, double *vsig,
               double *dt, double *scale_a, double *scale_u, int32_t *nforce,
               const double *alpha, double *divv, double *curlv)
{
    if (n < 0 || nsel < 0) return ORC_EINVAL;
    if (sel == NULL) nsel = n;
    const double gam = p->gamma;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nsel; k++) {
        int64_t i = sel ? sel[k] : k;
        double Pi = (gam - 1.0) * rho[i] * u[i];
        double ci = sqrt(gam * Pi / rho[i]);
        double Ai = Pi / (omega[i] * rho[i] * rho[i]);
        double hi2x4 = (supp(p) * h[i]) * (supp(p) * h[i]);
        double axi = 0.0, ayi = 0.0, azi = 0.0, dui = 0.0, sa = 0.0, su = 0.0;
        double vs_max = 2.0 * ci;
        int have_ngb = 0;
        int32_t cnt = 0;
        double dv = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
            double hj2x4 = (supp(p) * h[j]) * (supp(p) * h[j]);
            if (!(r2 < hi2x4 || r2 < hj2x4)) continue;
            cnt++;
            double Pj = (gam - 1.0) * rho[j] * u[j];
            double cj = sqrt(gam * Pj / rho[j]);
            if (r2 == 0.0) {
                double vs0 = ci + cj;
                if (!have_ngb || vs0 > vs_max) vs_max = vs0;
                have_ngb = 1;
                continue;
            }
            double Aj = Pj / (omega[j] * rho[j] * rho[j]);
            double r = sqrt(r2);
            double ex = dx / r, ey = dy / r, ez = dz / r;
            double gi = kdWdr(p, r, h[i]);
            double gj = kdWdr(p, r, h[j]);
            double vxij = vx[i] - vx[j], vyij = vy[i] - vy[j], vzij = vz[i] - vz[j];
            double w = (vxij * ex + vyij * ey) + vzij * ez;
            /* pressure term: vector coefficient along rhat */
            double cvec = -m[j] * (Ai * gi + Aj * gj);
            double cdu = Ai * m[j] * gi * w;
            double vs = ci + cj - p->beta * (w < 0.0 ? w : 0.0);
            if (!have_ngb || vs > vs_max) vs_max = vs;
            have_ngb = 1;
            if (w < 0.0) {
                double rhobar = 0.5 * (rho[i] + rho[j]);
                double gbar = 0.5 * (gi + gj);
                double aij = alpha ? 0.5 * (alpha[i] + alpha[j]) : p->alpha;
                cvec += (m[j] / rhobar) * aij * vs * w * gbar;
                cdu += -(m[j] / rhobar) * aij * vs * 0.5 * w * w * gbar;
            }
            /* v_ij . G_i = w gi and v_ij x G_i = gi (v_ij x rhat) */
            dv += m[j] * w * gi;
            cx += m[j] * gi * (vyij * ez - vzij * ey);
            cy += m[j] * gi * (vzij * ex - vxij * ez);
            cz += m[j] * gi * (vxij * ey - vyij * ex);
            if (p->alpha_ac != 0.0) {
                double rhobar = 0.5 * (rho[i] + rho[j]);
                double gbar = 0.5 * (gi + gj);
                double vc = p->ac_signal == 1 ? sqrt(fabs(Pi - Pj) / rhobar) : fabs(w);
                cdu += (m[j] / rhobar) * p->alpha_ac * vc * (u[i] - u[j]) * gbar;
            }
            axi += cvec * ex;
            ayi += cvec * ey;
            azi += cvec * ez;
            dui += cdu;
            sa += fabs(cvec);
            su += fabs(cdu);
        }
        ax[k] = axi;
        ay[k] = ayi;
        az[k] = azi;
        dudt[k] = dui;
        vsig[k] = vs_max;
        dt[k] = p->ccfl * h[i] / vs_max;
        scale_a[k] = sa;
        scale_u[k] = su;
        nforce[k] = cnt;
        if (divv) divv[k] = -dv / (omega[i] * rho[i]);
        if (curlv) curlv[k] = sqrt((cx * cx + cy * cy) + cz * cz) / (omega[i] * rho[i]);
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Artificial-viscosity switches (section 2.1.1 names both; the paper gives no
 * formulas, these are the published ones).
 *
 * Morris & Monaghan 1997: each particle carries alpha_i with
 *   d alpha_i / dt = -(alpha_i - alpha_min) ell c_i / h_i
 *                    + max(-divv_i, 0) (alpha_max - alpha_i)
 * (decay on tau = h/(ell c) towards alpha_min; the source max(-div v, 0) of
 * MM97 carries the (alpha_max - alpha) factor of Rosswog et al. 2000 that
 * keeps alpha below alpha_max).  alpha is integrated by the same
 * kick-drift-kick as u.
 * ------------------------------------------------------------------------- */
void orc_mm97_rate(const orc_params *p, int64_t n, const double *alpha, const double *divv,
                   const double *c, const double *h, double *adot)
{
    for (int64_t i = 0; i < n; i++) {
        double decay = -(alpha[i] - p->alpha_min) * p->av_ell * c[i] / h[i];
        double src = divv[i] < 0.0 ? -divv[i] * (p->alpha_max - alpha[i]) : 0.0;
        adot[i] = decay + src;
    }
}

/* ---------------------------------------------------------------------------
 * Cullen & Dehnen 2010, applied once per step after the forces at the end of
 * the step (step length dt):
 *   ddivv_i   = (divv_i - divv_prev_i) / dt      (finite-difference rate)
 *   xi_i      = |divv_i| / (|divv_i| + curlv_i + 1e-4 c_i / h_i)   (shear limiter)
 *   A_i       = xi_i max(-ddivv_i, 0)
 *   alpha_loc = alpha_max h_i^2 A_i / (vsig_i^2 + h_i^2 A_i), at least alpha_min
 *   alpha_i   = alpha_loc                                if alpha_i < alpha_loc
 *             = alpha_loc + (alpha_i - alpha_loc) exp(-dt 2 ell vsig_i / h_i)  otherwise
 * The rate of divv and the Balsara-type limiter stand in for CD10's
 * gradient-of-acceleration estimate and its R-weighted limiter.
 * ------------------------------------------------------------------------- */
void orc_cd10_update(const orc_params *p, int64_t n, double dt, double *alpha,
                     const double *divv, const double *divv_prev, const double *curlv,
                     const double *vsig, const double *c, const double *h)
{
    for (int64_t i = 0; i < n; i++) {
        double rate = (divv[i] - divv_prev[i]) / dt;
        double ad = fabs(divv[i]);
        double xi = ad / (ad + curlv[i] + 1e-4 * c[i] / h[i]);
        double A = rate < 0.0 ? -xi * rate : 0.0;
        double h2A = h[i] * h[i] * A;
        double aloc = p->alpha_max * h2A / (vsig[i] * vsig[i] + h2A);
        if (aloc < p->alpha_min) aloc = p->alpha_min;
        if (alpha[i] < aloc) alpha[i] = aloc;
        else alpha[i] = aloc + (alpha[i] - aloc) * exp(-dt * 2.0 * p->av_ell * vsig[i] / h[i]);
    }
}

/* ---------------------------------------------------------------------------
 * Neighbour lists, ascending j, for the selected particles.
 *   mode 0: density neighbours  j != i with r_ij^2 < (2 h_i)^2
 *   mode 1: force neighbours    j != i with r_ij^2 < (2 h_i)^2 or < (2 h_j)^2
 * counts[k] is always filled.  If idx != NULL, the lists are written back to
 * back (offsets = exclusive prefix sum of counts); ORC_ECAP if they exceed cap.
 * ------------------------------------------------------------------------- */
int orc_neighbours(const orc_params *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *h, int32_t mode, int64_t nsel,
                   const int64_t *sel, int64_t *counts, int32_t *idx, int64_t cap)
{
    if (n < 0 || nsel < 0 || (mode != 0 && mode != 1)) return ORC_EINVAL;
    if (sel == NULL) nsel = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nsel; k++) {
        int64_t i = sel ? sel[k] : k;
        double hi2x4 = (supp(p) * h[i]) * (supp(p) * h[i]);
        int64_t c = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
            int in = r2 < hi2x4;
            if (mode == 1) in = in || r2 < (supp(p) * h[j]) * (supp(p) * h[j]);
            if (in) c++;
        }
        counts[k] = c;
    }
    if (!idx) return ORC_OK;
    int64_t total = 0;
    for (int64_t k = 0; k < nsel; k++) total += counts[k];
    if (total > cap) return ORC_ECAP;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nsel + 1));
    if (!off) return ORC_ENOMEM;
    off[0] = 0;
    for (int64_t k = 0; k < nsel; k++) off[k + 1] = off[k] + counts[k];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nsel; k++) {
        int64_t i = sel ? sel[k] : k;
        double hi2x4 = (supp(p) * h[i]) * (supp(p) * h[i]);
        int64_t c = off[k];
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
            int in = r2 < hi2x4;
            if (mode == 1) in = in || r2 < (supp(p) * h[j]) * (supp(p) * h[j]);
            if (in) idx[c++] = (int32_t)j;
        }
    }
    free(off);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Kick-drift-kick leapfrog (eqs. EQN:LFKDK1, EQN:LFKDK2) with the SPH main
 * loop order of section 5.1: integrate, neighbours, h + forces, time-step,
 * closing kick.  The accelerations at step n+1 need velocities and internal
 * energies at n+1, so they are evaluated at the predicted values
 * v* = v^n + a^n dt and u* = u^n + du^n dt (the paper leaves this open).
 * u is integrated with the same kick-drift-kick pattern as v.
 *
 * On entry h holds a guess; a, du, dt_i are computed first.  dt_fixed > 0
 * fixes the step; otherwise each step uses min_i dt_i of the latest forces.
 * energy[s] = sum 1/2 m v^2 + sum m u after s steps (s = 0..nsteps),
 * dt_used[s] the step taken by step s+1.
 * ------------------------------------------------------------------------- */
static double total_energy(int64_t n, const double *m, const double *vx, const double *vy,
                           const double *vz, const double *u)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; i++)
        e += 0.5 * m[i] * ((vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i]) + m[i] * u[i];
    return e;
}

/* Density and forces of every particle.  av holds the switch state:
 * alpha (viscosity strength per particle, NULL without a switch) and the
 * outputs divv, curlv, vsig, c (sound speed) of this evaluation. */
typedef struct {
    const double *alpha;
    double *divv, *curlv, *vsig, *c;
} orc_av_io;

static int eval_all(const orc_params *p, int64_t n, const double *x, const double *y,
                    const double *z, const double *vx, const double *vy, const double *vz,
                    const double *m, const double *u, double *h, double *rho,
                    double *omega, double *ax, double *ay, double *az, double *du,
                    double *dt, double *work, orc_av_io av)
{
    double *hn = work, *drho = work + n, *sa = work + 3 * n, *su = work + 4 * n;
    int32_t *cnt = (int32_t *)(work + 5 * n);
    double *vsig = av.vsig ? av.vsig : work + 2 * n;
    int rc = orc_density(p, n, x, y, z, m, h, n, NULL, hn, rho, drho, omega, cnt);
    if (rc != ORC_OK) return rc;
    memcpy(h, hn, sizeof(double) * (size_t)n);
    rc = orc_forces(p, n, x, y, z, vx, vy, vz, m, u, h, rho, omega, n, NULL, ax, ay, az,
                    du, vsig, dt, sa, su, cnt, av.alpha, av.divv, av.curlv);
    if (rc == ORC_OK && av.c)
        for (int64_t i = 0; i < n; i++) av.c[i] = sqrt(p->gamma * (p->gamma - 1.0) * u[i]);
    return rc;
}

/* alpha (in/out, n values) is the per-particle viscosity strength of the
 * switch in p->av_switch; ignored (may be NULL) without a switch. */
int orc_kdk(const orc_params *p, int64_t n, double *x, double *y, double *z, double *vx,
            double *vy, double *vz, const double *m, double *u, double *h,
            int32_t nsteps, double dt_fixed, double *energy, double *dt_used, double *alpha)
{
    if (n <= 0 || nsteps < 0) return ORC_EINVAL;
    const int sw = p->av_switch;
    if (sw && !alpha) return ORC_EINVAL;
    size_t N = (size_t)n;
    double *buf = (double *)malloc(sizeof(double) * N * 30);
    if (!buf) return ORC_ENOMEM;
    double *rho = buf, *omega = buf + N, *ax = buf + 2 * N, *ay = buf + 3 * N,
           *az = buf + 4 * N, *du = buf + 5 * N, *dt = buf + 6 * N, *vxh = buf + 7 * N,
           *vyh = buf + 8 * N, *vzh = buf + 9 * N, *uh = buf + 10 * N, *vxp = buf + 11 * N,
           *vyp = buf + 12 * N, *vzp = buf + 13 * N, *up = buf + 14 * N, *work = buf + 15 * N;
    /* work: 5N doubles + N int32 (eval_all scratch) */
    double *divv = buf + 21 * N, *curlv = buf + 22 * N, *vsig = buf + 23 * N,
           *cs = buf + 24 * N, *adot = buf + 25 * N, *alh = buf + 26 * N, *alp = buf + 27 * N,
           *dprev = buf + 28 * N;
    orc_av_io av = {sw ? alpha : NULL, divv, curlv, vsig, cs};
    int rc = eval_all(p, n, x, y, z, vx, vy, vz, m, u, h, rho, omega, ax, ay, az, du, dt, work, av);
    if (rc != ORC_OK) { free(buf); return rc; }
    if (sw == 1) orc_mm97_rate(p, n, alpha, divv, cs, h, adot);
    if (sw == 2) memcpy(dprev, divv, sizeof(double) * N);
    if (energy) energy[0] = total_energy(n, m, vx, vy, vz, u);
    double L[3];
    for (int k = 0; k < 3; k++) L[k] = p->hi[k] - p->lo[k];
    for (int32_t s = 0; s < nsteps; s++) {
        double d = dt_fixed;
        if (!(d > 0.0)) {
            d = dt[0];
            for (int64_t i = 1; i < n; i++) if (dt[i] < d) d = dt[i];
        }
        if (dt_used) dt_used[s] = d;
        for (int64_t i = 0; i < n; i++) {
            vxh[i] = vx[i] + 0.5 * d * ax[i];
            vyh[i] = vy[i] + 0.5 * d * ay[i];
            vzh[i] = vz[i] + 0.5 * d * az[i];
            uh[i] = u[i] + 0.5 * d * du[i];
            double *pos[3] = {&x[i], &y[i], &z[i]};
            double vel[3] = {vxh[i], vyh[i], vzh[i]};
            for (int k = 0; k < 3; k++) {
                double q = *pos[k] + d * vel[k];
                if (p->periodic) {
                    if (q >= p->hi[k]) q -= L[k];
                    else if (q < p->lo[k]) q += L[k];
                }
                *pos[k] = q;
            }
            vxp[i] = vxh[i] + 0.5 * d * ax[i];
            vyp[i] = vyh[i] + 0.5 * d * ay[i];
            vzp[i] = vzh[i] + 0.5 * d * az[i];
            up[i] = uh[i] + 0.5 * d * du[i];
            if (sw == 1) {
                alh[i] = alpha[i] + 0.5 * d * adot[i];
                alp[i] = alh[i] + 0.5 * d * adot[i];
            }
        }
        /* the forces at the end of the step see the predicted alpha (MM97) or
         * the alpha of the start of the step (CD10) */
        av.alpha = sw == 1 ? alp : (sw == 2 ? alpha : NULL);
        rc = eval_all(p, n, x, y, z, vxp, vyp, vzp, m, up, h, rho, omega, ax, ay, az, du, dt,
                      work, av);
        if (rc != ORC_OK) { free(buf); return rc; }
        if (sw == 1) orc_mm97_rate(p, n, alp, divv, cs, h, adot);
        if (sw == 2) {
            orc_cd10_update(p, n, d, alpha, divv, dprev, curlv, vsig, cs, h);
            memcpy(dprev, divv, sizeof(double) * N);
        }
        for (int64_t i = 0; i < n; i++) {
            vx[i] = vxh[i] + 0.5 * d * ax[i];
            vy[i] = vyh[i] + 0.5 * d * ay[i];
            vz[i] = vzh[i] + 0.5 * d * az[i];
            u[i] = uh[i] + 0.5 * d * du[i];
            if (sw == 1) alpha[i] = alh[i] + 0.5 * d * adot[i];
        }
        if (energy) energy[s + 1] = total_energy(n, m, vx, vy, vz, u);
    }
    free(buf);
    return ORC_OK;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------------------
 * Meshless finite-volume geometry (section 2.2).
 *
 * Number density and smoothing length (eqs. EQN:MFV_NDENS, EQN:MFV_HN):
 * n_i = sum_j W(r_ij, h_i) with h_i = eta n_i^(-1/3) -- the density solve
 * above with every mass set to 1 (then rho_i = n_i and h^3 rho = eta^3).
 *
 * Given h_i and n_i, for each selected particle:
 *   psi_j(r_i)   = W(r_ij, h_i) / n_i
 *   E_i          = sum_j (r_j - r_i)(r_j - r_i)^T psi_j(r_i)    (EQN:MFVEMATRIX)
 *   B_i          = E_i^-1
 *   psit_j(r_i)  = B_i (r_j - r_i) psi_j(r_i)                   (EQN:MFVPSI)
 *   grad f_i     = sum_j (f_j - f_i) psit_j(r_i)                (EQN:MFVGRADIENT)
 * Condition number: cond_i = |E_i|_F |B_i|_F / 3 (Frobenius norms, 1 for a
 * multiple of the identity).  When it exceeds 100 the gradient is the
 * direct SPH estimate instead, psit_j -> V_i grad_i W(r_ij, h_i) with
 * V_i = 1/n_i (section 2.2.2).  The sums run over j with r_ij < 2 h_i (W
 * vanishes beyond); the particle itself contributes nothing (r = 0).
 * B is returned as xx, xy, xz, yy, yz, zz (6 per particle), grad as
 * nfields x 3 per particle.
 * ------------------------------------------------------------------------- */
static int inv3(const double E[3][3], double B[3][3])
{
    double c00 = E[1][1] * E[2][2] - E[1][2] * E[2][1];
    double c01 = E[1][2] * E[2][0] - E[1][0] * E[2][2];
    double c02 = E[1][0] * E[2][1] - E[1][1] * E[2][0];
    double det = E[0][0] * c00 + E[0][1] * c01 + E[0][2] * c02;
    if (det == 0.0 || !isfinite(det)) return 0;
    double id = 1.0 / det;
    B[0][0] = c00 * id;
    B[1][0] = c01 * id;
    B[2][0] = c02 * id;
    B[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) * id;
    B[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) * id;
    B[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) * id;
    B[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) * id;
    B[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) * id;
    B[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) * id;
    return 1;
}

int orc_mfv_gradients(const orc_params *p, int64_t n, const double *x, const double *y,
                      const double *z, const double *h, const double *ndens, int32_t nfields,
                      const double *const *f, int64_t nsel, const int64_t *sel, double *Bout,
                      double *cond, double *grad)
{
    if (n < 0 || nsel < 0 || nfields < 0 || nfields > 8) return ORC_EINVAL;
    if (sel == NULL) nsel = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nsel; k++) {
        int64_t i = sel ? sel[k] : k;
        double hi2x4 = (supp(p) * h[i]) * (supp(p) * h[i]);
        double E[3][3] = {{0}}, B[3][3];
        for (int64_t j = 0; j < n; j++) {
            double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
            if (!(r2 < hi2x4)) continue;
            double d[3] = {-dx, -dy, -dz};   /* r_j - r_i */
            double psi = kW(p, sqrt(r2), h[i]) / ndens[i];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) E[a][b] += d[a] * d[b] * psi;
        }
        int ok = inv3(E, B);
        double nE = 0.0, nB = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                nE += E[a][b] * E[a][b];
                nB += ok ? B[a][b] * B[a][b] : INFINITY;
            }
        double cn = sqrt(nE) * sqrt(nB) / 3.0;
        int sph = !(cn <= 100.0);
        for (int q = 0; q < nfields; q++)
            for (int a = 0; a < 3; a++) grad[(k * nfields + q) * 3 + a] = 0.0;
        for (int64_t j = 0; j < n; j++) {
            double dx, dy, dz, r2 = pair_r2(p, x, y, z, i, j, &dx, &dy, &dz);
            if (!(r2 < hi2x4) || r2 == 0.0) continue;
            double d[3] = {-dx, -dy, -dz};
            double r = sqrt(r2);
            double psit[3];
            if (!sph) {
                double psi = kW(p, r, h[i]) / ndens[i];
                for (int a = 0; a < 3; a++)
                    psit[a] = (B[a][0] * d[0] + B[a][1] * d[1] + B[a][2] * d[2]) * psi;
            } else {
                /* V_i grad_i W = (1/n_i) dW/dr (r_i - r_j)/r */
                double g = kdWdr(p, r, h[i]) / ndens[i] / r;
                for (int a = 0; a < 3; a++) psit[a] = -d[a] * g;
            }
            for (int q = 0; q < nfields; q++) {
                double df = f[q][j] - f[q][i];
                for (int a = 0; a < 3; a++) grad[(k * nfields + q) * 3 + a] += df * psit[a];
            }
        }
        if (Bout) {
            double *o = Bout + 6 * k;
            o[0] = B[0][0]; o[1] = B[0][1]; o[2] = B[0][2];
            o[3] = B[1][1]; o[4] = B[1][2]; o[5] = B[2][2];
        }
        if (cond) cond[k] = cn;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Hierarchical block time-steps (section 2.1.4) with a predictive and
 * reactive time-step limiter in the manner of Saitoh & Makino 2009
 * (section 2.1.5), kick-drift-kick.
 *
 * Timeline: one level-0 step of length dt_max holds 2^lmax integer ticks; a
 * particle on level l takes steps of 2^(lmax - l) ticks.  At a full
 * synchronisation (start, and whenever the level-0 step ends) dt_max is
 * recomputed from the CFL steps dt_i of every particle as
 *   dt_max = min_i dt_i 2^k,  k the largest integer with dt_max <= max_i dt_i
 * (the paper fixes dt_max from the time-steps available; this choice makes
 * the deepest occupied level step at exactly the smallest dt_i, and a set
 * whose dt_i lie within a factor 2 is integrated exactly as by the global
 * scheme), and every particle takes the level
 *   level(dt_i) = smallest l <= lmax with dt_max 2^-l <= dt_i
 * (the comparisons are exact: 2^k scales without rounding).  Each sub-step:
 *   T' = min_i t_end_i; every particle drifts x += v_half (T' - T); the
 *   particles with t_end_i = T' are active;
 *   all particles are predicted to T': v* = v_half + a (T' - t_mid), u
 *   likewise (t_mid the middle of the particle's step; for an active
 *   particle this is the usual predictor v_half + a dt/2);
 *   density (h solve) and forces for the active particles only, with the
 *   stored h, rho, Omega and the predicted v, u of inactive neighbours;
 *   limiter information, over the force neighbours j of each active i
 *   (r_ij < 2 max(h_i, h_j)): lmx_i = max level_j (old levels), and every
 *   inactive j with level_j < level_i - lim is marked with level_i;
 *   closing kick of the active particles with their new a, du;
 *   new levels of the active particles: any deeper level at once; one level
 *   shallower only when T' is a multiple of that shallower step, else the
 *   old level; never shallower than lmx_i - lim (predictive limiter);
 *   a marked inactive particle j moves to level mark_j - lim, its step ends
 *   at the first multiple of the new step after T', and its opening kick is
 *   corrected to the shortened step: v_half -= a (old - new step)/2, u
 *   likewise (reactive limiter);
 *   opening kick of the active particles with their new step.
 * At a full synchronisation the new levels are the fresh ones (with the
 * predictive limiter from this sub-step's neighbour levels; none at the
 * start).  The run stops after nfull level-0 steps, synchronised: x, v, u
 * are those of the synchronisation, the levels those assigned there for the
 * next level-0 step.  energy[k] = sum 1/2 m v^2 + m u at the k-th full
 * synchronisation; nsub = sub-steps taken; levels = final levels;
 * time_out = elapsed time; active_total = active particles summed over the
 * sub-steps (the particle updates the scheme made).  Returns ORC_EBOX-like errors of the solves, or
 * ORC_EINVAL if a particle needs a level beyond lmax.
 *
 * Viscosity switches (p->av_switch; alpha in/out as in orc_kdk, required
 * with a switch, ignored without one) follow each particle's own steps:
 *   MM97: alpha is integrated like u.  d alpha/dt comes from each force
 *   evaluation of the particle (from its predicted alpha, div v, c and h);
 *   alpha is opened, predicted to T' (the forces see the predicted alpha of
 *   every particle, active or not), closed, and its opening kick corrected
 *   by the reactive limiter exactly as u is.
 *   CD10: after the forces of a sub-step, each active particle's alpha is
 *   updated with its own step length (t_end - t_start) tick and the rate
 *   of div v since its previous evaluation; the forces see every
 *   particle's current alpha (that of the start of an active particle's
 *   step).  At the start, div v of the first evaluation is the previous one.
 * ------------------------------------------------------------------------- */
static double block_dtmax(int64_t n, const double *dt)
{
    double lo = dt[0], hi = dt[0];
    for (int64_t i = 1; i < n; i++) {
        if (dt[i] < lo) lo = dt[i];
        if (dt[i] > hi) hi = dt[i];
    }
    int k = 0;
    while (k < 1000 && ldexp(lo, k + 1) <= hi) k++;
    return ldexp(lo, k);
}

static int level_of(double dt, double dtmax, int lmax)
{
    int l = 0;
    while (l < lmax && ldexp(dtmax, -l) > dt) l++;
    return ldexp(dtmax, -l) > dt ? -1 : l;
}

int orc_kdk_block(const orc_params *p, int64_t n, double *x, double *y, double *z, double *vx,
                  double *vy, double *vz, const double *m, double *u, double *h, int32_t lmax,
                  int32_t lim, int32_t nfull, double *energy, int64_t *nsub, int32_t *levels,
                  double *time_out, int64_t *active_total, double *alpha)
{
    if (n <= 0 || lmax < 0 || lmax > 40 || lim < 0 || nfull < 0) return ORC_EINVAL;
    const int sw = p->av_switch;
    if (sw && !alpha) return ORC_EINVAL;
    size_t N = (size_t)n;
    double *buf = (double *)malloc(sizeof(double) * N * 31);
    int64_t *ib = (int64_t *)malloc(sizeof(int64_t) * N * 6);
    if (!buf || !ib) { free(buf); free(ib); return ORC_ENOMEM; }
    double *vhx = buf, *vhy = buf + N, *vhz = buf + 2 * N, *uh = buf + 3 * N, *ax = buf + 4 * N,
           *ay = buf + 5 * N, *az = buf + 6 * N, *du = buf + 7 * N, *rho = buf + 8 * N,
           *omega = buf + 9 * N, *dt = buf + 10 * N, *vpx = buf + 11 * N, *vpy = buf + 12 * N,
           *vpz = buf + 13 * N, *up = buf + 14 * N, *hn = buf + 15 * N, *t1 = buf + 16 * N,
           *t2 = buf + 17 * N, *t3 = buf + 18 * N, *t4 = buf + 19 * N, *t5 = buf + 20 * N,
           *t6 = buf + 21 * N, *t7 = buf + 22 * N, *t8 = buf + 23 * N, *t9 = buf + 24 * N;
    int64_t *ts = ib, *te = ib + N, *lev = ib + 2 * N, *lmx = ib + 3 * N, *mark = ib + 4 * N,
            *sel = ib + 5 * N;
    int32_t *cnt = (int32_t *)t9;
    /* switch state: alpha after the opening kick, predicted alpha and its
     * rate (MM97); div v of the previous evaluation (CD10); div v and curl v
     * of the selection */
    double *alh = buf + 25 * N, *alp = buf + 26 * N, *adot = buf + 27 * N, *dprev = buf + 28 * N,
           *dvs = buf + 29 * N, *cvs = buf + 30 * N;
    const double cfac = p->gamma * (p->gamma - 1.0);
    const int64_t P0 = (int64_t)1 << lmax;
    double Lb[3];
    for (int k = 0; k < 3; k++) Lb[k] = p->hi[k] - p->lo[k];
    int rc = ORC_OK;
    double tnow = 0.0;
    int64_t subs = 0, updates = 0;

    /* initial evaluation of every particle */
    rc = orc_density(p, n, x, y, z, m, h, n, NULL, hn, rho, t1, omega, cnt);
    if (rc != ORC_OK) goto out;
    memcpy(h, hn, sizeof(double) * N);
    rc = orc_forces(p, n, x, y, z, vx, vy, vz, m, u, h, rho, omega, n, NULL, ax, ay, az, du, t2,
                    dt, t3, t4, cnt, sw ? alpha : NULL, sw ? dvs : NULL, sw ? cvs : NULL);
    if (rc != ORC_OK) goto out;
    for (int64_t i = 0; sw && i < n; i++) {
        double c = sqrt(cfac * u[i]);
        if (sw == 1) orc_mm97_rate(p, 1, &alpha[i], &dvs[i], &c, &h[i], &adot[i]);
        else dprev[i] = dvs[i];
    }
    double dtmax = block_dtmax(n, dt);
    for (int64_t i = 0; i < n; i++) {
        int l = level_of(dt[i], dtmax, lmax);
        if (l < 0) { rc = ORC_EINVAL; goto out; }
        lev[i] = l;
        ts[i] = 0;
        te[i] = P0 >> l;
    }
    if (energy) energy[0] = total_energy(n, m, vx, vy, vz, u);
    int64_t T = 0;
    int32_t full = 0;
    double tick = dtmax / (double)P0;
    /* opening kicks */
    for (int64_t i = 0; i < n; i++) {
        double hs = 0.5 * (double)(te[i] - ts[i]) * tick;
        vhx[i] = vx[i] + ax[i] * hs;
        vhy[i] = vy[i] + ay[i] * hs;
        vhz[i] = vz[i] + az[i] * hs;
        uh[i] = u[i] + du[i] * hs;
        if (sw == 1) alh[i] = alpha[i] + adot[i] * hs;
    }
    while (full < nfull) {
        int64_t Tn = te[0];
        for (int64_t i = 1; i < n; i++) if (te[i] < Tn) Tn = te[i];
        double dlt = (double)(Tn - T) * tick;
        int64_t na = 0;
        for (int64_t i = 0; i < n; i++) {
            double *pos[3] = {&x[i], &y[i], &z[i]};
            double vel[3] = {vhx[i], vhy[i], vhz[i]};
            for (int k = 0; k < 3; k++) {
                double q = *pos[k] + dlt * vel[k];
                if (p->periodic) {
                    if (q >= p->hi[k]) q -= Lb[k];
                    else if (q < p->lo[k]) q += Lb[k];
                }
                *pos[k] = q;
            }
            double dm = ((double)Tn - 0.5 * (double)(ts[i] + te[i])) * tick;
            vpx[i] = vhx[i] + ax[i] * dm;
            vpy[i] = vhy[i] + ay[i] * dm;
            vpz[i] = vhz[i] + az[i] * dm;
            up[i] = uh[i] + du[i] * dm;
            if (sw == 1) alp[i] = alh[i] + adot[i] * dm;
            if (te[i] == Tn) sel[na++] = i;
            lmx[i] = 0;
            mark[i] = -1;
        }
        /* density and forces of the active particles */
        rc = orc_density(p, n, x, y, z, m, h, na, sel, t1, t2, t3, t4, cnt);
        if (rc != ORC_OK) goto out;
        for (int64_t k = 0; k < na; k++) {
            int64_t i = sel[k];
            h[i] = t1[k];
            rho[i] = t2[k];
            omega[i] = t4[k];
        }
        rc = orc_forces(p, n, x, y, z, vpx, vpy, vpz, m, up, h, rho, omega, na, sel, t1, t2, t3,
                        t4, t5, t6, t7, t8, cnt, sw == 1 ? alp : (sw == 2 ? alpha : NULL),
                        sw ? dvs : NULL, sw ? cvs : NULL);
        if (rc != ORC_OK) goto out;
        for (int64_t k = 0; k < na; k++) {
            int64_t i = sel[k];
            ax[i] = t1[k]; ay[i] = t2[k]; az[i] = t3[k]; du[i] = t4[k]; dt[i] = t6[k];
            /* the switch from this evaluation (c from the predicted u the
             * forces used; the step that ends now for CD10) */
            double c = sqrt(cfac * up[i]);
            if (sw == 1) orc_mm97_rate(p, 1, &alp[i], &dvs[k], &c, &h[i], &adot[i]);
            if (sw == 2) {
                double dti = (double)(te[i] - ts[i]) * tick;
                orc_cd10_update(p, 1, dti, &alpha[i], &dvs[k], &dprev[i], &cvs[k], &t5[k], &c,
                                &h[i]);
                dprev[i] = dvs[k];
            }
        }
        /* limiter information over the force neighbours of the active particles */
        for (int64_t k = 0; k < na; k++) {
            int64_t i = sel[k];
            double hi2x4 = (supp(p) * h[i]) * (supp(p) * h[i]);
            int64_t mx = 0;
            for (int64_t j = 0; j < n; j++) {
                if (j == i) continue;
                double ddx, ddy, ddz, r2 = pair_r2(p, x, y, z, i, j, &ddx, &ddy, &ddz);
                if (!(r2 < hi2x4 || r2 < (supp(p) * h[j]) * (supp(p) * h[j]))) continue;
                if (lev[j] > mx) mx = lev[j];
                if (te[j] != Tn && lev[j] < lev[i] - lim && lev[i] > mark[j]) mark[j] = lev[i];
            }
            lmx[i] = mx;
        }
        /* closing kicks */
        for (int64_t k = 0; k < na; k++) {
            int64_t i = sel[k];
            double hs = 0.5 * (double)(te[i] - ts[i]) * tick;
            vx[i] = vhx[i] + ax[i] * hs;
            vy[i] = vhy[i] + ay[i] * hs;
            vz[i] = vhz[i] + az[i] * hs;
            u[i] = uh[i] + du[i] * hs;
            if (sw == 1) alpha[i] = alh[i] + adot[i] * hs;
        }
        tnow += dlt;
        subs++;
        updates += na;
        if (Tn == P0) {
            /* full synchronisation: every particle is active */
            full++;
            if (energy) energy[full] = total_energy(n, m, vx, vy, vz, u);
            dtmax = block_dtmax(n, dt);
            tick = dtmax / (double)P0;
            for (int64_t i = 0; i < n; i++) {
                int l = level_of(dt[i], dtmax, lmax);
                if (l < 0) { rc = ORC_EINVAL; goto out; }
                if (l < lmx[i] - lim) l = (int)(lmx[i] - lim);
                if (l > lmax) { rc = ORC_EINVAL; goto out; }
                lev[i] = l;
                ts[i] = 0;
                te[i] = P0 >> l;
            }
            T = 0;
        } else {
            for (int64_t k = 0; k < na; k++) {
                int64_t i = sel[k];
                int l = level_of(dt[i], dtmax, lmax);
                if (l < 0) { rc = ORC_EINVAL; goto out; }
                int64_t cur = lev[i], nl;
                if (l > cur) nl = l;
                else if (l < cur && Tn % (P0 >> (cur - 1)) == 0) nl = cur - 1;
                else nl = cur;
                if (nl < lmx[i] - lim) nl = lmx[i] - lim;
                if (nl > lmax) { rc = ORC_EINVAL; goto out; }
                lev[i] = nl;
                ts[i] = Tn;
                te[i] = Tn + (P0 >> nl);
            }
            for (int64_t j = 0; j < n; j++) {
                /* only inactive particles were marked */
                if (mark[j] < 0 || lev[j] >= mark[j] - lim) continue;
                int64_t nl = mark[j] - lim;
                if (nl > lmax) { rc = ORC_EINVAL; goto out; }
                int64_t st = P0 >> nl;
                int64_t tn = (Tn / st + 1) * st;
                double cut = 0.5 * (double)((te[j] - ts[j]) - (tn - ts[j])) * tick;
                vhx[j] -= ax[j] * cut;
                vhy[j] -= ay[j] * cut;
                vhz[j] -= az[j] * cut;
                uh[j] -= du[j] * cut;
                if (sw == 1) alh[j] -= adot[j] * cut;
                lev[j] = nl;
                te[j] = tn;
            }
            T = Tn;
        }
        /* opening kicks of the particles that start a step */
        for (int64_t k = 0; k < na; k++) {
            int64_t i = sel[k];
            double hs = 0.5 * (double)(te[i] - ts[i]) * tick;
            vhx[i] = vx[i] + ax[i] * hs;
            vhy[i] = vy[i] + ay[i] * hs;
            vhz[i] = vz[i] + az[i] * hs;
            uh[i] = u[i] + du[i] * hs;
            if (sw == 1) alh[i] = alpha[i] + adot[i] * hs;
        }
        if (full == nfull && T == 0) break;
    }
    if (levels)
        for (int64_t i = 0; i < n; i++) levels[i] = (int32_t)lev[i];
out:
    if (nsub) *nsub = subs;
    if (time_out) *time_out = tnow;
    if (active_total) *active_total = updates;
    free(buf);
    free(ib);
    return rc;
}
