// Argument blocks of the pair kernels (density and h solve, forces,
// neighbour export, MFV geometry) and the launches of their instantiations.
// The kernels are built once per smoothing kernel of section 2 (M4 cubic
// spline, quintic spline), each in a translation unit of its own
// (pairs_m4.hip, pairs_quintic.hip; the kernel code is in pairs.hpp); the
// dispatching code (pairs.hip) sees only these declarations.
#pragma once

#include "sph_internal.hpp"

namespace sph {

template <class Args>
struct Batch {
    int32_t nreq;
    int32_t claim;   // home leaves per claim of the persistent loop (>= 1)
    int32_t stage;   // candidate leaves per staged group (1..128/G)
    uint32_t *work;
    double *cache;   // density loop: per-block candidate cache (nullptr: none)
    const Args *req[kMaxBatch];
};

struct DensArgs {
    int64_t n;
    const TreeInfo *tree;
    const uint32_t *lstart;
    uint32_t *work;
    Box box;
    const Node *nodes;
    const double *x, *y, *z, *m;
    const float *fx, *fy, *fz;
    double *h, *rho, *omega;
    int32_t *nngb;
    int32_t *status;
    int64_t *counts;
    const double *mrange;   // smallest and largest mass of the set
    int32_t count_tests;    // also count box and candidate tests (diagnostics)
    double eta3;
    double h_rtol;
    double walk_margin;
    int32_t max_iter;
    // block time-steps: particles that take part (nullptr: all) and their
    // count per leaf (leaves without any are skipped); the home leaves are
    // then leaf_list[0 .. *leaf_count) (nullptr: every leaf)
    const int32_t *active, *leaf_act;
    const uint32_t *leaf_list, *leaf_count;
};

struct ForceArgs {
    int64_t n;
    const TreeInfo *tree;
    const uint32_t *lstart;
    uint32_t *work;
    Box box;
    const Node *nodes;
    const double *x, *y, *z, *h;
    const ForceRec *rec;
    const ForceRec32 *rec32;   // FP32-pair: the single-precision records
    const float *fx, *fy, *fz;
    double *ax, *ay, *az, *du, *vsig, *dt;
    int32_t *nforce;
    int32_t *status;
    int64_t *counts;
    double alpha, beta, ccfl;
    // artificial conductivity: strength, 1 / (gamma (gamma - 1)), 1 / gamma,
    // and the signal speed (0: |v_ij . rhat_ij|, 1: sqrt(|P_i - P_j| / rhobar))
    double alpha_ac, u_per_c2, inv_gamma;
    int32_t ac_price;
    int32_t count_tests;    // also count box and candidate tests (diagnostics)
    // per-particle viscosity strengths (sorted; nullptr: alpha for every pair),
    // Omega (sorted) and the div v, |curl v| outputs (nullptr: not wanted)
    const double *alpha_p;
    const double *omega;
    double *divv, *curlv;
    // block time-steps: the active set (nullptr: all), its count per leaf, the
    // home leaves leaf_list[0 .. *leaf_count) (nullptr: every leaf), and the
    // limiter: levels, deepest neighbour level (out, active particles),
    // wake-up marks of inactive neighbours (atomic max), level spread lim
    const int32_t *active, *leaf_act;
    const uint32_t *leaf_list, *leaf_count;
    const int32_t *lev;
    int32_t *lmx, *mark;
    int32_t lim;
};

struct NgbArgs {
    int64_t n;
    const TreeInfo *tree;
    const uint32_t *lstart;
    uint32_t *work;
    Box box;
    const Node *nodes;
    const double *x, *y, *z, *h;
    const uint32_t *id;        // sorted -> caller index
    int32_t mode;
    int64_t *counts;           // sorted order (pass 1)
    const int64_t *offsets;    // caller order (pass 2)
    int32_t *idx;
    int64_t cap;
    int32_t *status;
};

constexpr int kMfvFields = 4;
struct MfvArgs {
    int64_t n;
    const TreeInfo *tree;
    const uint32_t *lstart;
    uint32_t *work;
    Box box;
    const Node *nodes;
    const double *x, *y, *z, *h, *ndens;
    int32_t nf;
    const double *f[kMfvFields];
    double *B[6];                  // xx, xy, xz, yy, yz, zz
    double *cond;
    double *grad[3 * kMfvFields];  // field q, axis a at 3 q + a
    int32_t *status;
};

// One launch of a pair kernel instantiated for smoothing kernel K
// (SPH_KERNEL_M4 or SPH_KERNEL_QUINTIC) at leaf size G (8, 16 or 32) and
// precision prec, on stream st.  ac / sw select the force variant carrying
// artificial conductivity / per-particle alpha and div v, curl v.
template <int K>
void launch_density(hipStream_t st, int G, int prec, unsigned grid, const Batch<DensArgs> &B);
template <int K>
void launch_forces(hipStream_t st, int G, int prec, bool ac, bool sw, unsigned grid,
                   const Batch<ForceArgs> &B);
template <int K>
void launch_neighbours(hipStream_t st, int G, unsigned grid, const NgbArgs &a, int pass);
template <int K>
void launch_mfv(hipStream_t st, int G, unsigned grid, const MfvArgs &a);

} // namespace sph
