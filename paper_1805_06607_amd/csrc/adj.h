// Device-side descriptors and launch entry points of the discrete adjoint
// (vector-Jacobian products of the right-hand side, the donor data and the
// objective), shared by the host runtime (runtime.cpp) and adjoint.hip.
#pragma once
#include "kern.h"

namespace mrk {

// Adjoint of one grid's right-hand side R(q, recv) at one evaluation:
//   lam_q    += (dR/dq)^T    lamF
//   lam_recv  = (dR/drecv)^T lamF   (rows of the receivers of g; the caller
//                                    zeroes them first)
// in three launches over the grid's points:
//   flux:  mu^m = adjoint of the directional flux of direction m, gathered
//          from the outputs whose SBP rows read the point (transposed rows);
//   point: the local Jacobians of the fluxes and SAT penalties at the point
//          (forward-mode dual numbers) -> direct adjoint of q (lqd), adjoint
//          of the index-space derivatives of the primitives (kap), adjoint of
//          the receiver row; points without SAT faces one lane each, the SAT
//          points (listed) one lane per (point, input direction), then one
//          lane per SAT point collects;
//   grad:  kap gathered through the transposed gradient rows and the
//          primitive map's Jacobian -> lam_q.
struct AdjRhs {
    GridDev g;              // g.recv: the forward receiver rows of this evaluation
    Phys ph;
    const double *q;        // forward state, nv x N
    const double *lamF;     // adjoint of R, nv x N
    double *mu;             // dim x nv x N scratch
    double *kap;            // dim x (dim+1) x N scratch
    double *lqd;            // nv x N scratch
    double *lam_recv;       // rows x (nv + dim (nv-1)), written at receiver rows
    double *lam_q;          // nv x N, accumulated
    const int32_t *bpts;    // the nb points ending a run in some direction (SAT points)
    int nb;
    double *bres;           // nb x (nv + dim (dim+1) + nv + dim (nv-1)) scratch
};

// Adjoint of one link's donor data at one time: the receiving grid's
// receiver-row adjoints (rows row0 .. row0 + nrecv - 1) pushed back onto the
// donor grid's input state y (an own-step state or an extrapolant):
//   unique donor points u: Lambda_u = sum over the entries naming u of
//          w * lam_recv row (entries listed per point, ascending), then the
//          local Jacobian of (q, F^V) at u -> uq (direct), uk (adjoint of
//          the index-space derivatives of the primitives at u);
//   stencil points c (every point a donor gradient reads): uk gathered
//          through the transposed rows, the primitive map's Jacobian and uq
//          when c is itself a donor point -> lam_y.
// Each point is written by one lane, so the result does not depend on the
// order in which lanes run.
struct AdjDonor {
    GridDev g;              // donor grid
    Phys ph;
    const double *y;        // donor input state, nv x N
    const double *lam_recv; // receiving grid's receiver-row adjoints
    int32_t row0;
    int S;
    const int32_t *upts;    // nu unique donor points
    int64_t nu;
    const int32_t *ustart;  // nu + 1
    const int32_t *uent;    // entry indices r * S + e of the link's receivers
    const double *w;        // nrecv x S weights of the link
    double *uq;             // nu x nv scratch
    double *uk;             // nu x dim x (dim+1) scratch
    const int32_t *cpts;    // nc stencil points
    int64_t nc;
    const int32_t *cstart;  // nc + 1
    const int32_t *cent;    // (u << 8) | (m << 4) | (o + 8): unique point u reads c at offset o along m
    const int32_t *cself;   // per stencil point: its unique index, or -1
    double *lam_y;          // nv x N, accumulated
};

// Pressure functional at listed points of one state: acc[0] += tau * sum_i
// w_i p(q(pts_i)) (one workgroup, fixed summation order), and its adjoint
// lam[v, pts_i] += tau * w_i * dp/dq_v.
struct Objective {
    const int32_t *pts;
    const double *w;
    int n;
    double gm1;
};

hipError_t launch_adj_rhs(const AdjRhs &a, int sbp, hipStream_t st);
hipError_t launch_adj_donor(const AdjDonor &a, int sbp, hipStream_t st);
hipError_t launch_obj(const Objective &o, const double *y, int64_t N, double tau, double *acc, hipStream_t st);
hipError_t launch_obj_adj(const Objective &o, const double *y, int64_t N, double tau, double *lam, hipStream_t st);
// adjoint of an extrapolant ext = y + sum_h beta_h hist_h at listed points:
// lam_y += lam_ext, lam_hist[h] += beta_h lam_ext, then lam_ext = 0 there
struct AdjExt {
    double *lam_ext, *lam_y;
    double *lam_hist[MAXH];
    double beta[MAXH];
    int m, nv;
    int64_t N;
    const int32_t *pts;
    int64_t np;
};
hipError_t launch_adj_ext(const AdjExt &a, hipStream_t st);
// dst[i][e] += coef[i] * src[e] for i < nd, e < n
hipError_t launch_adj_axpy(int64_t n, const double *src, int nd, double *const *dst, const double *coef,
                           hipStream_t st);

}  // namespace mrk
