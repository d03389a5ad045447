// gfx950 kernels of the discrete adjoint: vector-Jacobian products of the
// 2D right-hand side (fluxes, gradients, SAT penalties), of the donor data
// (interpolated states and viscous fluxes) and of a wall-pressure objective.
//
// The adjoint of a composition is taken piece by piece: the SBP rows are
// linear, so their transposes are gathers over the points whose rows read a
// given point (coefficients taken from the same row tables as the forward
// kernels); the pointwise maps (primitives, inviscid and viscous fluxes, SAT
// penalties with the closed-form flux-Jacobian product) are differentiated
// exactly by forward-mode dual numbers, one input direction at a time, and
// contracted with the incoming adjoint.  FP64 throughout.
#include "adj.h"
#include "sbp_dev.h"

namespace mrk {

// ------------------------------------------------------------ dual numbers
struct Dual {
    double v, d;
    Dual() = default;
    __device__ constexpr Dual(double x) : v(x), d(0.0) {}
    __device__ constexpr Dual(double x, double dx) : v(x), d(dx) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b)
{
    const double r = a.v / b.v;
    return {r, (a.d - r * b.d) / b.v};
}
__device__ __forceinline__ Dual &operator+=(Dual &a, Dual b) { return a = a + b; }
__device__ __forceinline__ Dual &operator-=(Dual &a, Dual b) { return a = a - b; }
__device__ __forceinline__ double sq_(double a) { return sqrt(a); }
__device__ __forceinline__ Dual sq_(Dual a)
{
    const double s = sqrt(a.v);
    return {s, 0.5 * a.d / s};
}
__device__ __forceinline__ double ab_(double a) { return fabs(a); }
__device__ __forceinline__ Dual ab_(Dual a) { return a.v < 0.0 ? -a : a; }
__device__ __forceinline__ double der(double) { return 0.0; }
__device__ __forceinline__ double der(Dual a) { return a.d; }

// ---------------------------------------- pointwise maps, generic in the type
// (the same formulas as the forward kernels)
template <int DIM, class T>
__device__ __forceinline__ void prim_t(const T *q, double gm1, T *w)
{
    T ri = T(1.0) / q[0];
    T ke = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        w[i] = q[1 + i] * ri;
        ke += w[i] * q[1 + i];
    }
    T p = gm1 * (q[DIM + 1] - 0.5 * ke);
    w[DIM] = p * ri;
}

template <int DIM, class T>
__device__ __forceinline__ void viscous_t(const Phys &ph, const T *u, T (*gr)[DIM], T (*Fv)[DIM + 1])
{
    const double mre = ph.mu / ph.Re, lre = ph.lam / ph.Re;
    const double kc = ph.mu * ph.gamma / ((ph.gamma - 1.0) * ph.Re * ph.Pr);
    T div = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) div += gr[i][i];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        T w = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            T tau = mre * (gr[i][j] + gr[j][i]);
            if (i == j) tau += lre * div;
            Fv[j][i] = tau;
            w += u[i] * tau;
        }
        Fv[j][DIM] = w + kc * gr[DIM][j];
    }
}

// sum_j A[j] (F^I_j - F^V_j) at one point (A: metric row m, or e_m on
// Cartesian grids)
template <int DIM, class T>
__device__ __forceinline__ void flux_t(const Phys &ph, const T *q, T (*gr)[DIM], const double *A, T *out)
{
    constexpr int NV = DIM + 2;
    const double gm1 = ph.gamma - 1.0;
    T ri = T(1.0) / q[0];
    T u[DIM], ke = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        u[i] = q[1 + i] * ri;
        ke += u[i] * q[1 + i];
    }
    T pr = gm1 * (q[NV - 1] - 0.5 * ke);
    T Fv[DIM][DIM + 1];
    viscous_t<DIM, T>(ph, u, gr, Fv);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        if (A[j] == 0.0) continue;
        out[0] += A[j] * q[1 + j];
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            T t = q[1 + i] * u[j] - Fv[j][i];
            if (i == j) t += pr;
            out[1 + i] += A[j] * t;
        }
        out[NV - 1] += A[j] * ((q[NV - 1] + pr) * u[j] - Fv[j][DIM]);
    }
}

template <int DIM, class T>
__device__ __forceinline__ void k_apply_t(double gamma, const T *q, const double *n, int sgn, const T *dQ, T *out)
{
    T rho = q[0], ri = T(1.0) / rho;
    T u[DIM], ke = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        u[i] = q[1 + i] * ri;
        ke += u[i] * u[i];
    }
    T p = (gamma - 1.0) * (q[DIM + 1] - 0.5 * rho * ke);
    T c2 = gamma * p * ri, c = sq_(c2);
    T H = (q[DIM + 1] + p) * ri;
    double L2 = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) L2 += n[j] * n[j];
    const double L = sqrt(L2), Li = 1.0 / L;
    double nh[DIM];
    T un = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        nh[j] = n[j] * Li;
        un += u[j] * nh[j];
    }
    T U = un * L;
    T drho = dQ[0];
    T du[DIM], udm = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        du[i] = (dQ[1 + i] - u[i] * drho) * ri;
        udm += u[i] * dQ[1 + i];
    }
    T dp = (gamma - 1.0) * (dQ[DIM + 1] - udm + 0.5 * ke * drho);
    T dun = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) dun += du[i] * nh[i];
    T ae = drho - dp / c2;
    T ap = (dp + rho * c * dun) / (2.0 * c2);
    T am = (dp - rho * c * dun) / (2.0 * c2);
    T l0 = U, lp = U + c * L, lm = U - c * L;
    T w0 = 0.5 * (ab_(l0) + (double)sgn * l0);
    T wp = 0.5 * (ab_(lp) + (double)sgn * lp);
    T wm = 0.5 * (ab_(lm) + (double)sgn * lm);
    T a0 = w0 * ae, bp = wp * ap, bm = wm * am;
    out[0] = a0 + bp + bm;
    T us = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        T s = rho * (du[i] - dun * nh[i]);
        us += u[i] * s;
        out[1 + i] = a0 * u[i] + w0 * s + bp * (u[i] + c * nh[i]) + bm * (u[i] - c * nh[i]);
    }
    out[DIM + 1] = a0 * 0.5 * ke + w0 * us + bp * (H + c * un) + bm * (H - c * un);
}

// SAT penalties at point p summed over the directions in which p ends a run
// (interface rows rb, far field, isothermal no-slip wall)
template <int DIM, int CART, class T>
__device__ __forceinline__ void sat_t(const GridDev &g, const Phys &ph, int64_t p, const T *qp, T (*gr)[DIM],
                                      const T *rb, T *r)
{
    constexpr int NV = DIM + 2;
    const int64_t N = g.npts;
#pragma unroll
    for (int v = 0; v < NV; ++v) r[v] = 0.0;
    T ri = T(1.0) / qp[0];
    T u[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) u[i] = qp[1 + i] * ri;
    T Fv[DIM][DIM + 1];
    viscous_t<DIM, T>(ph, u, gr, Fv);
    for (int m = 0; m < DIM; ++m) {
        const int c = g.cls[m * N + p];
        const int bc = (c >> 4) & 3;
        if (!bc) continue;
        const int sgn = ((c & 15) == 1) ? 1 : -1;
        double kap[DIM], k2 = 0.0;
        if constexpr (CART) {
#pragma unroll
            for (int j = 0; j < DIM; ++j) kap[j] = (j == m) ? g.inv_h[m] : 0.0;
        } else {
            const double Jp = g.metric[(int64_t)(DIM * DIM) * N + p];
#pragma unroll
            for (int j = 0; j < DIM; ++j) kap[j] = Jp * g.metric[(int64_t)(m * DIM + j) * N + p];
        }
#pragma unroll
        for (int j = 0; j < DIM; ++j) k2 += kap[j] * kap[j];
        T dQ[NV], dV[NV], s2[NV];
        double sigI, sig1 = ph.mu * k2 / (2.0 * ph.Re);
        bool use_s2 = true;
        s2[0] = 0.0;
#pragma unroll
        for (int v = 1; v < NV; ++v) {
            T s = 0.0;
#pragma unroll
            for (int j = 0; j < DIM; ++j) s += kap[j] * Fv[j][v - 1];
            s2[v] = s;
        }
        if (bc == 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                dQ[v] = qp[v] - rb[v];
                dV[v] = dQ[v];
            }
#pragma unroll
            for (int v = 1; v < NV; ++v) {
                T s = 0.0;
#pragma unroll
                for (int j = 0; j < DIM; ++j) s += kap[j] * rb[NV + j * (NV - 1) + (v - 1)];
                s2[v] -= s;
            }
            sigI = ph.sig_iface;
        } else if (bc == 2) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                dQ[v] = qp[v] - ph.q_inf[v];
                dV[v] = dQ[v];
            }
            sigI = ph.sig_bc;
        } else {
            const double kn = sqrt(k2);
            T mn = 0.0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) mn += qp[1 + i] * kap[i];
            mn = mn / kn;
            dQ[0] = 0.0;
            dV[0] = 0.0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                dQ[1 + i] = 2.0 * mn * kap[i] / kn;
                dV[1 + i] = qp[1 + i];
            }
            dQ[NV - 1] = 0.0;
            dV[NV - 1] = qp[NV - 1] - qp[0] * ph.T_wall / (ph.gamma - 1.0);
            sigI = ph.sig_bc;
            sig1 = ph.wall_visc * ph.mu * k2 / ph.Re;
            use_s2 = false;
        }
        T KdQ[NV];
        k_apply_t<DIM, T>(ph.gamma, qp, kap, sgn, dQ, KdQ);
        const double hs = 0.5 * sgn;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T pen = -(sigI * KdQ[v] + sig1 * dV[v]) * ph.p0inv;
            if (use_s2) pen += hs * s2[v] * ph.p0inv;
            r[v] += pen;
        }
    }
}

// ------------------------------------------------------- transposed rows
// coefficient of line offset o in the first-derivative row `row`
template <int SBP>
__device__ __forceinline__ double dcoef(int row, int o)
{
    return dsbp<SBP, 1>(row, [&](int oo) {
               Vec<1> r;
               r.v[0] = oo == o ? 1.0 : 0.0;
               return r;
           }).v[0];
}

// the point whose row, at line offset o along m, reads point x (-1 when the
// line ends first)
__device__ __forceinline__ int64_t reader(const GridDev &g, int64_t x, const int *ic, int m, int o)
{
    int j = ic[m] - o;
    if (g.periodic[m]) {
        j %= g.n[m];
        if (j < 0) j += g.n[m];
    } else if (j < 0 || j >= g.n[m]) {
        return -1;
    }
    return x + (int64_t)(j - ic[m]) * g.stride[m];
}

__device__ __forceinline__ bool hole(const GridDev &g, int64_t p) { return (g.cls[p] & 15) == CLS_HOLE; }

template <int SBP>
constexpr int reach() { return SBP == 21 ? 1 : 3; }

// ------------------------------------------------------ right-hand side
template <int DIM, int SBP, int CART>
__global__ void __launch_bounds__(256) k_adj_flux(AdjRhs a)
{
    constexpr int NV = DIM + 2;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const GridDev &g = a.g;
    const int64_t N = g.npts;
    if (x >= N) return;
    if (hole(g, x)) {
        for (int k = 0; k < DIM * NV; ++k) a.mu[k * N + x] = 0.0;
        return;
    }
    int ic[3];
    coords(g, x, ic);
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
        const double sc = CART ? g.inv_h[m] : 1.0;
#pragma unroll
        for (int o = -reach<SBP>(); o <= reach<SBP>(); ++o) {
            const int64_t p = reader(g, x, ic, m, o);
            if (p < 0 || hole(g, p)) continue;
            const double coef = dcoef<SBP>(g.cls[m * N + p] & 15, o);
            if (coef == 0.0) continue;
            const double Jp = CART ? 1.0 : g.metric[(int64_t)(DIM * DIM) * N + p];
            const double w = -Jp * sc * coef;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += w * a.lamF[v * N + p];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) a.mu[(int64_t)(m * NV + v) * N + x] = acc[v];
    }
}

// the local Jacobian products at point x for input direction i (inputs: q,
// then the gradients (u, v, T) x (x, y), then the receiver row): flux terms
// weighted by mu, SAT terms (when sat) weighted by the right-hand-side
// adjoint at x
template <int DIM, int SBP, int CART>
__device__ __forceinline__ void point_inputs(const AdjRhs &a, int64_t x, double *qx, double (*gr)[DIM])
{
    const int64_t N = a.g.npts;
    int ic[3];
    coords(a.g, x, ic);
    load_q<DIM>(a.q, N, x, qx);
    gradient<DIM, SBP, CART>(a.g, x, ic, a.ph.gamma - 1.0, [&](int64_t idx, double *o) { load_q<DIM>(a.q, N, idx, o); },
                             gr);
}

template <int DIM, int CART>
__device__ __forceinline__ double point_seed(const AdjRhs &a, int64_t x, const double *qx, const double (*gr)[DIM],
                                             int i, bool sat, bool iface)
{
    constexpr int NV = DIM + 2, NG = (DIM + 1) * DIM, RB = NV + DIM * (NV - 1);
    const GridDev &g = a.g;
    const int64_t N = g.npts;
    Dual qd[NV], grd[DIM + 1][DIM];
#pragma unroll
    for (int v = 0; v < NV; ++v) qd[v] = Dual(qx[v], i == v ? 1.0 : 0.0);
#pragma unroll
    for (int b = 0; b <= DIM; ++b)
#pragma unroll
        for (int j = 0; j < DIM; ++j) grd[b][j] = Dual(gr[b][j], i == NV + b * DIM + j ? 1.0 : 0.0);
    double s = 0.0;
    if (i < NV + NG) {
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            double A[DIM];
#pragma unroll
            for (int j = 0; j < DIM; ++j) A[j] = CART ? (j == m ? 1.0 : 0.0) : g.metric[(int64_t)(m * DIM + j) * N + x];
            Dual out[NV];
            flux_t<DIM, Dual>(a.ph, qd, grd, A, out);
#pragma unroll
            for (int v = 0; v < NV; ++v) s += a.mu[(int64_t)(m * NV + v) * N + x] * out[v].d;
        }
    }
    if (sat) {
        Dual rbd[RB];
        const double *rb = iface ? g.recv + (int64_t)g.recv_idx[x] * RB : nullptr;
#pragma unroll
        for (int t = 0; t < RB; ++t) rbd[t] = Dual(iface ? rb[t] : 0.0, i == NV + NG + t ? 1.0 : 0.0);
        Dual r[NV];
        sat_t<DIM, CART, Dual>(g, a.ph, x, qd, grd, rbd, r);
#pragma unroll
        for (int v = 0; v < NV; ++v) s += a.lamF[v * N + x] * r[v].d;
    }
    return s;
}

// results of the local Jacobians at x -> lqd, kap (and the receiver row)
template <int DIM, int CART>
__device__ __forceinline__ void point_store(const AdjRhs &a, int64_t x, const double *res, bool iface)
{
    constexpr int NV = DIM + 2, NG = (DIM + 1) * DIM, RB = NV + DIM * (NV - 1);
    const GridDev &g = a.g;
    const int64_t N = g.npts;
#pragma unroll
    for (int v = 0; v < NV; ++v) a.lqd[v * N + x] = res[v];
    const double Jx = CART ? 1.0 : g.metric[(int64_t)(DIM * DIM) * N + x];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int b = 0; b <= DIM; ++b) {
            double k;
            if constexpr (CART) {
                k = g.inv_h[m] * res[NV + b * DIM + m];
            } else {
                k = 0.0;
#pragma unroll
                for (int j = 0; j < DIM; ++j) k += g.metric[(int64_t)(m * DIM + j) * N + x] * res[NV + b * DIM + j];
                k *= Jx;
            }
            a.kap[(int64_t)(m * (DIM + 1) + b) * N + x] = k;
        }
    if (iface) {
        const int64_t row = g.recv_idx[x];
        for (int t = 0; t < RB; ++t) a.lam_recv[row * RB + t] = res[NV + NG + t];
    }
}

__device__ __forceinline__ void bc_flags(const GridDev &g, int dim, int64_t x, bool &anyb, bool &iface)
{
    anyb = iface = false;
    for (int m = 0; m < dim; ++m) {
        const int bc = (g.cls[m * g.npts + x] >> 4) & 3;
        anyb |= bc != 0;
        iface |= bc == 1;
    }
}

// points without a SAT face (holes: zeros); SAT points are left to the
// listed kernels below
template <int DIM, int SBP, int CART>
__global__ void __launch_bounds__(256) k_adj_point(AdjRhs a)
{
    constexpr int NV = DIM + 2, NG = (DIM + 1) * DIM;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const GridDev &g = a.g;
    const int64_t N = g.npts;
    if (x >= N) return;
    if (hole(g, x)) {
        for (int v = 0; v < NV; ++v) a.lqd[v * N + x] = 0.0;
        for (int k = 0; k < NG; ++k) a.kap[k * N + x] = 0.0;
        return;
    }
    bool anyb, iface;
    bc_flags(g, DIM, x, anyb, iface);
    if (anyb) return;
    double qx[NV], gr[DIM + 1][DIM];
    point_inputs<DIM, SBP, CART>(a, x, qx, gr);
    double res[NV + NG];
#pragma unroll 1
    for (int i = 0; i < NV + NG; ++i) {
        const double s = point_seed<DIM, CART>(a, x, qx, gr, i, false, false);
#pragma unroll
        for (int k = 0; k < NV + NG; ++k)
            if (k == i) res[k] = s;
    }
    point_store<DIM, CART>(a, x, res, false);
}

// SAT points: one lane per (listed point, input direction)
template <int DIM, int SBP, int CART>
__global__ void __launch_bounds__(256) k_adj_bnd(AdjRhs a)
{
    constexpr int NV = DIM + 2, NG = (DIM + 1) * DIM, RB = NV + DIM * (NV - 1), NIN = NV + NG + RB;
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = lane / NIN;
    const int i = (int)(lane % NIN);
    if (b >= a.nb) return;
    const int64_t x = a.bpts[b];
    bool anyb, iface;
    bc_flags(a.g, DIM, x, anyb, iface);
    double s = 0.0;
    if (i < NV + NG || iface) {
        double qx[NV], gr[DIM + 1][DIM];
        point_inputs<DIM, SBP, CART>(a, x, qx, gr);
        s = point_seed<DIM, CART>(a, x, qx, gr, i, true, iface);
    }
    a.bres[lane] = s;
}

template <int DIM, int CART>
__global__ void __launch_bounds__(256) k_adj_bnd_store(AdjRhs a)
{
    constexpr int NV = DIM + 2, NG = (DIM + 1) * DIM, RB = NV + DIM * (NV - 1), NIN = NV + NG + RB;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nb) return;
    const int64_t x = a.bpts[b];
    bool anyb, iface;
    bc_flags(a.g, DIM, x, anyb, iface);
    double res[NIN];
#pragma unroll
    for (int k = 0; k < NIN; ++k) res[k] = a.bres[b * NIN + k];
    point_store<DIM, CART>(a, x, res, iface);
}

// adjoint of the primitives at one state -> adjoint of q
template <int DIM>
__device__ __forceinline__ void prim_adjoint(const double *q, double gm1, const double *lw, double *lq)
{
    constexpr int NV = DIM + 2;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        Dual qd[NV], w[DIM + 1];
#pragma unroll
        for (int k = 0; k < NV; ++k) qd[k] = Dual(q[k], k == v ? 1.0 : 0.0);
        prim_t<DIM, Dual>(qd, gm1, w);
        double s = 0.0;
#pragma unroll
        for (int b = 0; b <= DIM; ++b) s += lw[b] * w[b].d;
        lq[v] = s;
    }
}

template <int DIM, int SBP, int CART>
__global__ void __launch_bounds__(256) k_adj_grad(AdjRhs a)
{
    constexpr int NV = DIM + 2;
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const GridDev &g = a.g;
    const int64_t N = g.npts;
    if (y >= N || hole(g, y)) return;
    int ic[3];
    coords(g, y, ic);
    double lw[DIM + 1];
#pragma unroll
    for (int b = 0; b <= DIM; ++b) lw[b] = 0.0;
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int o = -reach<SBP>(); o <= reach<SBP>(); ++o) {
            const int64_t x = reader(g, y, ic, m, o);
            if (x < 0 || hole(g, x)) continue;
            const double coef = dcoef<SBP>(g.cls[m * N + x] & 15, o);
            if (coef == 0.0) continue;
#pragma unroll
            for (int b = 0; b <= DIM; ++b) lw[b] += coef * a.kap[(int64_t)(m * (DIM + 1) + b) * N + x];
        }
    double qy[NV], lq[NV];
    load_q<DIM>(a.q, N, y, qy);
    prim_adjoint<DIM>(qy, a.ph.gamma - 1.0, lw, lq);
#pragma unroll
    for (int v = 0; v < NV; ++v) a.lam_q[v * N + y] += a.lqd[v * N + y] + lq[v];
}

// ------------------------------------------------------------- donor data
template <int DIM, int SBP, int CART>
__global__ void __launch_bounds__(256) k_adj_donor_u(AdjDonor a)
{
    constexpr int NV = DIM + 2, NG = (DIM + 1) * DIM, RB = NV + DIM * (NV - 1);
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= a.nu) return;
    const GridDev &g = a.g;
    const int64_t N = g.npts;
    double L[RB];
#pragma unroll
    for (int t = 0; t < RB; ++t) L[t] = 0.0;
    for (int k = a.ustart[u]; k < a.ustart[u + 1]; ++k) {
        const int e = a.uent[k];
        const double w = a.w[e];
        const double *lr = a.lam_recv + (int64_t)(a.row0 + e / a.S) * RB;
#pragma unroll
        for (int t = 0; t < RB; ++t) L[t] += w * lr[t];
    }
    const int64_t p = a.upts[u];
    int ic[3];
    coords(g, p, ic);
    double qp[NV];
    load_q<DIM>(a.y, N, p, qp);
    double gr[DIM + 1][DIM];
    gradient<DIM, SBP, CART>(g, p, ic, a.ph.gamma - 1.0, [&](int64_t idx, double *o) { load_q<DIM>(a.y, N, idx, o); },
                             gr);
    double res[NV + NG];
#pragma unroll 1
    for (int i = 0; i < NV + NG; ++i) {
        Dual qd[NV], grd[DIM + 1][DIM];
#pragma unroll
        for (int v = 0; v < NV; ++v) qd[v] = Dual(qp[v], i == v ? 1.0 : 0.0);
#pragma unroll
        for (int b = 0; b <= DIM; ++b)
#pragma unroll
            for (int j = 0; j < DIM; ++j) grd[b][j] = Dual(gr[b][j], i == NV + b * DIM + j ? 1.0 : 0.0);
        Dual ri = Dual(1.0) / qd[0];
        Dual uu[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) uu[k] = qd[1 + k] * ri;
        Dual Fv[DIM][DIM + 1];
        viscous_t<DIM, Dual>(a.ph, uu, grd, Fv);
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) s += L[v] * qd[v].d;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int v = 1; v < NV; ++v) s += L[NV + d * (NV - 1) + (v - 1)] * Fv[d][v - 1].d;
        res[i] = s;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) a.uq[u * NV + v] = res[v];
    const double Jp = CART ? 1.0 : g.metric[(int64_t)(DIM * DIM) * N + p];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int b = 0; b <= DIM; ++b) {
            double k;
            if constexpr (CART) {
                k = g.inv_h[m] * res[NV + b * DIM + m];
            } else {
                k = 0.0;
#pragma unroll
                for (int j = 0; j < DIM; ++j) k += g.metric[(int64_t)(m * DIM + j) * N + p] * res[NV + b * DIM + j];
                k *= Jp;
            }
            a.uk[(u * DIM + m) * (DIM + 1) + b] = k;
        }
}

template <int DIM, int SBP>
__global__ void __launch_bounds__(256) k_adj_donor_c(AdjDonor a)
{
    constexpr int NV = DIM + 2;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.nc) return;
    const GridDev &g = a.g;
    const int64_t N = g.npts;
    const int64_t pc = a.cpts[c];
    double lw[DIM + 1];
#pragma unroll
    for (int b = 0; b <= DIM; ++b) lw[b] = 0.0;
    for (int k = a.cstart[c]; k < a.cstart[c + 1]; ++k) {
        const int ent = a.cent[k];
        const int u = ent >> 8, m = (ent >> 4) & 15, o = (ent & 15) - 8;
        const double coef = dcoef<SBP>(g.cls[m * N + a.upts[u]] & 15, o);
#pragma unroll
        for (int b = 0; b <= DIM; ++b) lw[b] += coef * a.uk[((int64_t)u * DIM + m) * (DIM + 1) + b];
    }
    double qc[NV], lq[NV];
    load_q<DIM>(a.y, N, pc, qc);
    prim_adjoint<DIM>(qc, a.ph.gamma - 1.0, lw, lq);
    const int su = a.cself[c];
#pragma unroll
    for (int v = 0; v < NV; ++v) a.lam_y[v * N + pc] += lq[v] + (su >= 0 ? a.uq[(int64_t)su * NV + v] : 0.0);
}

// -------------------------------------------------------------- objective
__device__ __forceinline__ double pressure(const double *y, int64_t N, int64_t p, int dim, double gm1)
{
    const double rho = y[p];
    double ke = 0.0;
    for (int i = 0; i < dim; ++i) {
        const double m = y[(1 + i) * N + p];
        ke += (m / rho) * m;
    }
    return gm1 * (y[(dim + 1) * N + p] - 0.5 * ke);
}

__global__ void __launch_bounds__(256) k_obj(Objective o, int dim, const double *y, int64_t N, double tau,
                                             double *acc)
{
    __shared__ double s[256];
    double t = 0.0;
    for (int i = threadIdx.x; i < o.n; i += 256) t += o.w[i] * pressure(y, N, o.pts[i], dim, o.gm1);
    s[threadIdx.x] = t;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[0] += tau * s[0];
}

__global__ void __launch_bounds__(256) k_obj_adj(Objective o, int dim, const double *y, int64_t N, double tau,
                                                 double *lam)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= o.n) return;
    const int64_t p = o.pts[i];
    const double rho = y[p], f = tau * o.w[i] * o.gm1;
    double m2 = 0.0;
    for (int k = 0; k < dim; ++k) {
        const double m = y[(1 + k) * N + p];
        m2 += m * m;
        lam[(1 + k) * N + p] += -f * m / rho;
    }
    lam[p] += f * 0.5 * m2 / (rho * rho);
    lam[(dim + 1) * N + p] += f;
}

__global__ void __launch_bounds__(256) k_adj_ext(AdjExt a)
{
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= a.np * a.nv) return;
    const int v = (int)(lane / a.np);
    const int64_t el = (int64_t)v * a.N + a.pts[lane - (int64_t)v * a.np];
    const double l = a.lam_ext[el];
    a.lam_y[el] += l;
    for (int h = 0; h < a.m; ++h) a.lam_hist[h][el] += a.beta[h] * l;
    a.lam_ext[el] = 0.0;
}

struct AxpyList {
    int nd;
    double *dst[MAXH + 2];
    double coef[MAXH + 2];
};

__global__ void k_adj_axpy(int64_t n, const double *__restrict__ src, AxpyList L)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double s = src[e];
    for (int i = 0; i < L.nd; ++i) L.dst[i][e] += L.coef[i] * s;
}

// ---------------------------------------------------------------- launches
static inline unsigned nblk_(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int SBP, int CART>
static hipError_t adj_rhs_t(const AdjRhs &a, hipStream_t st)
{
    const unsigned nb = nblk_(a.g.npts, 256);
    hipLaunchKernelGGL((k_adj_flux<2, SBP, CART>), dim3(nb), dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_adj_point<2, SBP, CART>), dim3(nb), dim3(256), 0, st, a);
    if (a.nb > 0) {
        constexpr int NIN = 4 + 6 + 10;
        hipLaunchKernelGGL((k_adj_bnd<2, SBP, CART>), dim3(nblk_((int64_t)a.nb * NIN, 256)), dim3(256), 0, st, a);
        hipLaunchKernelGGL((k_adj_bnd_store<2, CART>), dim3(nblk_(a.nb, 256)), dim3(256), 0, st, a);
    }
    hipLaunchKernelGGL((k_adj_grad<2, SBP, CART>), dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_rhs(const AdjRhs &a, int sbp, hipStream_t st)
{
    if (a.g.dim != 2 || a.g.npts == 0) return hipErrorInvalidValue;
    if (sbp == 21) return a.g.cartesian ? adj_rhs_t<21, 1>(a, st) : adj_rhs_t<21, 0>(a, st);
    return a.g.cartesian ? adj_rhs_t<42, 1>(a, st) : adj_rhs_t<42, 0>(a, st);
}

template <int SBP, int CART>
static hipError_t adj_donor_t(const AdjDonor &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_adj_donor_u<2, SBP, CART>), dim3(nblk_(a.nu, 256)), dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_adj_donor_c<2, SBP>), dim3(nblk_(a.nc, 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_donor(const AdjDonor &a, int sbp, hipStream_t st)
{
    if (a.g.dim != 2) return hipErrorInvalidValue;
    if (a.nu == 0) return hipSuccess;
    if (sbp == 21) return a.g.cartesian ? adj_donor_t<21, 1>(a, st) : adj_donor_t<21, 0>(a, st);
    return a.g.cartesian ? adj_donor_t<42, 1>(a, st) : adj_donor_t<42, 0>(a, st);
}

hipError_t launch_obj(const Objective &o, const double *y, int64_t N, double tau, double *acc, hipStream_t st)
{
    if (o.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_obj, dim3(1), dim3(256), 0, st, o, 2, y, N, tau, acc);
    return hipGetLastError();
}

hipError_t launch_obj_adj(const Objective &o, const double *y, int64_t N, double tau, double *lam, hipStream_t st)
{
    if (o.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_obj_adj, dim3(nblk_(o.n, 256)), dim3(256), 0, st, o, 2, y, N, tau, lam);
    return hipGetLastError();
}

hipError_t launch_adj_ext(const AdjExt &a, hipStream_t st)
{
    if (a.m < 0 || a.m > MAXH) return hipErrorInvalidValue;
    if (a.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_ext, dim3(nblk_(a.np * a.nv, 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_axpy(int64_t n, const double *src, int nd, double *const *dst, const double *coef,
                           hipStream_t st)
{
    if (nd < 0 || nd > MAXH + 2) return hipErrorInvalidValue;
    if (nd == 0 || n == 0) return hipSuccess;
    AxpyList L{};
    L.nd = nd;
    for (int i = 0; i < nd; ++i) {
        L.dst[i] = dst[i];
        L.coef[i] = coef[i];
    }
    hipLaunchKernelGGL(k_adj_axpy, dim3(nblk_(n, 256)), dim3(256), 0, st, n, src, L);
    return hipGetLastError();
}

}  // namespace mrk
