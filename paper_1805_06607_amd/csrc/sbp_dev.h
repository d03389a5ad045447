// Device helpers shared by the forward kernels (kernels.hip) and their
// discrete adjoints (adjoint.hip): SBP first-derivative rows, neighbour
// indexing, primitives, gradients, viscous fluxes and the closed-form SAT
// flux-Jacobian product.
#pragma once
#include "kern.h"

#include <math.h>

namespace mrk {

template <int K>
struct Vec {
    double v[K];
};

// -------------------------------------------------------------- SBP rows
// Diagonal-norm SBP 4-2 closure rows (left end); the right end mirrors them
// with negated signs.  Interior: (1/12, -2/3, 0, 2/3, -1/12).
// SBP 2-1: closure (-1, 1); interior (-1/2, 0, 1/2).
#define C42_00 (-24.0 / 17.0)
#define C42_01 (59.0 / 34.0)
#define C42_02 (-4.0 / 17.0)
#define C42_03 (-3.0 / 34.0)
#define C42_20 (4.0 / 43.0)
#define C42_21 (-59.0 / 86.0)
#define C42_23 (59.0 / 86.0)
#define C42_24 (-4.0 / 43.0)
#define C42_30 (3.0 / 98.0)
#define C42_32 (-59.0 / 98.0)
#define C42_34 (32.0 / 49.0)
#define C42_35 (-4.0 / 49.0)

// First derivative (index spacing 1) of a K-vector field at a point whose
// class row is `row`; f(o) returns the field at line offset o.
template <int SBP, int K, class F>
__device__ __forceinline__ Vec<K> dsbp(int row, F &&f)
{
    Vec<K> r;
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = 0.0;
    auto add = [&](double c, int o) {
        Vec<K> x = f(o);
#pragma unroll
        for (int k = 0; k < K; ++k) r.v[k] += c * x.v[k];
    };
    if (row == 0) {
        if constexpr (SBP == 21) {
            add(-0.5, -1); add(0.5, 1);
        } else {
            add(1.0 / 12.0, -2); add(-2.0 / 3.0, -1); add(2.0 / 3.0, 1); add(-1.0 / 12.0, 2);
        }
    } else if constexpr (SBP == 21) {
        if (row == 1) { add(-1.0, 0); add(1.0, 1); }
        else          { add(1.0, 0); add(-1.0, -1); }
    } else {
        switch (row) {
        case 1: add(C42_00, 0); add(C42_01, 1); add(C42_02, 2); add(C42_03, 3); break;
        case 2: add(-0.5, -1); add(0.5, 1); break;
        case 3: add(C42_20, -2); add(C42_21, -1); add(C42_23, 1); add(C42_24, 2); break;
        case 4: add(C42_30, -3); add(C42_32, -1); add(C42_34, 1); add(C42_35, 2); break;
        case 5: add(-C42_00, 0); add(-C42_01, -1); add(-C42_02, -2); add(-C42_03, -3); break;
        case 6: add(0.5, 1); add(-0.5, -1); break;
        case 7: add(-C42_20, 2); add(-C42_21, 1); add(-C42_23, -1); add(-C42_24, -2); break;
        default: add(-C42_30, 3); add(-C42_32, 1); add(-C42_34, -1); add(-C42_35, -2); break;
        }
    }
    return r;
}

// neighbour along direction d at line offset o (periodic wrap)
__device__ __forceinline__ int64_t nbr(const GridDev &g, int64_t p, const int *ic, int d, int o)
{
    int j = ic[d] + o;
    if (g.periodic[d]) j = j < 0 ? j + g.n[d] : (j >= g.n[d] ? j - g.n[d] : j);
    return p + (int64_t)(j - ic[d]) * g.stride[d];
}

__device__ __forceinline__ void coords(const GridDev &g, int64_t p, int *ic)
{
    ic[0] = (int)(p % g.n[0]);
    int64_t r = p / g.n[0];
    ic[1] = (int)(r % g.n[1]);
    ic[2] = (int)(r / g.n[1]);
}

// primitives (u_1..u_D, T) of a conserved state
template <int DIM>
__device__ __forceinline__ Vec<DIM + 1> prim(const double *q, double gm1)
{
    Vec<DIM + 1> r;
    double ri = 1.0 / q[0];
    double ke = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        r.v[i] = q[1 + i] * ri;
        ke += r.v[i] * q[1 + i];
    }
    double p = gm1 * (q[DIM + 1] - 0.5 * ke);
    r.v[DIM] = p * ri;
    return r;
}

template <int DIM>
__device__ __forceinline__ void load_q(const double *q, int64_t N, int64_t p, double *out)
{
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) out[v] = q[v * N + p];
}

// metric terms of point p for grad_cart: M_mj row-major, then J
// (curvilinear grids only)
template <int DIM, int CART>
__device__ __forceinline__ void load_metric(const GridDev &g, int64_t p, double *met)
{
    if constexpr (!CART) {
        const int64_t N = g.npts;
        met[DIM * DIM] = g.metric[(int64_t)(DIM * DIM) * N + p];
#pragma unroll
        for (int m = 0; m < DIM * DIM; ++m) met[m] = g.metric[(int64_t)m * N + p];
    }
}

// Cartesian gradient of (u_1..u_D, T) from its index-space derivatives
// dxi[m] along each grid direction m (chain rule through the metric terms)
template <int DIM, int CART>
__device__ __forceinline__ void grad_cart(const GridDev &g, const Vec<DIM + 1> *dxi, const double *met,
                                          double gr[DIM + 1][DIM])
{
    if constexpr (CART) {
#pragma unroll
        for (int a = 0; a <= DIM; ++a)
#pragma unroll
            for (int j = 0; j < DIM; ++j) gr[a][j] = g.inv_h[j] * dxi[j].v[a];
    } else {
        const double J = met[DIM * DIM];
#pragma unroll
        for (int a = 0; a <= DIM; ++a)
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
                double s = 0.0;
#pragma unroll
                for (int m = 0; m < DIM; ++m) s += met[m * DIM + j] * dxi[m].v[a];
                gr[a][j] = J * s;
            }
    }
}

// gradient d(phi_a)/dx_j of (u_1..u_D, T) at point p; qload(idx, out[nv])
template <int DIM, int SBP, int CART, class QL>
__device__ __forceinline__ void gradient(const GridDev &g, int64_t p, const int *ic, double gm1, QL &&qload,
                                         double gr[DIM + 1][DIM])
{
    Vec<DIM + 1> dxi[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        int row = g.cls[m * g.npts + p] & 15;
        dxi[m] = dsbp<SBP, DIM + 1>(row, [&](int o) {
            double qq[DIM + 2];
            qload(nbr(g, p, ic, m, o), qq);
            return prim<DIM>(qq, gm1);
        });
    }
    double met[DIM * DIM + 1];
    load_metric<DIM, CART>(g, p, met);
    grad_cart<DIM, CART>(g, dxi, met, gr);
}

// the same gradient with every load issued before the first use: the
// point's class rows, metric terms (when `cart` is false) and the states of
// its whole +-R line windows (R = 1 for SBP 2-1, 3 for 4-2; positions past a
// non-periodic end are clamped and never read by a row), qp being its own
// state.  The rows are applied to the loaded windows exactly as gradient()
// applies them.
template <int DIM, int SBP>
__device__ __forceinline__ void gradient_window(const GridDev &g, int64_t p, const int *ic, bool cart, double gm1,
                                                const double *__restrict__ y, const double *qp,
                                                double gr[DIM + 1][DIM])
{
    constexpr int NV = DIM + 2, RW = SBP == 21 ? 1 : 3;
    const int64_t N = g.npts;
    int row[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m) row[m] = g.cls[m * N + p] & 15;
    double met[DIM * DIM + 1];
    if (!cart) load_metric<DIM, 0>(g, p, met);
    double win[DIM][2 * RW][NV];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int k = 0; k < 2 * RW; ++k) {
            const int o = k < RW ? k - RW : k - RW + 1;
            int jj = ic[m] + o;
            if (g.periodic[m]) jj = jj < 0 ? jj + g.n[m] : (jj >= g.n[m] ? jj - g.n[m] : jj);
            jj = jj < 0 ? 0 : (jj >= g.n[m] ? g.n[m] - 1 : jj);
            const int64_t idx = p + (int64_t)(jj - ic[m]) * g.stride[m];
#pragma unroll
            for (int v = 0; v < NV; ++v) win[m][k][v] = y[v * N + idx];
        }
    Vec<DIM + 1> dxi[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
        dxi[m] = dsbp<SBP, DIM + 1>(row[m], [&](int o) {
            const double *qq = o == 0 ? qp : win[m][o < 0 ? o + RW : o + RW - 1];
            return prim<DIM>(qq, gm1);
        });
    if (cart)
        grad_cart<DIM, 1>(g, dxi, met, gr);
    else
        grad_cart<DIM, 0>(g, dxi, met, gr);
}

// Cartesian viscous flux vectors (components 1..nv-1) at a point
template <int DIM>
__device__ __forceinline__ void viscous_flux(const Phys &ph, const double *u, double gr[DIM + 1][DIM],
                                             double Fv[DIM][DIM + 1])
{
    double mre = ph.mu / ph.Re, lre = ph.lam / ph.Re;
    double kc = ph.mu * ph.gamma / ((ph.gamma - 1.0) * ph.Re * ph.Pr);
    double div = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) div += gr[i][i];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        double w = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            double tau = mre * (gr[i][j] + gr[j][i]);
            if (i == j) tau += lre * div;
            Fv[j][i] = tau;
            w += u[i] * tau;
        }
        Fv[j][DIM] = w + kc * gr[DIM][j];
    }
}

// 3D: V layout (NVISC3 values per point, kern.h): tau_00, tau_11, tau_22,
// tau_01, tau_02, tau_12, then h_0, h_1, h_2
__device__ __forceinline__ int visc3_tau(int i, int j)
{
    return i == j ? i : (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5));
}

// V of a point from its gradients, the arithmetic of viscous_flux<3>
__device__ __forceinline__ void visc3_from_grad(const Phys &ph, double gr[4][3], double *V)
{
    double mre = ph.mu / ph.Re, lre = ph.lam / ph.Re;
    double kc = ph.mu * ph.gamma / ((ph.gamma - 1.0) * ph.Re * ph.Pr);
    double div = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) div += gr[i][i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            double tau = mre * (gr[i][j] + gr[j][i]);
            if (i == j) tau += lre * div;
            V[visc3_tau(i, j)] = tau;
        }
#pragma unroll
    for (int j = 0; j < 3; ++j) V[6 + j] = kc * gr[3][j];
}

// Cartesian viscous flux vectors (components 1..4) of a 3D point from V
__device__ __forceinline__ void viscous_flux3(const double *u, const double *V, double Fv[3][4])
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double w = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double tau = V[visc3_tau(i, j)];
            Fv[j][i] = tau;
            w += u[i] * tau;
        }
        Fv[j][3] = w + V[6 + j];
    }
}

// --------------------------------------------------------- SAT (closed form)
// K^{+-} dQ for the Euler flux Jacobian along the (non-normalised) direction
// n, at state q, via characteristic wave strengths (entropy + shear waves at
// U, acoustic waves at U +- c|n|); sgn = +1 for K+, -1 for K-.
template <int DIM>
__device__ __forceinline__ void k_apply(double gamma, const double *q, const double *n, int sgn, const double *dQ,
                                        double *out)
{
    double rho = q[0], ri = 1.0 / rho;
    double u[DIM], ke = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) { u[i] = q[1 + i] * ri; ke += u[i] * u[i]; }
    double p = (gamma - 1.0) * (q[DIM + 1] - 0.5 * rho * ke);
    double c2 = gamma * p * ri, c = sqrt(c2);
    double H = (q[DIM + 1] + p) * ri;
    double L2 = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) L2 += n[j] * n[j];
    double L = sqrt(L2), Li = 1.0 / L;
    double nh[DIM], un = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) { nh[j] = n[j] * Li; un += u[j] * nh[j]; }
    double U = un * L;
    // linearised primitive differences
    double drho = dQ[0];
    double du[DIM], udm = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) { du[i] = (dQ[1 + i] - u[i] * drho) * ri; udm += u[i] * dQ[1 + i]; }
    double dp = (gamma - 1.0) * (dQ[DIM + 1] - udm + 0.5 * ke * drho);
    double dun = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) dun += du[i] * nh[i];
    const double ic2 = 1.0 / c2, hc2 = 0.5 * ic2;
    double ae = drho - dp * ic2;
    double ap = (dp + rho * c * dun) * hc2;
    double am = (dp - rho * c * dun) * hc2;
    double l0 = U, lp = U + c * L, lm = U - c * L;
    double w0 = 0.5 * (fabs(l0) + sgn * l0);
    double wp = 0.5 * (fabs(lp) + sgn * lp);
    double wm = 0.5 * (fabs(lm) + sgn * lm);
    double a0 = w0 * ae, bp = wp * ap, bm = wm * am;
    out[0] = a0 + bp + bm;
    double us = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        double s = rho * (du[i] - dun * nh[i]);
        us += u[i] * s;
        out[1 + i] = a0 * u[i] + w0 * s + bp * (u[i] + c * nh[i]) + bm * (u[i] - c * nh[i]);
    }
    out[DIM + 1] = a0 * 0.5 * ke + w0 * us + bp * (H + c * un) + bm * (H - c * un);
}

__device__ __forceinline__ double add_nc(double acc, double c, double f)
{
#pragma clang fp contract(off)
    double t = c * f;
    return acc + t;
}

// XCD-aware order: consecutive workgroups go to different XCDs, so give each
// XCD a contiguous range of tiles (neighbours share halos in its L2); a
// bijection when the tile count is a multiple of 8, identity otherwise
__device__ __forceinline__ int xcd_tile(int b, int nblk)
{
    return (nblk % 8) ? b : (b % 8) * (nblk / 8) + b / 8;
}

}  // namespace mrk
