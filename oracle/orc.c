/*
 * Plain FP64 reference implementation of the semi-discrete right-hand side.
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path.
 *
 * Everything is written as whole-grid passes in the order of the definition
 * (primitives -> gradients -> fluxes -> derivative of the contravariant flux
 * -> SAT penalties), with no fusion or blocking.  Build: gcc -O2
 * -ffp-contract=off -fopenmp (results do not depend on the thread count:
 * there are no reductions).
 *
 * Paper references:
 *  - governing equations and viscous stress: Appendix "Spatial Accuracy of
 *    Right-Hand Sides" (conservation form, tau_ij with mu/Re and lambda/Re);
 *  - curvilinear form and metric terms: section "Timestep Calculation" (the
 *    metric terms (1/J) d(xi_i)/dx) and section "Compressible Navier-Stokes
 *    Equations on Overset Meshes";
 *  - second derivatives as two applications of the first-derivative operator:
 *    Appendix "Spatial Accuracy of Right-Hand Sides";
 *  - SAT interface penalty: eq. (int) with sigma^I = 1/2,
 *    sigma_1^V = |grad kappa|^2/(2 Re), sigma_2^{+-V} = +-1/2, and
 *    K^{+-} = T (|Lambda| +- Lambda)/2 T^{-1}; edge and corner points sum the
 *    terms of every direction in which they end a run;
 *  - timestep estimate: eq. (ts_inv), (ts_visc), (ts_overall).
 * Readings taken where the paper is silent (see the design notes): T = p/rho,
 * c_p = gamma/(gamma-1), constant mu, lambda = -2/3 mu, heat flux
 * -mu c_p/(Re Pr) grad T; p0^{-1} also multiplies the sigma_2 term; far-field
 * = interface form with target q_inf and zero target viscous flux; isothermal
 * wall = target (rho, 0, T_wall) without the sigma_2 term.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { BC_PERIODIC = 0, BC_INTERFACE = 1, BC_FARFIELD = 2, BC_WALL = 3 };

typedef struct {
    int32_t dim, nv, nb, cw, hw;   /* closure rows, closure width, interior half width */
    int32_t n[3];
    int32_t periodic[3];
    int32_t pad0;
    int64_t npts;
    double dint[5];                /* interior coefficients, offsets -2..2 */
    double dclo[4][6];             /* left closure rows */
    double p0;
    double gamma, Re, Pr, mu, lam;
    double sig_iface, sig_bc, T_wall, wall_visc;
    double q_inf[5];
    const double *metric;          /* (dim*dim+1) x N: M[m*dim+j] = J^{-1} dxi_m/dx_j, then J */
    const int32_t *pos[3];
    const int32_t *rlen[3];
    const int8_t *bclo[3];
    const int8_t *bchi[3];
    const int32_t *recv_idx;       /* per point: receiver row, or -1 */
} OrcGrid;

static int64_t nbr(const OrcGrid *g, int64_t p, int d, int off)
{
    int64_t c[3];
    c[0] = p % g->n[0];
    c[1] = (p / g->n[0]) % g->n[1];
    c[2] = p / ((int64_t)g->n[0] * g->n[1]);
    int64_t v = c[d] + off;
    if (g->periodic[d]) {
        v %= g->n[d];
        if (v < 0) v += g->n[d];
    }
    c[d] = v;
    return c[0] + (int64_t)g->n[0] * (c[1] + (int64_t)g->n[1] * c[2]);
}

/* first derivative along direction d at point p of the scalar field f, using
 * the run that contains p (closures at run ends, interior stencil inside,
 * periodic wrap on endless periodic lines) */
static double dapply(const OrcGrid *g, const double *f, int64_t p, int d)
{
    int L = g->rlen[d][p];
    int i = g->pos[d][p];
    double s = 0.0;
    if (L != 0 && i < g->nb) {
        for (int c = 0; c < g->cw; ++c) s = s + g->dclo[i][c] * f[nbr(g, p, d, c - i)];
    } else if (L != 0 && i >= L - g->nb) {
        int r = L - 1 - i;
        for (int c = 0; c < g->cw; ++c) s = s - g->dclo[r][c] * f[nbr(g, p, d, r - c)];
    } else {
        for (int o = -g->hw; o <= g->hw; ++o) {
            if (o == 0) continue;
            s = s + g->dint[o + 2] * f[nbr(g, p, d, o)];
        }
    }
    return s;
}

static int active(const OrcGrid *g, int64_t p) { return g->rlen[0][p] >= 0; }

static double Mmj(const OrcGrid *g, int64_t p, int m, int j)
{
    return g->metric[(int64_t)(m * g->dim + j) * g->npts + p];
}
static double Jac(const OrcGrid *g, int64_t p)
{
    return g->metric[(int64_t)(g->dim * g->dim) * g->npts + p];
}

/* ---------------------------------------------------------------- metrics */
/* derivative of a coordinate along d at p: as dapply, but a neighbour reached
 * across a periodic seam carries the coordinate jump per[d] (translation
 * periodic domains; zero for grids whose coordinates wrap by themselves) */
static double dcoord(const OrcGrid *g, const double *f, int64_t p, int d, const double *per)
{
    int64_t c[3];
    c[0] = p % g->n[0];
    c[1] = (p / g->n[0]) % g->n[1];
    c[2] = p / ((int64_t)g->n[0] * g->n[1]);
    int L = g->rlen[d][p];
    int i = g->pos[d][p];
    double s = 0.0;
#define VAL(off) (f[nbr(g, p, d, (off))] + ((c[d] + (off) >= g->n[d]) ? per[d] : ((c[d] + (off) < 0) ? -per[d] : 0.0)))
    if (L != 0 && i < g->nb) {
        for (int k = 0; k < g->cw; ++k) s = s + g->dclo[i][k] * VAL(k - i);
    } else if (L != 0 && i >= L - g->nb) {
        int r = L - 1 - i;
        for (int k = 0; k < g->cw; ++k) s = s - g->dclo[r][k] * VAL(r - k);
    } else {
        for (int o = -g->hw; o <= g->hw; ++o) {
            if (o == 0) continue;
            s = s + g->dint[o + 2] * VAL(o);
        }
    }
#undef VAL
    return s;
}

/* 2D metric terms from coordinates, full-line operator (run info must
 * describe the whole grid without holes).  perx[d], pery[d]: coordinate jumps
 * across the seam of direction d. */
int orc_metrics2d(const OrcGrid *g, const double *x, const double *y, const double *perx,
                  const double *pery, double *metric)
{
    int64_t N = g->npts;
    for (int64_t p = 0; p < N; ++p) {
        double xxi = dcoord(g, x, p, 0, perx), xeta = dcoord(g, x, p, 1, perx);
        double yxi = dcoord(g, y, p, 0, pery), yeta = dcoord(g, y, p, 1, pery);
        double jinv = xxi * yeta - xeta * yxi;
        metric[0 * N + p] = yeta;     /* J^{-1} xi_x  */
        metric[1 * N + p] = -xeta;    /* J^{-1} xi_y  */
        metric[2 * N + p] = -yxi;     /* J^{-1} eta_x */
        metric[3 * N + p] = xxi;      /* J^{-1} eta_y */
        metric[4 * N + p] = 1.0 / jinv;
    }
    return 0;
}

/* ------------------------------------------------------------- primitives */
typedef struct {
    double *rho, *u[3], *p, *T;
    double *grad;   /* (dim+1) x dim x N: d(phi_a)/dx_j, phi = (u_1..u_dim, T) */
} Work;

static void primitives(const OrcGrid *g, const double *q, Work *w)
{
    int64_t N = g->npts;
    int dim = g->dim;
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        if (!active(g, p)) {
            w->rho[p] = 0.0; w->p[p] = 0.0; w->T[p] = 0.0;
            for (int i = 0; i < dim; ++i) w->u[i][p] = 0.0;
            continue;
        }
        double rho = q[p];
        double ke = 0.0;
        for (int i = 0; i < dim; ++i) {
            double ui = q[(int64_t)(1 + i) * N + p] / rho;
            w->u[i][p] = ui;
            ke = ke + ui * ui;
        }
        double pr = (g->gamma - 1.0) * (q[(int64_t)(dim + 1) * N + p] - 0.5 * rho * ke);
        w->rho[p] = rho;
        w->p[p] = pr;
        w->T[p] = pr / rho;
    }
}

/* gradient of phi_a at point p: d phi/dx_j = J sum_m M_mj D_m phi */
static void gradient_at(const OrcGrid *g, const Work *w, int64_t p, double gr[4][3])
{
    int dim = g->dim;
    for (int a = 0; a <= dim; ++a) {
        const double *f = (a < dim) ? w->u[a] : w->T;
        double dxi[3];
        for (int m = 0; m < dim; ++m) dxi[m] = dapply(g, f, p, m);
        for (int j = 0; j < dim; ++j) {
            double s = 0.0;
            for (int m = 0; m < dim; ++m) s = s + Mmj(g, p, m, j) * dxi[m];
            gr[a][j] = Jac(g, p) * s;
        }
    }
}

/* Cartesian viscous flux vectors at point p: Fv[j][v], v = 0..nv-1 */
static void viscous_flux(const OrcGrid *g, const Work *w, int64_t p, double gr[4][3], double Fv[3][5])
{
    int dim = g->dim;
    double mu = g->mu, Re = g->Re;
    double cp = g->gamma / (g->gamma - 1.0);
    double kappa = mu * cp / (Re * g->Pr);
    double div = 0.0;
    for (int i = 0; i < dim; ++i) div = div + gr[i][i];
    for (int j = 0; j < dim; ++j) {
        Fv[j][0] = 0.0;
        double work = 0.0;
        for (int i = 0; i < dim; ++i) {
            double tau = (mu / Re) * (gr[i][j] + gr[j][i]);
            if (i == j) tau = tau + (g->lam / Re) * div;
            Fv[j][1 + i] = tau;
            work = work + w->u[i][p] * tau;
        }
        Fv[j][dim + 1] = work + kappa * gr[dim][j];
    }
}

static void inviscid_flux(const OrcGrid *g, const double *q, const Work *w, int64_t p, double Fi[3][5])
{
    int dim = g->dim;
    int64_t N = g->npts;
    double rho = w->rho[p], pr = w->p[p];
    double rE = q[(int64_t)(dim + 1) * N + p];
    for (int j = 0; j < dim; ++j) {
        double uj = w->u[j][p];
        Fi[j][0] = rho * uj;
        for (int i = 0; i < dim; ++i) {
            double v = rho * w->u[i][p] * uj;
            if (i == j) v = v + pr;
            Fi[j][1 + i] = v;
        }
        Fi[j][dim + 1] = (rE + pr) * uj;
    }
}

/* ------------------------------------------------ SAT: K^{+-} via T, T^{-1} */
static int invert(int n, double A[5][5], double X[5][5])
{
    double M[5][10];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            M[i][j] = (j < n) ? A[i][j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (M[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) { double t = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = t; }
        double d = M[c][c];
        for (int j = 0; j < 2 * n; ++j) M[c][j] = M[c][j] / d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = M[r][c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j) M[r][j] = M[r][j] - f * M[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) X[i][j] = M[i][j + n];
    return 0;
}

/* K = T diag((|lambda| + sgn*lambda)/2) T^{-1} for the Euler flux Jacobian in
 * direction nvec (not normalised), at the conserved state qp. */
int orc_kmatrix(int dim, double gamma, const double *qp, const double *nvec, int sgn, double *Kout)
{
    int nv = dim + 2;
    double rho = qp[0];
    double u[3] = {0, 0, 0}, ke = 0.0;
    for (int i = 0; i < dim; ++i) { u[i] = qp[1 + i] / rho; ke = ke + u[i] * u[i]; }
    double pr = (gamma - 1.0) * (qp[dim + 1] - 0.5 * rho * ke);
    double c = sqrt(gamma * pr / rho);
    double H = (qp[dim + 1] + pr) / rho;
    double L = 0.0;
    for (int j = 0; j < dim; ++j) L = L + nvec[j] * nvec[j];
    L = sqrt(L);
    double nh[3] = {0, 0, 0};
    for (int j = 0; j < dim; ++j) nh[j] = nvec[j] / L;
    double U = 0.0, un = 0.0;
    for (int j = 0; j < dim; ++j) { U = U + u[j] * nvec[j]; un = un + u[j] * nh[j]; }
    double T[5][5], lam[5];
    memset(T, 0, sizeof T);
    int col = 0;
    /* entropy wave */
    T[0][col] = 1.0;
    for (int i = 0; i < dim; ++i) T[1 + i][col] = u[i];
    T[dim + 1][col] = 0.5 * ke;
    lam[col++] = U;
    /* shear waves: orthonormal tangents */
    double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
    if (dim == 2) {
        t1[0] = -nh[1]; t1[1] = nh[0];
    } else {
        int k = 0;
        if (fabs(nh[1]) < fabs(nh[k])) k = 1;
        if (fabs(nh[2]) < fabs(nh[k])) k = 2;
        double e[3] = {0, 0, 0};
        e[k] = 1.0;
        double dot = nh[k];
        double s = 0.0;
        for (int i = 0; i < 3; ++i) { t1[i] = e[i] - dot * nh[i]; s = s + t1[i] * t1[i]; }
        s = sqrt(s);
        for (int i = 0; i < 3; ++i) t1[i] = t1[i] / s;
        t2[0] = nh[1] * t1[2] - nh[2] * t1[1];
        t2[1] = nh[2] * t1[0] - nh[0] * t1[2];
        t2[2] = nh[0] * t1[1] - nh[1] * t1[0];
    }
    for (int w = 0; w < dim - 1; ++w) {
        double *t = (w == 0) ? t1 : t2;
        T[0][col] = 0.0;
        double ut = 0.0;
        for (int i = 0; i < dim; ++i) { T[1 + i][col] = t[i]; ut = ut + u[i] * t[i]; }
        T[dim + 1][col] = ut;
        lam[col++] = U;
    }
    /* acoustic waves */
    for (int s = 1; s >= -1; s -= 2) {
        T[0][col] = 1.0;
        for (int i = 0; i < dim; ++i) T[1 + i][col] = u[i] + s * c * nh[i];
        T[dim + 1][col] = H + s * c * un;
        lam[col++] = U + s * c * L;
    }
    double Ti[5][5];
    if (invert(nv, T, Ti) != 0) return -1;
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            double s = 0.0;
            for (int k = 0; k < nv; ++k) {
                double dk = 0.5 * (fabs(lam[k]) + sgn * lam[k]);
                s = s + T[i][k] * dk * Ti[k][j];
            }
            Kout[i * nv + j] = s;
        }
    return 0;
}

/* SAT penalty of the run end (direction m, side sgn: +1 run start, -1 run
 * end) at point p with boundary flag bc: pen (nv values) */
static int sat_term(const OrcGrid *g, int64_t p, int m, int bc, int sgn, const double *qp, double Fvp[3][5],
                    const double *recv, int RB, double *pen)
{
    int dim = g->dim, nv = g->nv;
    double kap[3], k2 = 0.0;
    for (int j = 0; j < dim; ++j) { kap[j] = Jac(g, p) * Mmj(g, p, m, j); k2 = k2 + kap[j] * kap[j]; }
    double qt[5], qv[5];      /* targets of the K term and of the sigma_1 term */
    double Fvk[5], Fvkh[5];
    for (int v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int j = 0; j < dim; ++j) s = s + kap[j] * Fvp[j][v];
        Fvk[v] = s;
        Fvkh[v] = 0.0;
    }
    double sigI, sig1 = g->mu * k2 / (2.0 * g->Re);
    int use_s2 = 1;
    if (bc == BC_INTERFACE) {
        int ri = g->recv_idx[p];
        if (ri < 0) return -1;
        const double *rb = recv + (int64_t)ri * RB;
        for (int v = 0; v < nv; ++v) qt[v] = rb[v];
        for (int v = 1; v < nv; ++v) {
            double s = 0.0;
            for (int j = 0; j < dim; ++j) s = s + kap[j] * rb[nv + j * (nv - 1) + (v - 1)];
            Fvkh[v] = s;
        }
        for (int v = 0; v < nv; ++v) qv[v] = qt[v];
        sigI = g->sig_iface;
    } else if (bc == BC_FARFIELD) {
        for (int v = 0; v < nv; ++v) qt[v] = g->q_inf[v];
        for (int v = 0; v < nv; ++v) qv[v] = qt[v];
        sigI = g->sig_bc;
    } else if (bc == BC_WALL) {
        /* inviscid part: the point's own state with the normal momentum
         * reflected (characteristic no-penetration); viscous part: rest at the
         * wall temperature */
        double mn = 0.0, kn = sqrt(k2);
        for (int i = 0; i < dim; ++i) mn = mn + qp[1 + i] * kap[i] / kn;
        qt[0] = qp[0];
        for (int i = 0; i < dim; ++i) qt[1 + i] = qp[1 + i] - 2.0 * mn * kap[i] / kn;
        qt[dim + 1] = qp[dim + 1];
        qv[0] = qp[0];
        for (int i = 0; i < dim; ++i) qv[1 + i] = 0.0;
        qv[dim + 1] = qp[0] * g->T_wall / (g->gamma - 1.0);
        sigI = g->sig_bc;
        sig1 = g->wall_visc * g->mu * k2 / g->Re;
        use_s2 = 0;
    } else {
        return -1;
    }
    double K[25];
    if (orc_kmatrix(dim, g->gamma, qp, kap, sgn, K) != 0) return -1;
    double dQ[5], dV[5];
    for (int v = 0; v < nv; ++v) { dQ[v] = qp[v] - qt[v]; dV[v] = qp[v] - qv[v]; }
    double s2 = 0.5 * sgn;
    for (int v = 0; v < nv; ++v) {
        double kd = 0.0;
        for (int c2 = 0; c2 < nv; ++c2) kd = kd + K[v * nv + c2] * dQ[c2];
        double pv = -(sigI * kd + sig1 * dV[v]) / g->p0;
        if (use_s2) pv = pv + s2 * (Fvk[v] - Fvkh[v]) / g->p0;
        pen[v] = pv;
    }
    return 0;
}

/* ------------------------------------------------------------------- RHS */
static double *alloc(int64_t n) { return (double *)calloc((size_t)n, sizeof(double)); }

int orc_rhs(const OrcGrid *g, const double *q, const double *recv, double *dqdt)
{
    int dim = g->dim, nv = g->nv;
    int64_t N = g->npts;
    int RB = nv + dim * (nv - 1);
    Work w;
    w.rho = alloc(N); w.p = alloc(N); w.T = alloc(N);
    for (int i = 0; i < 3; ++i) w.u[i] = alloc(N);
    double *Fhat = alloc((int64_t)dim * nv * N);   /* contravariant fluxes [m][v][p] */
    double *Fvis = alloc((int64_t)dim * nv * N);   /* Cartesian viscous fluxes [j][v][p] */
    if (!w.rho || !w.p || !w.T || !w.u[2] || !Fhat || !Fvis) return -1;

    primitives(g, q, &w);

    /* fluxes at every active point */
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        if (!active(g, p)) continue;
        double gr[4][3], Fv[3][5], Fi[3][5];
        gradient_at(g, &w, p, gr);
        viscous_flux(g, &w, p, gr, Fv);
        inviscid_flux(g, q, &w, p, Fi);
        for (int j = 0; j < dim; ++j)
            for (int v = 0; v < nv; ++v) Fvis[((int64_t)j * nv + v) * N + p] = Fv[j][v];
        for (int m = 0; m < dim; ++m)
            for (int v = 0; v < nv; ++v) {
                double s = 0.0;
                for (int j = 0; j < dim; ++j) s = s + Mmj(g, p, m, j) * (Fi[j][v] - Fv[j][v]);
                Fhat[((int64_t)m * nv + v) * N + p] = s;
            }
    }

    /* divergence of the contravariant flux, then SAT */
    int err = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        if (!active(g, p)) {
            for (int v = 0; v < nv; ++v) dqdt[(int64_t)v * N + p] = 0.0;
            continue;
        }
        double r[5];
        for (int v = 0; v < nv; ++v) {
            double s = 0.0;
            for (int m = 0; m < dim; ++m) s = s + dapply(g, Fhat + ((int64_t)m * nv + v) * N, p, m);
            r[v] = -Jac(g, p) * s;
        }
        double qp[5];
        for (int v = 0; v < nv; ++v) qp[v] = q[(int64_t)v * N + p];
        for (int m = 0; m < dim; ++m) {
            int L = g->rlen[m][p];
            if (L <= 0) continue;
            for (int side = 0; side < 2; ++side) {
                int at_end = side == 0 ? (g->pos[m][p] == 0) : (g->pos[m][p] == L - 1);
                if (!at_end) continue;
                int bc = side == 0 ? g->bclo[m][p] : g->bchi[m][p];
                int sgn = side == 0 ? +1 : -1;      /* '+' face at the run start */
                double pen[5], Fvp[3][5];
                for (int j = 0; j < dim; ++j)
                    for (int v = 0; v < nv; ++v) Fvp[j][v] = Fvis[((int64_t)j * nv + v) * N + p];
                if (sat_term(g, p, m, bc, sgn, qp, Fvp, recv, RB, pen) != 0) { err = 1; continue; }
                for (int v = 0; v < nv; ++v) r[v] = r[v] + pen[v];
            }
        }
        for (int v = 0; v < nv; ++v) dqdt[(int64_t)v * N + p] = r[v];
    }

    free(w.rho); free(w.p); free(w.T);
    for (int i = 0; i < 3; ++i) free(w.u[i]);
    free(Fhat); free(Fvis);
    return err ? -2 : 0;
}

/* donor data at listed points: q (nv values) then the Cartesian viscous flux
 * vectors F^V_j (components 1..nv-1) for j = 0..dim-1 */
int orc_donor(const OrcGrid *g, const double *q, int64_t np, const int64_t *pts, double *out)
{
    int dim = g->dim, nv = g->nv;
    int64_t N = g->npts;
    int RB = nv + dim * (nv - 1);
    Work w;
    w.rho = alloc(N); w.p = alloc(N); w.T = alloc(N);
    for (int i = 0; i < 3; ++i) w.u[i] = alloc(N);
    primitives(g, q, &w);
    int err = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < np; ++r) {
        int64_t p = pts[r];
        if (p < 0 || p >= N || !active(g, p)) { err = 1; continue; }
        double gr[4][3], Fv[3][5];
        gradient_at(g, &w, p, gr);
        viscous_flux(g, &w, p, gr, Fv);
        double *o = out + r * RB;
        for (int v = 0; v < nv; ++v) o[v] = q[(int64_t)v * N + p];
        for (int j = 0; j < dim; ++j)
            for (int v = 1; v < nv; ++v) o[nv + j * (nv - 1) + (v - 1)] = Fv[j][v];
    }
    free(w.rho); free(w.p); free(w.T);
    for (int i = 0; i < 3; ++i) free(w.u[i]);
    return err ? -1 : 0;
}

/* per-point timestep estimate (holes: +inf) */
int orc_dt(const OrcGrid *g, const double *q, double *dt)
{
    int dim = g->dim;
    int64_t N = g->npts;
    double nu_coef = fmax(g->mu, g->gamma * g->mu / g->Pr);
    for (int64_t p = 0; p < N; ++p) {
        if (!active(g, p)) { dt[p] = INFINITY; continue; }
        double rho = q[p], ke = 0.0, u[3] = {0, 0, 0};
        for (int i = 0; i < dim; ++i) { u[i] = q[(int64_t)(1 + i) * N + p] / rho; ke = ke + u[i] * u[i]; }
        double pr = (g->gamma - 1.0) * (q[(int64_t)(dim + 1) * N + p] - 0.5 * rho * ke);
        double c = sqrt(g->gamma * pr / rho);
        double J = Jac(g, p);
        double adv = 0.0, sn = 0.0;
        for (int m = 0; m < dim; ++m) {
            double dot = 0.0, nrm = 0.0;
            for (int j = 0; j < dim; ++j) { dot = dot + u[j] * Mmj(g, p, m, j); nrm = nrm + Mmj(g, p, m, j) * Mmj(g, p, m, j); }
            adv = adv + fabs(dot);
            sn = sn + sqrt(nrm);
        }
        double nu = nu_coef / (rho * g->Re);
        dt[p] = fabs(1.0 / J) / (adv + c * sn + 2.0 * nu * fabs(J) * sn * sn);
    }
    return 0;
}

/* first derivative along direction d at every active point (0 at holes) */
int orc_deriv(const OrcGrid *g, const double *f, int d, double *out)
{
    for (int64_t p = 0; p < g->npts; ++p)
        out[p] = active(g, p) ? dapply(g, f, p, d) : 0.0;
    return 0;
}

/* right-hand side at listed points only (same definition as orc_rhs: the
 * contravariant fluxes at each point's stencil columns are evaluated where
 * needed instead of on the whole grid); for sampled checks of large grids */
int orc_rhs_points(const OrcGrid *g, const double *q, const double *recv, int64_t np, const int64_t *pts,
                   double *out)
{
    int dim = g->dim, nv = g->nv;
    int64_t N = g->npts;
    int RB = nv + dim * (nv - 1);
    Work w;
    w.rho = alloc(N); w.p = alloc(N); w.T = alloc(N);
    for (int i = 0; i < 3; ++i) w.u[i] = alloc(N);
    if (!w.rho || !w.p || !w.T || !w.u[2]) return -1;
    primitives(g, q, &w);
    int err = 0;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < np; ++r) {
        int64_t p = pts[r];
        double *o = out + r * nv;
        if (p < 0 || p >= N) { err = 1; continue; }
        if (!active(g, p)) { for (int v = 0; v < nv; ++v) o[v] = 0.0; continue; }
        /* contravariant flux of direction m at point s */
        double res[5] = {0, 0, 0, 0, 0};
        for (int m = 0; m < dim; ++m) {
            int L = g->rlen[m][p], i = g->pos[m][p];
            int cols[6], nc = 0;
            double cf[6];
            if (L != 0 && i < g->nb) {
                for (int c2 = 0; c2 < g->cw; ++c2) { cols[nc] = c2 - i; cf[nc++] = g->dclo[i][c2]; }
            } else if (L != 0 && i >= L - g->nb) {
                int rr = L - 1 - i;
                for (int c2 = 0; c2 < g->cw; ++c2) { cols[nc] = rr - c2; cf[nc++] = -g->dclo[rr][c2]; }
            } else {
                for (int o2 = -g->hw; o2 <= g->hw; ++o2) {
                    if (o2 == 0) continue;
                    cols[nc] = o2; cf[nc++] = g->dint[o2 + 2];
                }
            }
            double sum[5] = {0, 0, 0, 0, 0};
            for (int t = 0; t < nc; ++t) {
                int64_t s = nbr(g, p, m, cols[t]);
                double gr[4][3], Fv[3][5], Fi[3][5];
                gradient_at(g, &w, s, gr);
                viscous_flux(g, &w, s, gr, Fv);
                inviscid_flux(g, q, &w, s, Fi);
                for (int v = 0; v < nv; ++v) {
                    double fh = 0.0;
                    for (int j = 0; j < dim; ++j) fh = fh + Mmj(g, s, m, j) * (Fi[j][v] - Fv[j][v]);
                    sum[v] = sum[v] + cf[t] * fh;
                }
            }
            for (int v = 0; v < nv; ++v) res[v] = res[v] + sum[v];
        }
        for (int v = 0; v < nv; ++v) o[v] = -Jac(g, p) * res[v];
        /* SAT terms: reuse the whole-grid routine's definition on a one-point basis */
        double gr[4][3], Fvp[3][5];
        gradient_at(g, &w, p, gr);
        viscous_flux(g, &w, p, gr, Fvp);
        double qp[5];
        for (int v = 0; v < nv; ++v) qp[v] = q[(int64_t)v * N + p];
        for (int m = 0; m < dim; ++m) {
            int L = g->rlen[m][p];
            if (L <= 0) continue;
            for (int side = 0; side < 2; ++side) {
                int at_end = side == 0 ? (g->pos[m][p] == 0) : (g->pos[m][p] == L - 1);
                if (!at_end) continue;
                int bc = side == 0 ? g->bclo[m][p] : g->bchi[m][p];
                int sgn = side == 0 ? +1 : -1;
                double pen[5];
                if (sat_term(g, p, m, bc, sgn, qp, Fvp, recv, RB, pen) != 0) { err = 1; continue; }
                for (int v = 0; v < nv; ++v) o[v] = o[v] + pen[v];
            }
        }
    }
    free(w.rho); free(w.p); free(w.T);
    for (int i = 0; i < 3; ++i) free(w.u[i]);
    return err ? -2 : 0;
}

int orc_abi_version(void) { return 1; }
