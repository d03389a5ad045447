// gfx950 kernels of the SBP-SAT overset right-hand side and the AB/MRAB
// history combination.  FP64 throughout; the stencils are bandwidth bound and
// use no matrix cores.
//
// Paper: Mikida, Kloeckner, Bodony, "Multi-Rate Time Integration on Overset
// Meshes" -- governing equations and viscous stress (Appendix "Spatial
// Accuracy of Right-Hand Sides"), second derivatives as two applications of
// the first-derivative SBP operator (same Appendix), SAT interface penalty
// eq. (int), AB combination eq. (ab_general), timestep eq. (ts_inv)-(ts_overall).
#include "mrab.h"
#include "kern.h"
#include "sbp_dev.h"

#include <math.h>
#include <map>
#include <mutex>

namespace mrk {

// ------------------------------------------------------------ gradient pass
template <int DIM, int SBP, int CART>
__global__ void __launch_bounds__(256) k_grad(GridDev g, Phys ph, const double *__restrict__ q,
                                              double *__restrict__ grad)
{
    const double gm1 = ph.gamma - 1.0;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.npts) return;
    const int64_t N = g.npts;
    constexpr int NG = DIM == 3 ? NVISC3 : DIM * (DIM + 1);
    if ((g.cls[p] & 15) == CLS_HOLE) {
#pragma unroll
        for (int k = 0; k < NG; ++k) grad[k * N + p] = 0.0;
        return;
    }
    int ic[3];
    coords(g, p, ic);
    double gr[DIM + 1][DIM];
    gradient<DIM, SBP, CART>(g, p, ic, gm1, [&](int64_t idx, double *o) { load_q<DIM>(q, N, idx, o); }, gr);
    if constexpr (DIM == 3) {
        double V[NVISC3];
        visc3_from_grad(ph, gr, V);
#pragma unroll
        for (int k = 0; k < NVISC3; ++k) grad[(int64_t)k * N + p] = V[k];
    } else {
#pragma unroll
        for (int a = 0; a <= DIM; ++a)
#pragma unroll
            for (int j = 0; j < DIM; ++j) grad[(int64_t)(a * DIM + j) * N + p] = gr[a][j];
    }
}

// --------------------------------------------- fused flux divergence + SAT + AB
// contravariant flux of direction m at point idx (Cartesian grids: the flux
// vector of direction m), from the state and the stored gradients
template <int DIM, int CART>
__device__ __forceinline__ Vec<DIM + 2> fhat_at(const GridDev &g, const Phys &ph, const double *__restrict__ q,
                                                const double *__restrict__ grad, int m, int64_t idx)
{
    constexpr int NV = DIM + 2;
    const int64_t N = g.npts;
    const double gm1 = ph.gamma - 1.0;
    double qq[NV];
    load_q<DIM>(q, N, idx, qq);
    double ri = 1.0 / qq[0];
    double u[DIM], ke = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) { u[i] = qq[1 + i] * ri; ke += u[i] * qq[1 + i]; }
    double pr = gm1 * (qq[DIM + 1] - 0.5 * ke);
    double Fv[DIM][DIM + 1];
    if constexpr (DIM == 3) {
        double V[NVISC3];
#pragma unroll
        for (int k = 0; k < NVISC3; ++k) V[k] = grad[(int64_t)k * N + idx];
        viscous_flux3(u, V, Fv);
    } else {
        double gr[DIM + 1][DIM];
#pragma unroll
        for (int a = 0; a <= DIM; ++a)
#pragma unroll
            for (int j = 0; j < DIM; ++j) gr[a][j] = grad[(int64_t)(a * DIM + j) * N + idx];
        viscous_flux<DIM>(ph, u, gr, Fv);
    }
    Vec<NV> out;
    if constexpr (CART) {
        out.v[0] = qq[1 + m];
#pragma unroll
        for (int i = 0; i < DIM; ++i) out.v[1 + i] = qq[1 + i] * u[m] + (i == m ? pr : 0.0) - Fv[m][i];
        out.v[NV - 1] = (qq[NV - 1] + pr) * u[m] - Fv[m][DIM];
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) out.v[v] = 0.0;
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double Mmj = g.metric[(int64_t)(m * DIM + j) * N + idx];
            out.v[0] += Mmj * qq[1 + j];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
                out.v[1 + i] += Mmj * (qq[1 + i] * u[j] + (i == j ? pr : 0.0) - Fv[j][i]);
            out.v[NV - 1] += Mmj * ((qq[NV - 1] + pr) * u[j] - Fv[j][DIM]);
        }
    }
    return out;
}

// SAT penalties of point p added into r: at run ends, directions ascending
template <int DIM, int CART>
__device__ __forceinline__ void sat_point(const GridDev &g, const Phys &ph, const double *__restrict__ q,
                                          const double *__restrict__ grad, int64_t p, double *r)
{
    constexpr int NV = DIM + 2;
    const int64_t N = g.npts;
    // SAT penalties at run ends (directions ascending, run start first)
    bool any = false;
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        int c = g.cls[m * N + p];
        any |= ((c >> 4) & 3) != 0;
    }
    if (any) {
        double qp[NV];
        load_q<DIM>(q, N, p, qp);
        double u[DIM];
        double ri = 1.0 / qp[0];
#pragma unroll
        for (int i = 0; i < DIM; ++i) u[i] = qp[1 + i] * ri;
        double Fv[DIM][DIM + 1];
        if constexpr (DIM == 3) {
            double V[NVISC3];
#pragma unroll
            for (int k = 0; k < NVISC3; ++k) V[k] = grad[(int64_t)k * N + p];
            viscous_flux3(u, V, Fv);
        } else {
            double gr[DIM + 1][DIM];
#pragma unroll
            for (int a = 0; a <= DIM; ++a)
#pragma unroll
                for (int j = 0; j < DIM; ++j) gr[a][j] = grad[(int64_t)(a * DIM + j) * N + p];
            viscous_flux<DIM>(ph, u, gr, Fv);
        }
        for (int m = 0; m < DIM; ++m) {
            int c = g.cls[m * N + p];
            int bc = (c >> 4) & 3;
            if (!bc) continue;
            int row = c & 15;
            int sgn = (row == 1) ? 1 : -1;
            double kap[DIM], k2 = 0.0;
            if constexpr (CART) {
#pragma unroll
                for (int j = 0; j < DIM; ++j) kap[j] = (j == m) ? g.inv_h[m] : 0.0;
            } else {
                double Jp = g.metric[(int64_t)(DIM * DIM) * N + p];
#pragma unroll
                for (int j = 0; j < DIM; ++j) kap[j] = Jp * g.metric[(int64_t)(m * DIM + j) * N + p];
            }
#pragma unroll
            for (int j = 0; j < DIM; ++j) k2 += kap[j] * kap[j];
            double dQ[NV], dV[NV], s2[NV];
            double sigI, sig1 = k2 * (ph.mu / (2.0 * ph.Re));
            bool use_s2 = true;
#pragma unroll
            for (int v = 0; v < NV; ++v) s2[v] = 0.0;
            // own viscous flux along kappa (components 1..nv-1)
#pragma unroll
            for (int v = 1; v < NV; ++v) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < DIM; ++j) s += kap[j] * Fv[j][v - 1];
                s2[v] = s;
            }
            if (bc == 1) {
                const double *rb = g.recv + (int64_t)g.recv_idx[p] * (NV + DIM * (NV - 1));
#pragma unroll
                for (int v = 0; v < NV; ++v) { dQ[v] = qp[v] - rb[v]; dV[v] = dQ[v]; }
#pragma unroll
                for (int v = 1; v < NV; ++v) {
                    double s = 0.0;
#pragma unroll
                    for (int j = 0; j < DIM; ++j) s += kap[j] * rb[NV + j * (NV - 1) + (v - 1)];
                    s2[v] -= s;
                }
                sigI = ph.sig_iface;
            } else if (bc == 2) {
#pragma unroll
                for (int v = 0; v < NV; ++v) { dQ[v] = qp[v] - ph.q_inf[v]; dV[v] = dQ[v]; }
                sigI = ph.sig_bc;
            } else {
                // wall: reflected normal momentum (inviscid), rest at T_wall
                // (viscous); twice the normal momentum along kappa / |kappa|
                double mn = 0.0;
#pragma unroll
                for (int i = 0; i < DIM; ++i) mn += qp[1 + i] * kap[i];
                const double tm = 2.0 * mn / k2;
                dQ[0] = 0.0;
                dV[0] = 0.0;
#pragma unroll
                for (int i = 0; i < DIM; ++i) { dQ[1 + i] = tm * kap[i]; dV[1 + i] = qp[1 + i]; }
                dQ[NV - 1] = 0.0;
                dV[NV - 1] = qp[NV - 1] - qp[0] * (ph.T_wall / (ph.gamma - 1.0));
                sigI = ph.sig_bc;
                sig1 = k2 * (ph.wall_visc * ph.mu / ph.Re);
                use_s2 = false;
            }
            double KdQ[NV];
            k_apply<DIM>(ph.gamma, qp, kap, sgn, dQ, KdQ);
            double hs = 0.5 * sgn;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double pen = -(sigI * KdQ[v] + sig1 * dV[v]) * ph.p0inv;
                if (use_s2) pen += hs * s2[v] * ph.p0inv;
                r[v] += pen;
            }
        }
    }
}

// store F at p and, when fused, y_next = y + sum_j c_j F_j, oldest first, the
// new F last; each product and sum rounded separately
template <int DIM>
__device__ __forceinline__ void store_step(const double *__restrict__ q, double *__restrict__ F, const Combine &cb,
                                           int64_t N, int64_t p, const double *r)
{
    constexpr int NV = DIM + 2;
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v * N + p] = r[v];
    if (cb.m > 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            int64_t e = v * N + p;
            double acc = q[e];
#pragma unroll
            for (int j = 0; j < MAXH - 1; ++j)
                if (j < cb.m - 1) acc = add_nc(acc, cb.c[j], cb.hist[j][e]);
            acc = add_nc(acc, cb.c[cb.m - 1], r[v]);
            cb.y_next[e] = acc;
        }
    }
}

template <int DIM, int SBP, int CART>
__global__ void __launch_bounds__(256) k_rhs(GridDev g, Phys ph, const double *__restrict__ q,
                                             const double *__restrict__ grad, double *__restrict__ F,
                                             Combine cb)
{
    constexpr int NV = DIM + 2;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.npts) return;
    const int64_t N = g.npts;
    int c0 = g.cls[p] & 15;
    double r[NV];
    if (c0 == CLS_HOLE) {
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = 0.0;
    } else {
        int ic[3];
        coords(g, p, ic);
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            int row = g.cls[m * N + p] & 15;
            Vec<NV> d = dsbp<SBP, NV>(row, [&](int o) { return fhat_at<DIM, CART>(g, ph, q, grad, m, nbr(g, p, ic, m, o)); });
            double sc = CART ? g.inv_h[m] : 1.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += sc * d.v[v];
        }
        double J = CART ? 1.0 : g.metric[(int64_t)(DIM * DIM) * N + p];
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = -J * acc[v];
        sat_point<DIM, CART>(g, ph, q, grad, p, r);
    }
    store_step<DIM>(q, F, cb, N, p, r);
}

// 3D tiles of TX x TY x TZ outputs, one thread per output.  For each
// direction m, a quantity needed on the tile plus R points along m (R: the
// reach of a first-derivative row) is staged in LDS: the tile's own values
// come from registers (each thread evaluates its own point once, for every
// direction), only the 2R slabs of halo points are evaluated per direction.
// Periodic directions wrap; points off the grid or in holes stage zeros (no
// row of an active output reads them).
template <int TX, int TY, int TZ, int R>
struct Tile3 {
    static constexpr int NT = TX * TY * TZ;
    static constexpr int R0 = (TX + 2 * R) * TY * TZ, R1 = TX * (TY + 2 * R) * TZ, R2 = TX * TY * (TZ + 2 * R);
    static constexpr int RMAX = R0 > R1 ? (R0 > R2 ? R0 : R2) : (R1 > R2 ? R1 : R2);
    __device__ static constexpr int T(int m) { return m == 0 ? TX : (m == 1 ? TY : TZ); }
    // region extents of direction m
    __device__ static void ext(int m, int *e)
    {
        e[0] = TX + (m == 0 ? 2 * R : 0);
        e[1] = TY + (m == 1 ? 2 * R : 0);
        e[2] = TZ + (m == 2 ? 2 * R : 0);
    }
    // halo slab entry h of direction m -> region coordinates
    __device__ static void halo(int m, int h, int *c)
    {
        const int o1 = m == 0 ? 1 : 0, o2 = m == 2 ? 1 : 2;   // the other two directions, ascending
        const int n1 = T(o1);
        const int s = h % (2 * R), r = h / (2 * R);
        c[m] = s < R ? s : s + T(m);
        c[o1] = r % n1;
        c[o2] = r / n1;
    }
    // global index of region coordinates c of direction m (false: off the grid)
    __device__ static bool global(const GridDev &g, const int *t0, int m, const int *c, int64_t &idx)
    {
        idx = 0;
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int j = t0[d] + c[d] - (d == m ? R : 0);
            if (d == m && g.periodic[d]) j = j < 0 ? j + g.n[d] : (j >= g.n[d] ? j - g.n[d] : j);
            ok = ok && j >= 0 && j < g.n[d];
            idx += (int64_t)j * g.stride[d];
        }
        return ok;
    }
};

// the three directional flux vectors of a Cartesian 3D point from one load of
// its state and gradients (the formulas of fhat_at)
__device__ __forceinline__ void fluxes3(const GridDev &g, const Phys &ph, const double *__restrict__ q,
                                        const double *__restrict__ grad, int64_t idx, Vec<5> *out)
{
#pragma unroll
    for (int m = 0; m < 3; ++m) out[m] = fhat_at<3, 1>(g, ph, q, grad, m, idx);
}

// tile coordinates (in tiles) of the tile-th tile of a 3D launch: the tile
// rows are cut into slabs of sy rows along y (the last slab may be shorter);
// slab by slab, the tiles are taken in planes of constant z, each plane row by
// row, x fastest.  A tile's z neighbours then lie ntx * sy tiles away in this
// order (sy = nty: the plain x, y, z order).
__device__ __forceinline__ void tile3_origin(int tile, int ntx, int nty, int ntz, int sy, int *t)
{
    const int per = ntx * sy * ntz;   // tiles of a full slab
    const int s = tile / per, rem = tile - s * per;
    const int h = min(sy, nty - s * sy);
    const int z = rem / (ntx * h), r2 = rem - z * (ntx * h);
    t[0] = r2 % ntx;
    t[1] = s * sy + r2 / ntx;
    t[2] = z;
}

// 3D Cartesian gradient pass on tiles: grad[(a*3+j)*N + p] = d(u, v, w, T)_a / dx_j
// (zero at holes), the formulas of k_grad
template <int SBP, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX * TY * TZ) k_grad_tile3d(GridDev g, Phys ph, const double *__restrict__ q,
                                                              double *__restrict__ grad, int ntx, int nty, int ntz,
                                                              int sy)
{
    const double gm1 = ph.gamma - 1.0;
    constexpr int R = SBP == 21 ? 1 : 3;
    using C = Tile3<TX, TY, TZ, R>;
    __shared__ double sW[4][C::RMAX];
    int t0[3];
    tile3_origin(xcd_tile(blockIdx.x, ntx * nty * ntz), ntx, nty, ntz, sy, t0);
    t0[0] *= TX;
    t0[1] *= TY;
    t0[2] *= TZ;
    const int tid = threadIdx.x;
    const int lc[3] = {tid % TX, (tid / TX) % TY, tid / (TX * TY)};
    const int64_t N = g.npts;
    const bool inside = t0[0] + lc[0] < g.n[0] && t0[1] + lc[1] < g.n[1] && t0[2] + lc[2] < g.n[2];
    const int64_t p = inside ? (t0[0] + lc[0]) * g.stride[0] + (t0[1] + lc[1]) * g.stride[1] +
                                   (t0[2] + lc[2]) * g.stride[2]
                             : 0;
    // every global load of a point is issued before its class decides what
    // to keep (a hole's state is read but not used)
    int row[3] = {CLS_HOLE, CLS_HOLE, CLS_HOLE};
    double qo[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
    if (inside) {
#pragma unroll
        for (int m = 0; m < 3; ++m) row[m] = g.cls[m * N + p] & 15;
        load_q<3>(q, N, p, qo);
    }
    const bool active = row[0] != CLS_HOLE;
    Vec<4> own = prim<3>(qo, gm1);
    if (!active) {
#pragma unroll
        for (int a = 0; a < 4; ++a) own.v[a] = 0.0;
    }
    Vec<4> dxi[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        int ext[3];
        C::ext(m, ext);
        {
            // a tile slot past the grid's end holds the wrapped point of a
            // periodic direction m (zero otherwise)
            const int co[3] = {lc[0] + (m == 0 ? R : 0), lc[1] + (m == 1 ? R : 0), lc[2] + (m == 2 ? R : 0)};
            const int e = co[0] + ext[0] * (co[1] + ext[1] * co[2]);
            Vec<4> w = own;
            int64_t idx;
            if (!inside && C::global(g, t0, m, co, idx)) {
                double qq[5];
                load_q<3>(q, N, idx, qq);
                if ((g.cls[idx] & 15) != CLS_HOLE) w = prim<3>(qq, gm1);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) sW[a][e] = w.v[a];
        }
        const int nh = 2 * R * C::NT / C::T(m);
        // at most NHI entries per thread, unrolled so that their loads issue together
        constexpr int NHI = (2 * R * C::NT / (TX < TY ? (TX < TZ ? TX : TZ) : (TY < TZ ? TY : TZ)) + C::NT - 1) / C::NT;
#pragma unroll
        for (int it = 0; it < NHI; ++it) {
            const int h = tid + it * C::NT;
            if (h >= nh) break;
            int c[3];
            C::halo(m, h, c);
            int64_t idx;
            const bool ok = C::global(g, t0, m, c, idx);
            double qq[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
            int ch = CLS_HOLE;
            if (ok) {
                ch = g.cls[idx] & 15;
                load_q<3>(q, N, idx, qq);
            }
            Vec<4> w = prim<3>(qq, gm1);
            if (ch == CLS_HOLE) {
#pragma unroll
                for (int a = 0; a < 4; ++a) w.v[a] = 0.0;
            }
            const int e = c[0] + ext[0] * (c[1] + ext[1] * c[2]);
#pragma unroll
            for (int a = 0; a < 4; ++a) sW[a][e] = w.v[a];
        }
        __syncthreads();
        if (active) {
            const int base = (lc[0] + (m == 0 ? R : 0)) + ext[0] * ((lc[1] + (m == 1 ? R : 0)) + ext[1] * (lc[2] + (m == 2 ? R : 0)));
            const int step = m == 0 ? 1 : (m == 1 ? ext[0] : ext[0] * ext[1]);
            dxi[m] = dsbp<SBP, 4>(row[m], [&](int o) {
                Vec<4> x;
#pragma unroll
                for (int a = 0; a < 4; ++a) x.v[a] = sW[a][base + o * step];
                return x;
            });
        }
        __syncthreads();
    }
    if (!inside) return;
    double V[NVISC3];
    if (active) {
        double gr[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int j = 0; j < 3; ++j) gr[a][j] = g.inv_h[j] * dxi[j].v[a];
        visc3_from_grad(ph, gr, V);
    } else {
#pragma unroll
        for (int k = 0; k < NVISC3; ++k) V[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < NVISC3; ++k) grad[(int64_t)k * N + p] = V[k];
}

// 3D Cartesian flux divergence + SAT + AB on tiles, from the gradients of the
// gradient pass: the formulas of k_rhs, each directional flux computed about
// 1 + 2R / T_m times per output instead of once per stencil entry
template <int SBP, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX * TY * TZ) k_rhs_tile3d(GridDev g, Phys ph, const double *__restrict__ q,
                                                             const double *__restrict__ grad,
                                                             double *__restrict__ F, Combine cb, int ntx, int nty,
                                                             int ntz, int sy)
{
    constexpr int NV = 5, R = SBP == 21 ? 1 : 3;
    using C = Tile3<TX, TY, TZ, R>;
    __shared__ double sF[NV][C::RMAX];
    int t0[3];
    tile3_origin(xcd_tile(blockIdx.x, ntx * nty * ntz), ntx, nty, ntz, sy, t0);
    t0[0] *= TX;
    t0[1] *= TY;
    t0[2] *= TZ;
    const int tid = threadIdx.x;
    const int lc[3] = {tid % TX, (tid / TX) % TY, tid / (TX * TY)};
    const int64_t N = g.npts;
    const bool inside = t0[0] + lc[0] < g.n[0] && t0[1] + lc[1] < g.n[1] && t0[2] + lc[2] < g.n[2];
    const int64_t p = inside ? (t0[0] + lc[0]) * g.stride[0] + (t0[1] + lc[1]) * g.stride[1] +
                                   (t0[2] + lc[2]) * g.stride[2]
                             : 0;
    // every global load of a point is issued before its class decides what
    // to keep (a hole's state is read but not used)
    int row[3] = {CLS_HOLE, CLS_HOLE, CLS_HOLE};
    Vec<NV> own[3];
    if (inside) {
#pragma unroll
        for (int m = 0; m < 3; ++m) row[m] = g.cls[m * N + p] & 15;
        fluxes3(g, ph, q, grad, p, own);
    }
    const bool active = row[0] != CLS_HOLE;
    if (!active) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int v = 0; v < NV; ++v) own[m].v[v] = 0.0;
    }
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        int ext[3];
        C::ext(m, ext);
        const int co[3] = {lc[0] + (m == 0 ? R : 0), lc[1] + (m == 1 ? R : 0), lc[2] + (m == 2 ? R : 0)};
        const int base = co[0] + ext[0] * (co[1] + ext[1] * co[2]);
        {
            // a tile slot past the grid's end holds the wrapped point of a
            // periodic direction m (zero otherwise)
            Vec<NV> f = own[m];
            int64_t idx;
            if (!inside && C::global(g, t0, m, co, idx)) {
                Vec<NV> fw = fhat_at<3, 1>(g, ph, q, grad, m, idx);
                if ((g.cls[idx] & 15) != CLS_HOLE) f = fw;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) sF[v][base] = f.v[v];
        }
        const int nh = 2 * R * C::NT / C::T(m);
        // at most NHI entries per thread, unrolled so that their loads issue together
        constexpr int NHI = (2 * R * C::NT / (TX < TY ? (TX < TZ ? TX : TZ) : (TY < TZ ? TY : TZ)) + C::NT - 1) / C::NT;
#pragma unroll
        for (int it = 0; it < NHI; ++it) {
            const int h = tid + it * C::NT;
            if (h >= nh) break;
            int c[3];
            C::halo(m, h, c);
            int64_t idx;
            const bool ok = C::global(g, t0, m, c, idx);
            Vec<NV> f;
            int ch = CLS_HOLE;
            if (ok) {
                ch = g.cls[idx] & 15;
                f = fhat_at<3, 1>(g, ph, q, grad, m, idx);
            }
            if (ch == CLS_HOLE) {
#pragma unroll
                for (int v = 0; v < NV; ++v) f.v[v] = 0.0;
            }
            const int e = c[0] + ext[0] * (c[1] + ext[1] * c[2]);
#pragma unroll
            for (int v = 0; v < NV; ++v) sF[v][e] = f.v[v];
        }
        __syncthreads();
        if (active) {
            const int step = m == 0 ? 1 : (m == 1 ? ext[0] : ext[0] * ext[1]);
            Vec<NV> d = dsbp<SBP, NV>(row[m], [&](int o) {
                Vec<NV> x;
#pragma unroll
                for (int v = 0; v < NV; ++v) x.v[v] = sF[v][base + o * step];
                return x;
            });
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += g.inv_h[m] * d.v[v];
        }
        __syncthreads();
    }
    if (!inside) return;
    double r[NV];
    if (active) {
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = -1.0 * acc[v];
        sat_point<3, 1>(g, ph, q, grad, p, r);
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = 0.0;
    }
    store_step<3>(q, F, cb, N, p, r);
}

// coefficient of line offset o (|o| <= 3) in first-derivative row `row`: the
// rows dsbp applies, as a table (row 15, a hole, has none)
__constant__ double kRow42[9][7] = {
    {0.0, 1.0 / 12.0, -2.0 / 3.0, 0.0, 2.0 / 3.0, -1.0 / 12.0, 0.0},
    {0.0, 0.0, 0.0, C42_00, C42_01, C42_02, C42_03},
    {0.0, 0.0, -0.5, 0.0, 0.5, 0.0, 0.0},
    {0.0, C42_20, C42_21, 0.0, C42_23, C42_24, 0.0},
    {C42_30, 0.0, C42_32, 0.0, C42_34, C42_35, 0.0},
    {-C42_03, -C42_02, -C42_01, -C42_00, 0.0, 0.0, 0.0},
    {0.0, 0.0, -0.5, 0.0, 0.5, 0.0, 0.0},
    {0.0, -C42_24, -C42_23, 0.0, -C42_21, -C42_20, 0.0},
    {0.0, -C42_35, -C42_34, 0.0, -C42_32, 0.0, -C42_30},
};
__constant__ double kRow21[3][3] = {{-0.5, 0.0, 0.5}, {0.0, -1.0, 1.0}, {-1.0, 1.0, 0.0}};

template <int SBP>
__device__ __forceinline__ double row_coef(int row, int o)
{
    if constexpr (SBP == 21)
        return row <= 2 ? kRow21[row][o + 1] : 0.0;
    else
        return row <= 8 ? kRow42[row][o + 3] : 0.0;
}

// 3D Cartesian flux divergence and AB update, marching along z.  A workgroup
// of TX x TY threads owns TX x TY point columns and a chunk of zc planes of
// outputs (one output per thread and plane).  Per flux plane, each thread
// evaluates the three directional fluxes of its own point once (from q and the
// viscous quantities V of the gradient pass); the x and y fluxes of an output
// plane go to LDS with the in-plane halo (2R columns along x, 2R rows along y,
// one direction each, evaluated by the workgroup), the z flux is added at once,
// scaled by its row coefficient, into the sums of the 2R + 1 output planes it
// reaches (registers), which also receive their own plane's x and y
// derivative sums.  Each flux is evaluated about 1 + 2R/TX + 2R/TY (x, y) and
// 1 + 2R/zc (z) times per output.  SAT points are finished by k_sat3d, which
// adds their penalties to the stored F and redoes their AB update.
template <int SBP, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) k_rhs_zm3d(GridDev g, Phys ph, const double *__restrict__ q,
                                                      const double *__restrict__ vis, double *__restrict__ F,
                                                      Combine cb, int ntx, int nty, int nzc, int zc)
{
    constexpr int NV = 5, R = SBP == 21 ? 1 : 3, NT = TX * TY;
    constexpr int EX = TX + 2 * R, EY = TY + 2 * R;
    __shared__ double sX[NV][EX * TY];
    __shared__ double sY[NV][TX * EY];
    const int nblk = ntx * nty * nzc;
    const int b = xcd_tile(blockIdx.x, nblk);
    const int tx0 = (b % ntx) * TX, ty0 = ((b / ntx) % nty) * TY, z0 = (b / (ntx * nty)) * zc;
    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const int x = tx0 + lx, y = ty0 + ly;
    const int64_t N = g.npts;
    const bool col = x < g.n[0] && y < g.n[1];
    const int zend = min(z0 + zc, g.n[2]);
    const int nh = 2 * R * (TX + TY);
    const int64_t pc = col ? x * g.stride[0] + y * g.stride[1] : 0;   // column base

    // flux of direction m at in-plane point (i, j) of plane k (zero off the
    // grid and at holes); periodic directions wrap
    auto flux_at = [&](int i, int j, int k, int m) -> Vec<NV> {
        Vec<NV> f;
        const int c[3] = {i, j, k};
        int64_t idx = 0;
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int v = c[d];
            if (g.periodic[d]) v = v < 0 ? v + g.n[d] : (v >= g.n[d] ? v - g.n[d] : v);
            ok = ok && v >= 0 && v < g.n[d];
            idx += (int64_t)v * g.stride[d];
        }
        ok = ok && (g.cls[idx] & 15) != CLS_HOLE;
        if (ok) {
            f = fhat_at<3, 1>(g, ph, q, vis, m, idx);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) f.v[v] = 0.0;
        }
        return f;
    };
    // plane index inside the grid (periodic wrap), -1 off the grid
    auto plane = [&](int k) -> int {
        if (g.periodic[2]) k = k < 0 ? k + g.n[2] : (k >= g.n[2] ? k - g.n[2] : k);
        return k >= 0 && k < g.n[2] ? k : -1;
    };

    // acc[e]: sums of output plane k - R + e (e = 0 completes at flux plane k);
    // rz[e]: its z row
    Vec<NV> acc[2 * R + 1];
    int rz[2 * R + 1];
#pragma unroll
    for (int e = 0; e <= 2 * R; ++e) {
        rz[e] = CLS_HOLE;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[e].v[v] = 0.0;
    }
    const int nplanes = (zend - z0) + 2 * R;
    for (int s = 0; s < nplanes; ++s) {
        const int k = z0 - R + s;                 // flux plane
        const bool outp = k >= z0 && k < zend;    // an output plane of the chunk (uniform)
        // open the slot of output plane k + R
#pragma unroll
        for (int e = 0; e < 2 * R; ++e) {
            acc[e] = acc[e + 1];
            rz[e] = rz[e + 1];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[2 * R].v[v] = 0.0;
        {
            const int oz = k + R;
            rz[2 * R] = col && oz < zend ? g.cls[2 * N + pc + (int64_t)oz * g.stride[2]] & 15 : CLS_HOLE;
        }
        const int kw = plane(k);
        const int64_t p = pc + (int64_t)(kw < 0 ? 0 : kw) * g.stride[2];
        const bool act = col && kw >= 0 && (g.cls[p] & 15) != CLS_HOLE;
        Vec<NV> own[3];
        if (act) {
            if (outp) {
                fluxes3(g, ph, q, vis, p, own);
            } else {
                own[2] = fhat_at<3, 1>(g, ph, q, vis, 2, p);
            }
            // z flux into the sums of the output planes it reaches
#pragma unroll
            for (int e = 0; e <= 2 * R; ++e) {
                const double c = row_coef<SBP>(rz[e], R - e) * g.inv_h[2];
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[e].v[v] += c * own[2].v[v];
            }
        }
        if (outp) {
            if (col) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    sX[v][(lx + R) + EX * ly] = act ? own[0].v[v] : 0.0;
                    sY[v][lx + TX * (ly + R)] = act ? own[1].v[v] : 0.0;
                }
            } else {
                // a column past the grid's end (partial tile): the wrapped
                // point of a periodic direction, zero otherwise
                Vec<NV> fx = flux_at(x, y, k, 0), fy = flux_at(x, y, k, 1);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    sX[v][(lx + R) + EX * ly] = fx.v[v];
                    sY[v][lx + TX * (ly + R)] = fy.v[v];
                }
            }
            for (int h = tid; h < nh; h += NT) {
                if (h < 2 * R * TY) {
                    const int sd = h % (2 * R), r = h / (2 * R);
                    const int ex = sd < R ? sd : sd + TX;
                    Vec<NV> f = flux_at(tx0 + ex - R, ty0 + r, k, 0);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sX[v][ex + EX * r] = f.v[v];
                } else {
                    const int h2 = h - 2 * R * TY;
                    const int c = h2 % TX, sd = h2 / TX;
                    const int ey = sd < R ? sd : sd + TY;
                    Vec<NV> f = flux_at(tx0 + c, ty0 + ey - R, k, 1);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sY[v][c + TX * ey] = f.v[v];
                }
            }
            __syncthreads();
            if (act) {
                Vec<NV> dx = dsbp<SBP, NV>(g.cls[p] & 15, [&](int o) {
                    Vec<NV> r;
#pragma unroll
                    for (int v = 0; v < NV; ++v) r.v[v] = sX[v][(lx + R + o) + EX * ly];
                    return r;
                });
                Vec<NV> dy = dsbp<SBP, NV>(g.cls[N + p] & 15, [&](int o) {
                    Vec<NV> r;
#pragma unroll
                    for (int v = 0; v < NV; ++v) r.v[v] = sY[v][lx + TX * (ly + R + o)];
                    return r;
                });
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double a = acc[R].v[v];
                    a += g.inv_h[0] * dx.v[v];
                    a += g.inv_h[1] * dy.v[v];
                    acc[R].v[v] = a;
                }
            }
            __syncthreads();
        }
        // output plane k - R is complete
        const int oz = k - R;
        if (oz >= z0 && col) {
            const int64_t po = pc + (int64_t)oz * g.stride[2];
            double r[NV];
            const bool oact = rz[0] != CLS_HOLE;
#pragma unroll
            for (int v = 0; v < NV; ++v) r[v] = oact ? -1.0 * acc[0].v[v] : 0.0;
            store_step<3>(q, F, cb, N, po, r);
        }
    }
}

// SAT points of a 3D grid after k_rhs_zm3d: F holds the flux-divergence part;
// add the penalties, store F and redo the AB update
__global__ void __launch_bounds__(256) k_sat3d(GridDev g, Phys ph, const double *__restrict__ q,
                                               const double *__restrict__ vis, double *__restrict__ F, Combine cb,
                                               const int32_t *__restrict__ pts, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t N = g.npts, p = pts[i];
    double r[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] = F[v * N + p];
    sat_point<3, 1>(g, ph, q, vis, p, r);
    store_step<3>(q, F, cb, N, p, r);
}

// ------------------------------------------- fused LDS-tiled 2D right-hand side
// One workgroup of TM*TX*TY threads computes a TX x TY tile of outputs in one
// pass (the first TX*TY threads own one output each; all threads share the
// staging and flux phases, so small grids can still fill the CUs):
//   1. primitives (rho, u, v, T) and class bytes on the tile plus a halo of HP
//      points, metric terms on the flux region, all staged in LDS (every
//      global load of the phase is issued before the first use);
//   2. for xi then eta: the contravariant flux of that direction on the tile
//      plus HF points along it (gradients from the LDS primitives) in LDS,
//      then its SBP derivative at the outputs;
//   3. epilogue per output: scale, SAT penalties, store F, AB update.
// A first-derivative row reaches at most R = 3 points (SBP 4-2 closures; 1
// for SBP 2-1), so outputs need fluxes within HF = R and every flux point of
// that region has its whole stencil inside HP = HF + R, whatever the run
// layout.
template <int SBP, int TX_, int TY_, int TM_>
struct TileCfg {
    static constexpr int TX = TX_, TY = TY_, NO = TX_ * TY_, NT = TX_ * TY_ * TM_;
    static constexpr int R = SBP == 42 ? 3 : 1;
    static constexpr int HF = R, HP = 2 * R;
    static constexpr int PX = TX + 2 * HP, PY = TY + 2 * HP, PN = PX * PY;
    static constexpr int MX = TX + 2 * HF, MY = TY + 2 * HF, MN = MX * MY;   // metric region
    static constexpr int FN = (TX + 2 * HF) * TY > TX * (TY + 2 * HF) ? (TX + 2 * HF) * TY : TX * (TY + 2 * HF);
    static constexpr int NIT = (PN + NT - 1) / NT;
    // both directions' flux regions in one phase (one barrier less) when
    // that takes at most two passes of the threads and the second flux
    // buffer costs at most 16 KB of LDS
    static constexpr bool BOTH = (TX + 2 * HF) * TY + TX * (TY + 2 * HF) <= 2 * NT && 4 * FN * 8 <= 16 * 1024;
};

// periodic wrap of a line index (the remainder is taken only off the line)
__device__ __forceinline__ int wrap1(int i, int n)
{
    if (i < 0 || i >= n) {
        i %= n;
        if (i < 0) i += n;
    }
    return i;
}

// the work of one workgroup: the tile with corner (x0, y0) of grid g
template <int SBP, int CART, int TX_, int TY_, int TM_, bool NOEARLY = false>
__device__ __forceinline__ void rhs_tile2d_body(const GridDev &g, const Phys &ph, const double *__restrict__ q,
                                                double *__restrict__ F, const Combine &cb, int x0, int y0)
{
    using C = TileCfg<SBP, TX_, TY_, TM_>;
    constexpr int NT = C::NT;
    constexpr int TX = C::TX, TY = C::TY, HF = C::HF, HP = C::HP, PX = C::PX, PY = C::PY, PN = C::PN;
    constexpr int MX = C::MX, MN = C::MN;
    __shared__ double sP[4][PY][PX];                 // rho, u, v, T
    __shared__ double sF[4][C::FN];                  // contravariant flux of one direction
    __shared__ double sM[CART ? 1 : 5][CART ? 1 : MN];   // M00 M01 M10 M11 J on the flux region
    __shared__ int8_t sC[2][PY][PX];                 // class bytes

    const int nx = g.n[0], ny = g.n[1];
    const int64_t N = g.npts;
    const double gm1 = ph.gamma - 1.0;
    const int tid = threadIdx.x;

    // the thread's output point; its state and older history values are only
    // needed in the epilogue, so they are requested first
    const int tx = tid % TX, ty = tid / TX;
    const int cxo = HP + tx, cyo = HP + ty;
    const int gxo = x0 + tx, gyo = y0 + ty;
    const bool inside = tid < C::NO && gxo < nx && gyo < ny;
    const int64_t po = inside ? (int64_t)gyo * nx + gxo : 0;
    // (small, latency-bound tiles only: on large tiles the long live ranges
    // cost more occupancy than the early loads save)
    constexpr bool EARLY = TX_ * TY_ <= 128 && !NOEARLY;
    constexpr int HV = EARLY ? MAXH - 1 : 1;
    double hq[4], hv[HV][4];
    if constexpr (EARLY) {
#pragma unroll
        for (int v = 0; v < 4; ++v) hq[v] = inside ? q[v * N + po] : 0.0;
#pragma unroll
        for (int j = 0; j < HV; ++j)
            if (j < cb.m - 1 && inside) {
#pragma unroll
                for (int v = 0; v < 4; ++v) hv[j][v] = cb.hist[j][v * N + po];
            }
    }
    // NOEARLY (a kernel that must stay within 128 VGPRs): the same early
    // requests for the state and the HE oldest history values, parked in LDS
    // once the staging loads have landed instead of held in registers
    constexpr bool ELDS = NOEARLY && TX_ * TY_ <= 128;
    constexpr int HE = ELDS ? 3 : 1;
    __shared__ double sE[ELDS ? 4 * (1 + HE) : 1][ELDS ? C::NO : 1];
    double eq[4], eh[HE][4];
    if constexpr (ELDS) {
#pragma unroll
        for (int v = 0; v < 4; ++v) eq[v] = inside ? q[v * N + po] : 0.0;
#pragma unroll
        for (int j = 0; j < HE; ++j)
            if (j < cb.m - 1 && inside) {
#pragma unroll
                for (int v = 0; v < 4; ++v) eh[j][v] = cb.hist[j][v * N + po];
            }
    }

    // small tiles with early requests: a receiver's donor row (interface SAT
    // data) is requested once every staging load has been issued (its row
    // index first); other tiles read it in the epilogue
    constexpr bool RBE = EARLY;
    const int rrow = RBE && inside && g.recv_idx ? g.recv_idx[po] : -1;

    // 1. stage: issue every load first
    double lq[C::NIT][4];
    int8_t lc[C::NIT][2];
#pragma unroll
    for (int it = 0; it < C::NIT; ++it) {
        int e = tid + it * NT;
        lq[it][0] = lq[it][1] = lq[it][2] = lq[it][3] = 0.0;
        lc[it][0] = lc[it][1] = (int8_t)CLS_HOLE;
        if (e < PN) {
            int cx = e % PX, cy = e / PX;
            int gx = x0 - HP + cx, gy = y0 - HP + cy;
            bool ok = true;
            if (g.periodic[0]) gx = wrap1(gx, nx); else ok = ok && gx >= 0 && gx < nx;
            if (g.periodic[1]) gy = wrap1(gy, ny); else ok = ok && gy >= 0 && gy < ny;
            if (ok) {
                int64_t p = (int64_t)gy * nx + gx;
                lc[it][0] = g.cls[p];
                lc[it][1] = g.cls[N + p];
                lq[it][0] = q[p];
                lq[it][1] = q[N + p];
                lq[it][2] = q[2 * N + p];
                lq[it][3] = q[3 * N + p];
            }
        }
    }
    double rbv[RBE ? 10 : 1];
    auto rbload = [&]() {
        if constexpr (RBE) {
#pragma unroll
            for (int t = 0; t < 10; ++t) rbv[t] = rrow >= 0 ? g.recv[(int64_t)rrow * 10 + t] : 0.0;
        }
    };
    if constexpr (!CART) {
        constexpr int MIT = (MN + NT - 1) / NT;
        double lm[MIT][5];
#pragma unroll
        for (int it = 0; it < MIT; ++it) {
            int e = tid + it * NT;
            int mx = e % MX, my = e / MX;
            int gx = x0 - HF + mx, gy = y0 - HF + my;
            bool ok = e < MN;
            if (g.periodic[0]) gx = wrap1(gx, nx); else ok = ok && gx >= 0 && gx < nx;
            if (g.periodic[1]) gy = wrap1(gy, ny); else ok = ok && gy >= 0 && gy < ny;
            int64_t p = ok ? (int64_t)gy * nx + gx : 0;
#pragma unroll
            for (int kk = 0; kk < 5; ++kk) lm[it][kk] = ok ? g.metric[kk * N + p] : 0.0;
        }
        rbload();
#pragma unroll
        for (int it = 0; it < MIT; ++it) {
            int e = tid + it * NT;
            if (e < MN) {
#pragma unroll
                for (int kk = 0; kk < 5; ++kk) sM[kk][e] = lm[it][kk];
            }
        }
    } else {
        rbload();
    }
#pragma unroll
    for (int it = 0; it < C::NIT; ++it) {
        int e = tid + it * NT;
        if (e < PN) {
            int cx = e % PX, cy = e / PX;
            double r0 = 0.0, u = 0.0, v = 0.0, T = 0.0;
            if ((lc[it][0] & 15) != CLS_HOLE) {
                double ri = 1.0 / lq[it][0];
                u = lq[it][1] * ri;
                v = lq[it][2] * ri;
                double pr = gm1 * (lq[it][3] - 0.5 * (u * lq[it][1] + v * lq[it][2]));
                r0 = lq[it][0];
                T = pr * ri;
            }
            sP[0][cy][cx] = r0;
            sP[1][cy][cx] = u;
            sP[2][cy][cx] = v;
            sP[3][cy][cx] = T;
            sC[0][cy][cx] = lc[it][0];
            sC[1][cy][cx] = lc[it][1];
        }
    }
    if constexpr (ELDS) {
        if (inside) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sE[v][tid] = eq[v];
#pragma unroll
            for (int j = 0; j < HE; ++j)
                if (j < cb.m - 1) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) sE[4 + 4 * j + v][tid] = eh[j][v];
                }
        }
    }
    __syncthreads();

    // metric terms of box cell (cx, cy) (flux region only)
    auto metric_at = [&](int cx, int cy, int k) -> double {
        if constexpr (CART) {
            return 0.0;
        } else {
            return sM[k][(cy - (HP - HF)) * MX + (cx - (HP - HF))];
        }
    };

    // gradient of (u, v, T) at box cell (cx, cy)
    auto grad_at = [&](int cx, int cy, double gr[3][2]) {
        int rx = sC[0][cy][cx] & 15, ry = sC[1][cy][cx] & 15;
        Vec<3> dx = dsbp<SBP, 3>(rx, [&](int o) {
            Vec<3> r;
            r.v[0] = sP[1][cy][cx + o]; r.v[1] = sP[2][cy][cx + o]; r.v[2] = sP[3][cy][cx + o];
            return r;
        });
        Vec<3> dy = dsbp<SBP, 3>(ry, [&](int o) {
            Vec<3> r;
            r.v[0] = sP[1][cy + o][cx]; r.v[1] = sP[2][cy + o][cx]; r.v[2] = sP[3][cy + o][cx];
            return r;
        });
        if constexpr (CART) {
#pragma unroll
            for (int a = 0; a < 3; ++a) { gr[a][0] = g.inv_h[0] * dx.v[a]; gr[a][1] = g.inv_h[1] * dy.v[a]; }
        } else {
            double M00 = metric_at(cx, cy, 0), M01 = metric_at(cx, cy, 1);
            double M10 = metric_at(cx, cy, 2), M11 = metric_at(cx, cy, 3), J = metric_at(cx, cy, 4);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gr[a][0] = J * (M00 * dx.v[a] + M10 * dy.v[a]);
                gr[a][1] = J * (M01 * dx.v[a] + M11 * dy.v[a]);
            }
        }
    };

    // contravariant flux of direction m at box cell (cx, cy)
    auto flux_at = [&](int m, int cx, int cy, double *out) {
        double gr[3][2];
        grad_at(cx, cy, gr);
        double rho = sP[0][cy][cx], uu[2] = {sP[1][cy][cx], sP[2][cy][cx]}, T = sP[3][cy][cx];
        double pr = rho * T;
        double rE = pr / gm1 + 0.5 * rho * (uu[0] * uu[0] + uu[1] * uu[1]);
        double Fv[2][3];
        viscous_flux<2>(ph, uu, gr, Fv);
        if constexpr (CART) {
            out[0] = rho * uu[m];
            out[1] = rho * uu[0] * uu[m] + (m == 0 ? pr : 0.0) - Fv[m][0];
            out[2] = rho * uu[1] * uu[m] + (m == 1 ? pr : 0.0) - Fv[m][1];
            out[3] = (rE + pr) * uu[m] - Fv[m][2];
        } else {
            double M0 = metric_at(cx, cy, 2 * m), M1 = metric_at(cx, cy, 2 * m + 1);
            double U = M0 * uu[0] + M1 * uu[1];
            out[0] = rho * U;
            out[1] = rho * uu[0] * U + M0 * pr - (M0 * Fv[0][0] + M1 * Fv[1][0]);
            out[2] = rho * uu[1] * U + M1 * pr - (M0 * Fv[0][1] + M1 * Fv[1][1]);
            out[3] = (rE + pr) * U - (M0 * Fv[0][2] + M1 * Fv[1][2]);
        }
    };

    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // flux region of direction m: (TX + 2HF) x TY for xi, TX x (TY + 2HF) for eta
    constexpr int FN0 = (TX + 2 * HF) * TY, FN1 = TX * (TY + 2 * HF);
    auto flux_region = [&](int m, int e, double *f) {
        const int FX = m == 0 ? TX + 2 * HF : TX;
        const int ox = m == 0 ? HF : 0, oy = m == 0 ? 0 : HF;
        int fx = e % FX, fy = e / FX;
        int cx = HP - ox + fx, cy = HP - oy + fy;
#pragma unroll
        for (int v = 0; v < 4; ++v) f[v] = 0.0;
        if ((sC[0][cy][cx] & 15) != CLS_HOLE) flux_at(m, cx, cy, f);
    };
    auto divergence = [&](int m, double (*S)[C::FN]) {
        if (!inside) return;
        const int FX = m == 0 ? TX + 2 * HF : TX;
        int row = sC[m][cyo][cxo] & 15;
        if (row == CLS_HOLE) return;
        Vec<4> d = dsbp<SBP, 4>(row, [&](int o) {
            int fx = m == 0 ? tx + HF + o : tx;
            int fy = m == 0 ? ty : ty + HF + o;
            int e = fy * FX + fx;
            Vec<4> r;
            r.v[0] = S[0][e]; r.v[1] = S[1][e]; r.v[2] = S[2][e]; r.v[3] = S[3][e];
            return r;
        });
        double sc = CART ? g.inv_h[m] : 1.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += sc * d.v[v];
    };
    if constexpr (C::BOTH) {
        // enough threads for both flux regions at once: one phase, one barrier
        __shared__ double sF1[4][C::FN];
        for (int e = tid; e < FN0 + FN1; e += NT) {
            const int m = e < FN0 ? 0 : 1, ee = m ? e - FN0 : e;
            double f[4];
            flux_region(m, ee, f);
            double (*S)[C::FN] = m ? sF1 : sF;
#pragma unroll
            for (int v = 0; v < 4; ++v) S[v][ee] = f[v];
        }
        __syncthreads();
        divergence(0, sF);
        divergence(1, sF1);
    } else {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            for (int e = tid; e < (m ? FN1 : FN0); e += NT) {
                double f[4];
                flux_region(m, e, f);
#pragma unroll
                for (int v = 0; v < 4; ++v) sF[v][e] = f[v];
            }
            __syncthreads();
            divergence(m, sF);
            __syncthreads();
        }
    }

    // 3. epilogue
    if (!inside) return;
    if constexpr (ELDS) {
#pragma unroll
        for (int v = 0; v < 4; ++v) hq[v] = sE[v][tid];
    } else if constexpr (!EARLY) {
#pragma unroll
        for (int v = 0; v < 4; ++v) hq[v] = q[v * N + po];
    }
    const int64_t p = po;
    const int cx0 = sC[0][cyo][cxo], cy0 = sC[1][cyo][cxo];
    double r[4];
    if ((cx0 & 15) == CLS_HOLE) {
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] = 0.0;
    } else {
        double J = CART ? 1.0 : metric_at(cxo, cyo, 4);
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] = -J * acc[v];
        if (((cx0 >> 4) & 3) | ((cy0 >> 4) & 3)) {
            double qp[4] = {hq[0], hq[1], hq[2], hq[3]};
            // the viscous flux enters the interface and far-field penalties
            // only (a wall point's penalty has no flux term)
            const int b0 = (cx0 >> 4) & 3, b1 = (cy0 >> 4) & 3;
            double Fv[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
            if (b0 == 1 || b0 == 2 || b1 == 1 || b1 == 2) {
                double gr[3][2];
                grad_at(cxo, cyo, gr);
                double uu[2] = {sP[1][cyo][cxo], sP[2][cyo][cxo]};
                viscous_flux<2>(ph, uu, gr, Fv);
            }
            for (int m = 0; m < 2; ++m) {
                int c = m == 0 ? cx0 : cy0;
                int bc = (c >> 4) & 3;
                if (!bc) continue;
                int sgn = ((c & 15) == 1) ? 1 : -1;
                double kap[2];
                if constexpr (CART) {
                    kap[0] = m == 0 ? g.inv_h[0] : 0.0;
                    kap[1] = m == 1 ? g.inv_h[1] : 0.0;
                } else {
                    double Jp = metric_at(cxo, cyo, 4);
                    kap[0] = Jp * metric_at(cxo, cyo, 2 * m);
                    kap[1] = Jp * metric_at(cxo, cyo, 2 * m + 1);
                }
                double k2 = kap[0] * kap[0] + kap[1] * kap[1];
                double dQ[4], dV[4], s2[4] = {0.0, 0.0, 0.0, 0.0};
                double sigI, sig1 = k2 * (ph.mu / (2.0 * ph.Re));
                bool use_s2 = true;
#pragma unroll
                for (int v = 1; v < 4; ++v) s2[v] = kap[0] * Fv[0][v - 1] + kap[1] * Fv[1][v - 1];
                if (bc == 1) {
                    const double *rb = RBE ? rbv : g.recv + (int64_t)g.recv_idx[p] * 10;
#pragma unroll
                    for (int v = 0; v < 4; ++v) { dQ[v] = qp[v] - rb[v]; dV[v] = dQ[v]; }
#pragma unroll
                    for (int v = 1; v < 4; ++v) s2[v] -= kap[0] * rb[4 + (v - 1)] + kap[1] * rb[7 + (v - 1)];
                    sigI = ph.sig_iface;
                } else if (bc == 2) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) { dQ[v] = qp[v] - ph.q_inf[v]; dV[v] = dQ[v]; }
                    sigI = ph.sig_bc;
                } else {
                    // twice the normal momentum along the unit normal kappa / |kappa|
                    double mn = 0.0;
                    mn += qp[1] * kap[0];
                    mn += qp[2] * kap[1];
                    const double tm = 2.0 * mn / k2;
                    dQ[0] = 0.0; dV[0] = 0.0;
                    dQ[1] = tm * kap[0]; dV[1] = qp[1];
                    dQ[2] = tm * kap[1]; dV[2] = qp[2];
                    dQ[3] = 0.0; dV[3] = qp[3] - qp[0] * (ph.T_wall / gm1);
                    sigI = ph.sig_bc;
                    sig1 = k2 * (ph.wall_visc * ph.mu / ph.Re);
                    use_s2 = false;
                }
                double KdQ[4];
                k_apply<2>(ph.gamma, qp, kap, sgn, dQ, KdQ);
                double hs = 0.5 * sgn;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double pen = -(sigI * KdQ[v] + sig1 * dV[v]) * ph.p0inv;
                    if (use_s2) pen += hs * s2[v] * ph.p0inv;
                    r[v] += pen;
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) F[v * N + p] = r[v];
    if (cb.m > 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double a2 = hq[v];
#pragma unroll
            for (int j = 0; j < MAXH - 1; ++j)
                if (j < cb.m - 1) {
                    double h;
                    if constexpr (EARLY) h = hv[j < HV ? j : 0][v];
                    else if (ELDS && j < HE) h = sE[4 + 4 * (j < HE ? j : 0) + v][tid];
                    else h = cb.hist[j][v * N + p];
                    a2 = add_nc(a2, cb.c[j], h);
                }
            a2 = add_nc(a2, cb.c[cb.m - 1], r[v]);
            cb.y_next[v * N + p] = a2;
        }
    }
}

// one grid: tile blockIdx.x (XCD-ordered) of an ntx x nty tiling
template <int SBP, int CART, int TX_, int TY_, int TM_>
__global__ void __launch_bounds__(TX_ * TY_ * TM_, 2)
k_rhs_tile2d(GridDev g, Phys ph, const double *__restrict__ q, double *__restrict__ F, Combine cb, int ntx, int nty)
{
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    rhs_tile2d_body<SBP, CART, TX_, TY_, TM_>(g, ph, q, F, cb, (tile % ntx) * TX_, (tile / ntx) * TY_);
}

// a work list of grid evaluations (TileJob, ordered by first tile): the
// workgroup's tile in the concatenated tilings (XCD-ordered over the whole
// list), its job found by bisection on the first-tile offsets
template <int SBP, int CART, int TX_, int TY_, int TM_>
__global__ void __launch_bounds__(TX_ * TY_ * TM_, 2)
k_rhs_tiles(const TileJob *__restrict__ jobs, int njobs, int nblk, Phys ph)
{
    const int b = xcd_tile(blockIdx.x, nblk);
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= b) lo = mid; else hi = mid - 1;
    }
    const TileJob &J = jobs[lo];
    const int tile = b - J.tile0;
    rhs_tile2d_body<SBP, CART, TX_, TY_, TM_>(J.g, ph, J.q, J.F, J.cb, (tile % J.ntx) * TX_, (tile / J.ntx) * TY_);
}

// ---------------------------------------------------------------- donors
// Donor values: q and the Cartesian viscous flux vectors at each unique donor
// point, from the donor grid's state and its own SBP gradient.
template <int DIM, int SBP, int CART>
__global__ void __launch_bounds__(256) k_donor_vals(DonorLink a)
{
    constexpr int NV = DIM + 2;
    constexpr int RB = NV + DIM * (NV - 1);
    __shared__ double sv[256 * RB];
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nl = a.nu * a.nj;               // lanes with a row to write
    const int wl = threadIdx.x & 63;
    double *ws = sv + (threadIdx.x - wl) * RB;    // this wave's 64 rows
    if (lane < nl) {
        const int j = (int)(lane / a.nu);
        const int64_t u = lane - (int64_t)j * a.nu;
        const int64_t p = a.upts[u];
        const int64_t N = a.g.npts;
        const double *y = nullptr;
#pragma unroll
        for (int jj = 0; jj < MAXJ; ++jj)
            if (jj == j) y = a.ys[jj];
        auto qload = [&](int64_t idx, double *o) {
#pragma unroll
            for (int v = 0; v < NV; ++v) o[v] = y[v * N + idx];
        };
        double qp[NV];
        qload(p, qp);
        int ic[3];
        coords(a.g, p, ic);
        double gr[DIM + 1][DIM];
        gradient<DIM, SBP, CART>(a.g, p, ic, a.ph.gamma - 1.0, qload, gr);
        double u_[DIM];
        double ri = 1.0 / qp[0];
#pragma unroll
        for (int i = 0; i < DIM; ++i) u_[i] = qp[1 + i] * ri;
        double Fv[DIM][DIM + 1];
        viscous_flux<DIM>(a.ph, u_, gr, Fv);
        double *o = ws + wl * RB;
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = qp[v];
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int v = 1; v < NV; ++v) o[NV + d * (NV - 1) + (v - 1)] = Fv[d][v - 1];
    }
    __syncthreads();
    // lane (j, u) owns row j * nu + u of a.vals, so the wave's rows are one
    // contiguous block: written with consecutive lanes on consecutive doubles
    const int64_t lane0 = lane - wl;
#pragma unroll
    for (int c = 0; c < RB; ++c) {
        const int f = c * 64 + wl;
        if (lane0 + f / RB < nl) a.vals[lane0 * RB + f] = ws[f];
    }
}

// Receiver rows: Lagrange-weighted sum of the donor values; one lane per
// (slot, receiver, entry), summed over the S lanes of a receiver by a
// transposed butterfly.  At the step of lane offset 2^b every component's
// partial sum over a block of 2^b lanes meets its partner block's, as in a
// plain butterfly (so each component is the same tree of additions), but a
// lane keeps only half of its components (the upper half when bit b of its
// entry is set) and sends the other half: with RB padded to P components,
// log2(P) steps leave one component per lane and about P shuffles in all
// instead of RB per step.
template <int RB>
__global__ void __launch_bounds__(256) k_donor_gather(DonorLink a)
{
    constexpr int P = RB <= 16 ? 16 : 32;
    int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_slot = a.nrecv * a.S;
    const int j = (int)(lane / per_slot);
    if (j >= a.nj) return;                    // whole groups of S lanes leave together
    const int64_t rem = lane - (int64_t)j * per_slot;
    const int64_t k = rem / a.S;
    const int e = (int)(rem % a.S);
    double *outp = nullptr;
#pragma unroll
    for (int jj = 0; jj < MAXJ; ++jj)
        if (jj == j) outp = a.out[jj];
    const int64_t ent = k * a.S + e;
    const double w = a.w[ent];
    const double *vrow = a.vals + ((int64_t)j * a.nu + a.uid[ent]) * RB;
    double v[P];
#pragma unroll
    for (int t = 0; t < P; ++t) v[t] = t < RB ? w * vrow[t] : 0.0;
    int base = 0;       // component held in v[0]
    int halving = 0;    // halving steps taken
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const int off = 1 << b;
        if (off >= a.S) break;
        const int half = (P >> b) / 2;
        if (half >= 1) {
            const bool hi = (e & off) != 0;
#pragma unroll
            for (int i = 0; i < half; ++i) {
                const double send = hi ? v[i] : v[i + half];
                const double keep = hi ? v[i + half] : v[i];
                v[i] = keep + __shfl_xor(send, off, 64);
            }
            if (hi) base += half;
            ++halving;
        } else {
            v[0] = v[0] + __shfl_xor(v[0], off, 64);
        }
    }
    // lanes that differ only in bits past the halving steps hold the same sums
    if (e >> halving) return;
    const int cnt = P >> halving;
    double *o = outp + (int64_t)(a.row0 + k) * RB;
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (i < cnt && base + i < RB) o[base + i] = v[i];
}

// Receiver rows of one chunk of receivers for slot j = blockIdx.y in one
// workgroup: (EXT) the extrapolant at the points the chunk's gradient
// stencils read, each value with the same separately rounded products and
// sums as k_extrap, into LDS; q and the Cartesian viscous fluxes once per
// distinct donor point into LDS; then each receiver's S entries weighted and
// added by a plain butterfly over the S lanes (the same tree of additions,
// so the same bits, as k_donor_gather's transposed one).  The first 256
// threads do the work; threads past them (a larger workgroup shared with
// other work) only take part in the barriers.
template <int DIM, int SBP, int CART, int EXT>
__device__ __forceinline__ void donor_block_body(const DonorLink &a, const DonorBlocks &b, int ch, int j, double *sh)
{
    constexpr int NV = DIM + 2;
    constexpr int RB = NV + DIM * (NV - 1);
    constexpr int NT = 256;
    constexpr int KP = 1 + 4 * DIM;                    // stencil positions per donor point
    double *sV = sh;                                   // maxu x RB
    double *sQ = sh + (size_t)b.maxu * RB;             // NV x maxc
    int16_t *sP = reinterpret_cast<int16_t *>(sQ + (size_t)b.maxc * NV);   // maxu x KP
    const int tid = threadIdx.x;
    const double *y = nullptr;
    double *outp = nullptr;
    double bj[MAXH];
#pragma unroll
    for (int jj = 0; jj < MAXJ; ++jj)
        if (jj == j) {
            y = a.ys[jj];
            outp = a.out[jj];
#pragma unroll
            for (int hh = 0; hh < MAXH; ++hh) bj[hh] = a.beta[jj][hh];
        }
    const int64_t N = a.g.npts;
    // loads that depend on nothing the work computes are issued first: this
    // lane's receiver entry (weight, row of its donor point), its distinct
    // donor point (a chunk has at most 256, one per lane) with its stencil
    // positions, and the chunk's closure points (lists padded to maxu and
    // maxc per chunk, -1 past a chunk's count)
    const int kk = tid / a.S, e = tid - kk * a.S;
    const int64_t k = (int64_t)ch * b.rpc + kk;
    const bool ok = tid < NT && kk < b.rpc && k < a.nrecv;
    double w_ent = 0.0;
    int el_ent = 0;
    if (ok) {
        const int64_t ent = k * a.S + e;
        w_ent = a.w[ent];
        el_ent = b.eloc[ent];
    }
    const bool lane_u = tid < NT && tid < b.maxu;
    const int64_t p_own = lane_u ? b.upts[(int64_t)ch * b.maxu + tid] : -1;
    const bool own_u = p_own >= 0;
    if constexpr (EXT) {
        int16_t bp[KP];
#pragma unroll
        for (int r = 0; r < KP; ++r) bp[r] = lane_u ? b.bpos[((int64_t)ch * b.maxu + tid) * KP + r] : (int16_t)0;
        const int mh = a.m;
        const int nc = b.maxc;
        const int32_t *cp = b.cpts + (int64_t)ch * nc;
        // batches of XB items per thread: every load of a batch is issued
        // before the first sum
        constexpr int XB = 4;
        for (int base = 0; base < nc * NV; base += NT * XB) {
            double ly[XB], lh[XB][MAXH];
            int64_t el[XB];
            int32_t pt[XB];
#pragma unroll
            for (int r = 0; r < XB; ++r) {
                const int i = base + r * NT + tid;
                pt[r] = -1;
                if (tid < NT && i < nc * NV) pt[r] = cp[i - (i / nc) * nc];
            }
#pragma unroll
            for (int r = 0; r < XB; ++r) {
                const int i = base + r * NT + tid;
                el[r] = -1;
                if (pt[r] >= 0) {
                    const int v = i / nc;
                    el[r] = (int64_t)v * N + pt[r];
                    ly[r] = y[el[r]];
#pragma unroll
                    for (int hh = 0; hh < MAXH; ++hh)
                        if (hh < mh) lh[r][hh] = a.hist[hh][el[r]];
                }
            }
#pragma unroll
            for (int r = 0; r < XB; ++r) {
                const int i = base + r * NT + tid;
                if (el[r] < 0) continue;
                const int v = i / nc, ii = i - v * nc;
                double acc = ly[r];
#pragma unroll
                for (int hh = 0; hh < MAXH; ++hh)
                    if (hh < mh) acc = add_nc(acc, bj[hh], lh[r][hh]);
                sQ[(size_t)v * b.maxc + ii] = acc;
            }
        }
        if (own_u)
#pragma unroll
            for (int r = 0; r < KP; ++r) sP[(size_t)tid * KP + r] = bp[r];
        __syncthreads();
    }
    // EXT: the point's own entry, then its gradient stencil in the order
    // gradient() reads it (directions ascending, each row's offsets as the SBP
    // row applies them), as positions in the chunk's extrapolated points
    const int16_t *pos = nullptr;
    int cursor = 0;
    auto qload = [&](int64_t idx, double *o) {
        if constexpr (EXT) {
            const int at = pos[cursor++];
#pragma unroll
            for (int v = 0; v < NV; ++v) o[v] = sQ[(size_t)v * b.maxc + at];
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) o[v] = y[v * N + idx];
        }
    };
    if (own_u) {
        const int u = tid;
        const int64_t p = p_own;
        pos = sP + (size_t)u * KP;
        cursor = 0;
        double qp[NV];
        qload(p, qp);
        int ic[3];
        coords(a.g, p, ic);
        double gr[DIM + 1][DIM];
        if constexpr (!EXT && DIM == 2) {
            // current-time 2D links: the whole stencil requested at once
            const bool cart = CART == 2 ? a.g.cartesian : CART == 1;
            gradient_window<DIM, SBP>(a.g, p, ic, cart, a.ph.gamma - 1.0, y, qp, gr);
        } else if constexpr (CART == 2) {   // grid kind chosen per link at run time
            if (a.g.cartesian)
                gradient<DIM, SBP, 1>(a.g, p, ic, a.ph.gamma - 1.0, qload, gr);
            else
                gradient<DIM, SBP, 0>(a.g, p, ic, a.ph.gamma - 1.0, qload, gr);
        } else {
            gradient<DIM, SBP, CART>(a.g, p, ic, a.ph.gamma - 1.0, qload, gr);
        }
        double u_[DIM];
        double ri = 1.0 / qp[0];
#pragma unroll
        for (int i = 0; i < DIM; ++i) u_[i] = qp[1 + i] * ri;
        double Fv[DIM][DIM + 1];
        viscous_flux<DIM>(a.ph, u_, gr, Fv);
        double *o = sV + (size_t)u * RB;
#pragma unroll
        for (int v = 0; v < NV; ++v) o[v] = qp[v];
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int v = 1; v < NV; ++v) o[NV + d * (NV - 1) + (v - 1)] = Fv[d][v - 1];
    }
    __syncthreads();
    double val[RB];
    if (ok) {
        const double *vrow = sV + (size_t)el_ent * RB;
#pragma unroll
        for (int t = 0; t < RB; ++t) val[t] = w_ent * vrow[t];
    } else {
#pragma unroll
        for (int t = 0; t < RB; ++t) val[t] = 0.0;
    }
    for (int off = 1; off < a.S; off <<= 1) {
#pragma unroll
        for (int t = 0; t < RB; ++t) val[t] += __shfl_xor(val[t], off, 64);
    }
    if (ok && e == 0) {
        double *o = outp + (int64_t)(a.row0 + k) * RB;
#pragma unroll
        for (int t = 0; t < RB; ++t) o[t] = val[t];
    }
}

// one link: chunk blockIdx.x, slot blockIdx.y
template <int DIM, int SBP, int CART, int EXT>
__global__ void __launch_bounds__(256) k_donor_block(DonorLink a, DonorBlocks b)
{
    extern __shared__ double sh[];
    donor_block_body<DIM, SBP, CART, EXT>(a, b, blockIdx.x, blockIdx.y, sh);
}

// up to two links by value in one launch (their grid kinds may differ):
// chunk blockIdx.x of the two chunk lists, slot blockIdx.y
template <int DIM, int SBP, int EXT>
__global__ void __launch_bounds__(256) k_donor_block2(DonorLinks2 L)
{
    extern __shared__ double sh[];
    const int w = (L.n > 1 && (int)blockIdx.x >= L.chunk0[1]) ? 1 : 0;
    if ((int)blockIdx.y >= L.a[w].nj) return;
    donor_block_body<DIM, SBP, 2, EXT>(L.a[w], L.b[w], blockIdx.x - L.chunk0[w], blockIdx.y, sh);
}

// a work list of links (LinkJob, ordered by first chunk): chunk blockIdx.x
// of the concatenated chunk lists, slot blockIdx.y (workgroups past a link's
// slot count leave at once)
template <int DIM, int SBP, int CART, int EXT>
__global__ void __launch_bounds__(256) k_donor_blocks(const LinkJob *__restrict__ jobs, int njobs)
{
    extern __shared__ double sh[];
    const int bx = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].chunk0 <= bx) lo = mid; else hi = mid - 1;
    }
    const LinkJob &J = jobs[lo];
    if ((int)blockIdx.y >= J.a.nj) return;
    donor_block_body<DIM, SBP, CART, EXT>(J.a, J.b, bx - J.chunk0, blockIdx.y, sh);
}

// A grid's fused right-hand side and, in the same launch, the donor data of
// one chunked 2D link that neither reads nor writes anything the evaluation
// touches (another grid's mid-step data, gathered right after that grid
// evaluated at the same micro-time): workgroups below ntx * nty take the
// tiles (XCD-ordered as in k_rhs_tile2d), the rest take (chunk, slot) pairs
// of the link with the first 256 threads.  One launch less per pair.  The
// tiles here request their state and history values in the epilogue, which
// keeps the kernel within 128 VGPRs: two workgroups fit a CU, so the donor
// workgroups run beside the tiles rather than after them.
template <int SBP, int CART, int TX_, int TY_, int TM_>
__global__ void __launch_bounds__(TX_ * TY_ * TM_, 4)
k_rhs_tile2d_donor(GridDev g, Phys ph, const double *__restrict__ q, double *__restrict__ F, Combine cb, int ntx,
                   int nty, DonorLink a, DonorBlocks b)
{
    static_assert(TX_ * TY_ * TM_ >= 256, "the donor body needs 256 threads");
    extern __shared__ double sh[];
    const int ntile = ntx * nty;
    if ((int)blockIdx.x < ntile) {
        const int tile = xcd_tile(blockIdx.x, ntile);
        rhs_tile2d_body<SBP, CART, TX_, TY_, TM_, true>(g, ph, q, F, cb, (tile % ntx) * TX_, (tile / ntx) * TY_);
    } else {
        const int d = (int)blockIdx.x - ntile;
        if (d < b.nchunk * a.nj) donor_block_body<2, SBP, 2, 1>(a, b, d % b.nchunk, d / b.nchunk, sh);
    }
}

// extrapolated donor states at the donor-stencil points of mid-step links:
// one lane per (slot, point, variable)
__global__ void __launch_bounds__(256) k_extrap(Extrap a)
{
    int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = a.np * a.nv;
    const int j = (int)(lane / per);
    if (j >= a.nj) return;
    const int64_t rem = lane - (int64_t)j * per;
    const int v = (int)(rem / a.np);
    const int64_t i = rem - (int64_t)v * a.np;
    const int64_t el = (int64_t)v * a.N + a.pts[i];
    double bj[MAXH];
    double *outp = nullptr;
#pragma unroll
    for (int jj = 0; jj < MAXJ; ++jj)
        if (jj == j) {
            outp = a.out[jj];
#pragma unroll
            for (int hh = 0; hh < MAXH; ++hh) bj[hh] = a.beta[jj][hh];
        }
    double hv[MAXH];
#pragma unroll
    for (int hh = 0; hh < MAXH; ++hh)
        if (hh < a.m) hv[hh] = a.hist[hh][el];
    double acc = a.y[el];
#pragma unroll
    for (int hh = 0; hh < MAXH; ++hh)
        if (hh < a.m) acc = add_nc(acc, bj[hh], hv[hh]);
    outp[el] = acc;
}

hipError_t launch_extrap(const Extrap &a, hipStream_t st)
{
    if (a.np == 0 || a.nj == 0) return hipSuccess;
    int64_t lanes = a.np * a.nv * a.nj;
    hipLaunchKernelGGL(k_extrap, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- elementwise
__global__ void k_combine(int64_t n, const double *__restrict__ y, Combine cb)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double acc = y[e];
#pragma unroll
    for (int j = 0; j < MAXH; ++j)
        if (j < cb.m) acc = add_nc(acc, cb.c[j], cb.hist[j][e]);
    cb.y_next[e] = acc;
}

__global__ void k_axpy(int64_t n, const double *__restrict__ y, double a, const double *__restrict__ x,
                       double *__restrict__ out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = y[e] + a * x[e];
}

__global__ void k_rk3_final(int64_t n, const double *__restrict__ y, double a, const double *__restrict__ k1,
                            const double *__restrict__ k3, double *__restrict__ out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = y[e] + a * (k1[e] + 3.0 * k3[e]);
}

__global__ void k_rk4_final(int64_t n, const double *__restrict__ y, double a, const double *__restrict__ k1,
                            const double *__restrict__ k2, const double *__restrict__ k3,
                            const double *__restrict__ k4, double *__restrict__ out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = y[e] + a * (k1[e] + 2.0 * k2[e] + 2.0 * k3[e] + k4[e]);
}

// ---------------------------------------------------------------- setup
// 2D metric terms by the grid's own full-line SBP derivative of the
// coordinates (closures at non-periodic grid ends; coordinate jumps across
// periodic seams)
template <int SBP>
__global__ void k_metrics2d(GridDev g, const double *__restrict__ x, const double *__restrict__ y, double px0,
                            double px1, double py0, double py1, double *__restrict__ M)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.npts) return;
    constexpr int NB = SBP == 21 ? 1 : 4;
    int ic[3];
    coords(g, p, ic);
    double d[2][2];   // d[coord][dir]
    const double perx[2] = {px0, px1}, pery[2] = {py0, py1};
    for (int m = 0; m < 2; ++m) {
        int n = g.n[m], i = ic[m];
        int row = 0;
        if (!g.periodic[m]) row = i < NB ? 1 + i : (i >= n - NB ? 5 + (n - 1 - i) : 0);
        Vec<2> r = dsbp<SBP, 2>(row, [&](int o) {
            int j = i + o;
            double jx = 0.0, jy = 0.0;
            if (g.periodic[m]) {
                if (j < 0) { j += n; jx = -perx[m]; jy = -pery[m]; }
                else if (j >= n) { j -= n; jx = perx[m]; jy = pery[m]; }
            }
            int64_t idx = p + (int64_t)(j - i) * g.stride[m];
            Vec<2> v;
            v.v[0] = x[idx] + jx;
            v.v[1] = y[idx] + jy;
            return v;
        });
        d[0][m] = r.v[0];
        d[1][m] = r.v[1];
    }
    const int64_t N = g.npts;
    double jinv = d[0][0] * d[1][1] - d[0][1] * d[1][0];
    M[0 * N + p] = d[1][1];
    M[1 * N + p] = -d[0][1];
    M[2 * N + p] = -d[1][0];
    M[3 * N + p] = d[0][0];
    M[4 * N + p] = 1.0 / jinv;
}

template <int DIM>
__global__ void k_dt(GridDev g, Phys ph, const double *__restrict__ q, double *__restrict__ dt)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.npts) return;
    if ((g.cls[p] & 15) == CLS_HOLE) { dt[p] = INFINITY; return; }
    const int64_t N = g.npts;
    double qq[DIM + 2];
    load_q<DIM>(q, N, p, qq);
    double ri = 1.0 / qq[0], u[DIM], ke = 0.0;
    for (int i = 0; i < DIM; ++i) { u[i] = qq[1 + i] * ri; ke += u[i] * qq[1 + i]; }
    double pr = (ph.gamma - 1.0) * (qq[DIM + 1] - 0.5 * ke);
    double c = sqrt(ph.gamma * pr * ri);
    double J, adv = 0.0, sn = 0.0;
    if (g.cartesian) {
        double vol = 1.0;
        for (int m = 0; m < DIM; ++m) vol /= g.inv_h[m];
        J = 1.0 / vol;
        for (int m = 0; m < DIM; ++m) {
            double Mm = vol * g.inv_h[m];
            adv += fabs(u[m] * Mm);
            sn += Mm;
        }
    } else {
        J = g.metric[(int64_t)(DIM * DIM) * N + p];
        for (int m = 0; m < DIM; ++m) {
            double dot = 0.0, nrm = 0.0;
            for (int j = 0; j < DIM; ++j) {
                double Mmj = g.metric[(int64_t)(m * DIM + j) * N + p];
                dot += u[j] * Mmj;
                nrm += Mmj * Mmj;
            }
            adv += fabs(dot);
            sn += sqrt(nrm);
        }
    }
    double nu = fmax(ph.mu, ph.gamma * ph.mu / ph.Pr) * ri / ph.Re;
    dt[p] = fabs(1.0 / J) / (adv + c * sn + 2.0 * nu * fabs(J) * sn * sn);
}

__global__ void __launch_bounds__(256) k_reduce(int64_t n, const double *__restrict__ x, int mode,
                                                double *__restrict__ partial)
{
    __shared__ double sh[256];
    double acc = mode == 0 ? INFINITY : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double v = x[e];
        if (mode == 0) acc = fmin(acc, v);
        else acc = isfinite(v) ? fmax(acc, fabs(v)) : INFINITY;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            double o = sh[threadIdx.x + s];
            sh[threadIdx.x] = mode == 0 ? fmin(sh[threadIdx.x], o) : fmax(sh[threadIdx.x], o);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

#define DISPATCH_RHS(DIM, SBP, CART)                                                                  \
    hipLaunchKernelGGL((k_rhs<DIM, SBP, CART>), dim3(nblk(g.npts, 256)), dim3(256), 0, st, g, ph, q, \
                       grad, F, cb)

hipError_t launch_rhs(const GridDev &g, const GridDev *, int sbp, const Phys &ph, const double *q,
                      const double *grad, double *F, const Combine &cb, hipStream_t st)
{
    if (g.dim == 2 && sbp == 21 && g.cartesian) DISPATCH_RHS(2, 21, 1);
    else if (g.dim == 2 && sbp == 21) DISPATCH_RHS(2, 21, 0);
    else if (g.dim == 2 && sbp == 42 && g.cartesian) DISPATCH_RHS(2, 42, 1);
    else if (g.dim == 2 && sbp == 42) DISPATCH_RHS(2, 42, 0);
    else if (g.dim == 3 && sbp == 21 && g.cartesian) DISPATCH_RHS(3, 21, 1);
    else if (g.dim == 3 && sbp == 42 && g.cartesian) DISPATCH_RHS(3, 42, 1);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int TX, int TY, int TM>
static hipError_t tile2d_shape(const GridDev &g, int sbp, const Phys &ph, const double *q, double *F,
                               const Combine &cb, hipStream_t st)
{
    int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY;
    dim3 grid(ntx * nty), blk(TX * TY * TM);
    if (sbp == 21 && g.cartesian)
        hipLaunchKernelGGL((k_rhs_tile2d<21, 1, TX, TY, TM>), grid, blk, 0, st, g, ph, q, F, cb, ntx, nty);
    else if (sbp == 21)
        hipLaunchKernelGGL((k_rhs_tile2d<21, 0, TX, TY, TM>), grid, blk, 0, st, g, ph, q, F, cb, ntx, nty);
    else if (g.cartesian)
        hipLaunchKernelGGL((k_rhs_tile2d<42, 1, TX, TY, TM>), grid, blk, 0, st, g, ph, q, F, cb, ntx, nty);
    else
        hipLaunchKernelGGL((k_rhs_tile2d<42, 0, TX, TY, TM>), grid, blk, 0, st, g, ph, q, F, cb, ntx, nty);
    return hipGetLastError();
}

// Tile shapes (TX x TY outputs, TM threads per output).  Every shape evaluates
// the same formulas per output; results differ at most by rounding, where the
// compiler contracts a multiply-add differently in one instantiation.
const TileShape kTileShapes[NUM_TILE_SHAPES] = {
    {32, 16, 1}, {16, 8, 1}, {16, 8, 2}, {16, 8, 4}, {32, 8, 1}, {32, 8, 2}, {16, 16, 1}, {16, 16, 2},
};

// default: large grids 32 x 16 (less halo per output); small grids 16 x 8
// with four threads per output (enough waves to cover the 256 CUs)
int default_tile_shape(const GridDev &g)
{
    return g.npts >= (int64_t)128 * 1024 ? 0 : 3;
}

hipError_t launch_rhs_tile2d(const GridDev &g, int sbp, const Phys &ph, const double *q, double *F,
                             const Combine &cb, int shape, hipStream_t st)
{
    if (g.dim != 2) return hipErrorInvalidValue;
    switch (shape) {
    case 0: return tile2d_shape<32, 16, 1>(g, sbp, ph, q, F, cb, st);
    case 1: return tile2d_shape<16, 8, 1>(g, sbp, ph, q, F, cb, st);
    case 2: return tile2d_shape<16, 8, 2>(g, sbp, ph, q, F, cb, st);
    case 3: return tile2d_shape<16, 8, 4>(g, sbp, ph, q, F, cb, st);
    case 4: return tile2d_shape<32, 8, 1>(g, sbp, ph, q, F, cb, st);
    case 5: return tile2d_shape<32, 8, 2>(g, sbp, ph, q, F, cb, st);
    case 6: return tile2d_shape<16, 16, 1>(g, sbp, ph, q, F, cb, st);
    case 7: return tile2d_shape<16, 16, 2>(g, sbp, ph, q, F, cb, st);
    default: return hipErrorInvalidValue;
    }
}

template <int TX, int TY, int TM>
static hipError_t tile2d_donor_shape(const GridDev &g, int sbp, const Phys &ph, const double *q, double *F,
                                     const Combine &cb, const DonorLink &a, const DonorBlocks &b, size_t lds,
                                     hipStream_t st)
{
    if constexpr (TX * TY * TM < 256) {
        return hipErrorInvalidValue;
    } else {
        int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY;
        dim3 grid(ntx * nty + b.nchunk * a.nj), blk(TX * TY * TM);
        if (sbp == 21 && g.cartesian)
            hipLaunchKernelGGL((k_rhs_tile2d_donor<21, 1, TX, TY, TM>), grid, blk, lds, st, g, ph, q, F, cb, ntx, nty,
                               a, b);
        else if (sbp == 21)
            hipLaunchKernelGGL((k_rhs_tile2d_donor<21, 0, TX, TY, TM>), grid, blk, lds, st, g, ph, q, F, cb, ntx, nty,
                               a, b);
        else if (g.cartesian)
            hipLaunchKernelGGL((k_rhs_tile2d_donor<42, 1, TX, TY, TM>), grid, blk, lds, st, g, ph, q, F, cb, ntx, nty,
                               a, b);
        else
            hipLaunchKernelGGL((k_rhs_tile2d_donor<42, 0, TX, TY, TM>), grid, blk, lds, st, g, ph, q, F, cb, ntx, nty,
                               a, b);
        return hipGetLastError();
    }
}

bool tile2d_donor_ok(int shape)
{
    return shape >= 0 && shape < NUM_TILE_SHAPES && kTileShapes[shape].tx * kTileShapes[shape].ty * kTileShapes[shape].tm >= 256;
}

hipError_t launch_rhs_tile2d_donor(const GridDev &g, int sbp, const Phys &ph, const double *q, double *F,
                                   const Combine &cb, int shape, const DonorLink &a, const DonorBlocks &b,
                                   hipStream_t st)
{
    if (g.dim != 2 || a.g.dim != 2 || a.sbp != sbp || !tile2d_donor_ok(shape)) return hipErrorInvalidValue;
    if (a.nrecv == 0 || a.nj == 0) return launch_rhs_tile2d(g, sbp, ph, q, F, cb, shape, st);
    if (a.S < 1 || a.S > 64 || (a.S & (a.S - 1)) || b.rpc * a.S > 256 || a.nj > MAXJ || a.m < 1 ||
        a.m > MAXH || b.nchunk < 1 || (int64_t)b.nchunk * b.rpc < a.nrecv)
        return hipErrorInvalidValue;
    const size_t lds = donor_block_lds(2, b.maxu, b.maxc);
    switch (shape) {
    case 0: return tile2d_donor_shape<32, 16, 1>(g, sbp, ph, q, F, cb, a, b, lds, st);
    case 1: return tile2d_donor_shape<16, 8, 1>(g, sbp, ph, q, F, cb, a, b, lds, st);
    case 2: return tile2d_donor_shape<16, 8, 2>(g, sbp, ph, q, F, cb, a, b, lds, st);
    case 3: return tile2d_donor_shape<16, 8, 4>(g, sbp, ph, q, F, cb, a, b, lds, st);
    case 4: return tile2d_donor_shape<32, 8, 1>(g, sbp, ph, q, F, cb, a, b, lds, st);
    case 5: return tile2d_donor_shape<32, 8, 2>(g, sbp, ph, q, F, cb, a, b, lds, st);
    case 6: return tile2d_donor_shape<16, 16, 1>(g, sbp, ph, q, F, cb, a, b, lds, st);
    case 7: return tile2d_donor_shape<16, 16, 2>(g, sbp, ph, q, F, cb, a, b, lds, st);
    default: return hipErrorInvalidValue;
    }
}

#define DISPATCH_GRAD(DIM, SBP, CART) \
    hipLaunchKernelGGL((k_grad<DIM, SBP, CART>), dim3(nblk(g.npts, 256)), dim3(256), 0, st, g, ph, q, grad)

const TileShape3 kTile3dShapes[NUM_TILE3D_SHAPES] = {{8, 8, 8}, {16, 8, 4}, {32, 4, 4}, {16, 4, 4}, {16, 8, 8},
                                                      {32, 8, 4}};

template <int TX, int TY, int TZ>
static hipError_t grad3d_shape(const GridDev &g, int sbp, const Phys &ph, const double *q, double *vis, int slab,
                               hipStream_t st)
{
    const int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY, ntz = (g.n[2] + TZ - 1) / TZ;
    const int sy = slab > 0 && slab < nty ? slab : nty;
    const dim3 grid((unsigned)(ntx * nty * ntz)), block(TX * TY * TZ);
    if (sbp == 21)
        hipLaunchKernelGGL((k_grad_tile3d<21, TX, TY, TZ>), grid, block, 0, st, g, ph, q, vis, ntx, nty, ntz, sy);
    else
        hipLaunchKernelGGL((k_grad_tile3d<42, TX, TY, TZ>), grid, block, 0, st, g, ph, q, vis, ntx, nty, ntz, sy);
    return hipGetLastError();
}

static hipError_t grad3d_launch(const GridDev &g, int sbp, const Phys &ph, const double *q, double *vis, int shape,
                                int slab, hipStream_t st)
{
    switch (shape) {
    case 0: return grad3d_shape<8, 8, 8>(g, sbp, ph, q, vis, slab, st);
    case 1: return grad3d_shape<16, 8, 4>(g, sbp, ph, q, vis, slab, st);
    case 2: return grad3d_shape<32, 4, 4>(g, sbp, ph, q, vis, slab, st);
    case 3: return grad3d_shape<16, 4, 4>(g, sbp, ph, q, vis, slab, st);
    case 4: return grad3d_shape<16, 8, 8>(g, sbp, ph, q, vis, slab, st);
    case 5: return grad3d_shape<32, 8, 4>(g, sbp, ph, q, vis, slab, st);
    default: return hipErrorInvalidValue;
    }
}


template <int TX, int TY, int TZ>
static hipError_t flux3d_shape(const GridDev &g, int sbp, const Phys &ph, const double *q, const double *vis,
                               double *F, const Combine &cb, int slab, hipStream_t st)
{
    const int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY, ntz = (g.n[2] + TZ - 1) / TZ;
    const int sy = slab > 0 && slab < nty ? slab : nty;
    const dim3 grid((unsigned)(ntx * nty * ntz)), block(TX * TY * TZ);
    if (sbp == 21)
        hipLaunchKernelGGL((k_rhs_tile3d<21, TX, TY, TZ>), grid, block, 0, st, g, ph, q, vis, F, cb, ntx, nty, ntz,
                           sy);
    else
        hipLaunchKernelGGL((k_rhs_tile3d<42, TX, TY, TZ>), grid, block, 0, st, g, ph, q, vis, F, cb, ntx, nty, ntz,
                           sy);
    return hipGetLastError();
}

template <int TX, int TY>
static hipError_t zm3d_shape(const GridDev &g, int sbp, const Phys &ph, const double *q, const double *vis,
                             double *F, const Combine &cb, int zc, const int32_t *satpts, int nsat, hipStream_t st)
{
    const int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY;
    if (zc <= 0) {
        // about 768 workgroups (three per CU), chunks of at least 16 planes
        int nz = (768 + ntx * nty - 1) / (ntx * nty);
        nz = max(1, min(nz, g.n[2] / 16));
        zc = (g.n[2] + nz - 1) / nz;
    }
    const int nzc = (g.n[2] + zc - 1) / zc;
    const dim3 grid((unsigned)(ntx * nty * nzc)), block(TX * TY);
    if (sbp == 21)
        hipLaunchKernelGGL((k_rhs_zm3d<21, TX, TY>), grid, block, 0, st, g, ph, q, vis, F, cb, ntx, nty, nzc, zc);
    else
        hipLaunchKernelGGL((k_rhs_zm3d<42, TX, TY>), grid, block, 0, st, g, ph, q, vis, F, cb, ntx, nty, nzc, zc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsat == 0) return e;
    hipLaunchKernelGGL(k_sat3d, dim3(nblk(nsat, 256)), dim3(256), 0, st, g, ph, q, vis, F, cb, satpts, nsat);
    return hipGetLastError();
}

hipError_t launch_rhs_zm3d(const GridDev &g, int sbp, const Phys &ph, const double *q, double *vis, double *F,
                           const Combine &cb, int grad_shape, int slab, int shape, int zc, const int32_t *satpts,
                           int nsat, hipStream_t st)
{
    if (g.dim != 3 || !g.cartesian || (sbp != 21 && sbp != 42)) return hipErrorInvalidValue;
    hipError_t e = grad3d_launch(g, sbp, ph, q, vis, grad_shape, slab, st);
    if (e != hipSuccess) return e;
    switch (shape) {
    case 1: return zm3d_shape<16, 16>(g, sbp, ph, q, vis, F, cb, zc, satpts, nsat, st);
    case 2: return zm3d_shape<32, 8>(g, sbp, ph, q, vis, F, cb, zc, satpts, nsat, st);
    case 3: return zm3d_shape<16, 8>(g, sbp, ph, q, vis, F, cb, zc, satpts, nsat, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rhs_tile3d(const GridDev &g, int sbp, const Phys &ph, const double *q, double *grad,
                             double *F, const Combine &cb, int shape, int grad_shape, int slab, hipStream_t st)
{
    if (g.dim != 3 || !g.cartesian || (sbp != 21 && sbp != 42)) return hipErrorInvalidValue;
    hipError_t e = grad3d_launch(g, sbp, ph, q, grad, grad_shape < 0 ? shape : grad_shape, slab, st);
    if (e != hipSuccess) return e;
    switch (shape) {
    case 0: return flux3d_shape<8, 8, 8>(g, sbp, ph, q, grad, F, cb, slab, st);
    case 1: return flux3d_shape<16, 8, 4>(g, sbp, ph, q, grad, F, cb, slab, st);
    case 2: return flux3d_shape<32, 4, 4>(g, sbp, ph, q, grad, F, cb, slab, st);
    case 3: return flux3d_shape<16, 4, 4>(g, sbp, ph, q, grad, F, cb, slab, st);
    case 4: return flux3d_shape<16, 8, 8>(g, sbp, ph, q, grad, F, cb, slab, st);
    case 5: return flux3d_shape<32, 8, 4>(g, sbp, ph, q, grad, F, cb, slab, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_grad(const GridDev &g, int sbp, const Phys &ph, const double *q, double *grad, hipStream_t st)
{
    if (g.dim == 2 && sbp == 21 && g.cartesian) DISPATCH_GRAD(2, 21, 1);
    else if (g.dim == 2 && sbp == 21) DISPATCH_GRAD(2, 21, 0);
    else if (g.dim == 2 && sbp == 42 && g.cartesian) DISPATCH_GRAD(2, 42, 1);
    else if (g.dim == 2 && sbp == 42) DISPATCH_GRAD(2, 42, 0);
    else if (g.dim == 3 && sbp == 21 && g.cartesian) DISPATCH_GRAD(3, 21, 1);
    else if (g.dim == 3 && sbp == 42 && g.cartesian) DISPATCH_GRAD(3, 42, 1);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

#define DISPATCH_DONOR(DIM, SBP, CART) \
    hipLaunchKernelGGL((k_donor_vals<DIM, SBP, CART>), dim3(nblk(lanes, 256)), dim3(256), 0, st, a)

hipError_t launch_donor(const DonorLink &a, hipStream_t st)
{
    if (a.nrecv == 0 || a.nj == 0) return hipSuccess;
    int64_t lanes = a.nu * a.nj;
    const GridDev &g = a.g;
    if (g.dim == 2 && a.sbp == 21 && g.cartesian) DISPATCH_DONOR(2, 21, 1);
    else if (g.dim == 2 && a.sbp == 21) DISPATCH_DONOR(2, 21, 0);
    else if (g.dim == 2 && a.sbp == 42 && g.cartesian) DISPATCH_DONOR(2, 42, 1);
    else if (g.dim == 2 && a.sbp == 42) DISPATCH_DONOR(2, 42, 0);
    else if (g.dim == 3 && a.sbp == 21 && g.cartesian) DISPATCH_DONOR(3, 21, 1);
    else if (g.dim == 3 && a.sbp == 42 && g.cartesian) DISPATCH_DONOR(3, 42, 1);
    else return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t gl = a.nrecv * a.S * a.nj;
    if (g.dim == 2)
        hipLaunchKernelGGL((k_donor_gather<10>), dim3(nblk(gl, 256)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_donor_gather<17>), dim3(nblk(gl, 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

size_t donor_block_lds(int dim, int maxu, int maxc)
{
    int nv = dim + 2, rb = nv + dim * (nv - 1), kp = 1 + 4 * dim;
    return ((size_t)maxu * rb + (size_t)maxc * nv) * 8 + (maxc ? (size_t)maxu * kp * 2 : 0);
}

#define DISPATCH_BLOCK(DIM, SBP, CART)                                                                   \
    do {                                                                                                 \
        if (ext)                                                                                         \
            hipLaunchKernelGGL((k_donor_block<DIM, SBP, CART, 1>), grid, dim3(256), lds, st, a, b);      \
        else                                                                                             \
            hipLaunchKernelGGL((k_donor_block<DIM, SBP, CART, 0>), grid, dim3(256), lds, st, a, b);      \
    } while (0)

// every receiver's S entries share one wavefront; S * rpc <= 256
hipError_t launch_donor_block(const DonorLink &a, const DonorBlocks &b, hipStream_t st)
{
    if (a.nrecv == 0 || a.nj == 0) return hipSuccess;
    if (a.S < 1 || a.S > 64 || (a.S & (a.S - 1)) || b.rpc * a.S > 256 || a.nj > MAXJ || a.m < 0 ||
        a.m > MAXH || (int64_t)b.nchunk * b.rpc < a.nrecv)
        return hipErrorInvalidValue;
    const bool ext = a.m > 0;
    const GridDev &g = a.g;
    size_t lds = donor_block_lds(g.dim, b.maxu, ext ? b.maxc : 0);
    dim3 grid(b.nchunk, a.nj);
    // 2D: one body for both grid kinds (chosen per link at run time), so
    // every launch form runs the same code on a link
    if (g.dim == 2 && a.sbp == 21) DISPATCH_BLOCK(2, 21, 2);
    else if (g.dim == 2 && a.sbp == 42) DISPATCH_BLOCK(2, 42, 2);
    else if (g.dim == 3 && a.sbp == 21 && g.cartesian) DISPATCH_BLOCK(3, 21, 1);
    else if (g.dim == 3 && a.sbp == 42 && g.cartesian) DISPATCH_BLOCK(3, 42, 1);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int TX, int TY, int TM>
static hipError_t tiles_shape(const TileJob *jobs, int njobs, int nblk, int sbp, int cart, const Phys &ph,
                              hipStream_t st)
{
    dim3 grid(nblk), blk(TX * TY * TM);
    if (sbp == 21 && cart)
        hipLaunchKernelGGL((k_rhs_tiles<21, 1, TX, TY, TM>), grid, blk, 0, st, jobs, njobs, nblk, ph);
    else if (sbp == 21)
        hipLaunchKernelGGL((k_rhs_tiles<21, 0, TX, TY, TM>), grid, blk, 0, st, jobs, njobs, nblk, ph);
    else if (cart)
        hipLaunchKernelGGL((k_rhs_tiles<42, 1, TX, TY, TM>), grid, blk, 0, st, jobs, njobs, nblk, ph);
    else
        hipLaunchKernelGGL((k_rhs_tiles<42, 0, TX, TY, TM>), grid, blk, 0, st, jobs, njobs, nblk, ph);
    return hipGetLastError();
}

hipError_t launch_rhs_tiles(const TileJob *jobs, int njobs, int nblk, int sbp, int cart, int shape, const Phys &ph,
                            hipStream_t st)
{
    if (njobs <= 0 || nblk <= 0) return njobs == 0 ? hipSuccess : hipErrorInvalidValue;
    switch (shape) {
    case 0: return tiles_shape<32, 16, 1>(jobs, njobs, nblk, sbp, cart, ph, st);
    case 1: return tiles_shape<16, 8, 1>(jobs, njobs, nblk, sbp, cart, ph, st);
    case 2: return tiles_shape<16, 8, 2>(jobs, njobs, nblk, sbp, cart, ph, st);
    case 3: return tiles_shape<16, 8, 4>(jobs, njobs, nblk, sbp, cart, ph, st);
    case 4: return tiles_shape<32, 8, 1>(jobs, njobs, nblk, sbp, cart, ph, st);
    case 5: return tiles_shape<32, 8, 2>(jobs, njobs, nblk, sbp, cart, ph, st);
    case 6: return tiles_shape<16, 16, 1>(jobs, njobs, nblk, sbp, cart, ph, st);
    case 7: return tiles_shape<16, 16, 2>(jobs, njobs, nblk, sbp, cart, ph, st);
    default: return hipErrorInvalidValue;
    }
}

#define DISPATCH_BLOCKS(DIM, SBP, CART)                                                                  \
    do {                                                                                                 \
        if (ext)                                                                                         \
            hipLaunchKernelGGL((k_donor_blocks<DIM, SBP, CART, 1>), grid, dim3(256), lds, st, jobs, njobs); \
        else                                                                                             \
            hipLaunchKernelGGL((k_donor_blocks<DIM, SBP, CART, 0>), grid, dim3(256), lds, st, jobs, njobs); \
    } while (0)

hipError_t launch_donor_blocks(const LinkJob *jobs, int njobs, int nchunk, int maxnj, int dim, int sbp, int cart,
                               bool ext, size_t lds, hipStream_t st)
{
    if (njobs == 0 || nchunk == 0) return hipSuccess;
    if (njobs < 0 || nchunk < 0 || maxnj < 1 || maxnj > MAXJ || lds > 64 * 1024) return hipErrorInvalidValue;
    dim3 grid(nchunk, maxnj);
    (void)cart;
    if (dim == 2 && sbp == 21) DISPATCH_BLOCKS(2, 21, 2);
    else if (dim == 2 && sbp == 42) DISPATCH_BLOCKS(2, 42, 2);
    else if (dim == 3 && sbp == 21 && cart) DISPATCH_BLOCKS(3, 21, 1);
    else if (dim == 3 && sbp == 42 && cart) DISPATCH_BLOCKS(3, 42, 1);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_donor_block2(const DonorLinks2 &L, hipStream_t st)
{
    if (L.n < 1 || L.n > 2) return hipErrorInvalidValue;
    int nj = 0, dim = L.a[0].g.dim, sbp = L.a[0].sbp, chunks = L.chunk0[L.n];
    bool ext = L.a[0].m > 0;
    size_t lds = 0;
    for (int i = 0; i < L.n; ++i) {
        const DonorLink &a = L.a[i];
        const DonorBlocks &b = L.b[i];
        if (a.g.dim != dim || a.sbp != sbp || (a.m > 0) != ext || a.S < 1 || a.S > 64 || (a.S & (a.S - 1)) ||
            b.rpc * a.S > 256 || a.nj < 1 || a.nj > MAXJ || (int64_t)b.nchunk * b.rpc < a.nrecv ||
            L.chunk0[i + 1] - L.chunk0[i] != b.nchunk)
            return hipErrorInvalidValue;
        nj = a.nj > nj ? a.nj : nj;
        size_t s = donor_block_lds(dim, b.maxu, ext ? b.maxc : 0);
        lds = s > lds ? s : lds;
    }
    if (dim != 2 || lds > 64 * 1024) return hipErrorInvalidValue;
    dim3 grid(chunks, nj);
    if (sbp == 21 && ext) hipLaunchKernelGGL((k_donor_block2<2, 21, 1>), grid, dim3(256), lds, st, L);
    else if (sbp == 21) hipLaunchKernelGGL((k_donor_block2<2, 21, 0>), grid, dim3(256), lds, st, L);
    else if (ext) hipLaunchKernelGGL((k_donor_block2<2, 42, 1>), grid, dim3(256), lds, st, L);
    else hipLaunchKernelGGL((k_donor_block2<2, 42, 0>), grid, dim3(256), lds, st, L);
    return hipGetLastError();
}

hipError_t launch_combine(int64_t n, const double *y, const Combine &cb, hipStream_t st)
{
    hipLaunchKernelGGL(k_combine, dim3(nblk(n, 256)), dim3(256), 0, st, n, y, cb);
    return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, const double *y, double a, const double *x, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy, dim3(nblk(n, 256)), dim3(256), 0, st, n, y, a, x, out);
    return hipGetLastError();
}

hipError_t launch_rk3_final(int64_t n, const double *y, double a, const double *k1, const double *k3,
                            double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_rk3_final, dim3(nblk(n, 256)), dim3(256), 0, st, n, y, a, k1, k3, out);
    return hipGetLastError();
}

hipError_t launch_rk4_final(int64_t n, const double *y, double a, const double *k1, const double *k2,
                            const double *k3, const double *k4, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_rk4_final, dim3(nblk(n, 256)), dim3(256), 0, st, n, y, a, k1, k2, k3, k4, out);
    return hipGetLastError();
}

hipError_t launch_metrics2d(const GridDev &g, int sbp, const double *x, const double *y, const double per[2][2],
                            double *metric, hipStream_t st)
{
    if (sbp == 21)
        hipLaunchKernelGGL((k_metrics2d<21>), dim3(nblk(g.npts, 256)), dim3(256), 0, st, g, x, y, per[0][0],
                           per[1][0], per[0][1], per[1][1], metric);
    else
        hipLaunchKernelGGL((k_metrics2d<42>), dim3(nblk(g.npts, 256)), dim3(256), 0, st, g, x, y, per[0][0],
                           per[1][0], per[0][1], per[1][1], metric);
    return hipGetLastError();
}

hipError_t launch_dt(const GridDev &g, const Phys &ph, const double *q, double *dt, hipStream_t st)
{
    if (g.dim == 2)
        hipLaunchKernelGGL((k_dt<2>), dim3(nblk(g.npts, 256)), dim3(256), 0, st, g, ph, q, dt);
    else
        hipLaunchKernelGGL((k_dt<3>), dim3(nblk(g.npts, 256)), dim3(256), 0, st, g, ph, q, dt);
    return hipGetLastError();
}

// one wave waits until the device's constant-rate clock has advanced by
// `ticks` (bounded: it ends once the clock passes the mark)
__global__ void k_wait_ticks(uint64_t ticks)
{
    const uint64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(16);
}

hipError_t launch_wait_us(double us, hipStream_t st)
{
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    if (khz <= 0 || !(us >= 0.0) || us > 1e6) return hipErrorInvalidValue;
    const uint64_t ticks = (uint64_t)(us * 1e-3 * khz);
    hipLaunchKernelGGL(k_wait_ticks, dim3(1), dim3(64), 0, st, ticks);
    return hipGetLastError();
}

hipError_t launch_reduce(int64_t n, const double *x, int mode, double *partial, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3(nblocks), dim3(256), 0, st, n, x, mode, partial);
    return hipGetLastError();
}

}  // namespace mrk

// Library-owned workspace for callers that cannot allocate device memory
// (mr_bind_static_workspace).  Every device the library runs on holds its own
// copy from the load of the code object until the process ends.  Host code
// never uses this name as an address: the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[MR_STATIC_WORKSPACE_BYTES];

namespace mrk {

hipError_t static_workspace(int device, void **ptr)
{
    static std::mutex mu;
    static std::map<int, void *> addr;   // device -> address of its copy of the array
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
        hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p || (uintptr_t)p % 256) return hipErrorInvalidValue;
    addr[device] = p;
    *ptr = p;
    return hipSuccess;
}

}  // namespace mrk
