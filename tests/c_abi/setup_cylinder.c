/* A C-only caller of libmrab: sets up a cylinder-like overset system through
 * the ABI alone (host side, no device needed) -- a Cartesian background with
 * a disk hole and a body-fitted O-mesh, the library's own donor search
 * (mr_assemble_overset with no locate callback), then checks the assembled
 * stencils: every receiver's weights sum to one, and interpolating the donor
 * grid's coordinates with them gives the receiver's position (Lagrange
 * weights reproduce the coordinate interpolant the search inverts, exactly so
 * for the cubic stencils used here).  Prints "ok <receivers per grid>
 * <workspace bytes>" and exits 0, or prints the failure and exits 1. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "mrab.h"

#define NB 96      /* background points per direction on [-6, 6) */
#define NT 96      /* O-mesh points around */
#define NR 32      /* O-mesh points outward, r = 0.5 .. 2.5 */
#define PI 3.14159265358979323846

static double bg_x(int i) { return -6.0 + 12.0 * i / NB; }

static int fail_at(const char *what, mr_ctx *c)
{
    printf("FAILED %s: %s\n", what, c ? mr_last_error(c) : "");
    return 1;
}

int main(void)
{
    mr_params p = {0};
    p.dim = 2;
    p.sbp = MR_SBP_42;
    p.order = 4;
    p.hist_len = 4;
    p.interp_width = 4;
    p.gamma = 1.4;
    p.Re = 200.0;
    p.Pr = 0.72;
    p.mu = 1.0;
    p.lambda_over_mu = -2.0 / 3.0;
    p.sigma_I_iface = 0.5;
    p.sigma_I_bc = 0.5;
    p.T_wall = 1.0 / 1.4;
    p.wall_visc = 1.0;
    p.q_inf[0] = 1.0;
    p.q_inf[1] = 0.2;
    p.q_inf[3] = 1.0 / (1.4 * 0.4) + 0.02;
    p.cfl = 0.5;
    mr_ctx *c = NULL;
    if (mr_create(&p, NULL, &c) != MR_OK) return fail_at("mr_create", c);

    /* background: far-field faces, hole r < 1.6 */
    static int8_t ib0[NB * NB];
    for (int j = 0; j < NB; ++j)
        for (int i = 0; i < NB; ++i) {
            double x = bg_x(i), y = bg_x(j);
            ib0[i + NB * j] = (x * x + y * y < 1.6 * 1.6) ? 0 : 1;
        }
    mr_grid_desc g0 = {{NB, NB, 1}, {0, 0, 0}, MR_CARTESIAN, {-6.0, -6.0, 0.0}, {12.0 / NB, 12.0 / NB, 1.0}, NULL,
                       {{0}}, ib0, {MR_BC_FARFIELD, MR_BC_FARFIELD, MR_BC_FARFIELD, MR_BC_FARFIELD, 0, 0}, 1};
    int id0, id1;
    if (mr_add_grid(c, &g0, &id0) != MR_OK) return fail_at("mr_add_grid background", c);

    /* O-mesh: periodic around, wall inside, interface outside */
    static double xy[2 * NT * NR];
    for (int j = 0; j < NR; ++j)
        for (int i = 0; i < NT; ++i) {
            double r = 0.5 + 2.0 * j / (NR - 1), th = 2.0 * PI * i / NT;
            xy[i + NT * j] = r * cos(th);
            xy[NT * NR + i + NT * j] = r * sin(th);
        }
    mr_grid_desc g1 = {{NT, NR, 1}, {1, 0, 0}, MR_CURVILINEAR, {0, 0, 0}, {1, 1, 1}, xy, {{0}}, NULL,
                       {MR_BC_PERIODIC, MR_BC_PERIODIC, MR_BC_WALL, MR_BC_INTERFACE, 0, 0}, 4};
    if (mr_add_grid(c, &g1, &id1) != MR_OK) return fail_at("mr_add_grid O-mesh", c);

    const int prio[2] = {0, 1};
    if (mr_assemble_overset(c, 4, prio, NULL, NULL) != MR_OK) return fail_at("mr_assemble_overset", c);

    int64_t nrec[2];
    for (int g = 0; g < 2; ++g) {
        int64_t n = 0;
        if (mr_get_overset(c, g, &n, NULL, NULL, NULL, NULL) != MR_OK || n <= 0) return fail_at("mr_get_overset", c);
        int64_t *rp = malloc(sizeof(int64_t) * n), *dp = malloc(sizeof(int64_t) * n * 16);
        int *dg = malloc(sizeof(int) * n);
        double *w = malloc(sizeof(double) * n * 16);
        if (mr_get_overset(c, g, &n, rp, dg, dp, w) != MR_OK) return fail_at("mr_get_overset", c);
        for (int64_t r = 0; r < n; ++r) {
            double px, py, sx = 0.0, sy = 0.0, sw = 0.0;
            if (g == 0) { px = bg_x((int)(rp[r] % NB)); py = bg_x((int)(rp[r] / NB)); }
            else { px = xy[rp[r]]; py = xy[NT * NR + rp[r]]; }
            for (int e = 0; e < 16; ++e) {
                int64_t q = dp[r * 16 + e];
                double qx, qy;
                if (dg[r] == 0) { qx = bg_x((int)(q % NB)); qy = bg_x((int)(q / NB)); }
                else { qx = xy[q]; qy = xy[NT * NR + q]; }
                sx += w[r * 16 + e] * qx;
                sy += w[r * 16 + e] * qy;
                sw += w[r * 16 + e];
            }
            if (dg[r] == g || fabs(sw - 1.0) > 1e-12 || fabs(sx - px) > 1e-11 || fabs(sy - py) > 1e-11) {
                printf("FAILED receiver %lld of grid %d: donor grid %d, weight sum %.17g, position error %.3g %.3g\n",
                       (long long)rp[r], g, dg[r], sw, sx - px, sy - py);
                return 1;
            }
        }
        nrec[g] = n;
        free(rp);
        free(dp);
        free(dg);
        free(w);
    }
    size_t ws = 0;
    if (mr_finalize(c, &ws) != MR_OK) return fail_at("mr_finalize", c);
    printf("ok %lld %lld %zu\n", (long long)nrec[0], (long long)nrec[1], ws);
    mr_destroy(c);
    return 0;
}
