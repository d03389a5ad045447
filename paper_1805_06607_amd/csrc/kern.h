// Device-side descriptors and launch entry points shared by the host runtime
// (runtime.cpp) and the gfx950 kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrk {

constexpr int MAXG = 8;     // grids per context
constexpr int MAXH = 8;     // history length
// 3D grids store, per point, the viscous quantities a flux needs in place of
// the 12 gradients: the stress tau_ij (symmetric: 6 values) and the heat
// terms h_j = kc dT/dx_j (3)
constexpr int NVISC3 = 9;

// Class byte of a point along one direction:
//   bits 0-3  row: 0 interior, 1..4 left closure row 0..3, 5..8 right closure row 0..3, 15 hole
//   bits 4-5  SAT face flag at run ends (left row 0 / right row 0): 1 interface, 2 far-field, 3 wall
constexpr int CLS_HOLE = 15;

struct GridDev {
    int dim, nv;
    int n[3];
    int periodic[3];
    int64_t stride[3];
    int64_t npts;
    int cartesian;
    double inv_h[3];          // Cartesian grids: 1 / spacing
    const double *metric;     // curvilinear: (dim*dim + 1) x npts, M[m*dim+j] = J^-1 dxi_m/dx_j, then J
    const int8_t *cls;        // dim x npts class bytes
    const int32_t *recv_idx;  // per point: receiver row or -1 (null: no receivers)
    const double *recv;       // receiver rows: q_hat (nv), F_hat^V_j (nv-1 each)
};

struct Phys {
    double gamma, Re, Pr, mu, lam;
    double sig_iface, sig_bc, T_wall, wall_visc;
    double q_inf[5];
    double p0inv;
};

// y_next = y + sum_j c[j] * F_j (j = 0 oldest .. m-1 newest); F_{m-1} is the
// right-hand side computed by the same kernel when fused.
struct Combine {
    int m;
    double c[MAXH];
    const double *hist[MAXH];
    double *y_next;
};

// donor data of one link (receivers of one grid taking data from one donor
// grid) for nj target times at once, in two launches:
//   values: one lane per (slot j, unique donor point u): q and the Cartesian
//           viscous fluxes at the point from state ys[j] -> vals[j][u][RB]
//   gather: one lane per (slot j, receiver k, entry e): w[k][e] vals[j][uid]
//           summed by a fixed butterfly over e -> out[j] row (row0 + k)
constexpr int MAXJ = 8;
struct DonorLink {
    GridDev g;                 // donor grid
    int nj;
    const double *ys[MAXJ];
    double *out[MAXJ];
    int m;                     // block launch: extrapolant ys[j] + sum_h beta[j][h] hist[h] when m > 0
    double beta[MAXJ][MAXH];
    const double *hist[MAXH];
    double *vals;              // nj x nu x RB scratch
    Phys ph;
    int32_t row0;              // row of the link's first receiver
    const int32_t *upts;       // nu unique donor points
    int64_t nu;
    const int32_t *uid;        // nrecv x S indices into upts
    const double *w;           // nrecv x S weights
    int64_t nrecv;
    int S;
    int sbp;
};

// Receivers of a link cut into chunks of rpc consecutive receivers (rpc * S
// = 256 entries), one workgroup per (chunk, slot): the chunk's distinct donor
// points upts[c * maxu + u] (sorted, -1 past the chunk's count), each entry's
// index among them (eloc, receiver-major), the points their gradient stencils
// read, cpts[c * maxc + i] (sorted, -1 past the count; used when the state is
// an extrapolant), and per distinct donor point 1 + 4 dim positions in that
// list (bpos[(c * maxu + u) * (1 + 4 dim) + t]): the point, then its stencil
// in the order the gradient reads it (-1 past a short row).
// Dynamic LDS: maxu * RB + maxc * nv doubles, and maxu * (1 + 4 dim) int16
// when extrapolating.
struct DonorBlocks {
    const int32_t *upts, *cpts;
    const int16_t *eloc, *bpos;
    int nchunk, rpc, maxu, maxc;
};

// two 2D links' donor data in one launch by value: link i owns chunks
// chunk0[i] .. chunk0[i+1] - 1
struct DonorLinks2 {
    DonorLink a[2];
    DonorBlocks b[2];
    int chunk0[3];
    int n;
};

// one link's donor data in a work-list launch (chunks chunk0 .. chunk0 +
// b.nchunk - 1 of the concatenated list)
struct LinkJob {
    DonorLink a;
    DonorBlocks b;
    int chunk0;
};

// extrapolated donor states at listed points for nj target times:
// out[j][v*N + p] = y[v*N + p] + sum_h beta[j][h] hist[h][v*N + p]
struct Extrap {
    const double *y;
    int m, nv;
    int64_t N;
    const double *hist[MAXH];
    int nj;
    double beta[MAXJ][MAXH];
    double *out[MAXJ];
    const int32_t *pts;
    int64_t np;
};

// ---------------------------------------------------------------- launches
hipError_t launch_grad(const GridDev &g, int sbp, const Phys &ph, const double *q, double *grad, hipStream_t st);
hipError_t launch_rhs(const GridDev &g, const GridDev *g_dev, int sbp, const Phys &ph, const double *q,
                      const double *grad, double *F, const Combine &cb, hipStream_t st);
hipError_t launch_donor(const DonorLink &a, hipStream_t st);
// one launch: (extrapolation when a.m > 0,) values and gather per chunk
hipError_t launch_donor_block(const DonorLink &a, const DonorBlocks &b, hipStream_t st);
hipError_t launch_donor_block2(const DonorLinks2 &links, hipStream_t st);
size_t donor_block_lds(int dim, int maxu, int maxc);
hipError_t launch_extrap(const Extrap &a, hipStream_t st);
// fused LDS-tiled 2D right-hand side (gradients, fluxes, divergence, SAT, AB update)
struct TileShape { int tx, ty, tm; };
// one grid evaluation in a work-list launch: tiles tile0 .. tile0 + ntx*nty - 1
// of the concatenated list (g.recv: the receiver rows of this evaluation)
struct TileJob {
    GridDev g;
    const double *q;
    double *F;
    Combine cb;
    int ntx, nty, tile0;
};
// jobs (device, ordered by tile0, all of one kind: sbp, cart, shape), nblk
// tiles in all
hipError_t launch_rhs_tiles(const TileJob *jobs, int njobs, int nblk, int sbp, int cart, int shape, const Phys &ph,
                            hipStream_t st);
// jobs (device, ordered by chunk0, one kind: dim, sbp, cart, ext), nchunk
// chunks in all, up to maxnj slots, lds bytes per workgroup
hipError_t launch_donor_blocks(const LinkJob *jobs, int njobs, int nchunk, int maxnj, int dim, int sbp, int cart,
                               bool ext, size_t lds, hipStream_t st);
constexpr int NUM_TILE_SHAPES = 8;
extern const TileShape kTileShapes[NUM_TILE_SHAPES];
int default_tile_shape(const GridDev &g);
hipError_t launch_rhs_tile2d(const GridDev &g, int sbp, const Phys &ph, const double *q, double *F,
                             const Combine &cb, int shape, hipStream_t st);
// the same evaluation with one chunked 2D link's extrapolated donor data
// (a.m > 0) in extra workgroups of the launch; the link must not read or write
// anything the evaluation writes; shapes of at least 256 threads only
bool tile2d_donor_ok(int shape);
hipError_t launch_rhs_tile2d_donor(const GridDev &g, int sbp, const Phys &ph, const double *q, double *F,
                                   const Combine &cb, int shape, const DonorLink &a, const DonorBlocks &b,
                                   hipStream_t st);
// 3D Cartesian right-hand side on LDS tiles of shape 0..NUM_TILE3D_SHAPES-1:
// a gradient pass into grad (the NVISC3 x npts viscous quantities), then
// flux divergence + SAT + AB update
struct TileShape3 { int tx, ty, tz; };
constexpr int NUM_TILE3D_SHAPES = 6;
extern const TileShape3 kTile3dShapes[NUM_TILE3D_SHAPES];
// slab: tiles are taken in slabs of that many tile rows along y, z planes
// within a slab (<= 0 or >= the tile rows: the plain x, y, z order); the
// gradient pass takes tiles of grad_shape (-1: shape)
hipError_t launch_rhs_tile3d(const GridDev &g, int sbp, const Phys &ph, const double *q, double *grad,
                             double *F, const Combine &cb, int shape, int grad_shape, int slab, hipStream_t st);
// the same right-hand side with the flux pass marching along z (k_rhs_zm3d):
// gradient pass on tiles of grad_shape (kTile3dShapes), flux pass on columns of
// shape 1: 16 x 16, 2: 32 x 8, 3: 16 x 8, zc planes per chunk (0: chosen
// from the grid size), then the SAT penalties of the nsat points satpts
// (every active point that ends a run in some direction)
hipError_t launch_rhs_zm3d(const GridDev &g, int sbp, const Phys &ph, const double *q, double *vis, double *F,
                           const Combine &cb, int grad_shape, int slab, int shape, int zc, const int32_t *satpts,
                           int nsat, hipStream_t st);
hipError_t launch_combine(int64_t n, const double *y, const Combine &cb, hipStream_t st);
hipError_t launch_axpy(int64_t n, const double *y, double a, const double *x, double *out, hipStream_t st);
hipError_t launch_rk3_final(int64_t n, const double *y, double a, const double *k1, const double *k3,
                            double *out, hipStream_t st);
hipError_t launch_rk4_final(int64_t n, const double *y, double a, const double *k1, const double *k2,
                            const double *k3, const double *k4, double *out, hipStream_t st);
hipError_t launch_metrics2d(const GridDev &g, int sbp, const double *x, const double *y,
                            const double per[2][2], double *metric, hipStream_t st);
hipError_t launch_dt(const GridDev &g, const Phys &ph, const double *q, double *dt, hipStream_t st);
// occupy the stream for about `us` microseconds (at most 1 s) on one wave
// of the device: launches queued behind it then run back to back, so a timing
// of them measures the device, not the host's launch rate
hipError_t launch_wait_us(double us, hipStream_t st);
// block-partial reductions: mode 0 = min, 1 = max |x| (NaN/Inf -> +inf)
hipError_t launch_reduce(int64_t n, const double *x, int mode, double *partial, int nblocks, hipStream_t st);

// device address of the library's static workspace on `device`
// (MR_STATIC_WORKSPACE_BYTES bytes, 256-byte aligned), looked up once per device
hipError_t static_workspace(int device, void **ptr);

}  // namespace mrk
