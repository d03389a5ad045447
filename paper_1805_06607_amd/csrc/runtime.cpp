// Host runtime behind the C ABI of libmrab.so (include/mrab.h): run
// classification of every grid line, donor tables, workspace layout, the
// static multi-rate schedule and the RK bootstrap.  All device work is
// enqueued on the context's stream.
#include "../../include/mrab.h"
#include "kern.h"
#include "adj.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

using mrk::GridDev;

namespace {

constexpr size_t ALIGN = 256;

struct GridHost {
    int dim = 2, kind = 0, rate = 1;
    int n[3] = {1, 1, 1};
    int periodic[3] = {0, 0, 0};
    int64_t stride[3] = {1, 1, 1};
    int64_t npts = 0;
    double origin[3] = {0, 0, 0}, spacing[3] = {1, 1, 1};
    double coord_period[3][3] = {{0}};
    int face_bc[6] = {0};
    std::vector<double> coords;
    std::vector<int8_t> iblank;
    std::vector<int8_t> cls;          // dim x npts
    std::vector<int32_t> recv_idx;    // npts
    std::vector<int64_t> recv_pts;    // registered receivers, row order
    int64_t n_iface = 0;              // points ending a run on an interface face
    // device
    double *y[2] = {nullptr, nullptr};
    int cur = 0;
    double *hist = nullptr;
    double *metric = nullptr, *coords_d = nullptr, *grad = nullptr, *recv_buf = nullptr, *dt = nullptr;
    double *rk[5] = {nullptr};
    int8_t *cls_d = nullptr;
    int32_t *recv_idx_d = nullptr;
    GridDev dev{};
    int head = 0;
    int tile = -1;                    // 2D tile shape (-1: size-based default)
    // donor grid stepping slower than the fastest grid: its extrapolated
    // states at the points its donor stencils read, one buffer per mid-step
    std::vector<int32_t> closure;     // sorted donor-stencil points
    int32_t *closure_d = nullptr;
    std::vector<int32_t> satpts;      // 3D: active points ending a run in some direction (SAT points)
    int32_t *satpts_d = nullptr;
    std::vector<double *> ext;        // per mid-step offset jp = 1..per-1
};

}  // namespace

struct Link {
    int rg, dg;
    int64_t first, n;     // global receiver range
    int32_t row0;         // row of the first receiver in the receiving grid's buffer
    std::vector<int32_t> upts;   // unique donor points of the link
    int32_t *upts_d = nullptr;
    double *vals_d = nullptr;    // r_max x nu x RB donor values
    // chunked form for the one-launch donor kernel (mrk::DonorBlocks)
    bool blk = false;
    int nchunk = 0, rpc = 0, maxu = 0, maxc = 0;
    std::vector<int32_t> bup, bcp;
    std::vector<int16_t> bel, bpos;
    int32_t *bup_d = nullptr, *bcp_d = nullptr;
    int16_t *bel_d = nullptr, *bpos_d = nullptr;
};

// Cross-stream order inside one macrostep call.  Stream s (one per grid)
// counts the launches issued on it in this call (pos[s]; 0 is the call's
// start, which every stream has joined).  A launch is recorded right after
// it is issued when another stream may depend on it; a stream that needs
// position p of stream s waits on the first record at or after p unless its
// vector clock already covers p.  Receiver rows (link, k) remember their
// last writer and the receiving grid's slice k its last reader.
struct Order {
    struct Rec {
        int pos;
        hipEvent_t e;
        std::vector<int> clock;
    };
    static constexpr int POOL = 32;
    int G = 0, K = 0;
    std::vector<int> pos;
    std::vector<std::vector<int>> clock;          // [t][s]: position of s known complete before t's next launch
    std::vector<std::vector<Rec>> recs;           // per stream, this call
    const std::vector<std::vector<hipEvent_t>> *pool = nullptr;   // per stream (the call's event set)
    std::vector<int> used;
    std::vector<std::pair<int, int>> wr;          // [link * (K+1) + k]: (stream, pos) of the last write
    std::vector<std::pair<int, int>> rd;          // [grid * (K+1) + k]: (stream, pos) of the last read
};

// Below this many grid points the per-grid streams do not pay: the host's
// event calls and the cross-queue waits cost more than the overlap of the
// short launches saves.
constexpr int64_t kMultiStreamPoints = 4 << 20;

// Events of the macrostep calls.
struct EvSet {
    hipEvent_t join = nullptr;
    std::vector<hipEvent_t> done;                  // per grid
    std::vector<std::vector<hipEvent_t>> pool;     // per grid, Order::POOL each
};

struct AdjCtx;

struct mr_ctx {
    mr_params P{};
    hipStream_t st = nullptr;
    std::string err;
    std::vector<GridHost> G;
    int S = 0;
    std::vector<int32_t> rgrid, rrow;
    std::vector<int8_t> egrid;
    std::vector<int32_t> ept;
    std::vector<double> ew;
    bool finalized = false, bound = false, have_dt = false, started = false;
    bool stale = false;       // a state or history was set since the last start/resume
    size_t ws_bytes = 0;
    char *ws = nullptr;
    int rmax = 1;
    double H = 0, h = 0, t = 0;
    int64_t nmacro = 0;
    std::vector<std::vector<long double>> alpha_own;                 // per grid
    std::vector<std::vector<std::vector<long double>>> alpha_mid;   // per grid, per jp
    std::vector<std::vector<double>> c_own;
    std::vector<std::vector<std::vector<double>>> beta;
    std::vector<Link> links;
    std::vector<int32_t> euid;   // per entry: index into its link's unique points
    int32_t *euid_d = nullptr;
    double *ew_d = nullptr;
    GridDev *grids_d = nullptr;
    double *partial = nullptr;
    mrk::Phys ph{};
    // per-launch timing
    int tgrid = -1, tmax = 0, tcount = 0;    // tgrid -2: every grid
    std::vector<int> tgrid_of;                // grid of each timed launch
    bool two_pass = false;    // 2D: use the two-kernel (gradient pass) right-hand side
    bool donor_blocks = true; // one-launch donor data for links whose chunks fit one workgroup
    bool ride_donors = true;  // one stream: mid-step donor data in the next same-time 2D evaluation's launch
    int tile3d = 1;           // 3D passes: LDS tile shape (mrk::kTile3dShapes), -1 the per-point kernels
    int gtile3d = 4;          // 3D gradient pass: its own tile shape (-1: tile3d)
    int slab3d = 3;           // 3D passes: tile rows per slab of the tile order (0: plain x, y, z order)
    int flux3d = 0;           // 3D flux pass: 0 on tiles, 1..3 marching along z (columns 16x16, 32x8, 16x8)
    int zchunk3d = 0;         // 3D z-marching flux pass: planes per chunk (0: from the grid size)
    int period = 1;                            // macrosteps after which every pointer repeats
    int64_t version = 0;                       // bumped when a batch's launch plan must be rebuilt
    // macrosteps: one stream per grid, ordered by events (Order); -1: when
    // the grids hold at least kMultiStreamPoints points in all
    int multi_stream = -1;
    std::vector<hipStream_t> gs;                       // per grid
    Order ord;
    EvSet eager;
    std::vector<hipEvent_t> ev;
    AdjCtx *adj = nullptr;                     // discrete adjoint (mr_adj_*)
    int static_dev = -1;                       // device whose static workspace is bound, -1: caller memory
};

// Many independent systems advanced together: per micro-time of the batch,
// one work-list launch per kind of job (current donor data, fused 2D
// right-hand sides, mid-step donor data) over every system that steps then.
struct mr_batch {
    std::vector<mr_ctx *> ctx;
    hipStream_t st = nullptr;
    int R = 1, P = 1;                  // micro-times per macrostep, macrosteps per plan period
    size_t tj_cap = 0, lj_cap = 0, ws_bytes = 0;
    mrk::TileJob *tj_d = nullptr;
    mrk::LinkJob *lj_d = nullptr;
    struct Launch {
        int what;                      // 0 donor data at the current time, 1 right-hand sides, 2 mid-step donor data
        int first, njobs, nblk, maxnj; // job range, workgroups (tiles or chunks), slots
        int dim, sbp, cart, shape;
        size_t lds;
    };
    std::vector<std::vector<Launch>> plan;   // [p * (R + 1) + k]
    std::vector<int64_t> base, version;      // per system at the last plan build
    int64_t steps = 0;                       // batch macrosteps since that build
    bool built = false, bound = false;
    int shape = -1;                          // tile shape of every right-hand side (-1: each grid's own)
    std::string err;
};

namespace {

int fail(mr_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

// holder of each device's static workspace (mr_bind_static_workspace)
std::mutex g_static_mu;
std::map<int, const mr_ctx *> g_static_holder;

bool static_lost(const mr_ctx *c)
{
    if (c->static_dev < 0) return false;
    std::lock_guard<std::mutex> lock(g_static_mu);
    auto it = g_static_holder.find(c->static_dev);
    return it == g_static_holder.end() || it->second != c;
}

// MR_OK when the context's workspace is bound and still its own
int need_bound(mr_ctx *c, const char *what)
{
    if (!c->bound) return fail(c, MR_ERR_STATE, "%s before mr_bind_workspace", what);
    if (static_lost(c))
        return fail(c, MR_ERR_STATE, "%s: the static workspace of device %d is bound to another context", what,
                    c->static_dev);
    return MR_OK;
}

#define HIPCHK(c, expr)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(c, MR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int nclosure(int sbp) { return sbp == 21 ? 1 : 4; }

// ------------------------------------------------------- AB coefficients
// alpha (oldest first) for nodes -(m-1)..0 and target offset tau: Vandermonde
// transpose system for m == n, minimum-norm solution for m > n.
bool solve_ld(std::vector<std::vector<long double>> A, std::vector<long double> b, std::vector<long double> &x)
{
    int n = (int)A.size();
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0L) return false;
        std::swap(A[c], A[piv]);
        std::swap(b[c], b[piv]);
        for (int r = c + 1; r < n; ++r) {
            long double f = A[r][c] / A[c][c];
            for (int k = c; k < n; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    x.assign(n, 0.0L);
    for (int r = n - 1; r >= 0; --r) {
        long double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
    }
    return true;
}

bool ab_alpha(int n, int m, long double tau, std::vector<long double> &alpha)
{
    if (n < 1 || m < n || m > mrk::MAXH) return false;
    std::vector<long double> t(m);
    for (int j = 0; j < m; ++j) t[j] = -(long double)(m - 1 - j);
    std::vector<std::vector<long double>> V(m, std::vector<long double>(n));
    for (int j = 0; j < m; ++j) {
        long double v = 1.0L;
        for (int i = 0; i < n; ++i) { V[j][i] = v; v *= t[j]; }
    }
    std::vector<long double> b(n);
    long double tp = tau;
    for (int i = 0; i < n; ++i) { b[i] = tp / (long double)(i + 1); tp *= tau; }
    if (m == n) {
        std::vector<std::vector<long double>> VT(n, std::vector<long double>(n));
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) VT[i][j] = V[j][i];
        return solve_ld(VT, b, alpha);
    }
    std::vector<std::vector<long double>> N(n, std::vector<long double>(n, 0.0L));
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < m; ++j) N[i][k] += V[j][i] * V[j][k];
    std::vector<long double> z;
    if (!solve_ld(N, b, z)) return false;
    alpha.assign(m, 0.0L);
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) alpha[j] += V[j][i] * z[i];
    return true;
}

// -------------------------------------------------------- run classification
int classify(mr_ctx *c, GridHost &g)
{
    int nb = nclosure(c->P.sbp);
    int64_t N = g.npts;
    g.cls.assign((size_t)g.dim * N, 0);
    for (int d = 0; d < g.dim; ++d) {
        int nd = g.n[d];
        int o1 = (d + 1) % g.dim, o2 = (d + 2) % g.dim;
        int n1 = g.dim > 1 ? g.n[o1] : 1;
        int n2 = g.dim > 2 ? g.n[o2] : 1;
        std::vector<int64_t> idx(nd);
        std::vector<char> a(nd);
        for (int i2 = 0; i2 < n2; ++i2)
            for (int i1 = 0; i1 < n1; ++i1) {
                int64_t base = (int64_t)i1 * g.stride[o1] + (g.dim > 2 ? (int64_t)i2 * g.stride[o2] : 0);
                bool all = true, none = true;
                for (int i = 0; i < nd; ++i) {
                    idx[i] = base + (int64_t)i * g.stride[d];
                    a[i] = g.iblank[idx[i]] != 0;
                    all = all && a[i];
                    none = none && !a[i];
                }
                int8_t *cl = g.cls.data() + (size_t)d * N;
                for (int i = 0; i < nd; ++i)
                    if (!a[i]) cl[idx[i]] = mrk::CLS_HOLE;
                if (none) continue;
                if (all && g.periodic[d]) continue;   // endless periodic line: interior everywhere
                // runs (start, length); periodic lines start scanning after a hole
                int first = 0;
                if (g.periodic[d]) {
                    int h = 0;
                    while (a[h]) ++h;
                    first = h + 1;
                }
                int i = 0;
                while (i < nd) {
                    int k = (first + i) % nd;
                    if (!a[k]) { ++i; continue; }
                    int s = k, L = 0;
                    while (i < nd && a[(first + i) % nd]) { ++L; ++i; }
                    if (L < 2 * nb)
                        return fail(c, MR_ERR_SETUP,
                                    "run of %d points along direction %d shorter than two closures (%d)", L, d,
                                    2 * nb);
                    int e = (s + L - 1) % nd;
                    int lo = (!g.periodic[d] && s == 0) ? g.face_bc[2 * d] : MR_BC_INTERFACE;
                    int hi = (!g.periodic[d] && e == nd - 1) ? g.face_bc[2 * d + 1] : MR_BC_INTERFACE;
                    if (lo == MR_BC_PERIODIC || hi == MR_BC_PERIODIC)
                        return fail(c, MR_ERR_SETUP, "periodic flag on a non-periodic face (direction %d)", d);
                    for (int r = 0; r < L; ++r) {
                        int code = r < nb ? 1 + r : (r >= L - nb ? 5 + (L - 1 - r) : 0);
                        if (r == 0) code |= lo << 4;
                        if (r == L - 1) code |= hi << 4;
                        cl[idx[(s + r) % nd]] = (int8_t)code;
                    }
                }
            }
    }
    g.recv_idx.assign(N, -1);
    g.n_iface = 0;
    for (int64_t p = 0; p < N; ++p) {
        bool iface = false;
        for (int d = 0; d < g.dim; ++d) iface = iface || ((g.cls[(size_t)d * N + p] >> 4) & 3) == MR_BC_INTERFACE;
        g.n_iface += iface;
    }
    return MR_OK;
}

bool is_iface(const GridHost &g, int64_t p)
{
    for (int d = 0; d < g.dim; ++d)
        if (((g.cls[(size_t)d * g.npts + p] >> 4) & 3) == MR_BC_INTERFACE) return true;
    return false;
}

// offsets of the first-derivative row selected by a class code (the rows of
// the SBP operators used by the kernels)
void row_offsets(int sbp, int row, std::vector<int> &o)
{
    o.clear();
    if (sbp == 21) {
        if (row == 0) o = {-1, 1};
        else if (row == 1) o = {0, 1};
        else o = {0, -1};
        return;
    }
    switch (row) {
    case 0: o = {-2, -1, 1, 2}; break;
    case 1: o = {0, 1, 2, 3}; break;
    case 2: o = {-1, 1}; break;
    case 3: o = {-2, -1, 1, 2}; break;
    case 4: o = {-3, -1, 1, 2}; break;
    case 5: o = {0, -1, -2, -3}; break;
    case 6: o = {1, -1}; break;
    case 7: o = {2, 1, -1, -2}; break;
    default: o = {3, 1, -1, -2}; break;
    }
}

// points read by the donor kernel on donor grid D: every donor point and the
// points of its gradient stencil in each direction
void build_closure(const mr_ctx *c, int d, GridHost &D)
{
    std::vector<char> mark(D.npts, 0);
    std::vector<int> off;
    for (size_t e = 0; e < c->ept.size(); ++e) {
        if (c->egrid[e] != d) continue;
        int64_t p = c->ept[e];
        mark[p] = 1;
        int ic[3] = {(int)(p % D.n[0]), (int)((p / D.n[0]) % D.n[1]), (int)(p / ((int64_t)D.n[0] * D.n[1]))};
        for (int m = 0; m < D.dim; ++m) {
            row_offsets(c->P.sbp, D.cls[(size_t)m * D.npts + p] & 15, off);
            for (int o : off) {
                int j = ic[m] + o;
                if (D.periodic[m]) j = ((j % D.n[m]) + D.n[m]) % D.n[m];
                mark[p + (int64_t)(j - ic[m]) * D.stride[m]] = 1;
            }
        }
    }
    D.closure.clear();
    for (int64_t p = 0; p < D.npts; ++p)
        if (mark[p]) D.closure.push_back((int32_t)p);
}

// chunks of rpc = 256 / S consecutive receivers: distinct donor points,
// each entry's index among them, and the points their gradient stencils read;
// every chunk's lists padded to the longest chunk's (-1 past its end), so that
// a workgroup finds its chunk's lists without first reading their bounds
void build_blocks(const mr_ctx *c, Link &L)
{
    const GridHost &D = c->G[L.dg];
    const int S = c->S;
    const int kp = 1 + 4 * D.dim;
    L.rpc = 256 / S;
    L.nchunk = (int)((L.n + L.rpc - 1) / L.rpc);
    L.bel.assign((size_t)L.n * S, 0);
    L.maxu = L.maxc = 0;
    std::vector<std::vector<int32_t>> Us(L.nchunk), Cs(L.nchunk);
    std::vector<std::vector<int16_t>> Ps(L.nchunk);
    std::vector<int> off;
    for (int ch = 0; ch < L.nchunk; ++ch) {
        int64_t r0 = (int64_t)ch * L.rpc, r1 = std::min<int64_t>(L.n, r0 + L.rpc);
        std::vector<int32_t> &U = Us[ch];
        for (int64_t r = r0; r < r1; ++r)
            for (int e = 0; e < S; ++e) U.push_back(c->ept[(size_t)(L.first + r) * S + e]);
        std::sort(U.begin(), U.end());
        U.erase(std::unique(U.begin(), U.end()), U.end());
        for (int64_t r = r0; r < r1; ++r)
            for (int e = 0; e < S; ++e) {
                int32_t q = c->ept[(size_t)(L.first + r) * S + e];
                L.bel[(size_t)r * S + e] = (int16_t)(std::lower_bound(U.begin(), U.end(), q) - U.begin());
            }
        std::vector<int32_t> &C = Cs[ch];
        for (int32_t p : U) {
            C.push_back(p);
            int ic[3] = {(int)(p % D.n[0]), (int)((p / D.n[0]) % D.n[1]), (int)(p / ((int64_t)D.n[0] * D.n[1]))};
            for (int m = 0; m < D.dim; ++m) {
                row_offsets(c->P.sbp, D.cls[(size_t)m * D.npts + p] & 15, off);
                for (int o : off) {
                    int j = ic[m] + o;
                    if (D.periodic[m]) j = ((j % D.n[m]) + D.n[m]) % D.n[m];
                    C.push_back((int32_t)(p + (int64_t)(j - ic[m]) * D.stride[m]));
                }
            }
        }
        std::sort(C.begin(), C.end());
        C.erase(std::unique(C.begin(), C.end()), C.end());
        // per distinct point: its position in C, then its stencil's, in the
        // order the device gradient reads them
        auto at = [&](int64_t q) { return (int16_t)(std::lower_bound(C.begin(), C.end(), (int32_t)q) - C.begin()); };
        for (int32_t p : U) {
            std::vector<int16_t> row(kp, (int16_t)-1);
            int t = 0;
            row[t++] = at(p);
            int ic[3] = {(int)(p % D.n[0]), (int)((p / D.n[0]) % D.n[1]), (int)(p / ((int64_t)D.n[0] * D.n[1]))};
            for (int m = 0; m < D.dim; ++m) {
                row_offsets(c->P.sbp, D.cls[(size_t)m * D.npts + p] & 15, off);
                for (int o : off) {
                    int j = ic[m] + o;
                    if (D.periodic[m]) j = ((j % D.n[m]) + D.n[m]) % D.n[m];
                    row[t++] = at(p + (int64_t)(j - ic[m]) * D.stride[m]);
                }
            }
            Ps[ch].insert(Ps[ch].end(), row.begin(), row.end());
        }
        L.maxu = std::max(L.maxu, (int)U.size());
        L.maxc = std::max(L.maxc, (int)C.size());
    }
    L.bup.assign((size_t)L.nchunk * L.maxu, -1);
    L.bcp.assign((size_t)L.nchunk * L.maxc, -1);
    L.bpos.assign((size_t)L.nchunk * L.maxu * kp, (int16_t)-1);
    for (int ch = 0; ch < L.nchunk; ++ch) {
        std::copy(Us[ch].begin(), Us[ch].end(), L.bup.begin() + (size_t)ch * L.maxu);
        std::copy(Cs[ch].begin(), Cs[ch].end(), L.bcp.begin() + (size_t)ch * L.maxc);
        std::copy(Ps[ch].begin(), Ps[ch].end(), L.bpos.begin() + (size_t)ch * L.maxu * kp);
    }
    // one workgroup's LDS; stencils of 64 entries (3D) keep the two-launch form
    L.blk = S <= 16 && mrk::donor_block_lds(D.dim, L.maxu, L.maxc) <= 64 * 1024;
}

struct Carver {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count)
    {
        off = (off + ALIGN - 1) / ALIGN * ALIGN;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// lay out (base == nullptr: only measure) the workspace
size_t layout(mr_ctx *c, char *base)
{
    Carver cv{base};
    int m = c->P.hist_len;
    for (auto &g : c->G) {
        int nv = g.dim + 2;
        int64_t N = g.npts;
        g.y[0] = cv.take<double>((size_t)nv * N);
        g.y[1] = cv.take<double>((size_t)nv * N);
        g.hist = cv.take<double>((size_t)m * nv * N);
        g.grad = cv.take<double>((size_t)(g.dim == 3 ? mrk::NVISC3 : g.dim * (g.dim + 1)) * N);
        for (int k = 0; k < 5; ++k) g.rk[k] = cv.take<double>((size_t)nv * N);
        g.dt = cv.take<double>((size_t)N);
        g.cls_d = cv.take<int8_t>((size_t)g.dim * N);
        g.metric = g.kind == MR_CURVILINEAR ? cv.take<double>((size_t)(g.dim * g.dim + 1) * N) : nullptr;
        g.coords_d = g.kind == MR_CURVILINEAR ? cv.take<double>((size_t)g.dim * N) : nullptr;
        size_t nr = g.recv_pts.size();
        g.recv_idx_d = nr ? cv.take<int32_t>((size_t)N) : nullptr;
        g.recv_buf = nr ? cv.take<double>(nr * (nv + g.dim * (nv - 1)) * c->rmax) : nullptr;
        int per = c->rmax / g.rate;
        g.ext.assign(per > 1 && !g.closure.empty() ? per - 1 : 0, nullptr);
        for (auto &e : g.ext) e = cv.take<double>((size_t)nv * N);
        g.closure_d = g.closure.empty() ? nullptr : cv.take<int32_t>(g.closure.size());
        g.satpts_d = g.satpts.empty() ? nullptr : cv.take<int32_t>(g.satpts.size());
    }
    size_t R = c->rgrid.size();
    c->euid_d = cv.take<int32_t>(R * c->S + 1);
    c->ew_d = cv.take<double>(R * c->S + 1);
    int RB = (c->P.dim + 2) + c->P.dim * (c->P.dim + 1);
    for (Link &L : c->links) {
        L.upts_d = cv.take<int32_t>(L.upts.size() + 1);
        L.vals_d = cv.take<double>((size_t)c->rmax * L.upts.size() * RB + 1);
        L.bup_d = cv.take<int32_t>(L.bup.size() + 1);
        L.bcp_d = cv.take<int32_t>(L.bcp.size() + 1);
        L.bel_d = cv.take<int16_t>(L.bel.size() + 1);
        L.bpos_d = cv.take<int16_t>(L.bpos.size() + 1);
    }
    c->grids_d = cv.take<GridDev>(c->G.size());
    c->partial = cv.take<double>(1024);
    return cv.off + ALIGN;
}

double *slot(const mr_ctx *c, const GridHost &g, int j)   // j = 0 oldest .. m-1 newest
{
    int m = c->P.hist_len;
    int s = ((g.head - (m - 1) + j) % m + m) % m;
    return g.hist + (size_t)s * (g.dim + 2) * g.npts;
}

// receiver rows of grid g for micro-time k (1..rmax)
double *recv_slice(const mr_ctx *c, const GridHost &g, int k)
{
    if (!g.recv_buf) return nullptr;
    size_t rb = (size_t)(g.dim + 2) + (size_t)g.dim * (g.dim + 1);
    return g.recv_buf + (size_t)(k - 1) * g.recv_pts.size() * rb;
}

mrk::DonorLink link_base(const mr_ctx *c, const Link &L)
{
    mrk::DonorLink a{};
    a.g = c->G[L.dg].dev;
    a.ph = c->ph;
    a.row0 = L.row0;
    a.upts = L.upts_d;
    a.nu = (int64_t)L.upts.size();
    a.vals = L.vals_d;
    a.uid = c->euid_d + L.first * c->S;
    a.w = c->ew_d + L.first * c->S;
    a.nrecv = L.n;
    a.S = c->S;
    a.sbp = c->P.sbp;
    return a;
}

hipStream_t sst(const mr_ctx *c, int si) { return si < 0 ? c->st : c->gs[si]; }

// ---- cross-stream order (Order): si < 0 means the context's stream, untracked
void ord_reset(mr_ctx *c, const EvSet &ev)
{
    Order &o = c->ord;
    o.pool = &ev.pool;
    o.pos.assign(o.G, 0);
    o.clock.assign(o.G, std::vector<int>(o.G, 0));
    for (auto &r : o.recs) r.clear();
    o.used.assign(o.G, 0);
    std::fill(o.wr.begin(), o.wr.end(), std::make_pair(-1, 0));
    std::fill(o.rd.begin(), o.rd.end(), std::make_pair(-1, 0));
}

void ord_op(mr_ctx *c, int s)
{
    if (s < 0) return;
    Order &o = c->ord;
    o.clock[s][s] = ++o.pos[s];
}

int ord_mark(mr_ctx *c, int s)
{
    if (s < 0) return MR_OK;
    Order &o = c->ord;
    if (!o.recs[s].empty() && o.recs[s].back().pos == o.pos[s]) return MR_OK;
    Order::Rec r{o.pos[s], (*o.pool)[s][o.used[s]++ % Order::POOL], o.clock[s]};
    HIPCHK(c, hipEventRecord(r.e, c->gs[s]));
    o.recs[s].push_back(std::move(r));
    return MR_OK;
}

// stream t must not start its next launch before launch p of stream s ends
int ord_need(mr_ctx *c, int t, std::pair<int, int> dep)
{
    Order &o = c->ord;
    int s = dep.first, p = dep.second;
    if (t < 0 || s < 0 || s == t || p <= 0 || o.clock[t][s] >= p) return MR_OK;
    const Order::Rec *r = nullptr;
    for (const auto &x : o.recs[s])
        if (x.pos >= p) { r = &x; break; }
    if (!r) {
        int rc = ord_mark(c, s);
        if (rc) return rc;
        r = &o.recs[s].back();
    }
    HIPCHK(c, hipStreamWaitEvent(c->gs[t], r->e, 0));
    for (int u = 0; u < o.G; ++u) o.clock[t][u] = std::max(o.clock[t][u], r->clock[u]);
    return MR_OK;
}

std::pair<int, int> &ord_wr(mr_ctx *c, int link, int k) { return c->ord.wr[(size_t)link * (c->rmax + 1) + k]; }
std::pair<int, int> &ord_rd(mr_ctx *c, int g, int k) { return c->ord.rd[(size_t)g * (c->rmax + 1) + k]; }

int link_index(const mr_ctx *c, const Link &L) { return (int)(&L - c->links.data()); }

bool use_blocks(const mr_ctx *c, const Link &L) { return c->donor_blocks && L.blk; }

mrk::DonorBlocks link_blocks(const Link &L)
{
    mrk::DonorBlocks b{};
    b.upts = L.bup_d;
    b.cpts = L.bcp_d;
    b.eloc = L.bel_d;
    b.bpos = L.bpos_d;
    b.nchunk = L.nchunk;
    b.rpc = L.rpc;
    b.maxu = L.maxu;
    b.maxc = L.maxc;
    return b;
}

// donor data from the donor grid's state y into out (one target time; k > 0
// names the receiving grid's slice for the cross-stream order)
int link_current(mr_ctx *c, const Link &L, const double *y, double *out, int si, int k)
{
    mrk::DonorLink a = link_base(c, L);
    a.nj = 1;
    a.ys[0] = y;
    a.out[0] = out;
    if (si >= 0) {
        int rc = ord_need(c, si, ord_rd(c, L.rg, k));     // rows last read by the receiver at k
        if (rc) return rc;
    }
    if (use_blocks(c, L))
        HIPCHK(c, mrk::launch_donor_block(a, link_blocks(L), sst(c, si)));
    else
        HIPCHK(c, mrk::launch_donor(a, sst(c, si)));
    if (si >= 0) {
        ord_op(c, si);
        ord_wr(c, link_index(c, L), k) = {si, c->ord.pos[si]};
        return ord_mark(c, si);
    }
    return MR_OK;
}

// current-time donor data of one or two chunked 2D links in one launch
// (context stream): each from its donor grid's current state into its
// receiving grid's rows of micro-time k
int links_current2(mr_ctx *c, const std::vector<const Link *> &ls, int k)
{
    mrk::DonorLinks2 P{};
    P.n = (int)ls.size();
    P.chunk0[0] = 0;
    for (int i = 0; i < P.n; ++i) {
        const Link &L = *ls[i];
        const GridHost &D = c->G[L.dg];
        P.a[i] = link_base(c, L);
        P.a[i].nj = 1;
        P.a[i].ys[0] = D.y[D.cur];
        P.a[i].out[0] = recv_slice(c, c->G[L.rg], k);
        P.b[i] = link_blocks(L);
        P.chunk0[i + 1] = P.chunk0[i] + L.nchunk;
    }
    HIPCHK(c, mrk::launch_donor_block2(P, c->st));
    return MR_OK;
}

// a donor link's data launched inside another grid's right-hand side
struct Rider {
    mrk::DonorLink a;
    mrk::DonorBlocks b;
};

// the mid-step donor data of link L gathered right after its donor grid
// evaluated at micro-time k: one slot per later micro-time k' (receiver rows
// of k' into kps) before the donor's next step at which the receiving grid
// evaluates; from the extrapolant (chunked links) or the extrapolated
// buffers
void future_link(mr_ctx *c, const Link &L, int k, mrk::DonorLink &a, int *kps)
{
    const int d = L.dg;
    const GridHost &D = c->G[d];
    const GridHost &R = c->G[L.rg];
    const int per_d = c->rmax / D.rate, per_g = c->rmax / R.rate, m = c->P.hist_len;
    const bool blk = use_blocks(c, L);
    a = link_base(c, L);
    a.nj = 0;
    if (blk) {
        a.m = m;
        for (int j = 0; j < m; ++j) a.hist[j] = slot(c, D, j);
    }
    for (int jp = 1; jp < per_d; ++jp) {
        int kp = k + jp > c->rmax ? k + jp - c->rmax : k + jp;
        if (kp % per_g) continue;
        kps[a.nj] = kp;
        if (blk) {
            a.ys[a.nj] = D.y[D.cur];
            for (int j = 0; j < m; ++j) a.beta[a.nj][j] = c->beta[d][jp][j];
        } else {
            a.ys[a.nj] = D.ext[jp - 1];
        }
        a.out[a.nj] = recv_slice(c, R, kp);
        a.nj++;
    }
}

// the mid-step donor data of grid d (which just evaluated at micro-time k)
// when it is exactly one chunked 2D link with slots to fill, so that it can
// ride in the launch of another grid's fused right-hand side
bool future_rider(mr_ctx *c, int d, int k, Rider &r)
{
    const GridHost &D = c->G[d];
    if (D.dim != 2 || c->rmax / D.rate == 1 || D.closure.empty()) return false;
    int n = 0;
    for (const Link &L : c->links) {
        if (L.dg != d) continue;
        mrk::DonorLink a;
        int kps[mrk::MAXJ];
        future_link(c, L, k, a, kps);
        if (!a.nj) continue;
        if (!use_blocks(c, L) || ++n > 1) return false;
        r.a = a;
        r.b = link_blocks(L);
    }
    return n == 1;
}

// right after donor grid d evaluated at micro-time k: its extrapolant is
// fixed until its next step, so the donor data of every later micro-time
// k' < k + per_d at which a receiving grid evaluates is gathered now:
// first the extrapolated states at the donor-stencil points (one buffer per
// offset), then one batched gather per link
int donor_future(mr_ctx *c, int d, int k, int si)
{
    hipStream_t st = sst(c, si);
    GridHost &D = c->G[d];
    int per_d = c->rmax / D.rate;
    if (per_d == 1 || D.closure.empty()) return MR_OK;
    auto kprime = [&](int jp) { int kp = k + jp; return kp > c->rmax ? kp - c->rmax : kp; };
    mrk::Extrap x{};
    x.y = D.y[D.cur];
    x.m = c->P.hist_len;
    x.nv = D.dim + 2;
    x.N = D.npts;
    for (int j = 0; j < x.m; ++j) x.hist[j] = slot(c, D, j);
    x.pts = D.closure_d;
    x.np = (int64_t)D.closure.size();
    bool need[mrk::MAXJ + 1] = {};
    for (const Link &L : c->links) {
        if (L.dg != d || use_blocks(c, L)) continue;
        int per_g = c->rmax / c->G[L.rg].rate;
        for (int jp = 1; jp < per_d; ++jp)
            if (kprime(jp) % per_g == 0) need[jp] = true;
    }
    x.nj = 0;
    for (int jp = 1; jp < per_d; ++jp) {
        if (!need[jp]) continue;
        for (int j = 0; j < x.m; ++j) x.beta[x.nj][j] = c->beta[d][jp][j];
        x.out[x.nj] = D.ext[jp - 1];
        x.nj++;
    }
    if (x.nj) {
        HIPCHK(c, mrk::launch_extrap(x, st));
        ord_op(c, si);
    }
    for (const Link &L : c->links) {
        if (L.dg != d) continue;
        mrk::DonorLink a;
        int kps[mrk::MAXJ];
        future_link(c, L, k, a, kps);
        if (si >= 0)
            for (int j = 0; j < a.nj; ++j) {
                int rc = ord_need(c, si, ord_rd(c, L.rg, kps[j]));   // rows last read by the receiver
                if (rc) return rc;
            }
        if (!a.nj) continue;
        const bool blk = use_blocks(c, L);
        if (blk)
            HIPCHK(c, mrk::launch_donor_block(a, link_blocks(L), st));
        else
            HIPCHK(c, mrk::launch_donor(a, st));
        if (si >= 0) {
            ord_op(c, si);
            for (int j = 0; j < a.nj; ++j) ord_wr(c, link_index(c, L), kps[j]) = {si, c->ord.pos[si]};
        }
    }
    return ord_mark(c, si);
}

int shape_of(const GridHost &g);

// right-hand side of one grid from state q into F (+ optional fused combine,
// + optional rider: a donor link's data launched in the same kernel)

int grid_rhs(mr_ctx *c, int gi, const double *q, double *F, const mrk::Combine &cb, bool timed, int k, int si,
             const Rider *ride = nullptr)
{
    hipStream_t st = sst(c, si);
    if (si >= 0)
        for (const Link &L : c->links)
            if (L.rg == gi) {
                int rc = ord_need(c, si, ord_wr(c, link_index(c, L), k));   // receiver rows of k written
                if (rc) return rc;
            }
    GridHost &g = c->G[gi];
    GridDev dev = g.dev;
    dev.recv = recv_slice(c, g, k);
    bool rec = timed && (c->tgrid == gi || c->tgrid == -2) && c->tcount < c->tmax;
    if (rec) HIPCHK(c, hipEventRecord(c->ev[2 * c->tcount], st));
    if (ride) {
        HIPCHK(c, mrk::launch_rhs_tile2d_donor(dev, c->P.sbp, c->ph, q, F, cb, shape_of(g), ride->a, ride->b, st));
    } else if (g.dim == 2 && !c->two_pass) {
        int shape = g.tile >= 0 ? g.tile : mrk::default_tile_shape(dev);
        HIPCHK(c, mrk::launch_rhs_tile2d(dev, c->P.sbp, c->ph, q, F, cb, shape, st));
    } else if (g.dim == 3 && c->tile3d >= 0 && c->flux3d > 0) {
        HIPCHK(c, mrk::launch_rhs_zm3d(dev, c->P.sbp, c->ph, q, g.grad, F, cb, c->tile3d, c->slab3d, c->flux3d,
                                       c->zchunk3d, g.satpts_d, (int)g.satpts.size(), st));
    } else if (g.dim == 3 && c->tile3d >= 0) {
        HIPCHK(c, mrk::launch_rhs_tile3d(dev, c->P.sbp, c->ph, q, g.grad, F, cb, c->tile3d, c->gtile3d, c->slab3d,
                                         st));
    } else {
        HIPCHK(c, mrk::launch_grad(dev, c->P.sbp, c->ph, q, g.grad, st));
        HIPCHK(c, mrk::launch_rhs(dev, c->grids_d + gi, c->P.sbp, c->ph, q, g.grad, F, cb, st));
    }
    if (rec) {
        HIPCHK(c, hipEventRecord(c->ev[2 * c->tcount + 1], st));
        c->tgrid_of[c->tcount] = gi;
        c->tcount++;
    }
    if (si >= 0) {
        ord_op(c, si);
        ord_rd(c, gi, k) = {si, c->ord.pos[si]};
        return ord_mark(c, si);
    }
    return MR_OK;
}

// coupled right-hand side of all grids at one time
int rhs_all(mr_ctx *c, const double *const *q, double *const *F)
{
    for (const Link &L : c->links) {
        int rc = link_current(c, L, q[L.dg], recv_slice(c, c->G[L.rg], 1), -1, 1);
        if (rc) return rc;
    }
    mrk::Combine none{};
    for (size_t g = 0; g < c->G.size(); ++g) {
        int rc = grid_rhs(c, (int)g, q[g], F[g], none, false, 1, -1);
        if (rc) return rc;
    }
    return MR_OK;
}

int64_t nelem(const GridHost &g) { return (int64_t)(g.dim + 2) * g.npts; }

int make_evset(mr_ctx *c, EvSet &e)
{
    int G = (int)c->G.size();
    auto mk = [&](hipEvent_t *ev) { return hipEventCreateWithFlags(ev, hipEventDisableTiming); };
    HIPCHK(c, mk(&e.join));
    e.done.assign(G, nullptr);
    e.pool.assign(G, std::vector<hipEvent_t>(Order::POOL, nullptr));
    for (int g = 0; g < G; ++g) {
        HIPCHK(c, mk(&e.done[g]));
        for (auto &ev : e.pool[g]) HIPCHK(c, mk(&ev));
    }
    return MR_OK;
}

void free_evset(EvSet &e)
{
    if (e.join) (void)hipEventDestroy(e.join);
    for (auto ev : e.done)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &v : e.pool)
        for (auto ev : v)
            if (ev) (void)hipEventDestroy(ev);
    e = EvSet{};
}

// ---- launch tables
bool fused2d(const mr_ctx *c, const GridHost &g) { return g.dim == 2 && !c->two_pass; }

int shape_of(const GridHost &g) { return g.tile >= 0 ? g.tile : mrk::default_tile_shape(g.dev); }

// grid gi's evaluation at micro-time k as run_macrosteps issues it (after
// its state swap, before its ring head advances)
mrk::TileJob make_tile_job(const mr_ctx *c, int gi, int k)
{
    const GridHost &g = c->G[gi];
    const int m = c->P.hist_len;
    mrk::TileJob J{};
    J.g = g.dev;
    J.g.recv = recv_slice(c, g, k);
    J.q = g.y[g.cur];
    J.F = slot(c, g, 0);
    J.cb.m = m;
    for (int j = 0; j < m - 1; ++j) J.cb.hist[j] = slot(c, g, j + 1);
    for (int j = 0; j < m; ++j) J.cb.c[j] = c->c_own[gi][j];
    J.cb.y_next = g.y[1 - g.cur];
    const mrk::TileShape &s = mrk::kTileShapes[shape_of(g)];
    J.ntx = (g.n[0] + s.tx - 1) / s.tx;
    J.nty = (g.n[1] + s.ty - 1) / s.ty;
    return J;
}

mrk::LinkJob make_current_job(const mr_ctx *c, const Link &L, int k)
{
    mrk::LinkJob J{};
    const GridHost &D = c->G[L.dg];
    J.a = link_base(c, L);
    J.a.nj = 1;
    J.a.ys[0] = D.y[D.cur];
    J.a.out[0] = recv_slice(c, c->G[L.rg], k);
    J.b = link_blocks(L);
    return J;
}

// the mid-step receiver rows a chunked link provides right after its donor
// grid evaluated at micro-time k (its ring head already advanced)
mrk::LinkJob make_future_job(const mr_ctx *c, const Link &L, int k)
{
    mrk::LinkJob J{};
    const GridHost &D = c->G[L.dg];
    const GridHost &R = c->G[L.rg];
    const int m = c->P.hist_len, per_d = c->rmax / D.rate, per_g = c->rmax / R.rate;
    J.a = link_base(c, L);
    J.a.nj = 0;
    J.a.m = m;
    for (int j = 0; j < m; ++j) J.a.hist[j] = slot(c, D, j);
    for (int jp = 1; jp < per_d; ++jp) {
        int kp = k + jp;
        if (kp > c->rmax) kp -= c->rmax;
        if (kp % per_g) continue;
        J.a.ys[J.a.nj] = D.y[D.cur];
        for (int j = 0; j < m; ++j) J.a.beta[J.a.nj][j] = c->beta[L.dg][jp][j];
        J.a.out[J.a.nj] = recv_slice(c, R, kp);
        J.a.nj++;
    }
    J.b = link_blocks(L);
    return J;
}

// per-grid streams (default priority, not synchronising with the null
// stream) and their events, created on first use
int ensure_streams(mr_ctx *c)
{
    if (!c->gs.empty()) return MR_OK;
    int G = (int)c->G.size();
    Order &o = c->ord;
    o.G = G;
    o.K = c->rmax;
    o.recs.assign(G, {});
    o.wr.assign(c->links.size() * (c->rmax + 1), {-1, 0});
    o.rd.assign((size_t)G * (c->rmax + 1), {-1, 0});
    int rc = make_evset(c, c->eager);
    if (rc) return rc;
    c->gs.assign(G, nullptr);
    for (int g = 0; g < G; ++g) HIPCHK(c, hipStreamCreateWithFlags(&c->gs[g], hipStreamNonBlocking));
    return MR_OK;
}

// n macrosteps: on the context's stream, or (ms) on the per-grid streams
// between a join with the context's stream and a join back
int run_macrosteps(mr_ctx *c, int nsteps, bool ms, hipStream_t origin, const EvSet &ev)
{
    int m = c->P.hist_len;
    int G = (int)c->G.size();
    if (ms) {
        ord_reset(c, ev);
        HIPCHK(c, hipEventRecord(ev.join, origin));
        for (int g = 0; g < G; ++g) HIPCHK(c, hipStreamWaitEvent(c->gs[g], ev.join, 0));
    }
    auto gsi = [&](int g) { return ms ? g : -1; };
    for (int s = 0; s < nsteps; ++s) {
        for (int k = 1; k <= c->rmax; ++k) {
            bool ends[mrk::MAXG] = {};
            for (int g = 0; g < G; ++g) {
                ends[g] = k % (c->rmax / c->G[g].rate) == 0;
                if (ends[g]) c->G[g].cur ^= 1;   // the staged own step becomes current
            }
            // donor data from donors at their own step (on one stream, 2D
            // chunked links two to a launch); mid-step donor data was
            // gathered right after the donor grid's last evaluation
            std::vector<const Link *> pair;
            for (const Link &L : c->links) {
                if (!ends[L.rg] || !ends[L.dg]) continue;
                const GridHost &D = c->G[L.dg];
                if (!ms && D.dim == 2 && use_blocks(c, L)) {
                    pair.push_back(&L);
                    if (pair.size() == 2) {
                        int rc = links_current2(c, pair, k);
                        if (rc) return rc;
                        pair.clear();
                    }
                    continue;
                }
                int rc = link_current(c, L, D.y[D.cur], recv_slice(c, c->G[L.rg], k), gsi(L.dg), k);
                if (rc) return rc;
            }
            if (!pair.empty()) {
                int rc = links_current2(c, pair, k);
                if (rc) return rc;
            }
            // (one stream) a grid's mid-step donor data reads only that
            // grid's state and history and writes receiver rows of other
            // micro-times than k, so it rides in the launch of the next grid
            // evaluated at k when both fit the combined kernel
            bool rode[mrk::MAXG] = {};
            int pend = -1;
            Rider rider;
            for (int g = 0; g < G; ++g) {
                if (!ends[g]) continue;
                GridHost &Gh = c->G[g];
                mrk::Combine cb{};
                cb.m = m;
                for (int j = 0; j < m - 1; ++j) cb.hist[j] = slot(c, Gh, j + 1);
                for (int j = 0; j < m; ++j) cb.c[j] = c->c_own[g][j];
                cb.y_next = Gh.y[1 - Gh.cur];
                double *Fnew = slot(c, Gh, 0);      // the oldest slot is overwritten
                const bool timing = (c->tgrid == g || c->tgrid == -2) && c->tcount < c->tmax;
                const bool take = pend >= 0 && fused2d(c, Gh) && mrk::tile2d_donor_ok(shape_of(Gh)) && !timing;
                int rc = grid_rhs(c, g, Gh.y[Gh.cur], Fnew, cb, true, k, gsi(g), take ? &rider : nullptr);
                if (rc) return rc;
                if (take) {
                    rode[pend] = true;
                    pend = -1;
                }
                Gh.head = (Gh.head + 1) % m;
                if (!ms && c->ride_donors && pend < 0 && future_rider(c, g, k, rider)) pend = g;
            }
            for (int g = 0; g < G; ++g) {
                if (!ends[g] || rode[g]) continue;
                int rc = donor_future(c, g, k, gsi(g));
                if (rc) return rc;
            }
        }
        c->t += c->H;
        c->nmacro++;
    }
    if (ms)
        for (int g = 0; g < G; ++g) {
            HIPCHK(c, hipEventRecord(ev.done[g], c->gs[g]));
            HIPCHK(c, hipStreamWaitEvent(origin, ev.done[g], 0));
        }
    return MR_OK;
}

// from the current states and histories: stage every grid's first own step
// and, as if every grid had just evaluated, the donor data of the next
// macrostep's mid-step times
int restage(mr_ctx *c)
{
    int m = c->P.hist_len;
    for (size_t g = 0; g < c->G.size(); ++g) {
        GridHost &Gh = c->G[g];
        mrk::Combine cb{};
        cb.m = m;
        for (int j = 0; j < m; ++j) {
            cb.c[j] = c->c_own[g][j];
            cb.hist[j] = slot(c, Gh, j);
        }
        cb.y_next = Gh.y[1 - Gh.cur];
        HIPCHK(c, mrk::launch_combine(nelem(Gh), Gh.y[Gh.cur], cb, c->st));
    }
    for (int g = 0; g < (int)c->G.size(); ++g) {
        int rc = donor_future(c, g, c->rmax, -1);
        if (rc) return rc;
    }
    return MR_OK;
}

// macrostep H: the fastest grid's step h = H / r_max and every grid's own
// and mid-step AB coefficient rows scaled by its step H / r_g
int set_macrostep(mr_ctx *c, double Hm)
{
    if (!(Hm > 0) || !std::isfinite(Hm)) return fail(c, MR_ERR_SETUP, "invalid timestep %g", Hm);
    c->H = Hm;
    c->h = Hm / c->rmax;
    c->have_dt = true;
    int m = c->P.hist_len;
    c->c_own.assign(c->G.size(), std::vector<double>(m));
    c->beta.assign(c->G.size(), {});
    for (size_t g = 0; g < c->G.size(); ++g) {
        double Hg = Hm / c->G[g].rate;
        for (int j = 0; j < m; ++j) c->c_own[g][j] = (double)c->alpha_own[g][j] * Hg;
        int per = c->rmax / c->G[g].rate;
        c->beta[g].assign(per, std::vector<double>(m, 0.0));
        for (int jp = 1; jp < per; ++jp)
            for (int j = 0; j < m; ++j) c->beta[g][jp][j] = (double)c->alpha_mid[g][jp][j] * Hg;
    }
    return MR_OK;
}

// ---- batches
int bfail(mr_batch *b, int code, const char *msg)
{
    if (b) b->err = msg;
    return code;
}

#define BHIPCHK(b, call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return bfail(b, MR_ERR_HIP, hipGetErrorString(e_));          \
    } while (0)

// one system's bookkeeping for its micro-time ks (state swaps, ring heads)
// while collecting its jobs of that micro-time
void batch_collect(const mr_ctx *c, int ks, std::vector<mrk::LinkJob> &cur, std::vector<mrk::TileJob> &tiles,
                   std::vector<int> &tile_shape, std::vector<mrk::LinkJob> &fut)
{
    mr_ctx *cc = const_cast<mr_ctx *>(c);
    const int G = (int)c->G.size(), m = c->P.hist_len;
    bool ends[mrk::MAXG] = {};
    for (int g = 0; g < G; ++g) {
        ends[g] = ks % (c->rmax / c->G[g].rate) == 0;
        if (ends[g]) cc->G[g].cur ^= 1;
    }
    for (const Link &L : c->links)
        if (ends[L.rg] && ends[L.dg]) cur.push_back(make_current_job(c, L, ks));
    for (int g = 0; g < G; ++g) {
        if (!ends[g]) continue;
        tiles.push_back(make_tile_job(c, g, ks));
        tile_shape.push_back(shape_of(c->G[g]));
        cc->G[g].head = (cc->G[g].head + 1) % m;
    }
    for (const Link &L : c->links) {
        const GridHost &D = c->G[L.dg];
        if (!ends[L.dg] || c->rmax / D.rate == 1 || D.closure.empty()) continue;
        mrk::LinkJob J = make_future_job(c, L, ks);
        if (J.a.nj) fut.push_back(J);
    }
}

// group jobs of one kind by launch key, give each its offset in the
// concatenated list, append to the host tables and record the launches
template <class Job, class Key, class Count>
void batch_group(std::vector<Job> &jobs, Key key, Count count, int what, std::vector<Job> &table,
                 std::vector<mr_batch::Launch> &out)
{
    std::vector<std::array<int, 5>> keys;
    for (auto &j : jobs) {
        auto kk = key(j);
        if (std::find(keys.begin(), keys.end(), kk) == keys.end()) keys.push_back(kk);
    }
    for (auto &kk : keys) {
        mr_batch::Launch L{};
        L.what = what;
        L.first = (int)table.size();
        L.dim = kk[0];
        L.sbp = kk[1];
        L.cart = kk[2];
        L.shape = kk[3];
        int off = 0;
        for (auto &j : jobs) {
            if (key(j) != kk) continue;
            Job x = j;
            count(x, off, L);
            table.push_back(x);
            L.njobs++;
        }
        L.nblk = off;
        out.push_back(L);
    }
}

int batch_build(mr_batch *b)
{
    const int n = (int)b->ctx.size();
    std::vector<mrk::TileJob> tj;
    std::vector<mrk::LinkJob> lj;
    b->plan.assign((size_t)b->P * (b->R + 1), {});
    std::vector<std::vector<std::pair<int, int>>> saved(n);
    for (int s = 0; s < n; ++s)
        for (auto &g : b->ctx[s]->G) saved[s].push_back({g.cur, g.head});
    for (int p = 0; p < b->P; ++p)
        for (int k = 1; k <= b->R; ++k) {
            std::vector<mrk::LinkJob> cur, fut;
            std::vector<mrk::TileJob> tiles;
            std::vector<int> shapes;
            for (int s = 0; s < n; ++s) {
                const mr_ctx *c = b->ctx[s];
                if ((k * c->rmax) % b->R) continue;
                batch_collect(c, k * c->rmax / b->R, cur, tiles, shapes, fut);
            }
            if (b->shape >= 0)
                for (size_t i = 0; i < tiles.size(); ++i) {
                    const mrk::TileShape &t = mrk::kTileShapes[b->shape];
                    shapes[i] = b->shape;
                    tiles[i].ntx = (tiles[i].g.n[0] + t.tx - 1) / t.tx;
                    tiles[i].nty = (tiles[i].g.n[1] + t.ty - 1) / t.ty;
                }
            // a tile job's tile0 carries its tile shape until the jobs are
            // grouped by launch key; grouping then sets the real offsets
            for (size_t i = 0; i < tiles.size(); ++i) tiles[i].tile0 = shapes[i];
            auto &out = b->plan[(size_t)p * (b->R + 1) + k];
            auto lkey = [&](const mrk::LinkJob &j) {
                return std::array<int, 5>{j.a.g.dim, j.a.sbp, j.a.g.cartesian, 0, 0};
            };
            auto lcount = [&](mrk::LinkJob &j, int &off, mr_batch::Launch &L) {
                j.chunk0 = off;
                off += j.b.nchunk;
                L.maxnj = std::max(L.maxnj, j.a.nj);
                L.lds = std::max(L.lds, mrk::donor_block_lds(j.a.g.dim, j.b.maxu, L.what == 2 ? j.b.maxc : 0));
            };
            auto tkey = [&](const mrk::TileJob &j) {
                return std::array<int, 5>{2, 0, j.g.cartesian, j.tile0, 0};
            };
            auto tcount = [&](mrk::TileJob &j, int &off, mr_batch::Launch &L) {
                j.tile0 = off;
                off += j.ntx * j.nty;
                L.maxnj = 1;
            };
            batch_group(cur, lkey, lcount, 0, lj, out);
            batch_group(tiles, tkey, tcount, 1, tj, out);
            batch_group(fut, lkey, lcount, 2, lj, out);
            for (auto &L : out)
                if (L.what == 1) L.sbp = b->ctx[0]->P.sbp;
        }
    for (int s = 0; s < n; ++s)
        for (size_t g = 0; g < b->ctx[s]->G.size(); ++g) {
            b->ctx[s]->G[g].cur = saved[s][g].first;
            b->ctx[s]->G[g].head = saved[s][g].second;
        }
    if (tj.size() > b->tj_cap || lj.size() > b->lj_cap) return bfail(b, MR_ERR_STATE, "launch plan exceeds the workspace");
    if (!tj.empty())
        BHIPCHK(b, hipMemcpyAsync(b->tj_d, tj.data(), tj.size() * sizeof(mrk::TileJob), hipMemcpyHostToDevice, b->st));
    if (!lj.empty())
        BHIPCHK(b, hipMemcpyAsync(b->lj_d, lj.data(), lj.size() * sizeof(mrk::LinkJob), hipMemcpyHostToDevice, b->st));
    BHIPCHK(b, hipStreamSynchronize(b->st));
    b->base.resize(n);
    b->version.resize(n);
    for (int s = 0; s < n; ++s) {
        b->base[s] = b->ctx[s]->nmacro;
        b->version[s] = b->ctx[s]->version;
    }
    b->steps = 0;
    b->built = true;
    return MR_OK;
}

// a system's bookkeeping of one macrostep (what run_macrosteps leaves behind)
void advance_one(mr_ctx *c)
{
    const int m = c->P.hist_len;
    for (int k = 1; k <= c->rmax; ++k)
        for (auto &g : c->G)
            if (k % (c->rmax / g.rate) == 0) {
                g.cur ^= 1;
                g.head = (g.head + 1) % m;
            }
    c->t += c->H;
    c->nmacro++;
}

// ========================================================== discrete adjoint
// Reverse-mode derivative of a whole run (RK bootstrap, then MRAB
// macrosteps at the context's fixed macrostep H) of a wall-pressure
// objective, with respect to the initial states.  The run is re-expressed as
// a sequence of elementary operations on the integrator's quantities (own-step
// AB combination, extrapolant, donor data, right-hand side, history push,
// RK stage combinations); the reverse sweep applies their adjoints in the
// opposite order.  The forward pass the adjoint differentiates is the one in
// this section (same kernels and the same rounding order as the macrostep
// calls for the AB combinations and right-hand sides; donor data by the
// two-launch path).  Macrosteps are reversed under a binomial checkpointing
// schedule (optimal split by dynamic programming over the number of free
// snapshot slots); a snapshot holds every grid's state and history.

}  // namespace

struct AdjLink {
    std::vector<int32_t> ustart, uent, cpts, cstart, cent, cself;
    int32_t *ustart_d = nullptr, *uent_d = nullptr, *cpts_d = nullptr, *cstart_d = nullptr, *cent_d = nullptr,
            *cself_d = nullptr;
    double *uq = nullptr, *uk = nullptr;
};

struct AdjGrid {
    double *lam_y = nullptr, *lam_ext = nullptr, *lys = nullptr;
    double *lam_ring[mrk::MAXH] = {};
    double *mu = nullptr, *kap = nullptr, *lqd = nullptr;
    double *recv = nullptr, *lam_recv = nullptr;   // nslice slices of receiver rows
    double *ys = nullptr;                          // rate + 2 states: a macrostep's start, its own-step
                                                   // states, the next one's first (a ring from ys0)
    int ys0 = 0;
    double *ring[mrk::MAXH] = {};                  // forward history, oldest first
    double *ext = nullptr;                         // rmax extrapolants (by micro-time)
    double *snap = nullptr;                        // nsnap x (1 + m) states
    double *boot = nullptr;                        // nboot + 1 bootstrap states
    double *stg[4] = {}, *kk[4] = {}, *lk[4] = {}; // bootstrap stage states, derivatives, adjoints
    std::vector<int32_t> bpts;                     // points ending a run in some direction
    int32_t *bpts_d = nullptr;
    double *bres = nullptr;                        // their local-Jacobian results
};

struct AdjCtx {
    bool tables = false, bound = false;
    int nsnap = 0, nslice = 0, nboot = 0;
    size_t bytes = 0;
    char *ws = nullptr;
    int og = -1;
    std::vector<int32_t> opts;
    std::vector<double> ow;
    int32_t *opts_d = nullptr;
    double *ow_d = nullptr, *acc = nullptr;
    std::vector<AdjGrid> G;
    std::vector<AdjLink> L;
    std::vector<int> snap_pos;                     // macrostep held by each slot (-1 free)
};

namespace {

// per link: the entries of each unique donor point, and the points the
// donor gradients read with (unique point, direction, offset)
void adj_tables(mr_ctx *c)
{
    AdjCtx &A = *c->adj;
    if (A.tables) return;
    A.L.assign(c->links.size(), {});
    std::vector<int> off;
    for (size_t li = 0; li < c->links.size(); ++li) {
        const Link &L = c->links[li];
        AdjLink &T = A.L[li];
        const GridHost &D = c->G[L.dg];
        const int S = c->S;
        const size_t nu = L.upts.size();
        T.ustart.assign(nu + 1, 0);
        for (int64_t e = 0; e < L.n * S; ++e) T.ustart[c->euid[(size_t)L.first * S + e] + 1]++;
        for (size_t u = 0; u < nu; ++u) T.ustart[u + 1] += T.ustart[u];
        T.uent.assign((size_t)L.n * S, 0);
        std::vector<int32_t> fill(T.ustart.begin(), T.ustart.end() - 1);
        for (int64_t e = 0; e < L.n * S; ++e) T.uent[fill[c->euid[(size_t)L.first * S + e]]++] = (int32_t)e;
        struct E { int32_t c, code; };
        std::vector<E> es;
        for (size_t u = 0; u < nu; ++u) {
            int64_t p = L.upts[u];
            int ic[3] = {(int)(p % D.n[0]), (int)((p / D.n[0]) % D.n[1]), (int)(p / ((int64_t)D.n[0] * D.n[1]))};
            for (int m = 0; m < D.dim; ++m) {
                row_offsets(c->P.sbp, D.cls[(size_t)m * D.npts + p] & 15, off);
                for (int o : off) {
                    int j = ic[m] + o;
                    if (D.periodic[m]) j = ((j % D.n[m]) + D.n[m]) % D.n[m];
                    int32_t q = (int32_t)(p + (int64_t)(j - ic[m]) * D.stride[m]);
                    es.push_back({q, (int32_t)((u << 8) | (m << 4) | (o + 8))});
                }
            }
            es.push_back({(int32_t)p, -1});   // the point itself
        }
        std::stable_sort(es.begin(), es.end(), [](const E &a, const E &b) { return a.c < b.c; });
        T.cpts.clear();
        T.cstart.assign(1, 0);
        T.cent.clear();
        T.cself.clear();
        for (size_t i = 0; i < es.size();) {
            size_t k = i;
            int32_t self = -1;
            while (k < es.size() && es[k].c == es[i].c) {
                if (es[k].code < 0) {
                    self = (int32_t)(std::lower_bound(L.upts.begin(), L.upts.end(), es[k].c) - L.upts.begin());
                } else {
                    T.cent.push_back(es[k].code);
                }
                ++k;
            }
            T.cpts.push_back(es[i].c);
            T.cself.push_back(self);
            T.cstart.push_back((int32_t)T.cent.size());
            i = k;
        }
    }
    A.G.resize(c->G.size());
    for (size_t gi = 0; gi < c->G.size(); ++gi) {
        const GridHost &g = c->G[gi];
        std::vector<int32_t> &B = A.G[gi].bpts;
        B.clear();
        for (int64_t p = 0; p < g.npts; ++p) {
            if ((g.cls[p] & 15) == mrk::CLS_HOLE) continue;
            bool any = false;
            for (int d = 0; d < g.dim; ++d) any = any || ((g.cls[(size_t)d * g.npts + p] >> 4) & 3) != 0;
            if (any) B.push_back((int32_t)p);
        }
    }
    A.tables = true;
}

size_t adj_layout(mr_ctx *c, char *base)
{
    AdjCtx &A = *c->adj;
    Carver cv{base};
    const int m = c->P.hist_len;
    A.G.resize(c->G.size());
    for (size_t gi = 0; gi < c->G.size(); ++gi) {
        const GridHost &g = c->G[gi];
        AdjGrid &a = A.G[gi];
        const size_t ne = (size_t)(g.dim + 2) * g.npts, N = (size_t)g.npts;
        auto st = [&]() { return cv.take<double>(ne); };
        a.lam_y = st();
        a.lam_ext = st();
        a.lys = st();
        for (int j = 0; j < m; ++j) a.lam_ring[j] = st();
        a.mu = cv.take<double>((size_t)g.dim * (g.dim + 2) * N);
        a.kap = cv.take<double>((size_t)g.dim * (g.dim + 1) * N);
        a.lqd = st();
        const size_t rows = g.recv_pts.size() * (size_t)((g.dim + 2) + g.dim * (g.dim + 1));
        a.recv = rows ? cv.take<double>(rows * A.nslice) : nullptr;
        a.lam_recv = rows ? cv.take<double>(rows * A.nslice) : nullptr;
        a.ys = cv.take<double>(ne * (g.rate + 2));
        for (int j = 0; j < m; ++j) a.ring[j] = st();
        const bool donor_mid = c->rmax / g.rate > 1 && std::any_of(c->links.begin(), c->links.end(),
                                                                  [&](const Link &L) { return L.dg == (int)gi; });
        a.ext = donor_mid ? cv.take<double>(ne * c->rmax) : nullptr;
        a.snap = cv.take<double>(ne * (1 + m) * A.nsnap);
        a.boot = cv.take<double>(ne * (A.nboot + 1));
        for (int k = 0; k < 4; ++k) {
            a.stg[k] = st();
            a.kk[k] = st();
            a.lk[k] = st();
        }
        const size_t nv = g.dim + 2, ng = (size_t)g.dim * (g.dim + 1), rb = nv + (size_t)g.dim * (nv - 1);
        const size_t nin = nv + ng + rb;      // inputs of a SAT point's local Jacobian
        a.bpts_d = cv.take<int32_t>(a.bpts.size() + 1);
        a.bres = cv.take<double>(a.bpts.size() * nin + 1);
    }
    for (size_t li = 0; li < c->links.size(); ++li) {
        AdjLink &T = A.L[li];
        const int dim = c->G[c->links[li].dg].dim;
        const size_t nu = c->links[li].upts.size();
        T.ustart_d = cv.take<int32_t>(T.ustart.size());
        T.uent_d = cv.take<int32_t>(T.uent.size() + 1);
        T.cpts_d = cv.take<int32_t>(T.cpts.size() + 1);
        T.cstart_d = cv.take<int32_t>(T.cstart.size());
        T.cent_d = cv.take<int32_t>(T.cent.size() + 1);
        T.cself_d = cv.take<int32_t>(T.cself.size() + 1);
        T.uq = cv.take<double>(nu * (dim + 2) + 1);
        T.uk = cv.take<double>(nu * dim * (dim + 1) + 1);
    }
    int64_t maxn = 1;
    for (const GridHost &g : c->G) maxn = std::max(maxn, g.npts);
    A.opts_d = cv.take<int32_t>((size_t)maxn);
    A.ow_d = cv.take<double>((size_t)maxn);
    A.acc = cv.take<double>(1);
    return cv.off + ALIGN;
}

double *gstate(const AdjGrid &, const GridHost &g, double *base, int i)
{
    return base + (size_t)i * (g.dim + 2) * g.npts;
}
// state after e own steps of the current macrostep (e = 0: its start)
double *ysl(const AdjGrid &a, const GridHost &g, int e) { return gstate(a, g, a.ys, (a.ys0 + e) % (g.rate + 2)); }

double *rslice(const mr_ctx *c, const GridHost &g, double *base, int s)
{
    if (!base) return nullptr;
    return base + (size_t)s * g.recv_pts.size() * ((g.dim + 2) + g.dim * (g.dim + 1));
}
size_t rbytes(const GridHost &g) { return g.recv_pts.size() * ((g.dim + 2) + g.dim * (g.dim + 1)) * 8; }

mrk::Objective adj_obj(const mr_ctx *c)
{
    mrk::Objective o{};
    o.pts = c->adj->opts_d;
    o.w = c->adj->ow_d;
    o.n = (int)c->adj->opts.size();
    o.gm1 = c->P.gamma - 1.0;
    return o;
}

// donor data of link L from donor state Y into rows out (one launch per
// chunked link, else values then gather)
int adj_donor_fwd(mr_ctx *c, const Link &L, const double *Y, double *out)
{
    mrk::DonorLink a = link_base(c, L);
    a.nj = 1;
    a.ys[0] = Y;
    a.out[0] = out;
    if (use_blocks(c, L))
        HIPCHK(c, mrk::launch_donor_block(a, link_blocks(L), c->st));
    else
        HIPCHK(c, mrk::launch_donor(a, c->st));
    return MR_OK;
}

// right-hand side of grid gi from q with receiver rows recv into F (and the
// fused AB combination cb when cb.m > 0)
int adj_rhs_fwd(mr_ctx *c, int gi, const double *q, double *recv, double *F, const mrk::Combine &cb = mrk::Combine{})
{
    GridHost &g = c->G[gi];
    GridDev dev = g.dev;
    dev.recv = recv;
    HIPCHK(c, mrk::launch_rhs_tile2d(dev, c->P.sbp, c->ph, q, F, cb, shape_of(g), c->st));
    return MR_OK;
}

// every grid's first own step of the current macrostep from its start and
// history (the staging mr_mrab_resume does)
int adj_stage(mr_ctx *c)
{
    AdjCtx &A = *c->adj;
    const int m = c->P.hist_len;
    for (size_t g = 0; g < c->G.size(); ++g) {
        const GridHost &Gh = c->G[g];
        AdjGrid &a = A.G[g];
        mrk::Combine cb{};
        cb.m = m;
        for (int j = 0; j < m; ++j) {
            cb.c[j] = c->c_own[g][j];
            cb.hist[j] = a.ring[j];
        }
        cb.y_next = ysl(a, Gh, 1);
        HIPCHK(c, mrk::launch_combine(nelem(Gh), ysl(a, Gh, 0), cb, c->st));
    }
    return MR_OK;
}

// after a macrostep: its end state (and the staged next step) become the
// next macrostep's start
void adj_advance(mr_ctx *c)
{
    for (size_t g = 0; g < c->G.size(); ++g) {
        AdjGrid &a = c->adj->G[g];
        a.ys0 = (a.ys0 + c->G[g].rate) % (c->G[g].rate + 2);
    }
}

// lam_q += (dR/dq)^T lamF and lam_recv = (dR/drecv)^T lamF for grid gi
int adj_rhs_rev(mr_ctx *c, int gi, const double *q, double *recv, const double *lamF, double *lam_recv,
                double *lam_q)
{
    GridHost &g = c->G[gi];
    AdjGrid &a = c->adj->G[gi];
    if (lam_recv) HIPCHK(c, hipMemsetAsync(lam_recv, 0, rbytes(g), c->st));
    mrk::AdjRhs r{};
    r.g = g.dev;
    r.g.recv = recv;
    r.ph = c->ph;
    r.q = q;
    r.lamF = lamF;
    r.mu = a.mu;
    r.kap = a.kap;
    r.lqd = a.lqd;
    r.lam_recv = lam_recv;
    r.lam_q = lam_q;
    r.bpts = a.bpts_d;
    r.nb = (int)a.bpts.size();
    r.bres = a.bres;
    HIPCHK(c, mrk::launch_adj_rhs(r, c->P.sbp, c->st));
    return MR_OK;
}

// lam_Y += (d donor data / dY)^T lam_recv for link li
int adj_donor_rev(mr_ctx *c, int li, const double *Y, const double *lam_recv, double *lam_Y)
{
    const Link &L = c->links[li];
    AdjLink &T = c->adj->L[li];
    mrk::AdjDonor d{};
    d.g = c->G[L.dg].dev;
    d.ph = c->ph;
    d.y = Y;
    d.lam_recv = lam_recv;
    d.row0 = L.row0;
    d.S = c->S;
    d.upts = L.upts_d;
    d.nu = (int64_t)L.upts.size();
    d.ustart = T.ustart_d;
    d.uent = T.uent_d;
    d.w = c->ew_d + (size_t)L.first * c->S;
    d.uq = T.uq;
    d.uk = T.uk;
    d.cpts = T.cpts_d;
    d.nc = (int64_t)T.cpts.size();
    d.cstart = T.cstart_d;
    d.cent = T.cent_d;
    d.cself = T.cself_d;
    d.lam_y = lam_Y;
    HIPCHK(c, mrk::launch_adj_donor(d, c->P.sbp, c->st));
    return MR_OK;
}

// coupled right-hand side at one time: donor data from Y[dg] into slice s,
// then every grid's right-hand side into K
int adj_coupled_fwd(mr_ctx *c, const std::vector<double *> &Y, int s, const std::vector<double *> &K)
{
    AdjCtx &A = *c->adj;
    for (const Link &L : c->links) {
        int rc = adj_donor_fwd(c, L, Y[L.dg], rslice(c, c->G[L.rg], A.G[L.rg].recv, s));
        if (rc) return rc;
    }
    for (size_t g = 0; g < c->G.size(); ++g) {
        int rc = adj_rhs_fwd(c, (int)g, Y[g], rslice(c, c->G[g], A.G[g].recv, s), K[g]);
        if (rc) return rc;
    }
    return MR_OK;
}

// lamY += (coupled right-hand side at Y, slice s)^T lamK
int adj_coupled_rev(mr_ctx *c, const std::vector<double *> &Y, int s, const std::vector<double *> &lamK,
                    const std::vector<double *> &lamY)
{
    AdjCtx &A = *c->adj;
    for (size_t g = 0; g < c->G.size(); ++g) {
        const GridHost &G = c->G[g];
        int rc = adj_rhs_rev(c, (int)g, Y[g], rslice(c, G, A.G[g].recv, s), lamK[g],
                             rslice(c, G, A.G[g].lam_recv, s), lamY[g]);
        if (rc) return rc;
    }
    for (size_t li = 0; li < c->links.size(); ++li) {
        const Link &L = c->links[li];
        int rc = adj_donor_rev(c, (int)li, Y[L.dg], rslice(c, c->G[L.rg], A.G[L.rg].lam_recv, s), lamY[L.dg]);
        if (rc) return rc;
    }
    return MR_OK;
}

int adj_axpy(mr_ctx *c, int64_t n, const double *src, std::initializer_list<double *> dst,
             std::initializer_list<double> coef)
{
    std::vector<double *> d(dst);
    std::vector<double> k(coef);
    HIPCHK(c, mrk::launch_adj_axpy(n, src, (int)d.size(), d.data(), k.data(), c->st));
    return MR_OK;
}

// objective weight of the objective grid's state after own step i (i = 0:
// the start of the macrosteps) of a run of nmacro macrosteps: trapezoid rule
double adj_tau(const mr_ctx *c, int i, int nmacro)
{
    const GridHost &g = c->G[c->adj->og];
    const double hg = c->H / g.rate;
    const int last = nmacro * g.rate;
    return (i == 0 || i == last) ? 0.5 * hg : hg;
}

// bootstrap forward: boot[0] = y0, RK steps at h, history slots filled from
// the first-stage derivatives; leaves the MRAB start state in ys[0] and the
// history in ring[]
int adj_boot_fwd(mr_ctx *c)
{
    AdjCtx &A = *c->adj;
    const int G = (int)c->G.size(), m = c->P.hist_len;
    const double d = c->h;
    std::vector<double *> Y(G), K(G);
    for (int n = 0; n <= A.nboot; ++n) {
        for (int g = 0; g < G; ++g) {
            Y[g] = gstate(A.G[g], c->G[g], A.G[g].boot, n);
            K[g] = A.G[g].kk[0];
        }
        int rc = adj_coupled_fwd(c, Y, 0, K);
        if (rc) return rc;
        for (int g = 0; g < G; ++g) {
            const GridHost &Gh = c->G[g];
            const int per = c->rmax / Gh.rate, back = A.nboot - n;
            if (back % per == 0 && back / per < m)
                HIPCHK(c, hipMemcpyAsync(A.G[g].ring[m - 1 - back / per], A.G[g].kk[0], nelem(Gh) * 8,
                                         hipMemcpyDeviceToDevice, c->st));
        }
        if (n == A.nboot) break;
        auto stage_in = [&](int k) {
            for (int g = 0; g < G; ++g) {
                Y[g] = A.G[g].stg[k];
                K[g] = A.G[g].kk[k];
            }
        };
        for (int g = 0; g < G; ++g) {
            const GridHost &Gh = c->G[g];
            double *y = gstate(A.G[g], Gh, A.G[g].boot, n);
            HIPCHK(c, mrk::launch_axpy(nelem(Gh), y, c->P.order <= 3 ? d / 3.0 : d / 2.0, A.G[g].kk[0],
                                       A.G[g].stg[1], c->st));
        }
        stage_in(1);
        if ((rc = adj_coupled_fwd(c, Y, 1, K))) return rc;
        if (c->P.order <= 3) {
            for (int g = 0; g < G; ++g) {
                const GridHost &Gh = c->G[g];
                double *y = gstate(A.G[g], Gh, A.G[g].boot, n);
                HIPCHK(c, mrk::launch_axpy(nelem(Gh), y, 2.0 * d / 3.0, A.G[g].kk[1], A.G[g].stg[2], c->st));
            }
            stage_in(2);
            if ((rc = adj_coupled_fwd(c, Y, 2, K))) return rc;
            for (int g = 0; g < G; ++g) {
                const GridHost &Gh = c->G[g];
                double *y = gstate(A.G[g], Gh, A.G[g].boot, n);
                HIPCHK(c, mrk::launch_rk3_final(nelem(Gh), y, d / 4.0, A.G[g].kk[0], A.G[g].kk[2],
                                                gstate(A.G[g], Gh, A.G[g].boot, n + 1), c->st));
            }
        } else {
            for (int g = 0; g < G; ++g) {
                const GridHost &Gh = c->G[g];
                double *y = gstate(A.G[g], Gh, A.G[g].boot, n);
                HIPCHK(c, mrk::launch_axpy(nelem(Gh), y, d / 2.0, A.G[g].kk[1], A.G[g].stg[2], c->st));
            }
            stage_in(2);
            if ((rc = adj_coupled_fwd(c, Y, 2, K))) return rc;
            for (int g = 0; g < G; ++g) {
                const GridHost &Gh = c->G[g];
                double *y = gstate(A.G[g], Gh, A.G[g].boot, n);
                HIPCHK(c, mrk::launch_axpy(nelem(Gh), y, d, A.G[g].kk[2], A.G[g].stg[3], c->st));
            }
            stage_in(3);
            if ((rc = adj_coupled_fwd(c, Y, 3, K))) return rc;
            for (int g = 0; g < G; ++g) {
                const GridHost &Gh = c->G[g];
                double *y = gstate(A.G[g], Gh, A.G[g].boot, n);
                HIPCHK(c, mrk::launch_rk4_final(nelem(Gh), y, d / 6.0, A.G[g].kk[0], A.G[g].kk[1], A.G[g].kk[2],
                                                A.G[g].kk[3], gstate(A.G[g], Gh, A.G[g].boot, n + 1), c->st));
            }
        }
    }
    for (int g = 0; g < G; ++g) {
        A.G[g].ys0 = 0;
        HIPCHK(c, hipMemcpyAsync(ysl(A.G[g], c->G[g], 0), gstate(A.G[g], c->G[g], A.G[g].boot, A.nboot),
                                 nelem(c->G[g]) * 8, hipMemcpyDeviceToDevice, c->st));
    }
    return adj_stage(c);
}

// bootstrap reverse: on entry lam_y / lam_ring hold the adjoint of the MRAB
// start state and history; on exit lam_y holds the adjoint of boot[0]
int adj_boot_rev(mr_ctx *c)
{
    AdjCtx &A = *c->adj;
    const int G = (int)c->G.size(), m = c->P.hist_len;
    const double d = c->h;
    std::vector<double *> Y(G), LK(G), LY(G), LS(G);
    for (int g = 0; g < G; ++g) {
        LY[g] = A.G[g].lam_y;
        LS[g] = A.G[g].lys;
    }
    for (int n = A.nboot; n >= 0; --n) {
        // recompute the stages of step n
        for (int g = 0; g < G; ++g) Y[g] = gstate(A.G[g], c->G[g], A.G[g].boot, n);
        if (n < A.nboot) {
            // rerun step n's stages (fills stg[1..], kk[0..] and receiver slices 0..3)
            std::vector<double *> K(G);
            for (int g = 0; g < G; ++g) K[g] = A.G[g].kk[0];
            int rc = adj_coupled_fwd(c, Y, 0, K);
            if (rc) return rc;
            const int ns = c->P.order <= 3 ? 3 : 4;
            for (int s = 1; s < ns; ++s) {
                double coef = c->P.order <= 3 ? (s == 1 ? d / 3.0 : 2.0 * d / 3.0) : (s == 3 ? d : d / 2.0);
                for (int g = 0; g < G; ++g) {
                    HIPCHK(c, mrk::launch_axpy(nelem(c->G[g]), Y[g], coef, A.G[g].kk[s - 1], A.G[g].stg[s], c->st));
                }
                std::vector<double *> Ys(G);
                for (int g = 0; g < G; ++g) {
                    Ys[g] = A.G[g].stg[s];
                    K[g] = A.G[g].kk[s];
                }
                if ((rc = adj_coupled_fwd(c, Ys, s, K))) return rc;
            }
        } else {
            std::vector<double *> K(G);
            for (int g = 0; g < G; ++g) K[g] = A.G[g].kk[0];
            int rc = adj_coupled_fwd(c, Y, 0, K);   // receiver rows of slice 0 at y_n
            if (rc) return rc;
        }
        // first-stage adjoint: the history slot filled at n
        for (int g = 0; g < G; ++g) {
            const GridHost &Gh = c->G[g];
            const int per = c->rmax / Gh.rate, back = A.nboot - n;
            if (back % per == 0 && back / per < m)
                HIPCHK(c, hipMemcpyAsync(A.G[g].lk[0], A.G[g].lam_ring[m - 1 - back / per], nelem(Gh) * 8,
                                         hipMemcpyDeviceToDevice, c->st));
            else
                HIPCHK(c, hipMemsetAsync(A.G[g].lk[0], 0, nelem(Gh) * 8, c->st));
            for (int k = 1; k < 4; ++k) HIPCHK(c, hipMemsetAsync(A.G[g].lk[k], 0, nelem(Gh) * 8, c->st));
        }
        if (n < A.nboot) {
            auto stage_rev = [&](int s, double *const *to, std::initializer_list<double> coef) -> int {
                // lys = f_s^T lk[s]; lam_y += lys; lk[to] += coef * lys
                std::vector<double *> Ys(G);
                for (int g = 0; g < G; ++g) {
                    Ys[g] = A.G[g].stg[s];
                    LK[g] = A.G[g].lk[s];
                    HIPCHK(c, hipMemsetAsync(LS[g], 0, nelem(c->G[g]) * 8, c->st));
                }
                int rc = adj_coupled_rev(c, Ys, s, LK, LS);
                if (rc) return rc;
                for (int g = 0; g < G; ++g) {
                    const double k = *coef.begin();
                    rc = adj_axpy(c, nelem(c->G[g]), LS[g], {LY[g], to[g]}, {1.0, k});
                    if (rc) return rc;
                }
                return MR_OK;
            };
            int rc;
            std::vector<double *> to(G);
            if (c->P.order <= 3) {
                for (int g = 0; g < G; ++g)
                    if ((rc = adj_axpy(c, nelem(c->G[g]), LY[g], {A.G[g].lk[0], A.G[g].lk[2]},
                                       {d / 4.0, 3.0 * d / 4.0})))
                        return rc;
                for (int g = 0; g < G; ++g) to[g] = A.G[g].lk[1];
                if ((rc = stage_rev(2, to.data(), {2.0 * d / 3.0}))) return rc;
                for (int g = 0; g < G; ++g) to[g] = A.G[g].lk[0];
                if ((rc = stage_rev(1, to.data(), {d / 3.0}))) return rc;
            } else {
                for (int g = 0; g < G; ++g)
                    if ((rc = adj_axpy(c, nelem(c->G[g]), LY[g], {A.G[g].lk[0], A.G[g].lk[1], A.G[g].lk[2],
                                                                  A.G[g].lk[3]},
                                       {d / 6.0, d / 3.0, d / 3.0, d / 6.0})))
                        return rc;
                for (int g = 0; g < G; ++g) to[g] = A.G[g].lk[2];
                if ((rc = stage_rev(3, to.data(), {d}))) return rc;
                for (int g = 0; g < G; ++g) to[g] = A.G[g].lk[1];
                if ((rc = stage_rev(2, to.data(), {d / 2.0}))) return rc;
                for (int g = 0; g < G; ++g) to[g] = A.G[g].lk[0];
                if ((rc = stage_rev(1, to.data(), {d / 2.0}))) return rc;
            }
        }
        for (int g = 0; g < G; ++g) LK[g] = A.G[g].lk[0];
        int rc = adj_coupled_rev(c, Y, 0, LK, LY);
        if (rc) return rc;
    }
    return MR_OK;
}

// one MRAB macrostep (index n of nmacro) from its start (ysl 0, the staged
// first own step in ysl 1) and ring[], leaving every own-step state in ysl
// 1..rate, the next macrostep's staged first step in ysl rate + 1, the
// extrapolants in ext[k-1] and the receiver rows in slice k-1; adds the
// objective terms when obj.  adj_advance then makes its end the next start.
int adj_macro_fwd(mr_ctx *c, int n, int nmacro, bool obj)
{
    AdjCtx &A = *c->adj;
    const int G = (int)c->G.size(), m = c->P.hist_len;
    for (int k = 1; k <= c->rmax; ++k) {
        bool ends[mrk::MAXG] = {};
        for (int g = 0; g < G; ++g) ends[g] = k % (c->rmax / c->G[g].rate) == 0;
        // own steps ending at k were staged by the grid's previous evaluation
        if (obj && A.og >= 0 && ends[A.og]) {
            const GridHost &Gh = c->G[A.og];
            const int e = k / (c->rmax / Gh.rate);
            HIPCHK(c, mrk::launch_obj(adj_obj(c), ysl(A.G[A.og], Gh, e), Gh.npts, adj_tau(c, n * Gh.rate + e, nmacro),
                                      A.acc, c->st));
        }
        bool made[mrk::MAXG] = {};
        for (const Link &L : c->links) {
            if (!ends[L.rg]) continue;
            const GridHost &D = c->G[L.dg];
            AdjGrid &a = A.G[L.dg];
            const int per_d = c->rmax / D.rate, e = k / per_d, jp = k % per_d;
            const double *Y = ysl(a, D, e);
            if (jp) {
                // the extrapolant at the points the donor kernels read (the
                // donor grid's stencil closure); other points are not used
                double *X = gstate(a, D, a.ext, k - 1);
                if (!made[L.dg]) {
                    mrk::Extrap x{};
                    x.y = Y;
                    x.m = m;
                    x.nv = D.dim + 2;
                    x.N = D.npts;
                    for (int j = 0; j < m; ++j) {
                        x.hist[j] = a.ring[j];
                        x.beta[0][j] = c->beta[L.dg][jp][j];
                    }
                    x.nj = 1;
                    x.out[0] = X;
                    x.pts = D.closure_d;
                    x.np = (int64_t)D.closure.size();
                    HIPCHK(c, mrk::launch_extrap(x, c->st));
                    made[L.dg] = true;
                }
                Y = X;
            }
            int rc = adj_donor_fwd(c, L, Y, rslice(c, c->G[L.rg], A.G[L.rg].recv, k - 1));
            if (rc) return rc;
        }
        for (int g = 0; g < G; ++g) {
            if (!ends[g]) continue;
            const GridHost &Gh = c->G[g];
            AdjGrid &a = A.G[g];
            const int e = k / (c->rmax / Gh.rate);
            // the right-hand side into the oldest history slot, fused with the
            // next own step from the newer slots and the new value
            mrk::Combine cb{};
            cb.m = m;
            for (int j = 0; j < m - 1; ++j) cb.hist[j] = a.ring[j + 1];
            for (int j = 0; j < m; ++j) cb.c[j] = c->c_own[g][j];
            cb.y_next = ysl(a, Gh, e + 1);
            int rc = adj_rhs_fwd(c, g, ysl(a, Gh, e), rslice(c, Gh, a.recv, k - 1), a.ring[0], cb);
            if (rc) return rc;
            std::rotate(a.ring, a.ring + 1, a.ring + m);   // the new value is the newest
        }
    }
    return MR_OK;
}

// the reverse of macrostep n, right after adj_macro_fwd of the same
// macrostep (ys[1..rate], ext[] and the receiver slices still hold its
// quantities; the start state in ys[0] is not needed); lam_y / lam_ring:
// adjoint of the end state and history in, of the start ones out
int adj_macro_rev(mr_ctx *c, int n, int nmacro, double jscale)
{
    AdjCtx &A = *c->adj;
    const int G = (int)c->G.size(), m = c->P.hist_len;
    for (int k = c->rmax; k >= 1; --k) {
        bool ends[mrk::MAXG] = {};
        for (int g = 0; g < G; ++g) ends[g] = k % (c->rmax / c->G[g].rate) == 0;
        for (int g = 0; g < G; ++g) {
            if (!ends[g]) continue;
            const GridHost &Gh = c->G[g];
            AdjGrid &a = A.G[g];
            const int e = k / (c->rmax / Gh.rate);
            // undo the push: the newest slot's adjoint is the new value's
            std::rotate(a.lam_ring, a.lam_ring + m - 1, a.lam_ring + m);
            int rc = adj_rhs_rev(c, g, ysl(a, Gh, e), rslice(c, Gh, a.recv, k - 1), a.lam_ring[0],
                                 rslice(c, Gh, a.lam_recv, k - 1), a.lam_y);
            if (rc) return rc;
            HIPCHK(c, hipMemsetAsync(a.lam_ring[0], 0, nelem(Gh) * 8, c->st));
            if (g == A.og && jscale != 0.0)
                HIPCHK(c, mrk::launch_obj_adj(adj_obj(c), ysl(a, Gh, e), Gh.npts,
                                              jscale * adj_tau(c, n * Gh.rate + e, nmacro), a.lam_y, c->st));
        }
        for (int li = (int)c->links.size() - 1; li >= 0; --li) {
            const Link &L = c->links[li];
            if (!ends[L.rg]) continue;
            const GridHost &D = c->G[L.dg];
            AdjGrid &a = A.G[L.dg];
            const int per_d = c->rmax / D.rate, e = k / per_d, jp = k % per_d;
            const double *lr = rslice(c, c->G[L.rg], A.G[L.rg].lam_recv, k - 1);
            int rc;
            if (!jp) {
                rc = adj_donor_rev(c, li, ysl(a, D, e), lr, a.lam_y);
                if (rc) return rc;
                continue;
            }
            // lam_ext is zero outside the stencil closure and is cleared there
            // after each use
            rc = adj_donor_rev(c, li, gstate(a, D, a.ext, k - 1), lr, a.lam_ext);
            if (rc) return rc;
            mrk::AdjExt x{};
            x.lam_ext = a.lam_ext;
            x.lam_y = a.lam_y;
            for (int j = 0; j < m; ++j) {
                x.lam_hist[j] = a.lam_ring[j];
                x.beta[j] = c->beta[L.dg][jp][j];
            }
            x.m = m;
            x.nv = D.dim + 2;
            x.N = D.npts;
            x.pts = D.closure_d;
            x.np = (int64_t)D.closure.size();
            HIPCHK(c, mrk::launch_adj_ext(x, c->st));
        }
        for (int g = 0; g < G; ++g) {
            if (!ends[g]) continue;
            AdjGrid &a = A.G[g];
            std::vector<double> coef(c->c_own[g].begin(), c->c_own[g].end());
            HIPCHK(c, mrk::launch_adj_axpy(nelem(c->G[g]), a.lam_y, m, a.lam_ring, coef.data(), c->st));
        }
    }
    return MR_OK;
}

// snapshot slot s <- / -> the MRAB quantities (the start state, ring); a
// restore stages the first own step
int adj_snap(mr_ctx *c, int s, bool store)
{
    AdjCtx &A = *c->adj;
    const int m = c->P.hist_len;
    for (size_t g = 0; g < c->G.size(); ++g) {
        const GridHost &Gh = c->G[g];
        AdjGrid &a = A.G[g];
        const size_t nb = nelem(Gh) * 8;
        double *base = gstate(a, Gh, a.snap, s * (1 + m));
        for (int j = 0; j <= m; ++j) {
            double *dev = j == 0 ? ysl(a, Gh, 0) : a.ring[j - 1];
            double *sn = base + (size_t)j * nelem(Gh);
            HIPCHK(c, hipMemcpyAsync(store ? sn : dev, store ? dev : sn, nb, hipMemcpyDeviceToDevice, c->st));
        }
    }
    return store ? MR_OK : adj_stage(c);
}

// minimal forward macrosteps to reverse l macrosteps from a stored start
// with s free snapshot slots, and the first split that attains it
struct Sched {
    std::vector<std::vector<int64_t>> cost;
    std::vector<std::vector<int>> split;
    void build(int L, int S)
    {
        cost.assign(L + 1, std::vector<int64_t>(S + 1, 0));
        split.assign(L + 1, std::vector<int>(S + 1, 0));
        for (int l = 1; l <= L; ++l)
            for (int s = 0; s <= S; ++s) {
                if (l == 1) {
                    cost[l][s] = 1;
                    continue;
                }
                if (s == 0) {
                    cost[l][s] = (int64_t)l * (l + 1) / 2;
                    continue;
                }
                int64_t best = INT64_MAX;
                int bj = 1;
                for (int j = 1; j < l; ++j) {
                    int64_t v = j + cost[l - j][s - 1] + cost[j][s];
                    if (v < best) {
                        best = v;
                        bj = j;
                    }
                }
                cost[l][s] = best;
                split[l][s] = bj;
            }
    }
};

// reverse macrosteps [a, b) of nmacro; the start of a is in slot sa; s free
// slots beyond it
int adj_reverse(mr_ctx *c, const Sched &S, int a, int b, int sa, int s, int nmacro, double jscale, int64_t &nfwd)
{
    AdjCtx &A = *c->adj;
    if (b - a == 1) {
        int rc = adj_snap(c, sa, false);
        if (rc) return rc;
        if ((rc = adj_macro_fwd(c, a, nmacro, false))) return rc;
        nfwd++;
        return adj_macro_rev(c, a, nmacro, jscale);
    }
    if (s == 0) {
        for (int i = b - 1; i >= a; --i) {
            int rc = adj_snap(c, sa, false);
            if (rc) return rc;
            for (int k = a; k < i; ++k) {
                if ((rc = adj_macro_fwd(c, k, nmacro, false))) return rc;
                adj_advance(c);
                nfwd++;
            }
            if ((rc = adj_macro_fwd(c, i, nmacro, false))) return rc;
            nfwd++;
            if ((rc = adj_macro_rev(c, i, nmacro, jscale))) return rc;
        }
        return MR_OK;
    }
    const int j = S.split[b - a][s];
    int slot = -1;
    for (int i = 0; i < A.nsnap; ++i)
        if (A.snap_pos[i] < 0) {
            slot = i;
            break;
        }
    if (slot < 0) return fail(c, MR_ERR_STATE, "no free snapshot slot");
    int rc = adj_snap(c, sa, false);
    if (rc) return rc;
    for (int k = a; k < a + j; ++k) {
        if ((rc = adj_macro_fwd(c, k, nmacro, false))) return rc;
        adj_advance(c);
        nfwd++;
    }
    if ((rc = adj_snap(c, slot, true))) return rc;
    A.snap_pos[slot] = a + j;
    if ((rc = adj_reverse(c, S, a + j, b, slot, s - 1, nmacro, jscale, nfwd))) return rc;
    A.snap_pos[slot] = -1;
    return adj_reverse(c, S, a, a + j, sa, s, nmacro, jscale, nfwd);
}

int adj_check(mr_ctx *c, int nmacro)
{
    if (!c->adj || !c->adj->bound) return fail(c, MR_ERR_STATE, "adjoint workspace not bound");
    if (int rc_ = need_bound(c, "the adjoint")) return rc_;
    if (!c->have_dt) return fail(c, MR_ERR_STATE, "no macrostep set (mr_timestep or mr_set_macrostep)");
    if (nmacro < 0) return fail(c, MR_ERR_ARG, "negative macrostep count");
    return MR_OK;
}

// the whole forward run: bootstrap from y0, nmacro macrosteps; objective
// accumulated into acc (zeroed first)
int adj_run_fwd(mr_ctx *c, const double *const *y0, int nmacro, bool obj)
{
    AdjCtx &A = *c->adj;
    for (size_t g = 0; g < c->G.size(); ++g)
        HIPCHK(c, hipMemcpyAsync(A.G[g].boot, y0[g], nelem(c->G[g]) * 8, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipMemsetAsync(A.acc, 0, 8, c->st));
    int rc = adj_boot_fwd(c);
    if (rc) return rc;
    if (obj && A.og >= 0 && !A.opts.empty())
        HIPCHK(c, mrk::launch_obj(adj_obj(c), ysl(A.G[A.og], c->G[A.og], 0), c->G[A.og].npts, adj_tau(c, 0, nmacro),
                                  A.acc, c->st));
    for (int n = 0; n < nmacro; ++n) {
        if ((rc = adj_macro_fwd(c, n, nmacro, obj && A.og >= 0))) return rc;
        adj_advance(c);
    }
    return MR_OK;
}

int adj_upload_objective(mr_ctx *c)
{
    AdjCtx &A = *c->adj;
    if (!A.bound || A.opts.empty()) return MR_OK;
    HIPCHK(c, hipMemcpyAsync(A.opts_d, A.opts.data(), A.opts.size() * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(A.ow_d, A.ow.data(), A.ow.size() * 8, hipMemcpyHostToDevice, c->st));
    return MR_OK;
}

}  // namespace

// =================================================================== C ABI
namespace {

// ---------------------------------------------------------------------------
// Chimera donor-receiver search (section "SAT-Based Interpolation": donor
// search, Lagrange interpolation weights from Lagrange shape functions)
// ---------------------------------------------------------------------------

// physical position of point p of grid g
void point_position(const GridHost &g, int64_t p, double *x)
{
    if (g.kind == MR_CURVILINEAR) {
        for (int c = 0; c < g.dim; ++c) x[c] = g.coords[(size_t)c * g.npts + p];
        return;
    }
    int64_t r = p;
    for (int d = 0; d < g.dim; ++d) {
        const int64_t i = r % g.n[d];
        r /= g.n[d];
        x[d] = g.origin[d] + g.spacing[d] * (double)i;
    }
}

// coordinates of the (possibly out-of-range, periodic) index i[] of a
// curvilinear grid: wrapped, plus the coordinate jump of each seam crossed
void curv_coord(const GridHost &g, const int64_t *i, double *x)
{
    int64_t p = 0;
    double shift[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < g.dim; ++d) {
        int64_t k = i[d];
        if (g.periodic[d]) {
            const int64_t w = ((k % g.n[d]) + g.n[d]) % g.n[d];
            const int64_t turns = (k - w) / g.n[d];
            for (int c = 0; c < g.dim; ++c) shift[c] += (double)turns * g.coord_period[d][c];
            k = w;
        }
        p += k * g.stride[d];
    }
    for (int c = 0; c < g.dim; ++c) x[c] = g.coords[(size_t)c * g.npts + p] + shift[c];
}

// 1D Lagrange shape functions of the nodes 0..W-1 at t, and their derivatives
void lagrange_shape(double t, int W, double *L, double *dL)
{
    for (int a = 0; a < W; ++a) {
        double v = 1.0, dv = 0.0;
        for (int b = 0; b < W; ++b) {
            if (b == a) continue;
            const double f = (t - b) / (double)(a - b);
            dv = dv * f + v / (double)(a - b);
            v *= f;
        }
        L[a] = v;
        if (dL) dL[a] = dv;
    }
}

// fractional index of x in curvilinear grid g, the library's own search: the
// nearest grid point starts a Newton iteration on the grid's coordinates
// interpolated by 4-point (fewer on short non-periodic lines) Lagrange
// polynomials per direction; false when it does not converge
bool locate_curvilinear(const GridHost &g, const double *x, double *f)
{
    const int dim = g.dim;
    int64_t best = 0;
    double bd = INFINITY;
    for (int64_t p = 0; p < g.npts; ++p) {
        double d2 = 0.0;
        for (int c = 0; c < dim; ++c) {
            const double e = g.coords[(size_t)c * g.npts + p] - x[c];
            d2 += e * e;
        }
        if (d2 < bd) {
            bd = d2;
            best = p;
        }
    }
    double s[3];
    for (int d = 0; d < dim; ++d) s[d] = (double)((best / g.stride[d]) % g.n[d]);
    int W[3];
    for (int d = 0; d < dim; ++d) W[d] = g.periodic[d] ? 4 : std::min(4, g.n[d]);
    int polish = -1;
    for (int it = 0; it < 60; ++it) {
        int64_t base[3];
        double L[3][4], dL[3][4];
        for (int d = 0; d < dim; ++d) {
            base[d] = (int64_t)std::floor(s[d]) - (W[d] / 2 - 1);
            if (!g.periodic[d]) base[d] = std::min<int64_t>(std::max<int64_t>(base[d], 0), g.n[d] - W[d]);
            lagrange_shape(s[d] - (double)base[d], W[d], L[d], dL[d]);
        }
        double X[3] = {0, 0, 0}, J[3][3] = {{0}};
        const int ne = dim == 2 ? W[0] * W[1] : W[0] * W[1] * W[2];
        for (int e = 0; e < ne; ++e) {
            int a[3] = {e % W[0], (e / W[0]) % W[1], dim == 3 ? e / (W[0] * W[1]) : 0};
            int64_t idx[3];
            for (int d = 0; d < dim; ++d) idx[d] = base[d] + a[d];
            double xc[3];
            curv_coord(g, idx, xc);
            double w = 1.0, dw[3];
            for (int d = 0; d < dim; ++d) w *= L[d][a[d]];
            for (int k = 0; k < dim; ++k) {
                dw[k] = 1.0;
                for (int d = 0; d < dim; ++d) dw[k] *= d == k ? dL[d][a[d]] : L[d][a[d]];
            }
            for (int c = 0; c < dim; ++c) {
                X[c] += w * xc[c];
                for (int k = 0; k < dim; ++k) J[c][k] += dw[k] * xc[c];
            }
        }
        // Newton step: solve J step = X - x (Gaussian elimination, partial pivoting)
        double A[3][4];
        for (int c = 0; c < dim; ++c) {
            for (int k = 0; k < dim; ++k) A[c][k] = J[c][k];
            A[c][dim] = X[c] - x[c];
        }
        for (int k = 0; k < dim; ++k) {
            int piv = k;
            for (int c = k + 1; c < dim; ++c)
                if (std::fabs(A[c][k]) > std::fabs(A[piv][k])) piv = c;
            if (!(std::fabs(A[piv][k]) > 0.0)) return false;
            if (piv != k)
                for (int j = 0; j <= dim; ++j) std::swap(A[k][j], A[piv][j]);
            for (int c = k + 1; c < dim; ++c) {
                const double m = A[c][k] / A[k][k];
                for (int j = k; j <= dim; ++j) A[c][j] -= m * A[k][j];
            }
        }
        double step[3], big = 0.0;
        for (int k = dim - 1; k >= 0; --k) {
            double v = A[k][dim];
            for (int j = k + 1; j < dim; ++j) v -= A[k][j] * step[j];
            step[k] = v / A[k][k];
            big = std::max(big, std::fabs(step[k]));
        }
        for (int d = 0; d < dim; ++d) s[d] -= step[d];
        for (int d = 0; d < dim; ++d)
            if (!std::isfinite(s[d]) || std::fabs(s[d]) > 4.0 * g.n[d] + 8.0) return false;
        if (polish > 0 && --polish == 0) break;
        if (polish < 0 && big < 1e-12) polish = 2;   // two more steps at the rounding floor
        if (it == 59) return false;
    }
    for (int d = 0; d < dim; ++d) {
        if (g.periodic[d]) s[d] = s[d] - std::floor(s[d] / g.n[d]) * g.n[d];
        f[d] = s[d];
    }
    return true;
}

}  // namespace

extern "C" {

int mr_create(const mr_params *params, void *hip_stream, mr_ctx **out)
{
    if (!params || !out) return MR_ERR_ARG;
    const mr_params &P = *params;
    if ((P.dim != 2 && P.dim != 3) || (P.sbp != 21 && P.sbp != 42) || P.order < 1 || P.order > 4 ||
        P.hist_len < P.order || P.hist_len > mrk::MAXH || !(P.gamma > 1.0) || !(P.Re > 0.0) || !(P.Pr > 0.0))
        return MR_ERR_ARG;
    mr_ctx *c = new mr_ctx();
    c->P = P;
    c->st = (hipStream_t)hip_stream;
    c->ph.gamma = P.gamma;
    c->ph.Re = P.Re;
    c->ph.Pr = P.Pr;
    c->ph.mu = P.mu;
    c->ph.lam = P.lambda_over_mu * P.mu;
    c->ph.sig_iface = P.sigma_I_iface;
    c->ph.sig_bc = P.sigma_I_bc;
    c->ph.T_wall = P.T_wall;
    c->ph.wall_visc = P.wall_visc;
    for (int v = 0; v < 5; ++v) c->ph.q_inf[v] = P.q_inf[v];
    c->ph.p0inv = P.sbp == 21 ? 2.0 : 48.0 / 17.0;
    *out = c;
    return MR_OK;
}

int mr_add_grid(mr_ctx *c, const mr_grid_desc *d, int *grid_id)
{
    if (!c || !d) return MR_ERR_ARG;
    if (c->finalized) return fail(c, MR_ERR_STATE, "mr_add_grid after mr_finalize");
    if ((int)c->G.size() >= mrk::MAXG) return fail(c, MR_ERR_ARG, "at most %d grids", mrk::MAXG);
    GridHost g;
    g.dim = c->P.dim;
    g.kind = d->kind;
    g.rate = d->rate;
    if (g.rate < 1) return fail(c, MR_ERR_SETUP, "rate must be >= 1");
    if (g.kind == MR_CURVILINEAR && g.dim != 2)
        return fail(c, MR_ERR_UNSUPPORTED, "curvilinear grids are supported in 2D only");
    if (g.kind != MR_CARTESIAN && g.kind != MR_CURVILINEAR) return fail(c, MR_ERR_ARG, "bad grid kind");
    g.npts = 1;
    for (int k = 0; k < 3; ++k) {
        g.n[k] = k < g.dim ? d->n[k] : 1;
        g.periodic[k] = k < g.dim ? (d->periodic[k] != 0) : 0;
        if (g.n[k] < 1) return fail(c, MR_ERR_ARG, "bad size");
        g.stride[k] = g.npts;
        g.npts *= g.n[k];
        g.origin[k] = d->origin[k];
        g.spacing[k] = d->spacing[k];
        for (int j = 0; j < 3; ++j) g.coord_period[k][j] = d->coord_period[k][j];
    }
    if (g.npts >= ((int64_t)1 << 31)) return fail(c, MR_ERR_ARG, "grid too large for 32-bit point indices");
    for (int k = 0; k < 2 * g.dim; ++k) {
        g.face_bc[k] = d->face_bc[k];
        if (g.face_bc[k] < 0 || g.face_bc[k] > 3) return fail(c, MR_ERR_ARG, "bad face flag");
    }
    if (g.kind == MR_CARTESIAN)
        for (int k = 0; k < g.dim; ++k)
            if (!(g.spacing[k] > 0)) return fail(c, MR_ERR_ARG, "bad spacing");
    if (g.kind == MR_CURVILINEAR) {
        if (!d->coords) return fail(c, MR_ERR_ARG, "curvilinear grid without coordinates");
        g.coords.assign(d->coords, d->coords + (size_t)g.dim * g.npts);
    }
    g.iblank.assign(g.npts, 1);
    if (d->iblank)
        for (int64_t p = 0; p < g.npts; ++p) g.iblank[p] = d->iblank[p] ? 1 : 0;
    int rc = classify(c, g);
    if (rc) return rc;
    c->G.push_back(std::move(g));
    if (grid_id) *grid_id = (int)c->G.size() - 1;
    return MR_OK;
}

int mr_set_overset(mr_ctx *c, int rg, int dg, int64_t n, int S, const int64_t *recv_pt, const int64_t *donor_pt,
                   const double *w)
{
    if (!c) return MR_ERR_ARG;
    if (c->finalized) return fail(c, MR_ERR_STATE, "mr_set_overset after mr_finalize");
    if (rg < 0 || rg >= (int)c->G.size() || dg < 0 || dg >= (int)c->G.size() || rg == dg)
        return fail(c, MR_ERR_ARG, "bad grid ids");
    if (n < 0 || (n > 0 && (!recv_pt || !donor_pt || !w))) return fail(c, MR_ERR_ARG, "bad arrays");
    if (S < 1 || S > 64 || (S & (S - 1))) return fail(c, MR_ERR_ARG, "stencil size must be a power of two <= 64");
    if (c->S && c->S != S) return fail(c, MR_ERR_ARG, "stencil size differs from an earlier call");
    c->S = S;
    GridHost &R = c->G[rg];
    GridHost &D = c->G[dg];
    Link L{rg, dg, (int64_t)c->rgrid.size(), n, (int32_t)R.recv_pts.size()};
    for (int64_t r = 0; r < n; ++r) {
        int64_t p = recv_pt[r];
        if (p < 0 || p >= R.npts) return fail(c, MR_ERR_ARG, "receiver index out of range");
        if (!R.iblank[p] || !is_iface(R, p))
            return fail(c, MR_ERR_SETUP, "point %lld of grid %d is not an interface run end", (long long)p, rg);
        if (R.recv_idx[p] >= 0) return fail(c, MR_ERR_SETUP, "receiver %lld registered twice", (long long)p);
        for (int e = 0; e < S; ++e) {
            int64_t q = donor_pt[r * S + e];
            if (q < 0 || q >= D.npts) return fail(c, MR_ERR_ARG, "donor index out of range");
            if (!D.iblank[q]) return fail(c, MR_ERR_SETUP, "donor point %lld of grid %d is blanked", (long long)q, dg);
        }
        R.recv_idx[p] = (int32_t)R.recv_pts.size();
        c->rgrid.push_back(rg);
        c->rrow.push_back((int32_t)R.recv_pts.size());
        R.recv_pts.push_back(p);
        for (int e = 0; e < S; ++e) {
            c->egrid.push_back((int8_t)dg);
            c->ept.push_back((int32_t)donor_pt[r * S + e]);
            c->ew.push_back(w[r * S + e]);
        }
    }
    if (n) c->links.push_back(L);
    return MR_OK;
}


int mr_assemble_overset(mr_ctx *c, int W, const int *priority, mr_locate_fn locate, void *user)
{
    if (!c || !priority) return MR_ERR_ARG;
    if (c->finalized) return fail(c, MR_ERR_STATE, "mr_assemble_overset after mr_finalize");
    if (W < 1 || W > 8) return fail(c, MR_ERR_ARG, "stencil width must be 1..8");
    const int G = (int)c->G.size();
    if (G == 0) return fail(c, MR_ERR_STATE, "no grids");
    const int dim = c->P.dim;
    int S = 1;
    for (int d = 0; d < dim; ++d) S *= W;
    if (S > 64 || (S & (S - 1))) return fail(c, MR_ERR_ARG, "width^dim must be a power of two of at most 64");
    for (const GridHost &g : c->G)
        for (int64_t p = 0; p < g.npts; ++p)
            if (g.recv_idx[p] >= 0) return fail(c, MR_ERR_STATE, "receivers already registered");
    std::vector<int> order(G);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return priority[a] > priority[b]; });
    for (int g = 0; g < G; ++g) {
        const GridHost &R = c->G[g];
        std::vector<int64_t> recv;
        for (int64_t p = 0; p < R.npts; ++p)
            if (R.iblank[p] && is_iface(R, p)) recv.push_back(p);
        const int64_t nr = (int64_t)recv.size();
        std::vector<double> X((size_t)dim * nr);
        for (int64_t r = 0; r < nr; ++r) {
            double x[3];
            point_position(R, recv[r], x);
            for (int k = 0; k < dim; ++k) X[(size_t)k * nr + r] = x[k];
        }
        std::vector<char> todo(nr, 1);
        int64_t left = nr;
        for (int dg : order) {
            if (dg == g || left == 0) continue;
            const GridHost &D = c->G[dg];
            std::vector<int64_t> sel;
            for (int64_t r = 0; r < nr; ++r)
                if (todo[r]) sel.push_back(r);
            const int64_t ns = (int64_t)sel.size();
            std::vector<double> xs((size_t)dim * ns), fs((size_t)dim * ns, NAN);
            for (int64_t k = 0; k < ns; ++k)
                for (int d = 0; d < dim; ++d) xs[(size_t)d * ns + k] = X[(size_t)d * nr + sel[k]];
            if (D.kind == MR_CARTESIAN) {
                for (int64_t k = 0; k < ns; ++k)
                    for (int d = 0; d < dim; ++d)
                        fs[(size_t)d * ns + k] = (xs[(size_t)d * ns + k] - D.origin[d]) / D.spacing[d];
            } else if (locate) {
                if (locate(user, dg, ns, xs.data(), fs.data()) != 0)
                    return fail(c, MR_ERR_SETUP, "the locate callback failed for donor grid %d", dg);
            } else {
                for (int64_t k = 0; k < ns; ++k) {
                    double x[3], f[3];
                    for (int d = 0; d < dim; ++d) x[d] = xs[(size_t)d * ns + k];
                    if (locate_curvilinear(D, x, f))
                        for (int d = 0; d < dim; ++d) fs[(size_t)d * ns + k] = f[d];
                }
            }
            std::vector<int64_t> hit_r, hit_p;
            std::vector<double> hit_w;
            for (int64_t k = 0; k < ns; ++k) {
                bool ok = true;
                int64_t ids[3][8];
                double w1[3][8];
                for (int d = 0; d < dim && ok; ++d) {
                    const double f = fs[(size_t)d * ns + k];
                    if (!std::isfinite(f)) {
                        ok = false;
                        break;
                    }
                    const int64_t b = (int64_t)std::floor(f) - (W / 2 - 1);
                    if (!D.periodic[d] && (b < 0 || b + W - 1 > D.n[d] - 1)) {
                        ok = false;
                        break;
                    }
                    for (int a = 0; a < W; ++a) {
                        int64_t i = b + a;
                        if (D.periodic[d]) i = ((i % D.n[d]) + D.n[d]) % D.n[d];
                        ids[d][a] = i;
                    }
                    // shape function a: the product over b != a of (s - b) / (a - b)
                    const double s = f - (double)b;
                    for (int a = 0; a < W; ++a) {
                        double v = 1.0;
                        for (int bb = 0; bb < W; ++bb)
                            if (bb != a) v *= (s - (double)bb) / (double)(a - bb);
                        w1[d][a] = v;
                    }
                }
                if (!ok) continue;
                int64_t pts[64];
                double wts[64];
                for (int e = 0; e < S && ok; ++e) {
                    int64_t q = 0;
                    double w = 1.0;
                    int rest = e;
                    for (int d = 0; d < dim; ++d) {
                        const int a = rest % W;
                        rest /= W;
                        q += ids[d][a] * D.stride[d];
                        w *= w1[d][a];
                    }
                    if (!D.iblank[q]) ok = false;
                    pts[e] = q;
                    wts[e] = w;
                }
                if (!ok) continue;
                hit_r.push_back(recv[sel[k]]);
                hit_p.insert(hit_p.end(), pts, pts + S);
                hit_w.insert(hit_w.end(), wts, wts + S);
                todo[sel[k]] = 0;
                --left;
            }
            if (!hit_r.empty()) {
                int rc = mr_set_overset(c, g, dg, (int64_t)hit_r.size(), S, hit_r.data(), hit_p.data(), hit_w.data());
                if (rc) return rc;
            }
        }
        if (left) return fail(c, MR_ERR_SETUP, "grid %d: %lld receivers without a donor", g, (long long)left);
    }
    return MR_OK;
}

int mr_get_overset(const mr_ctx *c, int g, int64_t *n, int64_t *recv_pt, int *donor_grid, int64_t *donor_pt,
                   double *weights)
{
    if (!c || !n || g < 0 || g >= (int)c->G.size()) return MR_ERR_ARG;
    const GridHost &R = c->G[g];
    const int64_t k = (int64_t)R.recv_pts.size();
    if (!recv_pt && !donor_grid && !donor_pt && !weights) {
        *n = k;
        return MR_OK;
    }
    if (*n < k) return MR_ERR_ARG;
    const int S = c->S ? c->S : 1;
    for (size_t r = 0; r < c->rgrid.size(); ++r) {
        if (c->rgrid[r] != g) continue;
        const int32_t row = c->rrow[r];
        if (recv_pt) recv_pt[row] = R.recv_pts[row];
        if (donor_grid) donor_grid[row] = c->egrid[r * S];
        for (int e = 0; e < S; ++e) {
            if (donor_pt) donor_pt[(int64_t)row * S + e] = c->ept[r * S + e];
            if (weights) weights[(int64_t)row * S + e] = c->ew[r * S + e];
        }
    }
    *n = k;
    return MR_OK;
}

int mr_finalize(mr_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return MR_ERR_ARG;
    if (c->finalized) return fail(c, MR_ERR_STATE, "mr_finalize called twice");
    if (c->G.empty()) return fail(c, MR_ERR_STATE, "no grids");
    for (size_t g = 0; g < c->G.size(); ++g)
        if ((int64_t)c->G[g].recv_pts.size() != c->G[g].n_iface)
            return fail(c, MR_ERR_SETUP, "grid %zu: %lld interface run ends but %zu receivers with donors", g,
                        (long long)c->G[g].n_iface, c->G[g].recv_pts.size());
    if (c->S == 0) c->S = 1;
    c->rmax = 1;
    for (auto &g : c->G) c->rmax = std::max(c->rmax, g.rate);
    if (c->rmax > 63) return fail(c, MR_ERR_SETUP, "largest rate above 63");
    for (auto &g : c->G)
        if (c->rmax % g.rate) return fail(c, MR_ERR_SETUP, "rate %d does not divide %d", g.rate, c->rmax);
    int n = c->P.order, m = c->P.hist_len;
    // a grid's ring head returns after m / gcd(m, rate) macrosteps, its
    // state double buffer after 2 / gcd(2, rate)
    c->period = 1;
    for (auto &g : c->G) c->period = std::lcm(c->period, std::lcm(m / std::gcd(m, g.rate), 2 / std::gcd(2, g.rate)));
    c->alpha_own.assign(c->G.size(), {});
    c->alpha_mid.assign(c->G.size(), {});
    for (size_t g = 0; g < c->G.size(); ++g) {
        if (!ab_alpha(n, m, 1.0L, c->alpha_own[g])) return fail(c, MR_ERR_SETUP, "AB coefficients");
        int per = c->rmax / c->G[g].rate;
        c->alpha_mid[g].assign(per, {});
        for (int jp = 1; jp < per; ++jp)
            if (!ab_alpha(n, m, (long double)jp / (long double)per, c->alpha_mid[g][jp]))
                return fail(c, MR_ERR_SETUP, "AB coefficients");
    }
    for (size_t g = 0; g < c->G.size(); ++g)
        if (c->G[g].rate < c->rmax) build_closure(c, (int)g, c->G[g]);
    for (auto &g : c->G) {
        g.satpts.clear();
        if (g.dim != 3) continue;
        for (int64_t p = 0; p < g.npts; ++p) {
            if ((g.cls[p] & 15) == mrk::CLS_HOLE) continue;
            bool any = false;
            for (int d = 0; d < g.dim; ++d) any = any || ((g.cls[(size_t)d * g.npts + p] >> 4) & 3) != 0;
            if (any) g.satpts.push_back((int32_t)p);
        }
    }
    c->euid.assign(c->ept.size(), 0);
    for (Link &L : c->links) {
        size_t e0 = (size_t)L.first * c->S, e1 = (size_t)(L.first + L.n) * c->S;
        L.upts.assign(c->ept.begin() + e0, c->ept.begin() + e1);
        std::sort(L.upts.begin(), L.upts.end());
        L.upts.erase(std::unique(L.upts.begin(), L.upts.end()), L.upts.end());
        for (size_t e = e0; e < e1; ++e)
            c->euid[e] = (int32_t)(std::lower_bound(L.upts.begin(), L.upts.end(), c->ept[e]) - L.upts.begin());
        build_blocks(c, L);
    }
    c->ws_bytes = layout(c, nullptr);
    c->finalized = true;
    *bytes = c->ws_bytes;
    return MR_OK;
}

}  // extern "C"

namespace {

// clear the workspace, upload the tables, compute the metric terms
int bind_at(mr_ctx *c, void *dev)
{
    c->ws = (char *)dev;
    layout(c, c->ws);
    HIPCHK(c, hipMemsetAsync(c->ws, 0, c->ws_bytes, c->st));
    std::vector<GridDev> devs;
    for (size_t gi = 0; gi < c->G.size(); ++gi) {
        GridHost &g = c->G[gi];
        HIPCHK(c, hipMemcpyAsync(g.cls_d, g.cls.data(), g.cls.size(), hipMemcpyHostToDevice, c->st));
        if (!g.recv_pts.empty())
            HIPCHK(c, hipMemcpyAsync(g.recv_idx_d, g.recv_idx.data(), g.recv_idx.size() * 4, hipMemcpyHostToDevice,
                                     c->st));
        if (!g.closure.empty())
            HIPCHK(c, hipMemcpyAsync(g.closure_d, g.closure.data(), g.closure.size() * 4, hipMemcpyHostToDevice,
                                     c->st));
        if (!g.satpts.empty())
            HIPCHK(c, hipMemcpyAsync(g.satpts_d, g.satpts.data(), g.satpts.size() * 4, hipMemcpyHostToDevice,
                                     c->st));
        GridDev &D = g.dev;
        D.dim = g.dim;
        D.nv = g.dim + 2;
        for (int k = 0; k < 3; ++k) {
            D.n[k] = g.n[k];
            D.periodic[k] = g.periodic[k];
            D.stride[k] = g.stride[k];
            D.inv_h[k] = 1.0 / g.spacing[k];
        }
        D.npts = g.npts;
        D.cartesian = g.kind == MR_CARTESIAN;
        D.metric = g.metric;
        D.cls = g.cls_d;
        D.recv_idx = g.recv_idx_d;
        D.recv = g.recv_buf;
        if (g.kind == MR_CURVILINEAR) {
            HIPCHK(c, hipMemcpyAsync(g.coords_d, g.coords.data(), g.coords.size() * 8, hipMemcpyHostToDevice, c->st));
            double per[2][2] = {{g.coord_period[0][0], g.coord_period[0][1]}, {g.coord_period[1][0], g.coord_period[1][1]}};
            HIPCHK(c, mrk::launch_metrics2d(D, c->P.sbp, g.coords_d, g.coords_d + g.npts, per, g.metric, c->st));
        }
        devs.push_back(D);
    }
    size_t R = c->rgrid.size();
    if (R) {
        HIPCHK(c, hipMemcpyAsync(c->euid_d, c->euid.data(), R * c->S * 4, hipMemcpyHostToDevice, c->st));
        HIPCHK(c, hipMemcpyAsync(c->ew_d, c->ew.data(), R * c->S * 8, hipMemcpyHostToDevice, c->st));
    }
    for (Link &L : c->links) {
        HIPCHK(c, hipMemcpyAsync(L.upts_d, L.upts.data(), L.upts.size() * 4, hipMemcpyHostToDevice, c->st));
        if (!L.bup.empty())
            HIPCHK(c, hipMemcpyAsync(L.bup_d, L.bup.data(), L.bup.size() * 4, hipMemcpyHostToDevice, c->st));
        if (!L.bcp.empty())
            HIPCHK(c, hipMemcpyAsync(L.bcp_d, L.bcp.data(), L.bcp.size() * 4, hipMemcpyHostToDevice, c->st));
        if (!L.bel.empty())
            HIPCHK(c, hipMemcpyAsync(L.bel_d, L.bel.data(), L.bel.size() * 2, hipMemcpyHostToDevice, c->st));
        if (!L.bpos.empty())
            HIPCHK(c, hipMemcpyAsync(L.bpos_d, L.bpos.data(), L.bpos.size() * 2, hipMemcpyHostToDevice, c->st));
    }
    HIPCHK(c, hipMemcpyAsync(c->grids_d, devs.data(), devs.size() * sizeof(GridDev), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->bound = true;
    return MR_OK;
}

}  // namespace

extern "C" {

int mr_bind_workspace(mr_ctx *c, void *dev, size_t bytes)
{
    if (!c || !dev) return MR_ERR_ARG;
    if (!c->finalized) return fail(c, MR_ERR_STATE, "mr_bind_workspace before mr_finalize");
    if (c->bound) return fail(c, MR_ERR_STATE, "workspace already bound");
    if (bytes < c->ws_bytes) return fail(c, MR_ERR_ARG, "workspace too small (%zu < %zu)", bytes, c->ws_bytes);
    if ((uintptr_t)dev % ALIGN) return fail(c, MR_ERR_ARG, "workspace not 256-byte aligned");
    return bind_at(c, dev);
}

int mr_bind_static_workspace(mr_ctx *c)
{
    if (!c) return MR_ERR_ARG;
    if (!c->finalized) return fail(c, MR_ERR_STATE, "mr_bind_static_workspace before mr_finalize");
    if (c->bound) return fail(c, MR_ERR_STATE, "workspace already bound");
    if (c->ws_bytes > MR_STATIC_WORKSPACE_BYTES)
        return fail(c, MR_ERR_ARG,
                    "workspace of %zu bytes exceeds the static workspace (%zu bytes): bind caller memory "
                    "with mr_bind_workspace",
                    c->ws_bytes, (size_t)MR_STATIC_WORKSPACE_BYTES);
    int dev = 0;
    if (c->st) {
        HIPCHK(c, hipStreamGetDevice(c->st, &dev));
    } else {
        HIPCHK(c, hipGetDevice(&dev));
    }
    void *p = nullptr;
    HIPCHK(c, mrk::static_workspace(dev, &p));
    {
        // the previous holder's later calls fail; it must not be running now
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_holder[dev] = c;
    }
    c->static_dev = dev;
    return bind_at(c, p);
}

int mr_set_state(mr_ctx *c, int g, const double *q)
{
    if (!c || !q || g < 0 || g >= (int)c->G.size()) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_set_state")) return rc_;
    GridHost &G = c->G[g];
    HIPCHK(c, hipMemcpyAsync(G.y[G.cur], q, nelem(G) * 8, hipMemcpyDeviceToDevice, c->st));
    c->stale = true;
    return MR_OK;
}

int mr_get_state(mr_ctx *c, int g, double *q)
{
    if (!c || !q || g < 0 || g >= (int)c->G.size()) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_get_state")) return rc_;
    GridHost &G = c->G[g];
    HIPCHK(c, hipMemcpyAsync(q, G.y[G.cur], nelem(G) * 8, hipMemcpyDeviceToDevice, c->st));
    return MR_OK;
}

int mr_rhs(mr_ctx *c, double, const double *const *q, double *const *F)
{
    if (!c || !q || !F) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_rhs")) return rc_;
    for (size_t g = 0; g < c->G.size(); ++g)
        if (!q[g] || !F[g]) return fail(c, MR_ERR_ARG, "null state or output pointer");
    return rhs_all(c, q, F);
}

int mr_num_receivers(const mr_ctx *c, int g, int64_t *n)
{
    if (!c || !n || g < 0 || g >= (int)c->G.size()) return MR_ERR_ARG;
    *n = (int64_t)c->G[g].recv_pts.size();
    return MR_OK;
}

int mr_receiver_data(mr_ctx *c, int g, const double *const *q, double *out)
{
    if (!c || !q || !out || g < 0 || g >= (int)c->G.size()) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_receiver_data")) return rc_;
    for (const Link &L : c->links) {
        if (L.rg != g) continue;
        if (!q[L.dg]) return fail(c, MR_ERR_ARG, "null donor state");
        int rc = link_current(c, L, q[L.dg], out, -1, 1);
        if (rc) return rc;
    }
    return MR_OK;
}

int mr_timestep(mr_ctx *c, double *h, double *H)
{
    if (c) c->version++;
    if (!c) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_timestep")) return rc_;
    double Hm;
    if (c->P.dt_fixed > 0) {
        Hm = c->P.dt_fixed;
    } else {
        Hm = INFINITY;
        for (auto &g : c->G) {
            HIPCHK(c, mrk::launch_dt(g.dev, c->ph, g.y[g.cur], g.dt, c->st));
            int nb = 256;
            HIPCHK(c, mrk::launch_reduce(g.npts, g.dt, 0, c->partial, nb, c->st));
            HIPCHK(c, mrk::launch_reduce(nb, c->partial, 0, c->partial + 512, 1, c->st));
            double v = 0;
            HIPCHK(c, hipMemcpyAsync(&v, c->partial + 512, 8, hipMemcpyDeviceToHost, c->st));
            HIPCHK(c, hipStreamSynchronize(c->st));
            Hm = std::min(Hm, g.rate * v);
        }
        Hm *= c->P.cfl;
    }
    int rc = set_macrostep(c, Hm);
    if (rc) return rc;
    if (h) *h = c->h;
    if (H) *H = c->H;
    return MR_OK;
}

int mr_mrab_start(mr_ctx *c, double t0)
{
    if (c) c->version++;
    if (!c) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_mrab_start")) return rc_;
    if (!c->have_dt) {
        int rc = mr_timestep(c, nullptr, nullptr);
        if (rc) return rc;
    }
    int m = c->P.hist_len;
    int G = (int)c->G.size();
    double d = c->h;
    int nsteps = (m - 1) * c->rmax;
    std::vector<const double *> qv(G);
    std::vector<double *> fv(G);
    auto stage = [&](int which_q, int k) {   // which_q: 0 = y, 1 = rk[4] (ytmp)
        for (int g = 0; g < G; ++g) {
            qv[g] = which_q ? c->G[g].rk[4] : c->G[g].y[c->G[g].cur];
            fv[g] = c->G[g].rk[k];
        }
        return rhs_all(c, qv.data(), fv.data());
    };
    for (auto &g : c->G) g.head = m - 1;
    for (int n = 0; n <= nsteps; ++n) {
        int rc = stage(0, 0);
        if (rc) return rc;
        for (int g = 0; g < G; ++g) {
            GridHost &Gh = c->G[g];
            int per = c->rmax / Gh.rate;
            int back = nsteps - n;
            if (back % per == 0 && back / per < m) {
                int j = m - 1 - back / per;
                HIPCHK(c, hipMemcpyAsync(slot(c, Gh, j), Gh.rk[0], nelem(Gh) * 8, hipMemcpyDeviceToDevice, c->st));
            }
        }
        if (n == nsteps) break;
        if (c->P.order <= 3) {
            for (auto &g : c->G) HIPCHK(c, mrk::launch_axpy(nelem(g), g.y[g.cur], d / 3.0, g.rk[0], g.rk[4], c->st));
            if ((rc = stage(1, 1))) return rc;
            for (auto &g : c->G)
                HIPCHK(c, mrk::launch_axpy(nelem(g), g.y[g.cur], 2.0 * d / 3.0, g.rk[1], g.rk[4], c->st));
            if ((rc = stage(1, 2))) return rc;
            for (auto &g : c->G)
                HIPCHK(c, mrk::launch_rk3_final(nelem(g), g.y[g.cur], d / 4.0, g.rk[0], g.rk[2], g.y[g.cur], c->st));
        } else {
            for (auto &g : c->G) HIPCHK(c, mrk::launch_axpy(nelem(g), g.y[g.cur], d / 2.0, g.rk[0], g.rk[4], c->st));
            if ((rc = stage(1, 1))) return rc;
            for (auto &g : c->G) HIPCHK(c, mrk::launch_axpy(nelem(g), g.y[g.cur], d / 2.0, g.rk[1], g.rk[4], c->st));
            if ((rc = stage(1, 2))) return rc;
            for (auto &g : c->G) HIPCHK(c, mrk::launch_axpy(nelem(g), g.y[g.cur], d, g.rk[2], g.rk[4], c->st));
            if ((rc = stage(1, 3))) return rc;
            for (auto &g : c->G)
                HIPCHK(c, mrk::launch_rk4_final(nelem(g), g.y[g.cur], d / 6.0, g.rk[0], g.rk[1], g.rk[2], g.rk[3],
                                                 g.y[g.cur], c->st));
        }
    }
    int rc = restage(c);
    if (rc) return rc;
    c->t = t0 + nsteps * d;
    c->nmacro = 0;
    c->started = true;
    c->stale = false;
    return MR_OK;
}

int mr_mrab_macrostep(mr_ctx *c, int nsteps)
{
    if (!c || nsteps < 0) return MR_ERR_ARG;
    if (!c->started) return fail(c, MR_ERR_STATE, "mr_mrab_macrostep before mr_mrab_start");
    if (int rc_ = need_bound(c, "mr_mrab_macrostep")) return rc_;
    if (c->stale) return fail(c, MR_ERR_STATE, "state or history set: call mr_mrab_resume or mr_mrab_start first");
    if (nsteps == 0) return MR_OK;
    int64_t npts = 0;
    for (auto &g : c->G) npts += g.npts;
    const bool ms = c->G.size() > 1 && (c->multi_stream < 0 ? npts >= kMultiStreamPoints : c->multi_stream == 1);
    if (ms) {
        int rc = ensure_streams(c);
        if (rc) return rc;
    }
    return run_macrosteps(c, nsteps, ms, c->st, c->eager);
}

int mr_set_macrostep(mr_ctx *c, double H)
{
    if (c) c->version++;
    if (!c) return MR_ERR_ARG;
    if (!c->finalized) return fail(c, MR_ERR_STATE, "mr_set_macrostep before mr_finalize");
    int rc = set_macrostep(c, H);
    if (rc) return rc;
    c->stale = true;          // the staged own steps used the old coefficients
    return MR_OK;
}

int mr_set_history(mr_ctx *c, int g, int j, const double *in)
{
    if (!c || !in || g < 0 || g >= (int)c->G.size() || j < 0 || j >= c->P.hist_len) return MR_ERR_ARG;
    if (!c->started) return fail(c, MR_ERR_STATE, "mr_set_history before mr_mrab_start");
    if (int rc_ = need_bound(c, "mr_set_history")) return rc_;
    GridHost &G = c->G[g];
    HIPCHK(c, hipMemcpyAsync(slot(c, G, j), in, nelem(G) * 8, hipMemcpyDeviceToDevice, c->st));
    c->stale = true;
    return MR_OK;
}

int mr_mrab_resume(mr_ctx *c, double t)
{
    if (c) c->version++;
    if (!c) return MR_ERR_ARG;
    if (!c->started) return fail(c, MR_ERR_STATE, "mr_mrab_resume before mr_mrab_start");
    if (int rc_ = need_bound(c, "mr_mrab_resume")) return rc_;
    int rc = restage(c);
    if (rc) return rc;
    c->t = t;
    c->nmacro = 0;
    c->stale = false;
    return MR_OK;
}

int mr_get_history(mr_ctx *c, int g, int j, double *out)
{
    if (!c || !out || g < 0 || g >= (int)c->G.size() || j < 0 || j >= c->P.hist_len) return MR_ERR_ARG;
    if (!c->started) return fail(c, MR_ERR_STATE, "mr_get_history before mr_mrab_start");
    if (int rc_ = need_bound(c, "mr_get_history")) return rc_;
    GridHost &G = c->G[g];
    HIPCHK(c, hipMemcpyAsync(out, slot(c, G, j), nelem(G) * 8, hipMemcpyDeviceToDevice, c->st));
    return MR_OK;
}

int mr_time(const mr_ctx *c, double *t, int64_t *ms)
{
    if (!c) return MR_ERR_ARG;
    if (t) *t = c->t;
    if (ms) *ms = c->nmacro;
    return MR_OK;
}

int mr_ab_coeffs(int order, int hist_len, double spacing, double tau, double *out)
{
    if (!out || !(tau > 0.0) || tau > 1.0 || !(spacing > 0.0) || !std::isfinite(spacing)) return MR_ERR_ARG;
    std::vector<long double> a;
    if (!ab_alpha(order, hist_len, (long double)tau, a)) return MR_ERR_ARG;
    for (int j = 0; j < hist_len; ++j) out[j] = (double)a[j] * spacing;
    return MR_OK;
}

int mr_kernel_timing(mr_ctx *c, int grid, int max_events)
{
    if (!c || grid < -2 || grid >= (int)c->G.size() || max_events < 0) return MR_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (auto e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    c->tgrid = max_events ? grid : -1;
    c->tmax = max_events;
    c->tcount = 0;
    c->tgrid_of.assign(max_events, -1);
    for (int i = 0; i < 2 * max_events; ++i) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->ev.push_back(e);
    }
    return MR_OK;
}

int mr_kernel_time_grid(mr_ctx *c, int grid, double *total_ms, int *count)
{
    if (!c || !total_ms || !count || grid < -1 || grid >= (int)c->G.size()) return MR_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->st));
    double tot = 0;
    int n = 0;
    for (int i = 0; i < c->tcount; ++i) {
        if (grid >= 0 && c->tgrid_of[i] != grid) continue;
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
        tot += ms;
        n++;
    }
    *total_ms = tot;
    *count = n;
    return MR_OK;
}

int mr_kernel_time(mr_ctx *c, double *total_ms, int *count) { return mr_kernel_time_grid(c, -1, total_ms, count); }

}  // extern "C"

namespace {
// ---- checkpoints: 256-byte header, then per grid the state and the history
// values oldest first
// checkpoint header (256 bytes): the problem it belongs to (scheme, and per
// grid its sizes and rate) and the integrator's time, macrostep count and H
struct SaveHeader {
    char magic[8];
    uint32_t version, ngrids;
    int32_t hist_len, dim;
    double t, H;
    int64_t nmacro, npts_total;
    uint64_t bytes;
    int32_t sbp, order;
    int32_t grid[mrk::MAXG][4];   // n[0..2], rate
    char pad[256 - 64 - 8 - 16 * mrk::MAXG];
};

void save_problem(const mr_ctx *c, SaveHeader &h)
{
    h.sbp = c->P.sbp;
    h.order = c->P.order;
    for (size_t g = 0; g < c->G.size(); ++g) {
        for (int k = 0; k < 3; ++k) h.grid[g][k] = c->G[g].n[k];
        h.grid[g][3] = c->G[g].rate;
    }
}
static_assert(sizeof(SaveHeader) == 256, "checkpoint header size");

size_t save_bytes(const mr_ctx *c)
{
    size_t b = sizeof(SaveHeader);
    for (const GridHost &g : c->G) b += (size_t)(1 + c->P.hist_len) * nelem(g) * 8;
    return b;
}

int64_t npts_total(const mr_ctx *c)
{
    int64_t n = 0;
    for (const GridHost &g : c->G) n += g.npts;
    return n;
}

}  // namespace

extern "C" {

int mr_save_bytes(const mr_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return MR_ERR_ARG;
    *bytes = save_bytes(c);
    return MR_OK;
}

int mr_save(mr_ctx *c, void *dev, size_t bytes)
{
    if (!c || !dev) return MR_ERR_ARG;
    if (!c->started) return fail(c, MR_ERR_STATE, "mr_save before mr_mrab_start");
    if (int rc_ = need_bound(c, "mr_save")) return rc_;
    if (c->stale) return fail(c, MR_ERR_STATE, "state or history set since the last start/resume");
    const size_t need = save_bytes(c);
    if (bytes < need) return fail(c, MR_ERR_ARG, "checkpoint buffer too small (%zu < %zu)", bytes, need);
    if ((uintptr_t)dev % 8) return fail(c, MR_ERR_ARG, "checkpoint buffer not 8-byte aligned");
    SaveHeader h{};
    std::memcpy(h.magic, "MRABSAVE", 8);
    h.version = 2;
    h.ngrids = (uint32_t)c->G.size();
    save_problem(c, h);
    h.hist_len = c->P.hist_len;
    h.dim = c->P.dim;
    h.t = c->t;
    h.H = c->H;
    h.nmacro = c->nmacro;
    h.npts_total = npts_total(c);
    h.bytes = need;
    char *p = (char *)dev;
    HIPCHK(c, hipMemcpyAsync(p, &h, sizeof h, hipMemcpyHostToDevice, c->st));
    p += sizeof h;
    for (const GridHost &g : c->G) {
        const size_t nb = nelem(g) * 8;
        HIPCHK(c, hipMemcpyAsync(p, g.y[g.cur], nb, hipMemcpyDeviceToDevice, c->st));
        p += nb;
        for (int j = 0; j < c->P.hist_len; ++j) {
            HIPCHK(c, hipMemcpyAsync(p, slot(c, g, j), nb, hipMemcpyDeviceToDevice, c->st));
            p += nb;
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    return MR_OK;
}

int mr_load(mr_ctx *c, const void *dev, size_t bytes)
{
    if (c) c->version++;
    if (!c || !dev) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_load")) return rc_;
    if (bytes < sizeof(SaveHeader)) return fail(c, MR_ERR_ARG, "checkpoint buffer too small");
    if ((uintptr_t)dev % 8) return fail(c, MR_ERR_ARG, "checkpoint buffer not 8-byte aligned");
    SaveHeader h{};
    HIPCHK(c, hipStreamSynchronize(c->st));
    HIPCHK(c, hipMemcpy(&h, dev, sizeof h, hipMemcpyDeviceToHost));
    if (std::memcmp(h.magic, "MRABSAVE", 8) || h.version != 2) return fail(c, MR_ERR_SETUP, "not a checkpoint");
    SaveHeader mine{};
    save_problem(c, mine);
    if (h.ngrids != c->G.size() || h.hist_len != c->P.hist_len || h.dim != c->P.dim ||
        h.npts_total != npts_total(c) || h.bytes != save_bytes(c) || h.sbp != mine.sbp || h.order != mine.order ||
        std::memcmp(h.grid, mine.grid, sizeof h.grid))
        return fail(c, MR_ERR_SETUP, "checkpoint of a different problem (scheme, grid sizes or rates differ)");
    if (bytes < h.bytes) return fail(c, MR_ERR_ARG, "checkpoint buffer shorter than its header states");
    int rc = set_macrostep(c, h.H);
    if (rc) return rc;
    const char *p = (const char *)dev + sizeof h;
    for (GridHost &g : c->G) {
        const size_t nb = nelem(g) * 8;
        HIPCHK(c, hipMemcpyAsync(g.y[g.cur], p, nb, hipMemcpyDeviceToDevice, c->st));
        p += nb;
        for (int j = 0; j < c->P.hist_len; ++j) {
            HIPCHK(c, hipMemcpyAsync(slot(c, g, j), p, nb, hipMemcpyDeviceToDevice, c->st));
            p += nb;
        }
    }
    if ((rc = restage(c))) return rc;
    c->t = h.t;
    c->nmacro = h.nmacro;
    c->started = true;
    c->stale = false;
    HIPCHK(c, hipStreamSynchronize(c->st));
    return MR_OK;
}

int mr_set_option(mr_ctx *c, const char *name, int64_t value)
{
    if (c) c->version++;
    if (!c || !name) return MR_ERR_ARG;
    if (!strcmp(name, "rhs_two_pass")) {
        if (value != 0 && value != 1) return fail(c, MR_ERR_ARG, "rhs_two_pass must be 0 or 1");
        c->two_pass = value != 0;
    } else if (!strcmp(name, "multi_stream")) {
        if (value != 0 && value != 1) return fail(c, MR_ERR_ARG, "multi_stream must be 0 or 1");
        c->multi_stream = (int)value;
    } else if (!strcmp(name, "donor_blocks")) {
        if (value != 0 && value != 1) return fail(c, MR_ERR_ARG, "donor_blocks must be 0 or 1");
        c->donor_blocks = value != 0;
    } else if (!strcmp(name, "tile3d_slab")) {
        if (value < 0 || value > 1024) return fail(c, MR_ERR_ARG, "tile3d_slab must be 0 .. 1024");
        c->slab3d = (int)value;
    } else if (!strcmp(name, "grad_tile3d")) {
        if (value < -1 || value >= mrk::NUM_TILE3D_SHAPES)
            return fail(c, MR_ERR_ARG, "grad_tile3d must be -1 .. %d", mrk::NUM_TILE3D_SHAPES - 1);
        c->gtile3d = (int)value;
    } else if (!strcmp(name, "rhs_tile3d")) {
        if (value < -1 || value >= mrk::NUM_TILE3D_SHAPES)
            return fail(c, MR_ERR_ARG, "rhs_tile3d must be -1 .. %d", mrk::NUM_TILE3D_SHAPES - 1);
        c->tile3d = (int)value;
    } else if (!strcmp(name, "flux3d")) {
        if (value < 0 || value > 3) return fail(c, MR_ERR_ARG, "flux3d must be 0 .. 3");
        c->flux3d = (int)value;
    } else if (!strcmp(name, "zchunk3d")) {
        if (value < 0 || value > 4096) return fail(c, MR_ERR_ARG, "zchunk3d must be 0 .. 4096");
        c->zchunk3d = (int)value;
    } else if (!strcmp(name, "ride_donors")) {
        if (value != 0 && value != 1) return fail(c, MR_ERR_ARG, "ride_donors must be 0 or 1");
        c->ride_donors = value == 1;
    } else if (!strcmp(name, "graph")) {
        if (value != 0 && value != 1) return fail(c, MR_ERR_ARG, "graph must be 0 or 1");
        if (value) return fail(c, MR_ERR_UNSUPPORTED, "graph replay of macrosteps is switched off");
    } else {
        return fail(c, MR_ERR_ARG, "unknown option '%s'", name);
    }
    return MR_OK;
}

int mr_set_tile_shape(mr_ctx *c, int g, int shape)
{
    if (c) c->version++;
    if (!c || g < 0 || g >= (int)c->G.size() || shape < -1 || shape >= mrk::NUM_TILE_SHAPES) return MR_ERR_ARG;
    if (c->G[g].dim != 2) return fail(c, MR_ERR_UNSUPPORTED, "tile shapes apply to 2D grids");
    c->G[g].tile = shape;
    return MR_OK;
}

int mr_get_tile_shape(const mr_ctx *c, int g, int *shape, int *tx, int *ty, int *tm)
{
    if (!c || !shape || g < 0 || g >= (int)c->G.size()) return MR_ERR_ARG;
    const GridHost &G = c->G[g];
    int s = G.dim != 2 ? -1 : G.tile >= 0 ? G.tile : mrk::default_tile_shape(G.dev);
    *shape = s;
    const mrk::TileShape z{0, 0, 0};
    const mrk::TileShape &t = s >= 0 ? mrk::kTileShapes[s] : z;
    if (tx) *tx = t.tx;
    if (ty) *ty = t.ty;
    if (tm) *tm = t.tm;
    return MR_OK;
}

int mr_tile_shape_info(int shape, int *tx, int *ty, int *tm)
{
    if (shape < 0 || shape >= mrk::NUM_TILE_SHAPES) return MR_ERR_ARG;
    const mrk::TileShape &t = mrk::kTileShapes[shape];
    if (tx) *tx = t.tx;
    if (ty) *ty = t.ty;
    if (tm) *tm = t.tm;
    return MR_OK;
}

int mr_autotune(mr_ctx *c, int reps)
{
    if (c) c->version++;
    if (!c || reps < 1 || reps > 1000) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_autotune")) return rc_;
    if (c->two_pass) return MR_OK;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    int rc = MR_OK;
    for (size_t gi = 0; gi < c->G.size() && rc == MR_OK; ++gi) {
        GridHost &g = c->G[gi];
        if (g.dim != 2) continue;
        // time the fused step (right-hand side and an AB combination) of the
        // current state into the bootstrap scratch buffers
        mrk::Combine cb{};
        cb.m = c->P.hist_len;
        for (int j = 0; j < cb.m - 1; ++j) { cb.c[j] = 0.0; cb.hist[j] = slot(c, g, j); }
        cb.c[cb.m - 1] = 0.0;
        cb.y_next = g.rk[1];
        GridDev dev = g.dev;
        dev.recv = recv_slice(c, g, 1);
        double best = INFINITY;
        int pick = mrk::default_tile_shape(dev);
        for (int s = 0; s < mrk::NUM_TILE_SHAPES; ++s) {
            // a warm-up launch, then a wait on the device long enough for the
            // host to queue every timed launch behind it
            hipError_t e = mrk::launch_rhs_tile2d(dev, c->P.sbp, c->ph, g.y[g.cur], g.rk[0], cb, s, c->st);
            if (e == hipSuccess) e = mrk::launch_wait_us(50.0 * reps + 200.0, c->st);
            if (e == hipSuccess) e = hipEventRecord(e0, c->st);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = mrk::launch_rhs_tile2d(dev, c->P.sbp, c->ph, g.y[g.cur], g.rk[0], cb, s, c->st);
            if (e == hipSuccess) e = hipEventRecord(e1, c->st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { rc = fail(c, MR_ERR_HIP, hipGetErrorString(e)); break; }
            if (ms < best) { best = ms; pick = s; }
        }
        g.tile = pick;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int mr_guard(mr_ctx *c, double *maxabs)
{
    if (!c) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_guard")) return rc_;
    double mx = 0;
    for (auto &g : c->G) {
        HIPCHK(c, mrk::launch_reduce(nelem(g), g.y[g.cur], 1, c->partial, 256, c->st));
        HIPCHK(c, mrk::launch_reduce(256, c->partial, 1, c->partial + 512, 1, c->st));
        double v = 0;
        HIPCHK(c, hipMemcpyAsync(&v, c->partial + 512, 8, hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        mx = std::max(mx, v);
    }
    if (maxabs) *maxabs = mx;
    if (!std::isfinite(mx)) return fail(c, MR_ERR_NONFINITE, "non-finite value in a state");
    return MR_OK;
}

int mr_batch_create(mr_ctx *const *ctxs, int n, mr_batch **out)
{
    if (!ctxs || n < 1 || !out) return MR_ERR_ARG;
    *out = nullptr;
    for (int s = 0; s < n; ++s) {
        const mr_ctx *c = ctxs[s];
        if (!c || !c->finalized) return MR_ERR_STATE;
        if (c->P.dim != 2 || c->two_pass || c->P.sbp != ctxs[0]->P.sbp || c->st != ctxs[0]->st)
            return MR_ERR_UNSUPPORTED;
        for (const Link &L : c->links)
            if (!use_blocks(c, L)) return MR_ERR_UNSUPPORTED;
        for (int t = 0; t < s; ++t)
            if (ctxs[t] == c) return MR_ERR_ARG;
    }
    mr_batch *b = new mr_batch();
    b->ctx.assign(ctxs, ctxs + n);
    b->st = ctxs[0]->st;
    for (auto *c : b->ctx) {
        b->R = std::lcm(b->R, c->rmax);
        b->P = std::lcm(b->P, c->period);
    }
    if (b->R > 64 || b->P > 4096) {
        delete b;
        return MR_ERR_UNSUPPORTED;
    }
    size_t nt = 0, nl = 0;
    for (auto *c : b->ctx) {
        for (auto &g : c->G) nt += g.rate;
        nl += c->links.size() * 2 * c->rmax;
    }
    b->tj_cap = (size_t)b->P * nt;
    b->lj_cap = (size_t)b->P * nl;
    b->ws_bytes = (b->tj_cap * sizeof(mrk::TileJob) + ALIGN) / ALIGN * ALIGN + b->lj_cap * sizeof(mrk::LinkJob) + ALIGN;
    *out = b;
    return MR_OK;
}

int mr_batch_workspace_size(const mr_batch *b, size_t *bytes)
{
    if (!b || !bytes) return MR_ERR_ARG;
    *bytes = b->ws_bytes;
    return MR_OK;
}

int mr_batch_bind_workspace(mr_batch *b, void *dev, size_t bytes)
{
    if (!b || !dev) return MR_ERR_ARG;
    if (bytes < b->ws_bytes) return bfail(b, MR_ERR_ARG, "workspace too small");
    if ((uintptr_t)dev % ALIGN) return bfail(b, MR_ERR_ARG, "workspace not 256-byte aligned");
    char *base = (char *)dev;
    b->tj_d = reinterpret_cast<mrk::TileJob *>(base);
    size_t off = (b->tj_cap * sizeof(mrk::TileJob) + ALIGN) / ALIGN * ALIGN;
    b->lj_d = reinterpret_cast<mrk::LinkJob *>(base + off);
    b->bound = true;
    b->built = false;
    return MR_OK;
}

int mr_batch_macrostep(mr_batch *b, int nsteps)
{
    if (!b || nsteps < 0) return MR_ERR_ARG;
    if (!b->bound) return bfail(b, MR_ERR_STATE, "mr_batch_macrostep before mr_batch_bind_workspace");
    const int n = (int)b->ctx.size();
    bool rebuild = !b->built;
    for (int s = 0; s < n; ++s) {
        const mr_ctx *c = b->ctx[s];
        if (!c->started || c->stale) return bfail(b, MR_ERR_STATE, "a system is not started (or needs mr_mrab_resume)");
        if (static_lost(c)) return bfail(b, MR_ERR_STATE, "a system's static workspace is bound to another context");
        if (b->built && (c->version != b->version[s] || c->nmacro != b->base[s] + b->steps)) rebuild = true;
    }
    if (rebuild) {
        int rc = batch_build(b);
        if (rc) return rc;
    }
    for (int it = 0; it < nsteps; ++it) {
        const int p = (int)(b->steps % b->P);
        for (int k = 1; k <= b->R; ++k)
            for (const auto &L : b->plan[(size_t)p * (b->R + 1) + k]) {
                if (L.what == 1)
                    BHIPCHK(b, mrk::launch_rhs_tiles(b->tj_d + L.first, L.njobs, L.nblk, L.sbp, L.cart, L.shape,
                                                     b->ctx[0]->ph, b->st));
                else
                    BHIPCHK(b, mrk::launch_donor_blocks(b->lj_d + L.first, L.njobs, L.nblk, L.maxnj, L.dim, L.sbp,
                                                        L.cart, L.what == 2, L.lds, b->st));
            }
        for (auto *c : b->ctx) advance_one(c);
        b->steps++;
    }
    return MR_OK;
}

int mr_batch_autotune(mr_batch *b, int reps, int *shape, double *ms)
{
    if (!b || reps < 1 || reps > 1000) return MR_ERR_ARG;
    if (!b->bound) return bfail(b, MR_ERR_STATE, "mr_batch_autotune before mr_batch_bind_workspace");
    const int n = (int)b->ctx.size();
    for (int s = 0; s < n; ++s)
        if (!b->ctx[s]->started || static_lost(b->ctx[s]))
            return bfail(b, MR_ERR_STATE, "a system is not started");
    // one fused right-hand side of every grid of every system, from its
    // current state into its bootstrap scratch buffers (the states, histories
    // and the batch's plan period are not touched), per candidate: every
    // grid's own shape (-1), then each shape for all
    std::vector<mrk::TileJob> base;
    for (int s = 0; s < n; ++s) {
        mr_ctx *c = b->ctx[s];
        for (int gi = 0; gi < (int)c->G.size(); ++gi) {
            GridHost &g = c->G[gi];
            mrk::TileJob J{};
            J.g = g.dev;
            J.g.recv = recv_slice(c, g, 1);
            J.q = g.y[g.cur];
            J.F = g.rk[0];
            J.cb.m = c->P.hist_len;
            for (int j = 0; j < J.cb.m - 1; ++j) {
                J.cb.c[j] = 0.0;
                J.cb.hist[j] = slot(c, g, j);
            }
            J.cb.c[J.cb.m - 1] = 0.0;
            J.cb.y_next = g.rk[1];
            J.tile0 = shape_of(g);
            base.push_back(J);
        }
    }
    if (base.size() > b->tj_cap) return bfail(b, MR_ERR_STATE, "timing jobs exceed the workspace");
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    b->built = false;   // the timing jobs take the plan's job table
    double best = INFINITY;
    int pick = -1;
    int rc = MR_OK;
    for (int cand = -1; cand < mrk::NUM_TILE_SHAPES && rc == MR_OK; ++cand) {
        std::vector<mrk::TileJob> tiles = base, tj;
        for (auto &J : tiles) {
            const int sh = cand >= 0 ? cand : J.tile0;
            const mrk::TileShape &t = mrk::kTileShapes[sh];
            J.tile0 = sh;
            J.ntx = (J.g.n[0] + t.tx - 1) / t.tx;
            J.nty = (J.g.n[1] + t.ty - 1) / t.ty;
        }
        std::vector<mr_batch::Launch> out;
        auto tkey = [&](const mrk::TileJob &j) { return std::array<int, 5>{2, 0, j.g.cartesian, j.tile0, 0}; };
        auto tcount = [&](mrk::TileJob &j, int &off, mr_batch::Launch &L) {
            j.tile0 = off;
            off += j.ntx * j.nty;
            L.maxnj = 1;
        };
        batch_group(tiles, tkey, tcount, 1, tj, out);
        hipError_t e = hipMemcpyAsync(b->tj_d, tj.data(), tj.size() * sizeof(mrk::TileJob), hipMemcpyHostToDevice,
                                      b->st);
        auto all = [&]() {
            hipError_t x = hipSuccess;
            for (const auto &L : out)
                if (x == hipSuccess)
                    x = mrk::launch_rhs_tiles(b->tj_d + L.first, L.njobs, L.nblk, b->ctx[0]->P.sbp, L.cart, L.shape,
                                              b->ctx[0]->ph, b->st);
            return x;
        };
        // a warm-up pass, then a wait on the device long enough for the host
        // to queue every timed pass behind it
        if (e == hipSuccess) e = all();
        if (e == hipSuccess) e = mrk::launch_wait_us(100.0 * reps + 200.0, b->st);
        if (e == hipSuccess) e = hipEventRecord(e0, b->st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = all();
        if (e == hipSuccess) e = hipEventRecord(e1, b->st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) {
            rc = bfail(b, MR_ERR_HIP, hipGetErrorString(e));
            break;
        }
        const double per = (double)t / reps;
        if (ms) ms[cand + 1] = per;
        if (per < best) {
            best = per;
            pick = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    b->shape = pick;
    if (shape) *shape = pick;
    return MR_OK;
}

int mr_batch_set_tile_shape(mr_batch *b, int shape)
{
    if (!b || shape < -1 || shape >= mrk::NUM_TILE_SHAPES) return MR_ERR_ARG;
    b->shape = shape;
    b->built = false;
    return MR_OK;
}

const char *mr_batch_last_error(const mr_batch *b) { return b ? b->err.c_str() : "null batch"; }

void mr_batch_destroy(mr_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->st);
    delete b;
}

const char *mr_last_error(const mr_ctx *c) { return c ? c->err.c_str() : "null context"; }

// ------------------------------------------------------------ adjoint ABI
int mr_adj_set_objective(mr_ctx *c, int grid, int64_t n, const int64_t *pts, const double *w)
{
    if (!c || n < 0 || (n > 0 && (!pts || !w))) return MR_ERR_ARG;
    if (!c->finalized) return fail(c, MR_ERR_STATE, "mr_adj_set_objective before mr_finalize");
    if (grid < 0 || grid >= (int)c->G.size()) return fail(c, MR_ERR_ARG, "bad grid id");
    const GridHost &g = c->G[grid];
    std::vector<int64_t> sorted(pts, pts + n);
    std::sort(sorted.begin(), sorted.end());
    for (int64_t i = 0; i < n; ++i) {
        if (sorted[i] < 0 || sorted[i] >= g.npts) return fail(c, MR_ERR_ARG, "objective point out of range");
        if (i && sorted[i] == sorted[i - 1]) return fail(c, MR_ERR_ARG, "objective point listed twice");
        if (!g.iblank[sorted[i]]) return fail(c, MR_ERR_ARG, "objective point is blanked");
        if (!std::isfinite(w[i])) return fail(c, MR_ERR_ARG, "non-finite objective weight");
    }
    if (!c->adj) c->adj = new AdjCtx();
    AdjCtx &A = *c->adj;
    A.og = n ? grid : -1;
    A.opts.assign(pts, pts + n);
    A.ow.assign(w, w + n);
    return adj_upload_objective(c);
}

int mr_adj_workspace_size(mr_ctx *c, int nsnap, size_t *bytes)
{
    if (!c || !bytes || nsnap < 1) return MR_ERR_ARG;
    if (!c->finalized) return fail(c, MR_ERR_STATE, "mr_adj_workspace_size before mr_finalize");
    for (const GridHost &g : c->G)
        if (g.dim != 2) return fail(c, MR_ERR_UNSUPPORTED, "the adjoint covers 2D systems");
    if (!c->adj) c->adj = new AdjCtx();
    AdjCtx &A = *c->adj;
    if (A.bound) return fail(c, MR_ERR_STATE, "adjoint workspace already bound");
    adj_tables(c);
    A.nsnap = nsnap;
    A.nslice = std::max(c->rmax, 4);
    A.nboot = (c->P.hist_len - 1) * c->rmax;
    A.bytes = adj_layout(c, nullptr);
    *bytes = A.bytes;
    return MR_OK;
}

int mr_adj_bind_workspace(mr_ctx *c, void *dev, size_t bytes)
{
    if (!c || !dev) return MR_ERR_ARG;
    if (int rc_ = need_bound(c, "mr_adj_bind_workspace")) return rc_;
    if (!c->adj || !c->adj->bytes) return fail(c, MR_ERR_STATE, "mr_adj_bind_workspace before mr_adj_workspace_size");
    AdjCtx &A = *c->adj;
    if (A.bound) return fail(c, MR_ERR_STATE, "adjoint workspace already bound");
    if (bytes < A.bytes) return fail(c, MR_ERR_ARG, "adjoint workspace too small (%zu < %zu)", bytes, A.bytes);
    if ((uintptr_t)dev % ALIGN) return fail(c, MR_ERR_ARG, "adjoint workspace not 256-byte aligned");
    A.ws = (char *)dev;
    adj_layout(c, A.ws);
    HIPCHK(c, hipMemsetAsync(A.ws, 0, A.bytes, c->st));
    for (size_t li = 0; li < c->links.size(); ++li) {
        AdjLink &T = A.L[li];
        auto up = [&](int32_t *d, const std::vector<int32_t> &h) -> hipError_t {
            return h.empty() ? hipSuccess : hipMemcpyAsync(d, h.data(), h.size() * 4, hipMemcpyHostToDevice, c->st);
        };
        HIPCHK(c, up(T.ustart_d, T.ustart));
        HIPCHK(c, up(T.uent_d, T.uent));
        HIPCHK(c, up(T.cpts_d, T.cpts));
        HIPCHK(c, up(T.cstart_d, T.cstart));
        HIPCHK(c, up(T.cent_d, T.cent));
        HIPCHK(c, up(T.cself_d, T.cself));
    }
    for (size_t gi = 0; gi < c->G.size(); ++gi) {
        const AdjGrid &a = A.G[gi];
        if (!a.bpts.empty())
            HIPCHK(c, hipMemcpyAsync(a.bpts_d, a.bpts.data(), a.bpts.size() * 4, hipMemcpyHostToDevice, c->st));
    }
    A.snap_pos.assign(A.nsnap, -1);
    A.bound = true;
    int rc = adj_upload_objective(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->st));
    return MR_OK;
}

int mr_adj_rhs(mr_ctx *c, const double *const *q, const double *const *lamF, double *const *lam_q)
{
    if (!c || !q || !lamF || !lam_q) return MR_ERR_ARG;
    if (!c->adj || !c->adj->bound) return fail(c, MR_ERR_STATE, "adjoint workspace not bound");
    if (int rc_ = need_bound(c, "the adjoint")) return rc_;
    const int G = (int)c->G.size();
    std::vector<double *> Y(G), K(G), LF(G), LQ(G);
    for (int g = 0; g < G; ++g) {
        if (!q[g] || !lamF[g] || !lam_q[g]) return fail(c, MR_ERR_ARG, "null pointer");
        Y[g] = const_cast<double *>(q[g]);
        K[g] = c->adj->G[g].kk[0];
        LF[g] = const_cast<double *>(lamF[g]);
        LQ[g] = lam_q[g];
        HIPCHK(c, hipMemsetAsync(LQ[g], 0, nelem(c->G[g]) * 8, c->st));
    }
    int rc = adj_coupled_fwd(c, Y, 0, K);
    if (rc) return rc;
    return adj_coupled_rev(c, Y, 0, LF, LQ);
}

int mr_adj_forward(mr_ctx *c, int nmacro, const double *const *y0, double *const *yN, double *J)
{
    if (!c || !y0) return MR_ERR_ARG;
    int rc = adj_check(c, nmacro);
    if (rc) return rc;
    for (size_t g = 0; g < c->G.size(); ++g)
        if (!y0[g]) return fail(c, MR_ERR_ARG, "null initial state");
    if ((rc = adj_run_fwd(c, y0, nmacro, true))) return rc;
    AdjCtx &A = *c->adj;
    if (yN)
        for (size_t g = 0; g < c->G.size(); ++g)
            if (yN[g])
                HIPCHK(c, hipMemcpyAsync(yN[g], ysl(A.G[g], c->G[g], 0), nelem(c->G[g]) * 8, hipMemcpyDeviceToDevice,
                                         c->st));
    double v = 0.0;
    HIPCHK(c, hipMemcpyAsync(&v, A.acc, 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (J) *J = v;
    return MR_OK;
}

int mr_adj_gradient(mr_ctx *c, int nmacro, const double *const *y0, const double *const *lamN, double jscale,
                    double *const *grad, double *J, int64_t *nfwd)
{
    if (!c || !y0 || !grad) return MR_ERR_ARG;
    int rc = adj_check(c, nmacro);
    if (rc) return rc;
    if (nmacro > 4096) return fail(c, MR_ERR_ARG, "at most 4096 macrosteps per adjoint run");
    AdjCtx &A = *c->adj;
    const int G = (int)c->G.size(), m = c->P.hist_len;
    for (int g = 0; g < G; ++g)
        if (!y0[g] || !grad[g]) return fail(c, MR_ERR_ARG, "null initial state or gradient pointer");
    // forward: bootstrap, the start in slot 0, every macrostep (objective)
    for (int g = 0; g < G; ++g)
        HIPCHK(c, hipMemcpyAsync(A.G[g].boot, y0[g], nelem(c->G[g]) * 8, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipMemsetAsync(A.acc, 0, 8, c->st));
    if ((rc = adj_boot_fwd(c))) return rc;
    const bool obj = A.og >= 0;
    if (obj)
        HIPCHK(c, mrk::launch_obj(adj_obj(c), ysl(A.G[A.og], c->G[A.og], 0), c->G[A.og].npts, adj_tau(c, 0, nmacro),
                                  A.acc, c->st));
    std::fill(A.snap_pos.begin(), A.snap_pos.end(), -1);
    if ((rc = adj_snap(c, 0, true))) return rc;
    A.snap_pos[0] = 0;
    int64_t nf = 0;
    for (int n = 0; n < nmacro; ++n) {
        if ((rc = adj_macro_fwd(c, n, nmacro, obj))) return rc;
        adj_advance(c);
        nf++;
    }
    // reverse: terminal adjoint, macrosteps under the checkpointing schedule,
    // the start's objective term, the bootstrap
    for (int g = 0; g < G; ++g) {
        const size_t nb = nelem(c->G[g]) * 8;
        if (lamN && lamN[g])
            HIPCHK(c, hipMemcpyAsync(A.G[g].lam_y, lamN[g], nb, hipMemcpyDeviceToDevice, c->st));
        else
            HIPCHK(c, hipMemsetAsync(A.G[g].lam_y, 0, nb, c->st));
        for (int j = 0; j < m; ++j) HIPCHK(c, hipMemsetAsync(A.G[g].lam_ring[j], 0, nb, c->st));
        HIPCHK(c, hipMemsetAsync(A.G[g].lam_ext, 0, nb, c->st));
    }
    if (nmacro > 0) {
        Sched S;
        S.build(nmacro, A.nsnap - 1);
        if ((rc = adj_reverse(c, S, 0, nmacro, 0, A.nsnap - 1, nmacro, jscale, nf))) return rc;
    }
    if ((rc = adj_snap(c, 0, false))) return rc;
    if (obj && jscale != 0.0)
        HIPCHK(c, mrk::launch_obj_adj(adj_obj(c), ysl(A.G[A.og], c->G[A.og], 0), c->G[A.og].npts,
                                      jscale * adj_tau(c, 0, nmacro),
                                      A.G[A.og].lam_y, c->st));
    if ((rc = adj_boot_rev(c))) return rc;
    for (int g = 0; g < G; ++g)
        HIPCHK(c, hipMemcpyAsync(grad[g], A.G[g].lam_y, nelem(c->G[g]) * 8, hipMemcpyDeviceToDevice, c->st));
    double v = 0.0;
    HIPCHK(c, hipMemcpyAsync(&v, A.acc, 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (J) *J = v;
    if (nfwd) *nfwd = nf;
    return MR_OK;
}

int mr_adj_schedule(int nmacro, int nsnap, int64_t *nfwd)
{
    if (nmacro < 0 || nmacro > 4096 || nsnap < 1 || !nfwd) return MR_ERR_ARG;
    if (nmacro == 0) {
        *nfwd = 0;
        return MR_OK;
    }
    Sched S;
    S.build(nmacro, nsnap - 1);
    *nfwd = S.cost[nmacro][nsnap - 1];
    return MR_OK;
}

void mr_destroy(mr_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    for (auto s : c->gs)
        if (s) (void)hipStreamSynchronize(s);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    free_evset(c->eager);
    for (auto s : c->gs)
        if (s) (void)hipStreamDestroy(s);
    delete c->adj;
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        auto it = g_static_holder.find(c->static_dev);
        if (it != g_static_holder.end() && it->second == c) g_static_holder.erase(it);
    }
    delete c;
}

}  // extern "C"
