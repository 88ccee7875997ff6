// Host runtime of libgks: the C ABI of include/gks.h.
//
// Responsibilities: argument validation before any launch, the time step, the coefficients
// C1..C5 of the time-integrated flux (Sec. 3.1) and the sparse face operators derived from
// them, device buffers owned by a context (ping-pong state for gks_run, reduction scratch,
// source lists), kernel launches on the caller's stream, and error reporting.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "gks_internal.h"

using namespace gks;

struct gks_ctx {
    int32_t kind = 0, model = 0, prec = 0;
    int64_t batch = 1;
    int64_t n[3] = {1, 1, 1};
    double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, h[3] = {1, 1, 1};
    int32_t bc[6] = {0, 0, 0, 0, 0, 0};
    int64_t ncell = 0;
    int32_t nfields = 3;
    double c = 1, dt = 0, tau = 0, C[5] = {0, 0, 0, 0, 0};
    double chi = 0, gamma = 0;      // PHM couplings (GKS_TM2D_PHM)
    int32_t energy_every = 0;
    int32_t limiter = 0;            // 1: minmod-limited slopes (Cartesian grids)
    double unstable_growth = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int ncu = 256;                  // compute units of the device
    int32_t ntile_rows = 0;         // Cartesian 2D: tile rows of the step (entries of d_tiles)
    int32_t tiles_per_band = 0;     // Cartesian 2D: entries per band (one band per XCD)
    int32_t *d_tiles = nullptr;     // Cartesian 2D: [ntile_rows][4] tile rows in dispatch order
    int32_t pair_tiles_per_band = 0;  // Cartesian 2D TM: the paired (two-step) kernel's table,
    int32_t *d_pair_tiles = nullptr;  // null where that kernel does not apply
    int32_t tile_z = 64;            // planes per workgroup tile (Cartesian 3D)
    const void *epsinv = nullptr, *muinv = nullptr;

    // face operators in double precision: [orientation][...], sized for the largest tables
    static constexpr int MAX_N0 = std::max(std::max(EM_N0, TP_N0), EP_N0),
                         MAX_NE = std::max(std::max(EM_NE, TP_NE), EP_NE),
                         MAX_NH = std::max(std::max(EM_NH, TP_NH), EP_NH);
    double k0[3][MAX_N0], ke[3][MAX_NE], kh[3][MAX_NH];

    // point sources
    std::vector<int64_t> src_cells;
    std::vector<double> src_w;
    double J0 = 0, t0 = 0, sigma_t = 1;
    int64_t *d_src_cells = nullptr;
    double *d_src_w = nullptr;

    // owned device buffers
    void *d_ops = nullptr;          // face operators in the context's precision
    void *pingpong = nullptr;
    size_t pingpong_bytes = 0;
    double *d_partial = nullptr;
    int32_t nblk = 0;
    double *d_out = nullptr;        // energy records
    size_t d_out_count = 0;
    double *h_out = nullptr;        // pinned host mirror
    size_t h_out_count = 0;
    hipEvent_t rec_ev[2] = {nullptr, nullptr};   // gks_run: energy record r read back (r mod 2)
    void *adj_scratch = nullptr;    // adjoint: co-states and material gradients of the ghost positions
    size_t adj_scratch_bytes = 0;
    void *static_scratch = nullptr; // gks_adjoint_step_noalloc: this device's static scratch array
    int static_scratch_err = 0;     // its lookup's error (hipError_t) when static_scratch is NULL

    // triangle meshes: per cell-face neighbours and geometry, cell areas, gradient scratch
    int32_t *d_tri_nb = nullptr;
    void *d_tri_geo = nullptr;
    double *d_area = nullptr;       // cell areas (triangles) or volumes (tetrahedra), for the energy
    // tetrahedral meshes: per cell neighbours, face slots and geometry; per face cells and
    // geometry; the face-flux scratch
    int32_t *d_tet_nb = nullptr, *d_tet_cf = nullptr, *d_tet_fc = nullptr;
    void *d_tet_cgeo = nullptr, *d_tet_fgeo = nullptr, *d_flux = nullptr;
    int64_t nface = 0;
    void *d_grad = nullptr;

    std::string err;
};

static thread_local std::string g_init_error;

namespace {

gks_status fail(gks_ctx *ctx, gks_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_init_error = buf;
    return st;
}

gks_status hip_fail(gks_ctx *ctx, int e, const char *what)
{
    return fail(ctx, GKS_EDEVICE, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

size_t elem_size(const gks_ctx *x) { return x->prec == GKS_FP64 ? sizeof(double) : sizeof(float); }
size_t state_bytes(const gks_ctx *x) { return (size_t)x->batch * x->nfields * x->ncell * elem_size(x); }

gks_status check_device(gks_ctx *ctx)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ctx, GKS_EDEVICE, "hipGetDevice failed");
    if (dev != ctx->device)
        return fail(ctx, GKS_ESTATE, "the current HIP device (%d) is not the context's device (%d)", dev, ctx->device);
    return GKS_OK;
}

bool ranges_overlap(const void *a, const void *b, size_t n)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + n && pb < pa + n;
}

// Device form of a face operator: the kernels pass the sum of the two cells' 1/eps (1/mu)
// instead of their mean, so KE and KH are stored halved.
template <typename T, int N0, int NE, int NH>
void fill_op(FaceOp<T, N0, NE, NH> &o, const double *k0, const double *ke, const double *kh)
{
    for (int q = 0; q < N0; ++q) o.k0[q] = (T)k0[q];
    for (int q = 0; q < NE; ++q) o.ke[q] = (T)(0.5 * ke[q]);
    for (int q = 0; q < NH; ++q) o.kh[q] = (T)(0.5 * kh[q]);
}

// K0 + KH on the pattern pf (K0 of the folded operator), from K0 and KH on the pattern p; every
// entry of K0 and KH must have its place in pf.
bool fold_kh(const Pattern &p, const Pattern &pf, const double *k0, const double *kh, double *out)
{
    auto place = [&](int r, int c) {
        for (int q = 0; q < pf.n0; ++q)
            if (pf.r0[q] == r && pf.c0[q] == c) return q;
        return -1;
    };
    for (int q = 0; q < pf.n0; ++q) out[q] = 0.0;
    for (int q = 0; q < p.n0; ++q) {
        const int at = place(p.r0[q], p.c0[q]);
        if (at < 0) return false;
        out[at] += k0[q];
    }
    for (int q = 0; q < p.nH; ++q) {
        const int at = place(p.rH[q], p.cH[q]);
        if (at < 0) return false;
        out[at] += kh[q];
    }
    return true;
}

template <typename T>
bool pack_ops(const gks_ctx *x, std::vector<char> &buf)
{
    if (x->kind == GKS_TET3D) {
        std::vector<FaceOpEM<T>> ops(1);
        fill_op(ops[0], x->k0[0], x->ke[0], x->kh[0]);
        buf.assign((const char *)ops.data(), (const char *)(ops.data() + ops.size()));
    } else if (x->kind == GKS_TRI2D && x->model == GKS_TM2D_PHM) {
        std::vector<FaceOpTP<T>> ops(1);
        fill_op(ops[0], x->k0[0], x->ke[0], x->kh[0]);
        buf.assign((const char *)ops.data(), (const char *)(ops.data() + ops.size()));
    } else if (x->kind == GKS_TRI2D) {
        std::vector<FaceOpTM<T>> ops(1);
        fill_op(ops[0], x->k0[0], x->ke[0], x->kh[0]);
        buf.assign((const char *)ops.data(), (const char *)(ops.data() + ops.size()));
    } else if (x->model == GKS_TM2D) {
        // x and y faces, then the same with the 1/mu part folded into K0 for vacuum 1/mu (the
        // kernels pass the sum of the two cells' 1/mu, 2 in vacuum, against KH stored halved)
        std::vector<FaceOpTM<T>> ops(4);
        for (int ax = 0; ax < 2; ++ax) {
            fill_op(ops[ax], x->k0[ax], x->ke[ax], x->kh[ax]);
            double k0f[TM_N0];
            const Pattern &p = pattern_cart(x->model, ax);
            if (!fold_kh(p, p, x->k0[ax], x->kh[ax], k0f)) return false;
            fill_op(ops[2 + ax], k0f, x->ke[ax], x->kh[ax]);
        }
        buf.assign((const char *)ops.data(), (const char *)(ops.data() + ops.size()));
    } else if (x->model == GKS_TM2D_PHM) {
        std::vector<FaceOpTP<T>> ops(2);
        for (int ax = 0; ax < 2; ++ax) fill_op(ops[ax], x->k0[ax], x->ke[ax], x->kh[ax]);
        buf.assign((const char *)ops.data(), (const char *)(ops.data() + ops.size()));
    } else if (x->model == GKS_EM3D_PHM) {
        std::vector<FaceOpEP<T>> ops(3);
        for (int ax = 0; ax < 3; ++ax) fill_op(ops[ax], x->k0[ax], x->ke[ax], x->kh[ax]);
        buf.assign((const char *)ops.data(), (const char *)(ops.data() + ops.size()));
    } else {
        // x-, y- and z-faces, then the same with the 1/mu part folded into K0 (vacuum 1/mu)
        std::vector<FaceOpEM<T>> ops(3);
        std::vector<FaceOpEMF<T>> folded(3);
        for (int ax = 0; ax < 3; ++ax) {
            fill_op(ops[ax], x->k0[ax], x->ke[ax], x->kh[ax]);
            double k0f[EMF_N0];
            if (!fold_kh(pattern_cart(x->model, ax), pattern_cart_em_folded(ax), x->k0[ax], x->kh[ax], k0f))
                return false;
            fill_op(folded[ax], k0f, x->ke[ax], x->kh[ax]);
        }
        buf.assign((const char *)ops.data(), (const char *)(ops.data() + ops.size()));
        buf.insert(buf.end(), (const char *)folded.data(), (const char *)(folded.data() + folded.size()));
    }
    return true;
}

// Copies the face operators, rounded once to the storage precision, to device memory.
gks_status upload_ops(gks_ctx *x)
{
    std::vector<char> buf;
    const bool ok = (x->prec == GKS_FP64) ? pack_ops<double>(x, buf) : pack_ops<float>(x, buf);
    if (!ok) return fail(x, GKS_EINVAL, "internal: a 1/mu operator entry lies outside K0's pattern");
    if (hipMalloc(&x->d_ops, buf.size()) != hipSuccess) return fail(x, GKS_ENOMEM, "cannot allocate face operators");
    int e = hipMemcpy(x->d_ops, buf.data(), buf.size(), hipMemcpyHostToDevice);
    if (e) return hip_fail(x, e, "face operator upload");
    return GKS_OK;
}

}  // namespace

std::vector<int32_t> gks::cart2d_tile_table(int ny, int batch, int precision, int ntx, int32_t &tiles_per_band)
{
    // Workgroups reach the 8 XCDs round-robin (XCD = workgroup id mod 8) and each XCD starts its
    // workgroups in id order.  The tile rows are therefore cut in 8 bands of the (batch item,
    // row) sequence, one per XCD, each padded to the same length, and workgroup g works on band
    // g mod 8, taking that band's tiles in the table's order.  Each band lists tall tiles first
    // and short ones last: tall tiles re-read fewer halo rows (4 per tile), and the short ones
    // end the band, so the last waves of an XCD are short and the drain of the launch is short.
    // Measured on 4096^2 (fp32, per launch): uniform 14-row tiles 113.4 us; tall 32 / short 8
    // rows with the short rows 0.3 of each band 110.8 us (fp64 203.3 us, as with 16-row tiles).
    // A later sweep (batch-timed, fp32 / fp64 us): 32/8/0.3 108.3 / 201.4; tall 24, 28, 36, 40:
    // 108.6, 108.5, 109.0, 113.9 / 202.4, 202.1, 203.9, 206.0; short 6, 10, 12: 108.3, 109.5,
    // 109.6 / 203.0, 201.9, 202.6; short fraction 0.2, 0.4: 111.0, 108.5 / 200.6, 200.9.
    // A band whose last workgroup also ran the next band's first (tall) tiles cost up to 30%:
    // the padding keeps every band on its own XCD.  Vertically adjacent tiles of a band march in
    // opposite directions, so the halo rows they share are read at about the same time (the
    // second read hits the L2); tiles never straddle two batch items.
#ifndef GKS_TILE_TALL
#define GKS_TILE_TALL 32
#endif
#ifndef GKS_TILE_SHORT
#define GKS_TILE_SHORT 8
#endif
#ifndef GKS_TILE_SHORT_FRAC
#define GKS_TILE_SHORT_FRAC 0.3
#endif
    // (the three macros are build-time overrides for tuning sweeps)
    int tall = GKS_TILE_TALL, shrt = GKS_TILE_SHORT;
    double frac = GKS_TILE_SHORT_FRAC;
    (void)precision;
#ifdef GKS_FORCE_TILE_Y
    tall = shrt = GKS_FORCE_TILE_Y;   // build-time override for tuning sweeps: uniform tiles
    frac = 0.0;
#endif
    const int64_t total = (int64_t)ny * batch;
    std::vector<std::vector<int32_t>> bands(NBANDS);
    size_t most = 0;
    for (int64_t band = 0; band < NBANDS; ++band) {
        const int64_t r0 = total * band / NBANDS, r1 = total * (band + 1) / NBANDS;
        const int64_t split = r1 - (int64_t)(frac * (double)(r1 - r0) + 0.5);
        std::vector<int32_t> &tab = bands[band];
        int64_t r = r0;
        int k = 0;
        while (r < r1) {
            const int64_t b = r / ny, y = r % ny;
            const int64_t h = r < split ? tall : shrt;
            const int64_t lim = std::min(r < split ? split : r1, (b + 1) * ny);   // stay in the batch item
            const int64_t e = std::min(r + h, lim);
            tab.push_back((int32_t)b);
            tab.push_back((int32_t)y);
            tab.push_back((int32_t)(y + (e - r)));
            tab.push_back(k++ & 1);
            r = e;
        }
        most = std::max(most, tab.size() / 4);
    }
    // pad every band to the same number of tile rows, and that to whole workgroups of strips
    size_t per = most;
    while ((per * (size_t)ntx) % CART2D_WAVES_PER_BLOCK) ++per;
    std::vector<int32_t> out;
    for (auto &tab : bands) {
        out.insert(out.end(), tab.begin(), tab.end());
        for (size_t q = tab.size() / 4; q < per; ++q) {
            const int32_t pad[4] = {-1, 0, 0, 0};   // no tile: its waves exit at once
            out.insert(out.end(), pad, pad + 4);
        }
    }
    tiles_per_band = (int32_t)per;
    return out;
}

std::vector<int32_t> gks::cart2d_pair_tile_table(int ny, int batch, int precision, int ntx, int32_t &tiles_per_band)
{
    // The single-step table's bands and tile heights, with two constraints of the paired
    // kernel: a tile reads the intermediate state two rows beyond each end, so a cut between
    // tiles never falls one row from a side (it moves one row on), and a tile that touches the
    // lower side marches down, one that touches the upper side up (no tile may touch both).
    // A tile's stage 1 forms four rows more than it writes, so the paired kernel takes taller
    // tiles: on 4096^2 (fp32 / fp64 us per launch) tall 32 153.7 / 238.0, 48 150.4 / 232.3,
    // 64 150.3 / 230.5, 96 163.3 / 246.0, 128 174.8 / 234.7; tall 64 with short 16 150.0 / 226.3.
    // A later sweep (short 16): tall 56, 64, 72: 147.7, 143.8, 140.3 / 222.8, 226.4, 225.3; short
    // 24, 32: 143.8, 149.9 / 225.8, 232.0; short fraction 0.2, 0.4: 164.9, 142.7 / 246.3, 230.2.
#ifndef GKS_PAIR_TILE_TALL
#define GKS_PAIR_TILE_TALL ((precision == GKS_FP64) ? 56 : 72)
#endif
#ifndef GKS_PAIR_TILE_SHORT
#define GKS_PAIR_TILE_SHORT 16
#endif
    const int tall = GKS_PAIR_TILE_TALL, shrt = GKS_PAIR_TILE_SHORT;
    const double frac = GKS_TILE_SHORT_FRAC;
    tiles_per_band = 0;
    if (ny < 8) return {};
    const int64_t total = (int64_t)ny * batch;
    auto fix = [&](int64_t r) {   // a cut at row 1 or ny - 1 of an item moves one row on
        const int64_t y = r % ny;
        return (y == 1 || y == ny - 1) ? r + 1 : r;
    };
    std::vector<int64_t> cut(NBANDS + 1);
    for (int band = 0; band <= NBANDS; ++band) cut[band] = std::min(fix(total * band / NBANDS), total);
    std::vector<std::vector<int32_t>> bands(NBANDS);
    size_t most = 0;
    for (int band = 0; band < NBANDS; ++band) {
        const int64_t r0 = cut[band], r1 = cut[band + 1];
        const int64_t split = r1 - (int64_t)(frac * (double)(r1 - r0) + 0.5);
        std::vector<int32_t> &tab = bands[band];
        int64_t r = r0;
        int k = 0;
        while (r < r1) {
            const int64_t b = r / ny, y = r % ny;
            const int64_t h = r < split ? tall : shrt;
            const int64_t lim = std::min(r1, (b + 1) * ny);
            int64_t e = std::min(r + h, lim);
            if (e < lim) e = std::min(fix(e), lim);
            const int64_t ye = y + (e - r);
            int dn = k++ & 1;
            if (y == 0) dn = 1;
            if (ye == ny) dn = 0;
            if (y == 0 && ye == ny) return {};
            if ((y != 0 && y < 2) || (ye != ny && ye > ny - 2)) return {};
            tab.push_back((int32_t)b);
            tab.push_back((int32_t)y);
            tab.push_back((int32_t)ye);
            tab.push_back(dn);
            r = e;
        }
        most = std::max(most, tab.size() / 4);
    }
    size_t per = most;
    while ((per * (size_t)ntx) % CART2D_WAVES_PER_BLOCK) ++per;
    std::vector<int32_t> out;
    for (auto &tab : bands) {
        out.insert(out.end(), tab.begin(), tab.end());
        for (size_t q = tab.size() / 4; q < per; ++q) {
            const int32_t pad[4] = {-1, 0, 0, 0};
            out.insert(out.end(), pad, pad + 4);
        }
    }
    tiles_per_band = (int32_t)per;
    return out;
}

int gks::cart3d_pick_tile_z(int nx, int ny, int nz, int batch, int ncu, int precision, int nfields)
{
    // One workgroup per compute unit at a time (its LDS tile takes most of the unit): the step
    // takes about (rounds of workgroups) x (planes per tile + the three planes the march reads
    // beyond its tile).
    const int tx = cart3d_tile_x(precision), ty = cart3d_tile_y(precision, nfields);
    const int64_t per_z = (int64_t)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * batch;
    double best = 1e300;
    int pick = nz;
    for (int tz = std::min(4, nz); tz <= nz; ++tz) {
        const int64_t ntz = (nz + tz - 1) / tz;
        const int64_t rounds = (per_z * ntz + ncu - 1) / ncu;
        const double cost = (double)rounds * (tz + 3);
        if (cost < best) {
            best = cost;
            pick = tz;
        }
    }
    return pick;
}

namespace {

double source_pulse(const gks_ctx *x, double t)
{
    const double z = (t - x->t0) / x->sigma_t;
    return x->J0 * std::exp(-z * z);
}

template <typename T>
gks_status step_cart2d(gks_ctx *x, const void *Uin, void *Uout, double tn)
{
    Cart2DArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.U = (const T *)Uin;
    a.Unew = (T *)Uout;
    a.epsinv = (const T *)x->epsinv;
    a.muinv = (const T *)x->muinv;
    a.nx = (int32_t)x->n[0];
    a.ny = (int32_t)x->n[1];
    a.batch = (int32_t)x->batch;
    for (int i = 0; i < 4; ++i) a.bc[i] = x->bc[i];
    a.ntx = (a.nx + cart2d_tile_x(x->prec) - 1) / cart2d_tile_x(x->prec);
    a.nty = x->tiles_per_band;
    a.tiles = x->d_tiles;
    a.nfields = x->nfields;
    a.ops = x->d_ops;
    a.limiter = x->limiter;
    const int64_t ns = (int64_t)x->src_cells.size();
    // dt * S_z = -dt * J_z(t^n), scaled by 1/eps of the cell in the kernels
    const double amp = ns ? -x->dt * source_pulse(x, tn) : 0.0;
    a.src_row = -1;
    if (ns == 1) {   // a single source cell is added inside the step kernel
        a.src_row = (int32_t)(x->src_cells[0] / x->n[0]);
        a.src_col = (int32_t)(x->src_cells[0] % x->n[0]);
        a.src_amp = amp * x->src_w[0];
    }
    int e = launch_cart2d_step<T>(a, x->stream);
    if (e) return hip_fail(x, e, "GKS step launch");
    if (ns > 1) {
        e = launch_source_scatter<T>((T *)Uout, (const T *)x->epsinv, x->ncell, (int64_t)x->nfields * x->ncell,
                                     (int32_t)x->batch, 0, x->d_src_cells, x->d_src_w, amp, (int32_t)ns, x->stream);
        if (e) return hip_fail(x, e, "source launch");
    }
    return GKS_OK;
}

// The steps at tn and tn1 in one launch of the paired kernel (gks_run, where d_pair_tiles is set
// and at most one source cell is given): the same results as two calls of step_cart2d, bit for
// bit.
template <typename T>
gks_status step2_cart2d(gks_ctx *x, const void *Uin, void *Uout, double tn, double tn1)
{
    Cart2DArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.U = (const T *)Uin;
    a.Unew = (T *)Uout;
    a.epsinv = (const T *)x->epsinv;
    a.muinv = (const T *)x->muinv;
    a.nx = (int32_t)x->n[0];
    a.ny = (int32_t)x->n[1];
    a.batch = (int32_t)x->batch;
    for (int i = 0; i < 4; ++i) a.bc[i] = x->bc[i];
    a.ntx = (a.nx + cart2d_pair_tile_x(x->prec) - 1) / cart2d_pair_tile_x(x->prec);
    a.nty = x->pair_tiles_per_band;
    a.tiles = x->d_pair_tiles;
    a.nfields = x->nfields;
    a.ops = x->d_ops;
    a.limiter = x->limiter;
    a.src_row = -1;
    if (x->src_cells.size() == 1) {   // times formed as gks_run forms them for single steps
        a.src_row = (int32_t)(x->src_cells[0] / x->n[0]);
        a.src_col = (int32_t)(x->src_cells[0] % x->n[0]);
        a.src_amp = -x->dt * source_pulse(x, tn) * x->src_w[0];
        a.src_amp2 = -x->dt * source_pulse(x, tn1) * x->src_w[0];
    }
    const int e = launch_cart2d_pair<T>(a, x->stream);
    if (e) return hip_fail(x, e, "GKS paired step launch");
    return GKS_OK;
}

template <typename T>
gks_status step_cart3d(gks_ctx *x, const void *Uin, void *Uout, double tn)
{
    Cart3DArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.U = (const T *)Uin;
    a.Unew = (T *)Uout;
    a.epsinv = (const T *)x->epsinv;
    a.muinv = (const T *)x->muinv;
    a.nx = (int32_t)x->n[0];
    a.ny = (int32_t)x->n[1];
    a.nz = (int32_t)x->n[2];
    a.batch = (int32_t)x->batch;
    for (int i = 0; i < 6; ++i) a.bc[i] = x->bc[i];
    const int tx = cart3d_tile_x(x->prec), ty = cart3d_tile_y(x->prec, x->nfields);
    a.ntx = (a.nx + tx - 1) / tx;
    a.nty = (a.ny + ty - 1) / ty;
    a.tile_z = x->tile_z;
    a.ntz = (a.nz + a.tile_z - 1) / a.tile_z;
    a.nfields = x->nfields;
    a.ops = x->d_ops;
    a.limiter = x->limiter;
    int e = launch_cart3d_step<T>(a, x->stream);
    if (e) return hip_fail(x, e, "GKS 3D step launch");
    const int64_t ns = (int64_t)x->src_cells.size();
    if (ns > 0) {   // J_z drives Ez (field 2)
        const double amp = -x->dt * source_pulse(x, tn);
        e = launch_source_scatter<T>((T *)Uout, (const T *)x->epsinv, x->ncell, (int64_t)x->nfields * x->ncell,
                                     (int32_t)x->batch, 2, x->d_src_cells, x->d_src_w, amp, (int32_t)ns, x->stream);
        if (e) return hip_fail(x, e, "source launch");
    }
    return GKS_OK;
}

template <typename T>
gks_status step_tri(gks_ctx *x, const void *Uin, void *Uout, double tn)
{
    TriArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.U = (const T *)Uin;
    a.Unew = (T *)Uout;
    a.epsinv = (const T *)x->epsinv;
    a.muinv = (const T *)x->muinv;
    a.grad = (T *)x->d_grad;
    a.ncell = (int32_t)x->ncell;
    a.batch = (int32_t)x->batch;
    a.nfields = x->nfields;
    a.nb = x->d_tri_nb;
    a.geo = (const T *)x->d_tri_geo;
    a.op = x->d_ops;
    int e = launch_tri_step<T>(a, x->stream);
    if (e) return hip_fail(x, e, "triangle step launch");
    const int64_t ns = (int64_t)x->src_cells.size();
    if (ns > 0) {
        const double amp = -x->dt * source_pulse(x, tn);
        e = launch_source_scatter<T>((T *)Uout, (const T *)x->epsinv, x->ncell, (int64_t)x->nfields * x->ncell,
                                     (int32_t)x->batch, 0, x->d_src_cells, x->d_src_w, amp, (int32_t)ns, x->stream);
        if (e) return hip_fail(x, e, "source launch");
    }
    return GKS_OK;
}

template <typename T>
gks_status upload_tri(gks_ctx *x, const TriGeometry &g)
{
    const size_t nc = (size_t)g.ncell;
    // the device layout: vector components side by side (TGP_*), then the |l_k| / |Omega| rows
    std::vector<T> geo(g.geo.size());
    auto pair = [&](int p, int rx, int ry) {
        for (size_t c = 0; c < nc; ++c) {
            geo[((size_t)p * nc + c) * 2] = (T)g.geo[(size_t)rx * nc + c];
            geo[((size_t)p * nc + c) * 2 + 1] = (T)g.geo[(size_t)ry * nc + c];
        }
    };
    for (int k = 0; k < 3; ++k) {
        pair(TGP_N + k, TG_NX + k, TG_NY + k);
        pair(TGP_B + k, TG_BX + k, TG_BY + k);
        pair(TGP_W + k, TG_WX + k, TG_WY + k);
        for (size_t c = 0; c < nc; ++c)
            geo[2 * (size_t)TRI_GEO_PAIRS * nc + (size_t)k * nc + c] = (T)g.geo[(size_t)(TG_LW + k) * nc + c];
    }
    for (int k = 0; k < 2; ++k) pair(TGP_A + k, TG_AX + k, TG_AY + k);
    static_assert(2 * TRI_GEO_PAIRS + 3 == TRI_GEO_ROWS, "every geometry row is stored once");
    if (hipMalloc((void **)&x->d_tri_nb, 3 * nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&x->d_tri_geo, geo.size() * sizeof(T)) != hipSuccess ||
        hipMalloc((void **)&x->d_area, nc * sizeof(double)) != hipSuccess ||
        hipMalloc(&x->d_grad, (size_t)x->batch * 2 * x->nfields * nc * sizeof(T)) != hipSuccess)
        return fail(x, GKS_ENOMEM, "cannot allocate the triangle mesh arrays");
    int e = hipMemcpy(x->d_tri_nb, g.nb.data(), 3 * nc * sizeof(int32_t), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(x->d_tri_geo, geo.data(), geo.size() * sizeof(T), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(x->d_area, g.area.data(), nc * sizeof(double), hipMemcpyHostToDevice);
    if (e) return hip_fail(x, e, "triangle mesh upload");
    return GKS_OK;
}

template <typename T>
gks_status step_tet(gks_ctx *x, const void *Uin, void *Uout, double tn)
{
    TetArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.U = (const T *)Uin;
    a.Unew = (T *)Uout;
    a.epsinv = (const T *)x->epsinv;
    a.muinv = (const T *)x->muinv;
    a.grad = (T *)x->d_grad;
    a.flux = (T *)x->d_flux;
    a.ncell = (int32_t)x->ncell;
    a.nface = (int32_t)x->nface;
    a.batch = (int32_t)x->batch;
    a.nb = x->d_tet_nb;
    a.cf = x->d_tet_cf;
    a.fc = x->d_tet_fc;
    a.cgeo = (const T *)x->d_tet_cgeo;
    a.fgeo = (const T *)x->d_tet_fgeo;
    a.op = x->d_ops;
    int e = launch_tet_step<T>(a, x->stream);
    if (e) return hip_fail(x, e, "tetrahedral step launch");
    const int64_t ns = (int64_t)x->src_cells.size();
    if (ns > 0) {   // J_z drives Ez (field 2)
        const double amp = -x->dt * source_pulse(x, tn);
        e = launch_source_scatter<T>((T *)Uout, (const T *)x->epsinv, x->ncell, (int64_t)x->nfields * x->ncell,
                                     (int32_t)x->batch, 2, x->d_src_cells, x->d_src_w, amp, (int32_t)ns, x->stream);
        if (e) return hip_fail(x, e, "source launch");
    }
    return GKS_OK;
}

template <typename T>
gks_status upload_tet(gks_ctx *x, const TetGeometry &g)
{
    const size_t nc = (size_t)g.ncell, nf = (size_t)g.nface;
    std::vector<T> cg(g.cgeo.size()), fg(g.fgeo.size());
    for (size_t q = 0; q < cg.size(); ++q) cg[q] = (T)g.cgeo[q];
    for (size_t q = 0; q < fg.size(); ++q) fg[q] = (T)g.fgeo[q];
    if (hipMalloc((void **)&x->d_tet_nb, 4 * nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&x->d_tet_cf, 4 * nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&x->d_tet_fc, 2 * nf * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&x->d_tet_cgeo, cg.size() * sizeof(T)) != hipSuccess ||
        hipMalloc(&x->d_tet_fgeo, fg.size() * sizeof(T)) != hipSuccess ||
        hipMalloc((void **)&x->d_area, nc * sizeof(double)) != hipSuccess ||
        hipMalloc(&x->d_grad, (size_t)x->batch * 18 * nc * sizeof(T)) != hipSuccess ||
        hipMalloc(&x->d_flux, (size_t)x->batch * 6 * nf * sizeof(T)) != hipSuccess)
        return fail(x, GKS_ENOMEM, "cannot allocate the tetrahedral mesh arrays");
    int e = hipMemcpy(x->d_tet_nb, g.nb.data(), 4 * nc * sizeof(int32_t), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(x->d_tet_cf, g.cf.data(), 4 * nc * sizeof(int32_t), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(x->d_tet_fc, g.fc.data(), 2 * nf * sizeof(int32_t), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(x->d_tet_cgeo, cg.data(), cg.size() * sizeof(T), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(x->d_tet_fgeo, fg.data(), fg.size() * sizeof(T), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(x->d_area, g.vol.data(), nc * sizeof(double), hipMemcpyHostToDevice);
    if (e) return hip_fail(x, e, "tetrahedral mesh upload");
    return GKS_OK;
}

gks_status do_step(gks_ctx *x, const void *Uin, void *Uout, double tn)
{
    if (x->kind == GKS_TET3D)
        return x->prec == GKS_FP64 ? step_tet<double>(x, Uin, Uout, tn) : step_tet<float>(x, Uin, Uout, tn);
    if (x->kind == GKS_TRI2D)
        return x->prec == GKS_FP64 ? step_tri<double>(x, Uin, Uout, tn) : step_tri<float>(x, Uin, Uout, tn);
    if (x->kind == GKS_CART2D)
        return x->prec == GKS_FP64 ? step_cart2d<double>(x, Uin, Uout, tn) : step_cart2d<float>(x, Uin, Uout, tn);
    if (x->kind == GKS_CART3D)
        return x->prec == GKS_FP64 ? step_cart3d<double>(x, Uin, Uout, tn) : step_cart3d<float>(x, Uin, Uout, tn);
    return fail(x, GKS_ESTATE, "this mesh kind has no step kernel");
}

// Bytes of adjoint scratch one call needs: padg [batch][2][npos] doubles, then padpsi
// [batch][3][npos] of the field type, over the npos ghost positions around the grid.
size_t adjoint_scratch_bytes(const gks_ctx *x)
{
    const size_t npos = (size_t)adjoint_ring_positions((int)x->n[0], (int)x->n[1]);
    return (size_t)x->batch * npos * (2 * sizeof(double) + 3 * elem_size(x));
}

template <typename T>
gks_status adjoint_cart2d(gks_ctx *x, const void *Un, const void *lam_np1, void *lam_n, double *g_epsinv,
                          double *g_muinv, double tn, void *scratch)
{
    const size_t npos = (size_t)adjoint_ring_positions((int)x->n[0], (int)x->n[1]);
    double *padg = (double *)scratch;
    T *padpsi = (T *)(padg + (size_t)x->batch * 2 * npos);
    Cart2DAdjArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.U = (const T *)Un;
    a.lam = (const T *)lam_np1;
    a.lam_out = (T *)lam_n;
    a.g_epsinv = g_epsinv;
    a.g_muinv = g_muinv;
    a.epsinv = (const T *)x->epsinv;
    a.muinv = (const T *)x->muinv;
    a.nx = (int32_t)x->n[0];
    a.ny = (int32_t)x->n[1];
    a.batch = (int32_t)x->batch;
    for (int i = 0; i < 4; ++i) a.bc[i] = x->bc[i];
    a.ncu = x->ncu;
    a.ops = (const FaceOpTM<T> *)x->d_ops;
    int e = launch_cart2d_adjoint<T>(a, padpsi, padg, x->stream);
    if (e) return hip_fail(x, e, "adjoint launch");
    const int64_t ns = (int64_t)x->src_cells.size();
    if (ns > 0 && g_epsinv) {
        const double amp = -x->dt * source_pulse(x, tn);
        e = launch_adjoint_source<T>((const T *)lam_np1, g_epsinv, x->ncell, (int64_t)x->nfields * x->ncell,
                                     (int32_t)x->batch, x->d_src_cells, x->d_src_w, amp, (int32_t)ns, x->stream);
        if (e) return hip_fail(x, e, "adjoint source launch");
    }
    return GKS_OK;
}

// Checks shared by the adjoint entry points (no launch, no allocation).
gks_status check_adjoint(gks_ctx *ctx, const void *U_n, const void *lam_np1, void *lam_n, double *g_epsinv,
                         double *g_muinv, double t_n)
{
    if (ctx->kind != GKS_CART2D) return fail(ctx, GKS_ESTATE, "the adjoint step exists for Cartesian 2D TM contexts only");
    if (ctx->limiter)
        return fail(ctx, GKS_ESTATE, "the adjoint step is that of the linear (unlimited) step; this context limits slopes");
    if (ctx->model != GKS_TM2D) return fail(ctx, GKS_ESTATE, "the adjoint step is built for the TM fields without PHM");
    if (!U_n || !lam_np1 || !lam_n) return fail(ctx, GKS_EINVAL, "U_n, lam_np1 or lam_n is NULL");
    const size_t sb = state_bytes(ctx), gb = (size_t)ctx->batch * ctx->ncell * sizeof(double);
    if (ranges_overlap(lam_n, lam_np1, sb) || ranges_overlap(lam_n, U_n, sb))
        return fail(ctx, GKS_EINVAL, "lam_n overlaps lam_np1 or U_n");
    if (g_epsinv && g_muinv && ranges_overlap(g_epsinv, g_muinv, gb))
        return fail(ctx, GKS_EINVAL, "g_epsinv and g_muinv overlap");
    if (!std::isfinite(t_n)) return fail(ctx, GKS_EINVAL, "t_n is not finite");
    return check_device(ctx);
}

gks_status ensure_out(gks_ctx *x, size_t count)
{
    if (x->d_out_count < count) {
        if (x->d_out) hipFree(x->d_out);
        x->d_out = nullptr;
        x->d_out_count = 0;
        if (hipMalloc((void **)&x->d_out, count * sizeof(double)) != hipSuccess)
            return fail(x, GKS_ENOMEM, "cannot allocate %zu doubles of device memory", count);
        x->d_out_count = count;
    }
    if (x->h_out_count < count) {
        if (x->h_out) hipHostFree(x->h_out);
        x->h_out = nullptr;
        x->h_out_count = 0;
        if (hipHostMalloc((void **)&x->h_out, count * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return fail(x, GKS_ENOMEM, "cannot allocate %zu doubles of pinned host memory", count);
        x->h_out_count = count;
    }
    return GKS_OK;
}

gks_status launch_energy_into(gks_ctx *x, const void *U, double *dst)
{
    const double vol = x->h[0] * x->h[1] * (x->kind == GKS_CART3D ? x->h[2] : 1.0);
    const double *cell_vol = (x->kind == GKS_TRI2D || x->kind == GKS_TET3D) ? x->d_area : nullptr;
    // E components first, then H, then the potentials (weight 1)
    const bool em = x->model == GKS_EM3D || x->model == GKS_EM3D_PHM;
    const int nE = em ? 3 : 1, nH = em ? 3 : 2;
    int e;
    if (x->prec == GKS_FP64)
        e = launch_energy<double>((const double *)U, (const double *)x->epsinv, (const double *)x->muinv, x->ncell,
                                  x->nfields, nE, nH, (int32_t)x->batch, cell_vol, vol, x->d_partial, x->nblk, dst,
                                  x->stream);
    else
        e = launch_energy<float>((const float *)U, (const float *)x->epsinv, (const float *)x->muinv, x->ncell,
                                 x->nfields, nE, nH, (int32_t)x->batch, cell_vol, vol, x->d_partial, x->nblk, dst,
                                 x->stream);
    if (e) return hip_fail(x, e, "energy launch");
    return GKS_OK;
}

gks_status validate_box(gks_ctx *x, const int64_t *box)
{
    if (!box) return fail(x, GKS_EINVAL, "box is NULL");
    if (x->kind == GKS_TRI2D || x->kind == GKS_TET3D) return fail(x, GKS_ESTATE, "probe boxes need a Cartesian mesh");
    for (int d = 0; d < 3; ++d) {
        const int64_t a = box[2 * d], b = box[2 * d + 1];
        if (a < 0 || b > x->n[d] || a >= b) return fail(x, GKS_EINVAL, "box axis %d [%lld, %lld) outside [0, %lld)", d,
                                                          (long long)a, (long long)b, (long long)x->n[d]);
    }
    return GKS_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" const char *gks_last_error(const gks_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

extern "C" gks_status gks_init_mesh(const gks_mesh_desc *m, const gks_params *p, void *hip_stream, gks_ctx **out)
{
    if (!out) return fail(nullptr, GKS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!m || !p) return fail(nullptr, GKS_EINVAL, "mesh or params is NULL");
    if (m->precision != GKS_FP64 && m->precision != GKS_FP32) return fail(nullptr, GKS_EINVAL, "bad precision %d", m->precision);
    if (m->batch < 1 || m->batch > 4096) return fail(nullptr, GKS_EINVAL, "batch %lld not in [1, 4096]", (long long)m->batch);
    if (!(p->c > 0) || !std::isfinite(p->c)) return fail(nullptr, GKS_EINVAL, "c must be positive and finite");
    if (!(p->tau_over_dt >= 0)) return fail(nullptr, GKS_EINVAL, "tau_over_dt must be >= 0");
    if (p->energy_every < 0) return fail(nullptr, GKS_EINVAL, "energy_every must be >= 0");
    if (!(p->unstable_growth >= 0)) return fail(nullptr, GKS_EINVAL, "unstable_growth must be >= 0");
    if (p->gradient != GKS_GRAD_GREEN_GAUSS && p->gradient != GKS_GRAD_LSQ)
        return fail(nullptr, GKS_EINVAL, "gradient %d is neither Green-Gauss (0) nor least squares (1)", p->gradient);
    if (p->limiter != GKS_LIMITER_NONE && p->limiter != GKS_LIMITER_MINMOD)
        return fail(nullptr, GKS_EINVAL, "limiter %d is neither none (0) nor minmod (1)", p->limiter);
    if (p->limiter != GKS_LIMITER_NONE && (m->kind == GKS_TRI2D || m->kind == GKS_TET3D))
        return fail(nullptr, GKS_EINVAL, "the slope limiter is defined on Cartesian grids only");
    if (m->kind == GKS_TET3D && p->gradient != GKS_GRAD_GREEN_GAUSS)
        return fail(nullptr, GKS_EINVAL, "tetrahedral meshes take Green-Gauss gradients (least squares grows there)");
    const bool phm = m->model == GKS_TM2D_PHM || m->model == GKS_EM3D_PHM;
    if (phm) {
        if (!(p->chi >= 0.0 && p->chi <= 1.0) || !(p->gamma >= 0.0 && p->gamma <= 1.0))
            return fail(nullptr, GKS_EINVAL, "chi and gamma must lie in [0, 1] (divergence waves at most as fast as c)");
        if (m->kind == GKS_TRI2D && m->model != GKS_TM2D_PHM)
            return fail(nullptr, GKS_EINVAL, "triangle meshes carry TM2D or TM2D_PHM fields");
        if (m->kind == GKS_TET3D) return fail(nullptr, GKS_EINVAL, "tetrahedral meshes carry EM3D fields");
        if (p->limiter != GKS_LIMITER_NONE)
            return fail(nullptr, GKS_EINVAL, "the slope limiter is not available with the PHM fields");
    } else if (p->chi != 0.0 || p->gamma != 0.0) {
        return fail(nullptr, GKS_EINVAL, "chi and gamma are PHM couplings: they must be 0 for model %d", m->model);
    }

    TriGeometry tri;
    TetGeometry tet;
    gks_ctx *x = new (std::nothrow) gks_ctx();
    if (!x) return fail(nullptr, GKS_ENOMEM, "cannot allocate the context");
    x->kind = m->kind;
    x->model = m->model;
    x->prec = m->precision;
    x->batch = m->batch;
    x->c = p->c;
    if (phm) {
        x->chi = p->chi;
        x->gamma = p->gamma;
    }
    x->energy_every = p->energy_every;
    x->limiter = p->limiter;
    x->unstable_growth = p->unstable_growth;
    x->stream = (hipStream_t)hip_stream;
    auto bail = [&](gks_status st) {
        g_init_error = x->err;
        gks_destroy(x);
        return st;
    };

    if (m->kind == GKS_CART2D || m->kind == GKS_CART3D) {
        const int nd = (m->kind == GKS_CART2D) ? 2 : 3;
        if ((m->kind == GKS_CART2D && m->model != GKS_TM2D && m->model != GKS_TM2D_PHM) ||
            (m->kind == GKS_CART3D && m->model != GKS_EM3D && m->model != GKS_EM3D_PHM))
            return bail(fail(x, GKS_EINVAL,
                             "Cartesian 2D grids carry TM2D (or TM2D_PHM) fields and 3D grids EM3D (or EM3D_PHM) fields"));
        for (int d = 0; d < 3; ++d) {
            const int64_t nn = (d < nd) ? m->n[d] : 1;
            if (d < nd && (nn < 2 || nn > (1 << 30)))
                return bail(fail(x, GKS_EINVAL, "n[%d] = %lld must be in [2, 2^30]", d, (long long)m->n[d]));
            if (d < nd && !(m->hi[d] > m->lo[d]))
                return bail(fail(x, GKS_EINVAL, "hi[%d] must exceed lo[%d]", d, d));
            x->n[d] = nn;
            x->lo[d] = (d < nd) ? m->lo[d] : 0.0;
            x->hi[d] = (d < nd) ? m->hi[d] : 1.0;
            x->h[d] = (x->hi[d] - x->lo[d]) / (double)nn;
        }
        for (int s = 0; s < 2 * nd; ++s) {
            if (m->bc[s] < GKS_BC_PERIODIC || m->bc[s] > GKS_BC_PEC)
                return bail(fail(x, GKS_EINVAL, "bc[%d] = %d is not a boundary type", s, m->bc[s]));
            x->bc[s] = m->bc[s];
        }
        for (int d = 0; d < nd; ++d)
            if ((x->bc[2 * d] == GKS_BC_PERIODIC) != (x->bc[2 * d + 1] == GKS_BC_PERIODIC))
                return bail(fail(x, GKS_EINVAL, "axis %d is periodic on one side only", d));
        x->ncell = x->n[0] * x->n[1] * x->n[2];
        x->nfields = (m->model == GKS_TM2D) ? 3 : (m->model == GKS_TM2D_PHM) ? 4 : (m->model == GKS_EM3D) ? 6 : 8;
        if ((int64_t)x->nfields * x->ncell > ((int64_t)1 << 31) - 1)
            return bail(fail(x, GKS_EINVAL, "grid too large for 32-bit field indexing"));
        // the kernels address one batch item's fields with 32-bit byte offsets
        const int64_t esz = (m->precision == GKS_FP64) ? 8 : 4;
        if ((int64_t)x->nfields * x->ncell * esz > (int64_t)0xFFFFFFFF)
            return bail(fail(x, GKS_EINVAL, "grid too large: one batch item's fields exceed 4 GiB"));
        const double hmin = (nd == 2) ? std::min(x->h[0], x->h[1]) : std::min(x->h[0], std::min(x->h[1], x->h[2]));
        x->dt = (p->dt > 0) ? p->dt : p->cfl * hmin / p->c;
        if (!(x->dt > 0) || !std::isfinite(x->dt)) return bail(fail(x, GKS_EINVAL, "dt must be positive (set dt or cfl)"));
        const double nu = p->c * x->dt / hmin;
        // Largest Courant numbers at which the amplification factor of every Fourier mode
        // stays <= 1 (tau <= 0.01 dt).  2D: 0.5 for the D2Q4 step; with the psi coupling the
        // limit falls with gamma (0.49, 0.47, 0.44, 0.42 at gamma = 1/4 .. 1; at 0.5 and
        // gamma = 1 a mode gains 11% per step).  3D: the D3Q4 step grows above 1/3 (about 10%
        // per step at 1/2); with the potentials coupled (chi = gamma = 1) above 0.30 (2.6%
        // per step at 1/3).
        const bool cleaning = (m->model == GKS_TM2D_PHM && p->gamma > 0.0) ||
                              (m->model == GKS_EM3D_PHM && (p->chi > 0.0 || p->gamma > 0.0));
        const double numax = (nd == 2) ? (cleaning ? 0.42 : 0.5) : (cleaning ? 0.3 : 1.0 / 3.0);
        const char *lim = (nd == 2) ? (cleaning ? "0.42" : "0.5") : (cleaning ? "0.3" : "1/3");
        if (nu > numax * (1 + 1e-12))
            return bail(fail(x, GKS_EINVAL, "Courant number c dt / h = %g exceeds the stability limit %s of the %dD %sstep",
                             nu, lim, nd, cleaning ? "PHM " : ""));
    } else if (m->kind == GKS_TRI2D) {
        if (m->model != GKS_TM2D && m->model != GKS_TM2D_PHM)
            return bail(fail(x, GKS_EINVAL, "triangle meshes carry TM2D or TM2D_PHM fields"));
        char err[256];
        if (!build_tri_geometry(m, p->gradient, tri, err, sizeof err)) return bail(fail(x, GKS_EINVAL, "%s", err));
        x->ncell = m->ncells;
        x->n[0] = m->ncells;
        x->nfields = (m->model == GKS_TM2D_PHM) ? 4 : 3;
        if ((int64_t)x->nfields * x->ncell * ((m->precision == GKS_FP64) ? 8 : 4) > (int64_t)0xFFFFFFFF)
            return bail(fail(x, GKS_EINVAL, "mesh too large: one batch item's fields exceed 4 GiB"));
        // the step is stable for c dt <= 0.5 x (smallest inradius 2|Omega|/perimeter)
        x->dt = (p->dt > 0) ? p->dt : p->cfl * tri.rmin / p->c;
        if (!(x->dt > 0) || !std::isfinite(x->dt)) return bail(fail(x, GKS_EINVAL, "dt must be positive (set dt or cfl)"));
        const double nu = p->c * x->dt / tri.rmin;
        if (nu > 0.5 * (1 + 1e-12))
            return bail(fail(x, GKS_EINVAL, "c dt / (smallest inradius) = %g exceeds 0.5", nu));
    } else if (m->kind == GKS_TET3D) {
        if (m->model != GKS_EM3D) return bail(fail(x, GKS_EINVAL, "tetrahedral meshes carry EM3D fields"));
        char err[256];
        if (!build_tet_geometry(m, tet, err, sizeof err)) return bail(fail(x, GKS_EINVAL, "%s", err));
        x->ncell = m->ncells;
        x->nface = m->nfaces;
        x->n[0] = m->ncells;
        x->nfields = 6;
        if ((int64_t)6 * std::max(x->ncell, x->nface) * ((m->precision == GKS_FP64) ? 8 : 4) > (int64_t)0xFFFFFFFF)
            return bail(fail(x, GKS_EINVAL, "mesh too large: one batch item's fields or face fluxes exceed 4 GiB"));
        // as on triangles: c dt <= 0.5 x (smallest inradius 3|Omega|/surface)
        x->dt = (p->dt > 0) ? p->dt : p->cfl * tet.rmin / p->c;
        if (!(x->dt > 0) || !std::isfinite(x->dt)) return bail(fail(x, GKS_EINVAL, "dt must be positive (set dt or cfl)"));
        const double nu = p->c * x->dt / tet.rmin;
        if (nu > 0.5 * (1 + 1e-12))
            return bail(fail(x, GKS_EINVAL, "c dt / (smallest inradius) = %g exceeds 0.5", nu));
    } else {
        return bail(fail(x, GKS_EINVAL, "bad mesh kind %d", m->kind));
    }

    x->tau = p->tau_over_dt * x->dt;
    flux_coefficients(x->dt, x->tau, x->C);

    // face operators: local frames of the x-, y- (and z-) faces
    char err[256];
    if (x->kind == GKS_TRI2D &&
        !tri_face_operator(x->model, x->c, x->chi, x->gamma, x->C, x->k0[0], x->ke[0], x->kh[0], err, sizeof err))
        return bail(fail(x, GKS_EINVAL, "%s", err));
    if (x->kind == GKS_TET3D && !tet_face_operator(x->c, x->C, x->k0[0], x->ke[0], x->kh[0], err, sizeof err))
        return bail(fail(x, GKS_EINVAL, "%s", err));
    if (x->kind == GKS_CART2D || x->kind == GKS_CART3D) {
        // the kernels feed full central differences U(i+1) - U(i-1) = 2 h dU/dx
        const int nax = (x->kind == GKS_CART2D) ? 2 : 3;
        for (int ax = 0; ax < nax; ++ax)
            if (!cart_face_operator(x->model, ax, x->c, x->chi, x->gamma, x->C, x->h, 2.0, x->k0[ax], x->ke[ax],
                                    x->kh[ax], err, sizeof err))
                return bail(fail(x, GKS_EINVAL, "%s", err));
    }

    if (hipGetDevice(&x->device) != hipSuccess) return bail(fail(x, GKS_EDEVICE, "no HIP device"));
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, x->device) == hipSuccess && ncu > 0)
            x->ncu = ncu;
    }
    if (x->kind == GKS_CART2D) {
        const int ntx = (int)((x->n[0] + cart2d_tile_x(x->prec) - 1) / cart2d_tile_x(x->prec));
        const std::vector<int32_t> tab = cart2d_tile_table((int)x->n[1], (int)x->batch, x->prec, ntx, x->tiles_per_band);
        x->ntile_rows = (int32_t)(tab.size() / 4);
        if (hipMalloc((void **)&x->d_tiles, tab.size() * sizeof(int32_t)) != hipSuccess)
            return bail(fail(x, GKS_ENOMEM, "cannot allocate the tile table"));
        const int e = hipMemcpy(x->d_tiles, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e) return bail(hip_fail(x, e, "tile table upload"));
        // the paired kernel: TM fields (with or without psi; the limiter, TM only)
        if (x->model == GKS_TM2D || x->model == GKS_TM2D_PHM) {
            const int ntx2 = (int)((x->n[0] + cart2d_pair_tile_x(x->prec) - 1) / cart2d_pair_tile_x(x->prec));
            const std::vector<int32_t> tab2 =
                cart2d_pair_tile_table((int)x->n[1], (int)x->batch, x->prec, ntx2, x->pair_tiles_per_band);
            if (!tab2.empty()) {
                if (hipMalloc((void **)&x->d_pair_tiles, tab2.size() * sizeof(int32_t)) != hipSuccess)
                    return bail(fail(x, GKS_ENOMEM, "cannot allocate the paired tile table"));
                const int e2 = hipMemcpy(x->d_pair_tiles, tab2.data(), tab2.size() * sizeof(int32_t),
                                         hipMemcpyHostToDevice);
                if (e2) return bail(hip_fail(x, e2, "paired tile table upload"));
            }
        }
    }
    if (x->kind == GKS_CART2D && x->model == GKS_TM2D) {
        // the device address of the allocation-free adjoint's static scratch (once per device)
        x->static_scratch_err = adjoint_static_scratch(&x->static_scratch);
        if (x->static_scratch_err) x->static_scratch = nullptr;
    }
    if (x->kind == GKS_CART3D)
        x->tile_z = cart3d_pick_tile_z((int)x->n[0], (int)x->n[1], (int)x->n[2], (int)x->batch, x->ncu, x->prec,
                                       x->nfields);
    if (x->kind == GKS_TRI2D) {
        gks_status st = (x->prec == GKS_FP64) ? upload_tri<double>(x, tri) : upload_tri<float>(x, tri);
        if (st) return bail(st);
    }
    if (x->kind == GKS_TET3D) {
        gks_status st = (x->prec == GKS_FP64) ? upload_tet<double>(x, tet) : upload_tet<float>(x, tet);
        if (st) return bail(st);
    }
    {
        gks_status st = upload_ops(x);
        if (st) return bail(st);
    }
    x->nblk = 1024;
    if (hipMalloc((void **)&x->d_partial, sizeof(double) * x->nblk * x->batch) != hipSuccess)
        return bail(fail(x, GKS_ENOMEM, "cannot allocate reduction scratch"));
    *out = x;
    return GKS_OK;
}

extern "C" gks_status gks_destroy(gks_ctx *ctx)
{
    if (!ctx) return GKS_OK;
    if (ctx->d_ops) hipFree(ctx->d_ops);
    if (ctx->d_tiles) hipFree(ctx->d_tiles);
    if (ctx->d_pair_tiles) hipFree(ctx->d_pair_tiles);
    if (ctx->pingpong) hipFree(ctx->pingpong);
    if (ctx->d_partial) hipFree(ctx->d_partial);
    if (ctx->d_out) hipFree(ctx->d_out);
    if (ctx->h_out) hipHostFree(ctx->h_out);
    for (hipEvent_t &ev : ctx->rec_ev)
        if (ev) hipEventDestroy(ev);
    if (ctx->d_src_cells) hipFree(ctx->d_src_cells);
    if (ctx->d_src_w) hipFree(ctx->d_src_w);
    if (ctx->adj_scratch) hipFree(ctx->adj_scratch);
    if (ctx->d_tri_nb) hipFree(ctx->d_tri_nb);
    if (ctx->d_tri_geo) hipFree(ctx->d_tri_geo);
    if (ctx->d_area) hipFree(ctx->d_area);
    if (ctx->d_tet_nb) hipFree(ctx->d_tet_nb);
    if (ctx->d_tet_cf) hipFree(ctx->d_tet_cf);
    if (ctx->d_tet_fc) hipFree(ctx->d_tet_fc);
    if (ctx->d_tet_cgeo) hipFree(ctx->d_tet_cgeo);
    if (ctx->d_tet_fgeo) hipFree(ctx->d_tet_fgeo);
    if (ctx->d_flux) hipFree(ctx->d_flux);
    if (ctx->d_grad) hipFree(ctx->d_grad);
    delete ctx;
    return GKS_OK;
}

extern "C" gks_status gks_get_dt(const gks_ctx *ctx, double *dt_out)
{
    if (!ctx || !dt_out) return GKS_EINVAL;
    *dt_out = ctx->dt;
    return GKS_OK;
}

extern "C" gks_status gks_set_material(gks_ctx *ctx, const void *epsinv, const void *muinv)
{
    if (!ctx) return GKS_EINVAL;
    ctx->epsinv = epsinv;
    ctx->muinv = muinv;
    return GKS_OK;
}

extern "C" gks_status gks_set_point_source(gks_ctx *ctx, int64_t n, const int64_t *cells, const double *weight,
                                           double J0, double t0, double sigma_t)
{
    if (!ctx) return GKS_EINVAL;
    if (n < 0 || n > 4096) return fail(ctx, GKS_EINVAL, "source count %lld not in [0, 4096]", (long long)n);
    if (n > 0 && (!cells || !weight)) return fail(ctx, GKS_EINVAL, "cells or weight is NULL");
    if (n > 0 && !(sigma_t > 0)) return fail(ctx, GKS_EINVAL, "sigma_t must be positive");
    // merge repeated cells (the scatter kernel writes each cell once)
    std::map<int64_t, double> merged;
    for (int64_t s = 0; s < n; ++s) {
        if (cells[s] < 0 || cells[s] >= ctx->ncell)
            return fail(ctx, GKS_EINVAL, "source cell %lld outside [0, %lld)", (long long)cells[s], (long long)ctx->ncell);
        merged[cells[s]] += weight[s];
    }
    ctx->src_cells.clear();
    ctx->src_w.clear();
    for (auto &kv : merged) {
        ctx->src_cells.push_back(kv.first);
        ctx->src_w.push_back(kv.second);
    }
    ctx->J0 = J0;
    ctx->t0 = t0;
    ctx->sigma_t = (n > 0) ? sigma_t : 1.0;
    if (ctx->d_src_cells) hipFree(ctx->d_src_cells);
    if (ctx->d_src_w) hipFree(ctx->d_src_w);
    ctx->d_src_cells = nullptr;
    ctx->d_src_w = nullptr;
    const size_t m = ctx->src_cells.size();
    if (m > 0) {
        if (hipMalloc((void **)&ctx->d_src_cells, m * sizeof(int64_t)) != hipSuccess ||
            hipMalloc((void **)&ctx->d_src_w, m * sizeof(double)) != hipSuccess)
            return fail(ctx, GKS_ENOMEM, "cannot allocate the source list");
        int e = hipMemcpy(ctx->d_src_cells, ctx->src_cells.data(), m * sizeof(int64_t), hipMemcpyHostToDevice);
        if (!e) e = hipMemcpy(ctx->d_src_w, ctx->src_w.data(), m * sizeof(double), hipMemcpyHostToDevice);
        if (e) return hip_fail(ctx, e, "source upload");
    }
    return GKS_OK;
}

extern "C" gks_status gks_step(gks_ctx *ctx, const void *U_in, void *U_out, double t_n)
{
    if (!ctx) return GKS_EINVAL;
    if (!U_in || !U_out) return fail(ctx, GKS_EINVAL, "U_in or U_out is NULL");
    if (ranges_overlap(U_in, U_out, state_bytes(ctx)))
        return fail(ctx, GKS_EINVAL, "U_in and U_out overlap (the step is out of place)");
    if (!std::isfinite(t_n)) return fail(ctx, GKS_EINVAL, "t_n is not finite");
    gks_status st = check_device(ctx);
    if (st) return st;
    return do_step(ctx, U_in, U_out, t_n);
}

namespace {

// Checks energy record r (host copy in ctx->h_out) of gks_run: not finite -> GKS_ENONFINITE,
// above unstable_growth times the first record -> GKS_EUNSTABLE.
gks_status check_record(gks_ctx *x, int64_t r, int64_t every)
{
    for (int64_t b = 0; b < x->batch; ++b) {
        const double w = x->h_out[r * x->batch + b], w0 = x->h_out[b];
        if (!std::isfinite(w))
            return fail(x, GKS_ENONFINITE, "energy of batch item %lld is not finite after step %lld", (long long)b,
                        (long long)((r + 1) * every));
        if (x->unstable_growth > 0 && w > x->unstable_growth * w0)
            return fail(x, GKS_EUNSTABLE, "energy of batch item %lld grew by %g after step %lld", (long long)b, w / w0,
                        (long long)((r + 1) * every));
    }
    return GKS_OK;
}

}  // namespace

extern "C" gks_status gks_run(gks_ctx *ctx, void *U, int64_t nsteps, double t0, double *energy_host)
{
    if (!ctx) return GKS_EINVAL;
    if (!U) return fail(ctx, GKS_EINVAL, "U is NULL");
    if (nsteps < 0) return fail(ctx, GKS_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(t0)) return fail(ctx, GKS_EINVAL, "t0 is not finite");
    gks_status st = check_device(ctx);
    if (st) return st;
    const size_t bytes = state_bytes(ctx);
    if (ctx->pingpong_bytes < bytes) {
        if (ctx->pingpong) hipFree(ctx->pingpong);
        ctx->pingpong = nullptr;
        ctx->pingpong_bytes = 0;
        if (hipMalloc(&ctx->pingpong, bytes) != hipSuccess)
            return fail(ctx, GKS_ENOMEM, "cannot allocate the %zu-byte ping-pong state", bytes);
        ctx->pingpong_bytes = bytes;
    }
    const int64_t every = (energy_host && ctx->energy_every > 0) ? ctx->energy_every : 0;
    const int64_t nrec = every ? nsteps / every : 0;
    if (nrec) {
        st = ensure_out(ctx, (size_t)nrec * ctx->batch);
        if (st) return st;
        for (hipEvent_t &ev : ctx->rec_ev)
            if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
                return fail(ctx, GKS_EDEVICE, "cannot create the energy record events");
    }
    // Each energy record is copied to pinned host memory as soon as it is computed; record r - 1
    // is checked once record r has been enqueued (the host then waits for the GPU to finish the
    // steps of record r - 1 only, so that the steps of record r keep it busy meanwhile).  The run
    // stops at the first failing record, at most energy_every steps after it.
    void *cur = U, *nxt = ctx->pingpong;
    int64_t nenq = 0, nchecked = 0;   // records enqueued / checked
    gks_status bad = GKS_OK;
    int e = 0;
    // Two steps per launch where the paired kernel applies, except across an energy record.
    const bool pair = ctx->kind == GKS_CART2D && ctx->d_pair_tiles && ctx->src_cells.size() <= 1;
    for (int64_t k = 0; k < nsteps && bad == GKS_OK;) {
        const bool two = pair && k + 1 < nsteps && !(every && (k + 1) % every == 0);
        const double tk = t0 + (double)k * ctx->dt, tk1 = t0 + (double)(k + 1) * ctx->dt;
        if (two)
            st = ctx->prec == GKS_FP64 ? step2_cart2d<double>(ctx, cur, nxt, tk, tk1)
                                       : step2_cart2d<float>(ctx, cur, nxt, tk, tk1);
        else
            st = do_step(ctx, cur, nxt, tk);
        if (st) return st;
        std::swap(cur, nxt);
        k += two ? 2 : 1;
        if (every && k % every == 0) {
            const int64_t r = nenq++;
            double *dst = ctx->d_out + r * ctx->batch;
            st = launch_energy_into(ctx, cur, dst);
            if (st) return st;
            e = hipMemcpyAsync(ctx->h_out + r * ctx->batch, dst, ctx->batch * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream);
            if (!e) e = hipEventRecord(ctx->rec_ev[r & 1], ctx->stream);
            if (e) return hip_fail(ctx, e, "energy readback");
            if (r >= 1) {
                e = hipEventSynchronize(ctx->rec_ev[(r - 1) & 1]);
                if (e) return hip_fail(ctx, e, "energy readback");
                bad = check_record(ctx, r - 1, every);
                nchecked = r;
            }
        }
    }
    if (cur != U) {
        e = hipMemcpyAsync(U, cur, bytes, hipMemcpyDeviceToDevice, ctx->stream);
        if (e) return hip_fail(ctx, e, "state copy");
    }
    if (nenq) {
        e = hipStreamSynchronize(ctx->stream);
        if (e) return hip_fail(ctx, e, "energy readback");
        for (int64_t r = nchecked; r < nenq && bad == GKS_OK; ++r) bad = check_record(ctx, r, every);
        std::memcpy(energy_host, ctx->h_out, (size_t)nenq * ctx->batch * sizeof(double));
    }
    return bad;
}

extern "C" gks_status gks_energy(gks_ctx *ctx, const void *U, double *out_host)
{
    if (!ctx) return GKS_EINVAL;
    if (!U || !out_host) return fail(ctx, GKS_EINVAL, "U or out_host is NULL");
    gks_status st = check_device(ctx);
    if (st) return st;
    st = ensure_out(ctx, (size_t)ctx->batch);
    if (st) return st;
    st = launch_energy_into(ctx, U, ctx->d_out);
    if (st) return st;
    int e = hipMemcpyAsync(ctx->h_out, ctx->d_out, ctx->batch * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (!e) e = hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(ctx, e, "energy readback");
    std::memcpy(out_host, ctx->h_out, ctx->batch * sizeof(double));
    return GKS_OK;
}

extern "C" gks_status gks_probe_energy(gks_ctx *ctx, const void *U, const int64_t *box, double *out_host)
{
    if (!ctx) return GKS_EINVAL;
    if (!U || !out_host) return fail(ctx, GKS_EINVAL, "U or out_host is NULL");
    gks_status st = validate_box(ctx, box);
    if (st) return st;
    st = check_device(ctx);
    if (st) return st;
    st = ensure_out(ctx, (size_t)ctx->batch);
    if (st) return st;
    const double vol = ctx->h[0] * ctx->h[1] * (ctx->kind == GKS_CART3D ? ctx->h[2] : 1.0);
    const int ezf = (ctx->model == GKS_EM3D || ctx->model == GKS_EM3D_PHM) ? 2 : 0;
    int e = (ctx->prec == GKS_FP64)
                ? launch_probe_energy<double>((const double *)U, ctx->n[0], ctx->n[1], ctx->n[2], ctx->nfields, ezf,
                                              (int32_t)ctx->batch, box, vol, ctx->d_partial, ctx->nblk, ctx->d_out,
                                              ctx->stream)
                : launch_probe_energy<float>((const float *)U, ctx->n[0], ctx->n[1], ctx->n[2], ctx->nfields, ezf,
                                             (int32_t)ctx->batch, box, vol, ctx->d_partial, ctx->nblk, ctx->d_out,
                                             ctx->stream);
    if (!e) e = hipMemcpyAsync(ctx->h_out, ctx->d_out, ctx->batch * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (!e) e = hipStreamSynchronize(ctx->stream);
    if (e) return hip_fail(ctx, e, "probe energy");
    std::memcpy(out_host, ctx->h_out, ctx->batch * sizeof(double));
    return GKS_OK;
}

extern "C" gks_status gks_probe_energy_grad(gks_ctx *ctx, const void *U, const int64_t *box, void *lam)
{
    if (!ctx) return GKS_EINVAL;
    if (!U || !lam) return fail(ctx, GKS_EINVAL, "U or lam is NULL");
    if (ranges_overlap(U, lam, state_bytes(ctx))) return fail(ctx, GKS_EINVAL, "U and lam overlap");
    gks_status st = validate_box(ctx, box);
    if (st) return st;
    st = check_device(ctx);
    if (st) return st;
    const double vol = ctx->h[0] * ctx->h[1] * (ctx->kind == GKS_CART3D ? ctx->h[2] : 1.0);
    const int ezf = (ctx->model == GKS_EM3D || ctx->model == GKS_EM3D_PHM) ? 2 : 0;
    int e = (ctx->prec == GKS_FP64)
                ? launch_probe_grad<double>((const double *)U, (double *)lam, ctx->n[0], ctx->n[1], ctx->n[2],
                                            ctx->nfields, ezf, (int32_t)ctx->batch, box, vol, ctx->stream)
                : launch_probe_grad<float>((const float *)U, (float *)lam, ctx->n[0], ctx->n[1], ctx->n[2],
                                           ctx->nfields, ezf, (int32_t)ctx->batch, box, vol, ctx->stream);
    if (e) return hip_fail(ctx, e, "probe gradient");
    return GKS_OK;
}

extern "C" gks_status gks_adjoint_step(gks_ctx *ctx, const void *U_n, const void *lam_np1, void *lam_n,
                                       double *g_epsinv, double *g_muinv, double t_n)
{
    if (!ctx) return GKS_EINVAL;
    gks_status st = check_adjoint(ctx, U_n, lam_np1, lam_n, g_epsinv, g_muinv, t_n);
    if (st) return st;
    const size_t bytes = adjoint_scratch_bytes(ctx);
    if (ctx->adj_scratch_bytes < bytes) {
        if (ctx->adj_scratch) hipFree(ctx->adj_scratch);
        ctx->adj_scratch = nullptr;
        ctx->adj_scratch_bytes = 0;
        if (hipMalloc(&ctx->adj_scratch, bytes) != hipSuccess)
            return fail(ctx, GKS_ENOMEM, "cannot allocate the %zu-byte adjoint scratch", bytes);
        ctx->adj_scratch_bytes = bytes;
    }
    return ctx->prec == GKS_FP64
               ? adjoint_cart2d<double>(ctx, U_n, lam_np1, lam_n, g_epsinv, g_muinv, t_n, ctx->adj_scratch)
               : adjoint_cart2d<float>(ctx, U_n, lam_np1, lam_n, g_epsinv, g_muinv, t_n, ctx->adj_scratch);
}

// ---------------------------------------------------------------- allocation-free adjoint step
extern "C" gks_status gks_adjoint_step_noalloc(gks_ctx *ctx, const void *U_n, const void *lam_np1, void *lam_n,
                                               double *g_epsinv, double *g_muinv, double t_n)
{
    if (!ctx) return GKS_EINVAL;
    if (ctx->kind == GKS_CART2D && ctx->model == GKS_TM2D) {
        const size_t bytes = adjoint_scratch_bytes(ctx);
        if (bytes > ADJ_STATIC_SCRATCH_BYTES)
            return fail(ctx, GKS_EINVAL,
                        "this grid and batch need %zu bytes of adjoint scratch; the static scratch holds %zu "
                        "(use gks_adjoint_step)",
                        bytes, (size_t)ADJ_STATIC_SCRATCH_BYTES);
    }
    gks_status st = check_adjoint(ctx, U_n, lam_np1, lam_n, g_epsinv, g_muinv, t_n);
    if (st) return st;
    if (!ctx->static_scratch)
        return fail(ctx, GKS_EDEVICE, "the static adjoint scratch of this device is not available (lookup failed: %s)",
                    hipGetErrorString((hipError_t)ctx->static_scratch_err));
    return ctx->prec == GKS_FP64
               ? adjoint_cart2d<double>(ctx, U_n, lam_np1, lam_n, g_epsinv, g_muinv, t_n, ctx->static_scratch)
               : adjoint_cart2d<float>(ctx, U_n, lam_np1, lam_n, g_epsinv, g_muinv, t_n, ctx->static_scratch);
}
