// Reverse-mode adjoint of the 2D TM Cartesian GKS step.
//
// The forward step is U' = U - M^{-1} div Phi(pad(U)) + dt M^{-1} S, with pad() the ghost
// extension of the grid by the boundary conditions (periodic wrap, PEC mirror with signs,
// non-reflecting clamp for the Green-Gauss gradient) and Phi the face fluxes, each a sparse
// linear form K(m_s) w_f of the left/right states and central differences (the same operators
// as the forward kernel).  For lambda' = dJ/dU' the adjoint is
//     lambda = pad^T psi,   psi(p) = lambda'(p) - sum_f W_f^T K(m_s)^T a_f,
//     a_f = mu_L - mu_R,    mu = (1/eps, 1/mu) lambda' on cells, 0 on ghost positions,
// and the material gradients collect, per cell, -lambda'.div(Phi) (the 1/eps, 1/mu factors of
// the update) plus, per face, -a_f . d Phi_f / d m for both cells of the face (the mean face
// material of the equilibrium time derivative).  Three kernels:
//   1. faces:  one thread per padded position p next to a cell gathers the 13-point stencil of
//      U (mapped through the boundary conditions), lambda' and the materials, evaluates the four
//      faces of p (forward flux, transposed operator, material sensitivities) and stores p's
//      share: the direct adjoint Ubar(p) and the adjoints of its two central differences
//      (Dxbar, Dybar), and its material-gradient contributions;
//   2. psi:    the transposed differences, psi(p) = [cell] lambda'(p) - Ubar(p)
//              - Dxbar(p-x) + Dxbar(p+x) - Dybar(p-y) + Dybar(p+y), written to lambda on cells
//              and to a ghost buffer on ghost positions;
//   3. fold:   each cell within two cells of a side adds the psi and material gradients of the
//      ghost positions that read it (pad^T), with the mirror signs.
// Everything runs in a fixed order (no atomics), so the adjoint is deterministic.
#include "gks_device.h"

namespace gks {

constexpr int ADJ_BLOCK = 256;

struct Pad2D {
    int nx, ny, px;   // px = nx + 4
    __device__ __forceinline__ int64_t idx(int i, int j) const { return (int64_t)(j + 2) * px + (i + 2); }
    __device__ __forceinline__ int64_t size() const { return (int64_t)(ny + 4) * px; }
};

template <typename T>
struct Pos {
    T u[3];        // padded field values (mirror signs applied)
    T lam[3];      // lambda' (0 on ghost positions)
    T mE, mH;      // materials of the cell read
    bool ghost;    // outside the grid
    bool nr;       // non-reflecting ghost (its side of a boundary face carries nothing)
};

template <typename T, bool HAS_EPS, bool HAS_MU>
__device__ __forceinline__ void gather(const Cart2DAdjArgs<T> &a, const T *Ub, const T *Lb, const T *Eb, const T *Mb,
                                       int64_t ncell, int i, int j, Pos<T> &p)
{
    bool mx, nrx, my, nry;
    const int sx = map_axis(i, a.nx, a.bc[0], a.bc[1], mx, nrx);
    const int sy = map_axis(j, a.ny, a.bc[2], a.bc[3], my, nry);
    const int64_t c = (int64_t)sy * a.nx + sx;
    const T sgx = mx ? T(-1) : T(1), sgy = my ? T(-1) : T(1);
    p.u[0] = Ub[c] * (sgx * sgy);      // Ez: odd in both mirrors
    p.u[1] = Ub[ncell + c] * sgx;      // Hx: odd in the x mirror
    p.u[2] = Ub[2 * ncell + c] * sgy;  // Hy: odd in the y mirror
    p.mE = HAS_EPS ? Eb[c] : T(1);
    p.mH = HAS_MU ? Mb[c] : T(1);
    p.ghost = i < 0 || i >= a.nx || j < 0 || j >= a.ny;
    p.nr = nrx || nry;
#pragma unroll
    for (int f = 0; f < 3; ++f) p.lam[f] = p.ghost ? T(0) : Lb[f * ncell + c];
}

// One face: L/R positions with their central differences dL, dR ([dn(3) dt(3)]).  Adds p's
// share (side = 0: p is L, 1: p is R) of the transposed operator to ubar/dbar, returns the
// forward flux in phi and accumulates p's material sensitivity.
template <typename P, typename T, typename Op>
__device__ __forceinline__ void face_adjoint(const Pos<T> &L, const Pos<T> &R, const T (&dL)[6], const T (&dR)[6],
                                             int side, Op K, T (&ubar)[3], T (&dnbar)[3], T (&dtbar)[3], T (&phi)[3],
                                             double &gE, double &gH)
{
    const bool zl = L.ghost && L.nr, zr = R.ghost && R.nr;
    T w[18];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        w[f] = zl ? T(0) : L.u[f];
        w[3 + f] = zr ? T(0) : R.u[f];
        w[6 + f] = zl ? T(0) : dL[f];
        w[9 + f] = zl ? T(0) : dL[3 + f];
        w[12 + f] = zr ? T(0) : dR[f];
        w[15 + f] = zr ? T(0) : dR[3 + f];
    }
    const T mE = L.mE + R.mE, mH = L.mH + R.mH;
    apply_op<P>(w, mE, mH, K, phi);
    T abar[3], mu_l[3], mu_r[3];
    mu_l[0] = L.mE * L.lam[0];
    mu_l[1] = L.mH * L.lam[1];
    mu_l[2] = L.mH * L.lam[2];
    mu_r[0] = R.mE * R.lam[0];
    mu_r[1] = R.mH * R.lam[1];
    mu_r[2] = R.mH * R.lam[2];
#pragma unroll
    for (int f = 0; f < 3; ++f) abar[f] = mu_l[f] - mu_r[f];
    T wbar[18];
#pragma unroll
    for (int q = 0; q < 18; ++q) wbar[q] = T(0);
    apply_op_transpose<P>(abar, mE, mH, K, wbar);
    const bool drop = side == 0 ? zl : zr;   // the ghost side of a non-reflecting face is not read
    if (!drop) {
        const int o = side == 0 ? 0 : 3, od = side == 0 ? 6 : 12;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            ubar[f] += wbar[o + f];
            dnbar[f] += wbar[od + f];
            dtbar[f] += wbar[od + 3 + f];
        }
    }
    T sE, sH;
    material_sens<P>(abar, w, K, sE, sH);
    gE -= (double)sE;
    gH -= (double)sH;
}

template <typename T, bool HAS_EPS, bool HAS_MU>
__global__ __launch_bounds__(ADJ_BLOCK) void adj2d_faces_kernel(Cart2DAdjArgs<T> a, T *pad9, double *padg)
{
    const Pad2D pd{a.nx, a.ny, a.nx + 4};
    const int64_t npos = pd.size();
    const int64_t t = (int64_t)blockIdx.x * ADJ_BLOCK + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= npos) return;
    const int i = (int)(t % pd.px) - 2, j = (int)(t / pd.px) - 2;
    const int64_t ncell = (int64_t)a.nx * a.ny;
    T *out = pad9 + (int64_t)b * 9 * npos;
    double *gout = padg + (int64_t)b * 2 * npos;
    // positions two layers outside the grid touch no face of a cell
    if (i < -1 || i > a.nx || j < -1 || j > a.ny) {
#pragma unroll
        for (int q = 0; q < 9; ++q) out[q * npos + t] = T(0);
        gout[t] = 0.0;
        gout[npos + t] = 0.0;
        return;
    }
    const T *Ub = a.U + (int64_t)b * 3 * ncell;
    const T *Lb = a.lam + (int64_t)b * 3 * ncell;
    const T *Eb = HAS_EPS ? a.epsinv + (int64_t)b * ncell : nullptr;
    const T *Mb = HAS_MU ? a.muinv + (int64_t)b * ncell : nullptr;

    // 13-point stencil: c = p, x-/x+ = p -+ 1, xx-/xx+ = p -+ 2, same in y, and the diagonals
    Pos<T> c, xm, xp, xmm, xpp, ym, yp, ymm, ypp, mm, pm, mp, pp;
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i, j, c);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i - 1, j, xm);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i + 1, j, xp);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i - 2, j, xmm);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i + 2, j, xpp);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i, j - 1, ym);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i, j + 1, yp);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i, j - 2, ymm);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i, j + 2, ypp);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i - 1, j - 1, mm);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i + 1, j - 1, pm);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i - 1, j + 1, mp);
    gather<T, HAS_EPS, HAS_MU>(a, Ub, Lb, Eb, Mb, ncell, i + 1, j + 1, pp);

    // central differences [d/dx(3) d/dy(3)] of the five positions p, p-+x, p-+y
    T Dc[6], Dxm[6], Dxp[6], Dym[6], Dyp[6];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        Dc[f] = xp.u[f] - xm.u[f];
        Dc[3 + f] = yp.u[f] - ym.u[f];
        Dxm[f] = c.u[f] - xmm.u[f];
        Dxm[3 + f] = mp.u[f] - mm.u[f];
        Dxp[f] = xpp.u[f] - c.u[f];
        Dxp[3 + f] = pp.u[f] - pm.u[f];
        Dym[f] = pm.u[f] - mm.u[f];
        Dym[3 + f] = c.u[f] - ymm.u[f];
        Dyp[f] = pp.u[f] - mp.u[f];
        Dyp[3 + f] = ypp.u[f] - c.u[f];
    }
    // re-ordered [dn dt] per face orientation: x-faces [dx dy], y-faces [dy dx]
    auto nt_x = [](const T (&D)[6], T (&o)[6]) {
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = D[q];
    };
    auto nt_y = [](const T (&D)[6], T (&o)[6]) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            o[f] = D[3 + f];
            o[3 + f] = D[f];
        }
    };
    T ubar[3] = {T(0), T(0), T(0)}, dxbar[3] = {T(0), T(0), T(0)}, dybar[3] = {T(0), T(0), T(0)};
    T div[3] = {T(0), T(0), T(0)};
    double gE = 0.0, gH = 0.0;
    const auto opx = scalar_ptr(a.ops), opy = scalar_ptr(a.ops + 1);
    T dA[6], dB[6], phi[3];
    // x-face left of p (p is R), x-face right of p (p is L); a face with two ghost sides touches no cell
    if (!(xm.ghost && c.ghost)) {
        nt_x(Dxm, dA);
        nt_x(Dc, dB);
        face_adjoint<PatTMx>(xm, c, dA, dB, 1, opx, ubar, dxbar, dybar, phi, gE, gH);
#pragma unroll
        for (int f = 0; f < 3; ++f) div[f] -= phi[f];
    }
    if (!(c.ghost && xp.ghost)) {
        nt_x(Dc, dA);
        nt_x(Dxp, dB);
        face_adjoint<PatTMx>(c, xp, dA, dB, 0, opx, ubar, dxbar, dybar, phi, gE, gH);
#pragma unroll
        for (int f = 0; f < 3; ++f) div[f] += phi[f];
    }
    if (!(ym.ghost && c.ghost)) {
        nt_y(Dym, dA);
        nt_y(Dc, dB);
        face_adjoint<PatTMy>(ym, c, dA, dB, 1, opy, ubar, dybar, dxbar, phi, gE, gH);
#pragma unroll
        for (int f = 0; f < 3; ++f) div[f] -= phi[f];
    }
    if (!(c.ghost && yp.ghost)) {
        nt_y(Dc, dA);
        nt_y(Dyp, dB);
        face_adjoint<PatTMy>(c, yp, dA, dB, 0, opy, ubar, dybar, dxbar, phi, gE, gH);
#pragma unroll
        for (int f = 0; f < 3; ++f) div[f] += phi[f];
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        out[f * npos + t] = ubar[f];
        out[(3 + f) * npos + t] = dxbar[f];
        out[(6 + f) * npos + t] = dybar[f];
    }
    if (!c.ghost) {
        // the 1/eps, 1/mu factors of the cell update: d/dm (-m lambda'.div) = -lambda'.div
        gE -= (double)c.lam[0] * (double)div[0];
        gH -= (double)c.lam[1] * (double)div[1] + (double)c.lam[2] * (double)div[2];
        const int64_t cc = (int64_t)j * a.nx + i;
        if (a.g_epsinv) a.g_epsinv[(int64_t)b * ncell + cc] += gE;
        if (a.g_muinv) a.g_muinv[(int64_t)b * ncell + cc] += gH;
        gout[t] = 0.0;
        gout[npos + t] = 0.0;
    } else {
        gout[t] = gE;
        gout[npos + t] = gH;
    }
}

template <typename T>
__global__ __launch_bounds__(ADJ_BLOCK) void adj2d_psi_kernel(Cart2DAdjArgs<T> a, const T *pad9, T *padpsi)
{
    const Pad2D pd{a.nx, a.ny, a.nx + 4};
    const int64_t npos = pd.size();
    const int64_t t = (int64_t)blockIdx.x * ADJ_BLOCK + threadIdx.x;
    const int b = blockIdx.y;
    if (t >= npos) return;
    const int i = (int)(t % pd.px) - 2, j = (int)(t / pd.px) - 2;
    const int64_t ncell = (int64_t)a.nx * a.ny;
    const T *in = pad9 + (int64_t)b * 9 * npos;
    auto at = [&](int q, int ii, int jj) -> T {
        if (ii < -2 || ii >= a.nx + 2 || jj < -2 || jj >= a.ny + 2) return T(0);
        return in[q * npos + pd.idx(ii, jj)];
    };
    const bool cell = i >= 0 && i < a.nx && j >= 0 && j < a.ny;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        T v = cell ? a.lam[((int64_t)b * 3 + f) * ncell + (int64_t)j * a.nx + i] : T(0);
        v -= at(f, i, j);
        v -= at(3 + f, i - 1, j);
        v += at(3 + f, i + 1, j);
        v -= at(6 + f, i, j - 1);
        v += at(6 + f, i, j + 1);
        if (cell) a.lam_out[((int64_t)b * 3 + f) * ncell + (int64_t)j * a.nx + i] = v;
        else padpsi[((int64_t)b * 3 + f) * npos + t] = v;
    }
}

// Cells within two cells of a side (the only ones a ghost position reads): the first and
// last two rows in full, then the first and last two columns of the rows between.
struct Band2D {
    int nx, ny, nrow, ncol;   // band rows (all rows if ny <= 4), band columns of the middle rows
    __host__ __device__ Band2D(int nx_, int ny_) : nx(nx_), ny(ny_), nrow(ny_ <= 4 ? ny_ : 4), ncol(nx_ <= 4 ? nx_ : 4) {}
    __host__ __device__ int64_t count() const { return (int64_t)nrow * nx + (int64_t)(ny > 4 ? ny - 4 : 0) * ncol; }
    __device__ void cell(int64_t t, int &i, int &j) const
    {
        if (t < (int64_t)nrow * nx) {
            const int r = (int)(t / nx);
            i = (int)(t % nx);
            j = (ny <= 4 || r < 2) ? r : ny - 4 + r;
        } else {
            const int64_t u = t - (int64_t)nrow * nx;
            const int c = (int)(u % ncol);
            j = 2 + (int)(u / ncol);
            i = (nx <= 4 || c < 2) ? c : nx - 4 + c;
        }
    }
};

// pad^T: each cell within two cells of a side gathers the ghost positions that read it.
template <typename T>
__global__ __launch_bounds__(ADJ_BLOCK) void adj2d_fold_kernel(Cart2DAdjArgs<T> a, const T *padpsi, const double *padg)
{
    const Pad2D pd{a.nx, a.ny, a.nx + 4};
    const int64_t npos = pd.size();
    const int64_t ncell = (int64_t)a.nx * a.ny;
    const int b = blockIdx.y;
    const Band2D band(a.nx, a.ny);
    const int64_t tb = (int64_t)blockIdx.x * ADJ_BLOCK + threadIdx.x;
    if (tb >= band.count()) return;
    int i, j;
    band.cell(tb, i, j);
    const int64_t t = (int64_t)j * a.nx + i;
    // candidate images along each axis: the cell itself and the ghost indices that map to it
    int cx[5], cy[5], nxc = 0, nyc = 0;
    T sx[5], sy[5];
    cx[nxc] = i; sx[nxc++] = T(1);
    for (int g = -2; g <= a.nx + 1; g += (g == -1 ? a.nx + 1 : 1)) {
        bool m, nr;
        if (map_axis(g, a.nx, a.bc[0], a.bc[1], m, nr) == i) { cx[nxc] = g; sx[nxc++] = m ? T(-1) : T(1); }
    }
    cy[nyc] = j; sy[nyc++] = T(1);
    for (int g = -2; g <= a.ny + 1; g += (g == -1 ? a.ny + 1 : 1)) {
        bool m, nr;
        if (map_axis(g, a.ny, a.bc[2], a.bc[3], m, nr) == j) { cy[nyc] = g; sy[nyc++] = m ? T(-1) : T(1); }
    }
    T add[3] = {T(0), T(0), T(0)};
    double gE = 0.0, gH = 0.0;
    for (int u = 0; u < nxc; ++u)
        for (int v = 0; v < nyc; ++v) {
            if (u == 0 && v == 0) continue;
            const int64_t p = pd.idx(cx[u], cy[v]);
            // signs: Ez odd in both mirrors, Hx odd in the x mirror, Hy odd in the y mirror
            add[0] += sx[u] * sy[v] * padpsi[((int64_t)b * 3 + 0) * npos + p];
            add[1] += sx[u] * padpsi[((int64_t)b * 3 + 1) * npos + p];
            add[2] += sy[v] * padpsi[((int64_t)b * 3 + 2) * npos + p];
            gE += padg[((int64_t)b * 2 + 0) * npos + p];
            gH += padg[((int64_t)b * 2 + 1) * npos + p];
        }
#pragma unroll
    for (int f = 0; f < 3; ++f) a.lam_out[((int64_t)b * 3 + f) * ncell + t] += add[f];
    if (a.g_epsinv) a.g_epsinv[(int64_t)b * ncell + t] += gE;
    if (a.g_muinv) a.g_muinv[(int64_t)b * ncell + t] += gH;
}

// Material gradient of the explicit source: U'_Ez += (1/eps) A, A = dt S_z, so
// g_epsinv += lambda'_Ez A on the source cells.
template <typename T>
__global__ void adj_source_kernel(const T *lam, double *g_epsinv, int64_t ncell, int64_t fstride, const int64_t *cells,
                                  const double *weight, double amp, int32_t n)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (s >= n) return;
    const int64_t c = cells[s];
    g_epsinv[(int64_t)b * ncell + c] += (double)lam[(int64_t)b * fstride + c] * (amp * weight[s]);
}

template <typename T>
int launch_cart2d_adjoint(const Cart2DAdjArgs<T> &a, T *pad9, T *padpsi, double *padg, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int64_t npos = (int64_t)(a.nx + 4) * (a.ny + 4);
    const int64_t nband = Band2D(a.nx, a.ny).count();
    dim3 gpad((unsigned)((npos + ADJ_BLOCK - 1) / ADJ_BLOCK), a.batch), gband((unsigned)((nband + ADJ_BLOCK - 1) / ADJ_BLOCK), a.batch);
    if (a.epsinv && a.muinv) hipLaunchKernelGGL((adj2d_faces_kernel<T, true, true>), gpad, dim3(ADJ_BLOCK), 0, s, a, pad9, padg);
    else if (a.epsinv) hipLaunchKernelGGL((adj2d_faces_kernel<T, true, false>), gpad, dim3(ADJ_BLOCK), 0, s, a, pad9, padg);
    else if (a.muinv) hipLaunchKernelGGL((adj2d_faces_kernel<T, false, true>), gpad, dim3(ADJ_BLOCK), 0, s, a, pad9, padg);
    else hipLaunchKernelGGL((adj2d_faces_kernel<T, false, false>), gpad, dim3(ADJ_BLOCK), 0, s, a, pad9, padg);
    hipLaunchKernelGGL(adj2d_psi_kernel<T>, gpad, dim3(ADJ_BLOCK), 0, s, a, (const T *)pad9, padpsi);
    hipLaunchKernelGGL(adj2d_fold_kernel<T>, gband, dim3(ADJ_BLOCK), 0, s, a, (const T *)padpsi, (const double *)padg);
    return (int)hipGetLastError();
}

template <typename T>
int launch_adjoint_source(const T *lam, double *g_epsinv, int64_t ncell, int64_t fstride, int32_t batch,
                          const int64_t *cells, const double *weight, double amp, int32_t n, void *stream)
{
    hipLaunchKernelGGL(adj_source_kernel<T>, dim3((n + 255) / 256, batch), dim3(256), 0, (hipStream_t)stream, lam,
                       g_epsinv, ncell, fstride, cells, weight, amp, n);
    return (int)hipGetLastError();
}

template int launch_cart2d_adjoint<float>(const Cart2DAdjArgs<float> &, float *, float *, double *, void *);
template int launch_cart2d_adjoint<double>(const Cart2DAdjArgs<double> &, double *, double *, double *, void *);
template int launch_adjoint_source<float>(const float *, double *, int64_t, int64_t, int32_t, const int64_t *,
                                          const double *, double, int32_t, void *);
template int launch_adjoint_source<double>(const double *, double *, int64_t, int64_t, int32_t, const int64_t *,
                                           const double *, double, int32_t, void *);

}  // namespace gks
