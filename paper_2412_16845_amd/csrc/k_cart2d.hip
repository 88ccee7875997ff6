// Fused GKS step on a 2D Cartesian grid, TM fields (Ez, Hx, Hy).
//
// One wavefront owns a strip of 64 columns (60 written, 2 halo columns on each side) and
// marches TILE_Y rows upwards, keeping three rows of fields, two rows of gradients and the
// previous horizontal-face flux in registers.  Each field value is loaded once per strip row;
// neighbours along x come from the adjacent lanes through DPP moves, so no LDS and no
// barriers are needed.  Per row the wave:
//   1. loads the next row (structure-of-arrays, 64 consecutive values per field: coalesced),
//      mapping ghost rows/columns through the boundary conditions;
//   2. forms the Green-Gauss (central) half-differences of the middle row (Sec. 3.1);
//   3. evaluates the GKS flux of the horizontal face below the middle row and of the vertical
//      face right of each lane, as sparse linear forms of the stencil values (the closed-form
//      moments of Sec. 3.1 folded into coefficients on the host);
//   4. sums the four face terms of the row it finishes in double precision, adds the old
//      value and the explicit source, and stores once.
// Non-reflecting sides: the ghost side of a boundary face carries no distribution (zero state
// and slopes); the ghost value used by the Green-Gauss gradient is the cell's own.  PEC
// sides: mirror ghosts (Ez and the normal H odd, the tangential H even).  Periodic sides wrap.
#include "gks_device.h"

namespace gks {

constexpr int HALO = 2;
constexpr int OUTX = WAVE - 2 * HALO;   // columns written per wave
constexpr int TILE_Y = 64;              // rows written per wave

template <typename T>
struct Row2D {
    T u[3];      // Ez, Hx, Hy (mirror signs applied)
    T mE, mH;    // 1/eps, 1/mu of the cell read
    bool nr;     // non-reflecting ghost
};

template <typename T, bool HAS_EPS, bool HAS_MU>
__device__ __forceinline__ void load_row(const Cart2DArgs<T> &a, const T *Ub, const T *Eb, const T *Mb, int64_t ncell,
                                         int sx, T sgx0, T sgx1, bool nrx, int gy, Row2D<T> &r)
{
    bool mir, nry;
    const int sy = map_axis(gy, a.ny, a.bc[2], a.bc[3], mir, nry);
    const int64_t c = (int64_t)sy * a.nx + sx;
    // y-mirror signs: Ez odd, Hx (tangential) even, Hy (normal) odd
    const T sy0 = mir ? T(-1) : T(1);
    r.u[0] = Ub[c] * (sgx0 * sy0);
    r.u[1] = Ub[ncell + c] * sgx0;
    r.u[2] = Ub[2 * ncell + c] * (sgx1 * sy0);
    r.mE = HAS_EPS ? Eb[c] : T(1);
    r.mH = HAS_MU ? Mb[c] : T(1);
    r.nr = nry || nrx;
}

template <typename T, bool HAS_EPS, bool HAS_MU>
__global__ __launch_bounds__(256) void cart2d_step_kernel(Cart2DArgs<T> a)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
    const int per_b = a.ntx * a.nty;
    const int b = wave / per_b;
    if (b >= a.batch) return;
    const int rem = wave - b * per_b;
    const int ty = rem / a.ntx;
    const int tx = rem - ty * a.ntx;

    const int64_t ncell = (int64_t)a.nx * a.ny;
    const T *Ub = a.U + (int64_t)b * 3 * ncell;
    T *Ob = a.Unew + (int64_t)b * 3 * ncell;
    const T *Eb = HAS_EPS ? a.epsinv + (int64_t)b * ncell : nullptr;
    const T *Mb = HAS_MU ? a.muinv + (int64_t)b * ncell : nullptr;

    // column of this lane and its boundary mapping
    const int gx = tx * OUTX - HALO + lane;
    bool mirx, nrx;
    const int sx = map_axis(gx, a.nx, a.bc[0], a.bc[1], mirx, nrx);
    const T sgx0 = mirx ? T(-1) : T(1);   // Ez and Hx (normal to an x wall) are odd
    const T sgx1 = T(1);                  // Hy is even
    const bool writer = lane >= HALO && lane < WAVE - HALO && gx < a.nx;

    const int y0 = ty * TILE_Y;
    const int y1 = min(y0 + TILE_Y, a.ny);   // rows [y0, y1) are written

    Row2D<T> rs, rc, rn;                      // rows q-2, q-1, q
    load_row<T, HAS_EPS, HAS_MU>(a, Ub, Eb, Mb, ncell, sx, sgx0, sgx1, nrx, y0 - 2, rs);
    load_row<T, HAS_EPS, HAS_MU>(a, Ub, Eb, Mb, ncell, sx, sgx0, sgx1, nrx, y0 - 1, rc);
    T Ds[6], Dc[6];                           // half-differences (d/dx, d/dy) x (Ez,Hx,Hy)
    T fyS[3] = {T(0), T(0), T(0)};            // flux of the horizontal face below row q-2

    for (int q = y0; q <= y1 + 1; ++q) {
        load_row<T, HAS_EPS, HAS_MU>(a, Ub, Eb, Mb, ncell, sx, sgx0, sgx1, nrx, q, rn);
        // gradient of row q-1 (Green-Gauss on a uniform grid = central half-differences)
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            Dc[f] = T(0.5) * (from_right(rc.u[f]) - from_left(rc.u[f]));
            Dc[3 + f] = T(0.5) * (rn.u[f] - rs.u[f]);
        }
        if (q >= y0 + 1) {
            // horizontal face between rows q-2 (left) and q-1 (right), local frame
            // (x~, y~) = (y, -x): (Ez, Hx, Hy) -> (Ez, Hy, -Hx), d1 = d/dy, d2 = -d/dx
            T w[18];
            const bool zl = rs.nr, zr = rc.nr;
            w[0] = zl ? T(0) : rs.u[0];
            w[1] = zl ? T(0) : rs.u[2];
            w[2] = zl ? T(0) : -rs.u[1];
            w[3] = zr ? T(0) : rc.u[0];
            w[4] = zr ? T(0) : rc.u[2];
            w[5] = zr ? T(0) : -rc.u[1];
            w[6] = zl ? T(0) : Ds[3];
            w[7] = zl ? T(0) : Ds[5];
            w[8] = zl ? T(0) : -Ds[4];
            w[9] = zl ? T(0) : -Ds[0];
            w[10] = zl ? T(0) : -Ds[2];
            w[11] = zl ? T(0) : Ds[1];
            w[12] = zr ? T(0) : Dc[3];
            w[13] = zr ? T(0) : Dc[5];
            w[14] = zr ? T(0) : -Dc[4];
            w[15] = zr ? T(0) : -Dc[0];
            w[16] = zr ? T(0) : -Dc[2];
            w[17] = zr ? T(0) : Dc[1];
            // face material: mean of the two cells (a ghost reads its interior cell, so a
            // boundary face gets the interior value)
            const T mE = T(0.5) * (rs.mE + rc.mE);
            const T mH = T(0.5) * (rs.mH + rc.mH);
            T p[3];
            apply_tm(w, mE, mH, a.fy, p);
            T fyN[3] = {p[0], -p[2], p[1]};   // back to (Ez, Hx, Hy)

            if (q >= y0 + 2) {
                // vertical face right of this lane, row q-2 (local frame = global frame)
                const bool me_nr = rs.nr;
                T ul[3], dl[6];
#pragma unroll
                for (int f = 0; f < 3; ++f) ul[f] = me_nr ? T(0) : rs.u[f];
#pragma unroll
                for (int f = 0; f < 6; ++f) dl[f] = me_nr ? T(0) : Ds[f];
                T v[18];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    v[f] = ul[f];
                    v[3 + f] = from_right(ul[f]);
                    v[6 + f] = dl[f];
                    v[9 + f] = dl[3 + f];
                    v[12 + f] = from_right(dl[f]);
                    v[15 + f] = from_right(dl[3 + f]);
                }
                const T mEx = T(0.5) * (rs.mE + from_right(rs.mE));
                const T mHx = T(0.5) * (rs.mH + from_right(rs.mH));
                T fx[3];
                apply_tm(v, mEx, mHx, a.fx, fx);
                T fxl[3];
#pragma unroll
                for (int f = 0; f < 3; ++f) fxl[f] = from_left(fx[f]);

                const int r = q - 2;
                if (writer) {
                    const int64_t c = (int64_t)r * a.nx + gx;
                    double src = 0.0;
                    for (int s = 0; s < a.nsrc; ++s)
                        if (c == a.src_cell[s]) src += a.src_amp[s];
                    const double m[3] = {(double)rs.mE, (double)rs.mH, (double)rs.mH};
                    const double add[3] = {src, 0.0, 0.0};
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const double div = ((double)fx[f] - (double)fxl[f]) + ((double)fyN[f] - (double)fyS[f]);
                        Ob[(int64_t)f * ncell + c] = (T)((double)rs.u[f] + m[f] * (add[f] - div));
                    }
                }
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) fyS[f] = fyN[f];
        }
        rs = rc;
        rc = rn;
#pragma unroll
        for (int f = 0; f < 6; ++f) Ds[f] = Dc[f];
    }
}

template <typename T>
int launch_cart2d_step(const Cart2DArgs<T> &a, void *stream)
{
    const int waves = a.ntx * a.nty * a.batch;
    const int wpb = 256 / WAVE;
    dim3 grid((waves + wpb - 1) / wpb), block(256);
    hipStream_t s = (hipStream_t)stream;
    if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart2d_step_kernel<T, true, true>), grid, block, 0, s, a);
    else if (a.epsinv) hipLaunchKernelGGL((cart2d_step_kernel<T, true, false>), grid, block, 0, s, a);
    else if (a.muinv) hipLaunchKernelGGL((cart2d_step_kernel<T, false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((cart2d_step_kernel<T, false, false>), grid, block, 0, s, a);
    return (int)hipGetLastError();
}

template int launch_cart2d_step<float>(const Cart2DArgs<float> &, void *);
template int launch_cart2d_step<double>(const Cart2DArgs<double> &, void *);

int cart2d_tile_x() { return OUTX; }
int cart2d_tile_y() { return TILE_Y; }

}  // namespace gks
