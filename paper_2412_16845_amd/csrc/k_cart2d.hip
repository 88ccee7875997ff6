// Fused GKS step on a 2D Cartesian grid, TM fields (Ez, Hx, Hy).
//
// One wavefront owns a strip of 64 columns (60 written, 2 halo columns on each side) and
// marches a tile of rows upwards (the tile height is chosen by the host to balance the
// workgroups over the compute units).  Each field value is loaded once per strip row; neighbours along
// x come from the adjacent lanes through DPP moves, so no LDS and no barriers are needed.
// Per row the wave:
//   1. issues the loads of the row PF rows ahead (structure-of-arrays, 64 consecutive values
//      per field: coalesced), so that several rows of loads are in flight while it computes;
//   2. forms the Green-Gauss (central) differences of the middle row of its three-row window;
//   3. evaluates the GKS flux of the horizontal face below the middle row and of the vertical
//      face right of each lane, as sparse linear forms of the stencil values (the closed-form
//      moments of Sec. 3.1 folded into coefficients on the host);
//   4. sums the four face terms of the row it finishes in double precision, adds the old value
//      and the explicit source, and stores once.
// The row loop is unrolled six times so that the rotating window (six row slots, two gradient
// slots, two flux slots) lives in fixed registers without copies.
// Strips that touch no domain side take a path without index mapping.  On the others, ghost
// rows/columns follow the boundary condition: non-reflecting sides give the ghost side of a
// boundary face no distribution (zero state and slopes) and the Green-Gauss gradient the cell's
// own value; PEC sides read mirror ghosts (Ez and the normal H odd, the tangential H even);
// periodic sides wrap.
#include "gks_device.h"

namespace gks {

constexpr int HALO = 2;
constexpr int OUTX = WAVE - 2 * HALO;   // columns written per wave
constexpr int PF = 3;   // rows loaded ahead of use: with the three-row window, six row slots

template <typename T>
struct Row2D {
    T u[3];      // Ez, Hx, Hy (mirror signs applied)
    T mE, mH;    // 1/eps, 1/mu of the cell read
    bool nr;     // non-reflecting ghost (boundary strips only)
};

template <typename T, bool HAS_EPS, bool HAS_MU, bool BND>
struct Strip2D {
    const Cart2DArgs<T> &a;
    Rsrc rU, rE, rM, rO;   // this batch item's fields, 1/eps, 1/mu, output fields
    uint32_t fbytes;       // bytes per field array
    uint32_t vx;           // byte offset of this lane's column (mapped column on boundary strips)
    uint32_t vlane;        // byte offset of this lane inside the strip
    int x0;                // first column of the strip (uniform; -2 on the first strip)
    int gx;                // column of this lane
    T sgx;                 // x-mirror sign of Ez and Hx
    bool nrx;
    bool writer;
    int y0, y1;

    __device__ __forceinline__ void load(int gy, Row2D<T> &r) const
    {
        if constexpr (BND) {
            bool mir, nry;
            const int sy = map_axis(gy, a.ny, a.bc[2], a.bc[3], mir, nry);
            const uint32_t so = (uint32_t)sy * (uint32_t)a.nx * (uint32_t)sizeof(T);
            const T sgy = mir ? T(-1) : T(1);   // y mirror: Ez and Hy odd, Hx even
            r.u[0] = buf_load<T>(rU, vx, so) * (sgx * sgy);
            r.u[1] = buf_load<T>(rU, vx, so + fbytes) * sgx;
            r.u[2] = buf_load<T>(rU, vx, so + 2 * fbytes) * sgy;
            r.mE = HAS_EPS ? buf_load<T>(rE, vx, so) : T(1);
            r.mH = HAS_MU ? buf_load<T>(rM, vx, so) : T(1);
            r.nr = nry || nrx;
        } else {
            const uint32_t so = ((uint32_t)gy * (uint32_t)a.nx + (uint32_t)x0) * (uint32_t)sizeof(T);
            r.u[0] = buf_load<T>(rU, vx, so);
            r.u[1] = buf_load<T>(rU, vx, so + fbytes);
            r.u[2] = buf_load<T>(rU, vx, so + 2 * fbytes);
            r.mE = HAS_EPS ? buf_load<T>(rE, vx, so) : T(1);
            r.mH = HAS_MU ? buf_load<T>(rM, vx, so) : T(1);
            r.nr = false;
        }
    }

    // One row step at index q: window rows q-2 (Rs), q-1 (Rc), q (Rn); Rp receives row q+PF.
    __device__ __forceinline__ void body(int q, Row2D<T> &Rs, Row2D<T> &Rc, Row2D<T> &Rn, Row2D<T> &Rp,
                                         T (&Ds)[6], T (&Dc)[6], T (&fyS)[3], T (&fyN)[3]) const
    {
        // rows beyond y1 + 1 are not needed: re-read row y1 + 1 instead (already cached), which
        // keeps the load unconditional so the loads in flight are counted exactly
        load(min(q + PF, y1 + 1), Rp);
        // central differences of row q-1: [d/dx x (Ez,Hx,Hy), d/dy x (Ez,Hx,Hy)] times 2h
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            Dc[f] = from_right(Rc.u[f]) - from_left(Rc.u[f]);
            Dc[3 + f] = Rn.u[f] - Rs.u[f];
        }
        if (q < y0 + 1) return;

        // horizontal face between rows q-2 and q-1: inputs [UL UR dyL dxL dyR dxR]
        {
            const bool zl = BND && Rs.nr, zr = BND && Rc.nr;
            T w[18];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                w[f] = zl ? T(0) : Rs.u[f];
                w[3 + f] = zr ? T(0) : Rc.u[f];
                w[6 + f] = zl ? T(0) : Ds[3 + f];
                w[9 + f] = zl ? T(0) : Ds[f];
                w[12 + f] = zr ? T(0) : Dc[3 + f];
                w[15 + f] = zr ? T(0) : Dc[f];
            }
            // face material: the two cells' values (a ghost reads its interior cell); the
            // operator applies their mean
            apply_op<PatTMy>(w, Rs.mE + Rc.mE, Rs.mH + Rc.mH, scalar_ptr(a.ops + 1), fyN);
        }
        if (q < y0 + 2) return;

        // vertical face right of this lane, row q-2: inputs [UL UR dxL dyL dxR dyR]
        const bool me_nr = BND && Rs.nr;
        T ul[3], dl[6];
#pragma unroll
        for (int f = 0; f < 3; ++f) ul[f] = me_nr ? T(0) : Rs.u[f];
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
        T fx[3];
        apply_op<PatTMx>(v, Rs.mE + from_right(Rs.mE), Rs.mH + from_right(Rs.mH), scalar_ptr(a.ops), fx);
        T fxl[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) fxl[f] = from_left(fx[f]);

        if (writer) {
            // per-cell flux divergence (FP32 in FP32 mode), then the old value and the source
            // added in FP64 with a single rounding
            // interior strips: uniform offset of the strip start + lane offset; boundary strips
            // (whose first column may be a ghost): uniform row start + the lane's own column
            const uint32_t rowc = (uint32_t)(q - 2) * (uint32_t)a.nx;
            const uint32_t so = BND ? rowc * (uint32_t)sizeof(T) : (rowc + (uint32_t)x0) * (uint32_t)sizeof(T);
            const uint32_t vo = BND ? (uint32_t)gx * (uint32_t)sizeof(T) : vlane;
            const int c = (int)rowc + gx;
            double src = 0.0;
            for (int s = 0; s < a.nsrc; ++s)
                if (c == a.src_cell[s]) src += a.src_amp[s];
            const double mE = (double)Rs.mE, mH = (double)Rs.mH;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const T div = (fx[f] - fxl[f]) + (fyN[f] - fyS[f]);
                const double m = (f == 0) ? mE : mH;
                const double add = (f == 0) ? src : 0.0;
                buf_store((T)((double)Rs.u[f] + m * (add - (double)div)), rO, vo, so + f * fbytes);
            }
        }
    }

    __device__ __forceinline__ void run() const
    {
        Row2D<T> R0, R1, R2, R3, R4, R5;
        T D0[6], D1[6];
        T F0[3] = {T(0), T(0), T(0)}, F1[3] = {T(0), T(0), T(0)};
        load(y0 - 2, R0);
        load(y0 - 1, R1);
        load(y0, R2);
        load(y0 + 1, R3);
        load(y0 + 2, R4);
        const int qend = y1 + 1;
        for (int q = y0; q <= qend; q += 6) {
            body(q, R0, R1, R2, R5, D0, D1, F0, F1);
            if (q + 1 > qend) break;
            body(q + 1, R1, R2, R3, R0, D1, D0, F1, F0);
            if (q + 2 > qend) break;
            body(q + 2, R2, R3, R4, R1, D0, D1, F0, F1);
            if (q + 3 > qend) break;
            body(q + 3, R3, R4, R5, R2, D1, D0, F1, F0);
            if (q + 4 > qend) break;
            body(q + 4, R4, R5, R0, R3, D0, D1, F0, F1);
            if (q + 5 > qend) break;
            body(q + 5, R5, R0, R1, R4, D1, D0, F1, F0);
        }
    }
};

template <typename T, bool HAS_EPS, bool HAS_MU>
__global__ __launch_bounds__(256) void cart2d_step_kernel(Cart2DArgs<T> a)
{
    const int lane = threadIdx.x & (WAVE - 1);
    // the wave's index inside the block is uniform: say so, so that everything derived from it
    // (tile, batch item, buffer resources, row offsets) lives in scalar registers
    const int wave = xcd_logical_block() * (256 / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int per_b = a.ntx * a.nty;
    const int b = wave / per_b;
    if (b >= a.batch) return;
    const int rem = wave - b * per_b;
    const int ty = rem / a.ntx;
    const int tx = rem - ty * a.ntx;

    const int64_t ncell = (int64_t)a.nx * a.ny;
    const uint32_t fbytes = (uint32_t)(ncell * (int64_t)sizeof(T));
    const Rsrc rU = make_rsrc(a.U + (int64_t)b * 3 * ncell, 3ull * fbytes);
    const Rsrc rO = make_rsrc(a.Unew + (int64_t)b * 3 * ncell, 3ull * fbytes);
    const Rsrc rE = make_rsrc(HAS_EPS ? a.epsinv + (int64_t)b * ncell : a.U, fbytes);
    const Rsrc rM = make_rsrc(HAS_MU ? a.muinv + (int64_t)b * ncell : a.U, fbytes);

    const int x0 = tx * OUTX - HALO;
    const int gx = x0 + lane;
    const int y0 = ty * a.tile_y;
    const int y1 = min(y0 + a.tile_y, a.ny);   // rows [y0, y1) are written
    const uint32_t vlane = (uint32_t)lane * (uint32_t)sizeof(T);

    const bool interior = x0 >= 0 && x0 + WAVE - 1 <= a.nx - 1 && y0 - 2 >= 0 && y1 + 1 <= a.ny - 1;
    if (interior) {
        Strip2D<T, HAS_EPS, HAS_MU, false> s{a, rU, rE, rM, rO, fbytes, vlane, vlane, x0, gx, T(1), false,
                                             lane >= HALO && lane < WAVE - HALO, y0, y1};
        s.run();
    } else {
        bool mirx, nrx;
        const int sx = map_axis(gx, a.nx, a.bc[0], a.bc[1], mirx, nrx);
        Strip2D<T, HAS_EPS, HAS_MU, true> s{a, rU, rE, rM, rO, fbytes, (uint32_t)sx * (uint32_t)sizeof(T), vlane, x0, gx,
                                            mirx ? T(-1) : T(1), nrx,
                                            lane >= HALO && lane < WAVE - HALO && gx < a.nx, y0, y1};
        s.run();
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

}  // namespace gks
