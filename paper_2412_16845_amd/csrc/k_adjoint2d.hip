// Reverse-mode adjoint of the 2D TM Cartesian GKS step.
//
// The forward step is U' = U - M^{-1} div Phi(pad(U)) + dt M^{-1} S, with pad() the ghost
// extension of the grid by the boundary conditions (periodic wrap, PEC mirror with signs,
// non-reflecting clamp for the Green-Gauss gradient) and Phi the face fluxes, each a sparse
// linear form K(m_s) w_f of the left/right states and central differences (the operators of
// the forward kernel).  For lambda' = dJ/dU' the adjoint is
//     lambda = pad^T psi,   psi(p) = lambda'(p) - ubar(p) - Dxbar(p-x) + Dxbar(p+x)
//                                   - Dybar(p-y) + Dybar(p+y),
// where, over the faces f of p, ubar(p), Dxbar(p), Dybar(p) collect p's share of
// wbar_f = K(m_s)^T a_f (its state, x-difference and y-difference parts), a_f = mu_L - mu_R and
// mu = (1/eps, 1/mu) lambda' on cells, 0 on ghost positions.  The material gradients collect, per
// cell, -lambda'.div(Phi) (the 1/eps, 1/mu factors of the update) and, per face and for both of
// its cells, -a_f . d Phi_f / d m_s (the face material of the equilibrium time derivative).
//
// One kernel marches it, in the forward kernel's layout: a wave owns a strip of 64 columns (two
// halo columns each side) and marches a tile of rows.  Per row step (head row q) it loads row
// q+1, forms the central differences of row q-1, evaluates the x faces of row q-1 and the y
// face between rows q-2 and q-1 (forward flux with its material parts, transposed operator,
// material sensitivities), accumulates their shares per position (the right cell's share of an
// x face by DPP), and finishes row q-3, whose faces and whose neighbours' faces are then all
// known.  Cells receive lambda and their gradients; ghost positions (two layers around the
// grid) write psi and their material gradients to a scratch array of the ghost positions that
// a small kernel then adds, with the mirror signs, onto the cells they image.  Everything runs in a fixed order
// (no atomics), so the adjoint is deterministic.
#include <mutex>

#include "gks_device.h"

namespace gks {

constexpr int ADJ_BLOCK = 256;
// Coefficient chunk of the face operators: small chunks keep fewer scalar registers live and
// halve the scalar spills of the march (1024^2 x 8 adjoint step with separate forward and
// transposed passes: 221.5 -> 208.9 us in fp32 and 482.7 -> 433.1 us in fp64 with 4 instead of
// 12; 3, 5, 6 and 8 were slower).  With the fused pass below fp32 takes chunks of 6 (160.5 ->
// 157 us).
template <typename T> constexpr int adj_chunk() { return sizeof(T) == 4 ? 6 : 4; }
// fp32: the forward and the transposed operator of a face in one pass over its coefficients,
// each loaded once (163 -> 160.5 us with chunks of 4, 154 instead of 167 VGPRs); fp64 keeps two
// passes that load them twice (one pass raises its scalar spills from 603 to 722).
#ifndef GKS_ADJ_FUSED
#define GKS_ADJ_FUSED 1
#endif
template <typename T> constexpr bool adj_fused() { return GKS_ADJ_FUSED != 0 && sizeof(T) == 4; }
// One wave per workgroup for the march: its waves finish at different times, and a single-wave
// workgroup lets a freed slot take the next tile at once (4-wave workgroups wait for four free
// slots on one compute unit).  Measured on 1024^2 x 8: 231 vs 241 us (fp32), 503 vs 552 us (fp64).
constexpr int ADJ_MARCH_BLOCK = 64;
// Rows per wave tile: a wave marches its tile's rows plus five (the halo and the pipeline), and
// all tiles are alike, so the march takes about ceil(tiles / wave slots) x (rows + 5) row steps,
// the wave slots being the device's compute units times the waves one unit holds of the kernel
// variant.  The height is picked in [16, 40] to minimise that (a last round that is almost empty
// costs a whole tile's time: 1024^2 x 8 in fp32, three waves per SIMD, had 6192 tiles of 24
// rows for 3072 slots).
int adj_tile_rows(int nx, int ny, int batch, int64_t slots)
{
    const int64_t ntx = (nx + (WAVE - 4) - 1) / (WAVE - 4);
    int pick = 24;
    double best = 1e300;
    for (int ty = 16; ty <= 40; ++ty) {
        const int64_t tiles = ntx * ((ny + ty - 1) / ty) * batch;
        const int64_t rounds = (tiles + slots - 1) / std::max<int64_t>(slots, 1);
        const double cost = (double)rounds * (ty + 5);
        if (cost < best) {
            best = cost;
            pick = ty;
        }
    }
    return pick;
}

// The ghost positions of an nx x ny grid: the two layers of positions (i, j) around it,
// -2 <= i <= nx+1 and -2 <= j <= ny+1 outside [0, nx) x [0, ny).  Numbered row by row for the
// two ghost rows below and the two above, then four per grid row (columns -2, -1, nx, nx+1):
// 4 (nx + 4) + 4 ny positions, the only ones whose co-states and material gradients go through
// scratch memory.
struct Ring2D {
    int nx, ny;
    __host__ __device__ int64_t size() const { return 4 * (int64_t)(nx + 4) + 4 * (int64_t)ny; }
    __device__ __forceinline__ int64_t idx(int i, int j) const
    {
        const int64_t w = nx + 4;
        if (j < 0) return (j + 2) * w + (i + 2);
        if (j >= ny) return (2 + j - ny) * w + (i + 2);
        return 4 * w + 4 * (int64_t)j + (i < 0 ? i + 2 : i - nx + 2);
    }
};

template <typename T>
struct APos {
    T u[3];        // fields (ghosts: the imaged cell with mirror signs)
    T l[3];        // lambda' (0 on ghost positions)
    T mE, mH;      // materials of the cell read
};

template <typename T>
struct AAcc {
    T ub[3], dxb[3], dyb[3];   // adjoints of the state and of the two central differences
    T div[3];                  // forward flux divergence
    T sE, sH;                  // sum of the faces' material sensitivities a . (dPhi / dm_s)
};

template <typename T>
__device__ __forceinline__ void zero_acc(AAcc<T> &A)
{
#pragma unroll
    for (int f = 0; f < 3; ++f) A.ub[f] = A.dxb[f] = A.dyb[f] = A.div[f] = T(0);
    A.sE = A.sH = T(0);
}

__device__ __forceinline__ bool row_is_nr(int gy, int ny, int bclo, int bchi)
{
    return (gy < 0 && bclo == GKS_BC_NONREFLECT) || (gy >= ny && bchi == GKS_BC_NONREFLECT);
}

// HM = false (vacuum 1/mu and no 1/mu gradient asked for): the operators' 1/mu parts are
// folded into K0 on the host (the second pair of operators), which drops their products from
// the forward and the transposed evaluation of every face.
template <typename T, bool HAS_EPS, bool HAS_MU, bool HM, bool BND>
struct AdjStrip {
    static constexpr int OPS0 = HM ? 0 : 2;
    const Cart2DAdjArgs<T> &a;
    Rsrc rU, rL, rE, rM;
    uint32_t fbytes;
    int lane, x, x0;
    uint32_t vx;        // byte offset of the column this lane reads
    T sgx;              // x-mirror sign of the column this lane reads (Ez, Hx odd)
    bool gx, nrx;       // this lane's column is a ghost / a non-reflecting ghost
    bool nrx1;          // the next column is a non-reflecting ghost
    bool own_x;         // this wave writes this lane's positions
    int R0, R1;         // rows finished by this wave: [R0, R1)
    bool first_y, last_y;
    int64_t ncell;
    int b;
    T *padpsi;
    double *padg;

    __device__ __forceinline__ void load(int gy, APos<T> &p) const
    {
        if constexpr (BND) {
            bool my, nry;
            const int sy = map_axis(gy, a.ny, a.bc[2], a.bc[3], my, nry);
            const bool gyst = gy < 0 || gy >= a.ny;
            const uint32_t so = (uint32_t)sy * (uint32_t)a.nx * (uint32_t)sizeof(T);
            const T sgy = my ? T(-1) : T(1);
            p.u[0] = buf_load<T>(rU, vx, so) * (sgx * sgy);
            p.u[1] = buf_load<T>(rU, vx, so + fbytes) * sgx;
            p.u[2] = buf_load<T>(rU, vx, so + 2 * fbytes) * sgy;
            const bool ghost = gx || gyst;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const T v = buf_load<T>(rL, vx, so + f * fbytes);
                p.l[f] = ghost ? T(0) : v;
            }
            p.mE = HAS_EPS ? buf_load<T>(rE, vx, so) : T(1);
            p.mH = HAS_MU ? buf_load<T>(rM, vx, so) : T(1);
        } else {
            const uint32_t so = ((uint32_t)gy * (uint32_t)a.nx + (uint32_t)x0) * (uint32_t)sizeof(T);
            const uint32_t vo = (uint32_t)lane * (uint32_t)sizeof(T);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                p.u[f] = buf_load<T>(rU, vo, so + f * fbytes);
                p.l[f] = buf_load<T>(rL, vo, so + f * fbytes);
            }
            p.mE = HAS_EPS ? buf_load<T>(rE, vo, so) : T(1);
            p.mH = HAS_MU ? buf_load<T>(rM, vo, so) : T(1);
        }
    }

    __device__ __forceinline__ bool pos_nr(int gy) const
    {
        return BND && (nrx || row_is_nr(gy, a.ny, a.bc[2], a.bc[3]));
    }

    // One face: L/R data, inputs w (already zeroed on non-reflecting ghost sides).  Returns the
    // forward flux phi, the transposed operator wbar = K^T a and the sensitivities.
    template <typename P, typename Op>
    __device__ __forceinline__ void face(const T (&w)[18], T mEs, T mHs, const T (&ad)[3], Op K, T (&phi)[3],
                                         T (&wbar)[18], T &sE, T &sH) const
    {
        T e[3], h[3];
#pragma unroll
        for (int q = 0; q < 18; ++q) wbar[q] = T(0);
        if constexpr (adj_fused<T>()) {
            apply_op_both<P, adj_chunk<T>(), HM>(w, ad, mEs, mHs, K, phi, e, h, wbar);
        } else {
            apply_op_parts<P, adj_chunk<T>(), HM>(w, mEs, mHs, K, phi, e, h);
            // reload the coefficients for the transposed pass rather than keeping them live
            asm volatile("" : "+s"(K) : "v"(phi[2]));
            apply_op_transpose<P, adj_chunk<T>(), HM>(ad, mEs, mHs, K, wbar);
        }
        sE = ad[0] * e[0] + ad[1] * e[1] + ad[2] * e[2];
        sH = HM ? ad[0] * h[0] + ad[1] * h[1] + ad[2] * h[2] : T(0);
    }

    // Step i of the march (head row q = qs + i); I = i mod 4 selects the register slots:
    // data row q-k in P[(i-k)&3], accumulators of row q-k in S[(i-k)&3], differences of row
    // q-k in G[(i-k)&1].
    template <int I>
    __device__ __forceinline__ void step(int i, int qs, APos<T> (&P)[4], AAcc<T> (&S)[4], T (&G)[2][6]) const
    {
        const int q = qs + i;
        APos<T> &P3 = P[(I + 1) & 3], &P2 = P[(I + 2) & 3], &P1 = P[(I + 3) & 3], &P0 = P[I];
        AAcc<T> &A4 = S[I], &A3 = S[(I + 1) & 3], &A2 = S[(I + 2) & 3], &A1 = S[(I + 3) & 3];
        T(&G2)[6] = G[I & 1];
        T(&G1)[6] = G[(I + 1) & 1];
        // lambda' of row q-3 (finished below), then row q+1 into its slot
        T lf[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) lf[f] = P3.l[f];
        load(min(q + 1, R1 + 2), P3);
        zero_acc(A1);

        // central differences of row q-1: [d/dx(3) d/dy(3)]
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            G1[f] = from_right(P1.u[f]) - from_left(P1.u[f]);
            G1[3 + f] = P0.u[f] - P2.u[f];
        }

        // x faces of row q-1: inputs [UL UR dxL dyL dxR dyR], R the next lane
        {
            const bool nr = pos_nr(q - 1);
            T su[3], sg[6], mu[3];
#pragma unroll
            for (int f = 0; f < 3; ++f) su[f] = nr ? T(0) : P1.u[f];
#pragma unroll
            for (int k = 0; k < 6; ++k) sg[k] = nr ? T(0) : G1[k];
            mu[0] = P1.mE * P1.l[0];
            mu[1] = P1.mH * P1.l[1];
            mu[2] = P1.mH * P1.l[2];
            T w[18], ad[3];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                w[f] = su[f];
                w[3 + f] = from_right(su[f]);
                w[6 + f] = sg[f];
                w[9 + f] = sg[3 + f];
                w[12 + f] = from_right(sg[f]);
                w[15 + f] = from_right(sg[3 + f]);
                ad[f] = mu[f] - from_right(mu[f]);
            }
            const T mEs = P1.mE + from_right(P1.mE), mHs = P1.mH + from_right(P1.mH);
            T phi[3], wbar[18], sE, sH;
            face<PatTMx>(w, mEs, mHs, ad, scalar_ptr_after(a.ops + OPS0, G1[5]), phi, wbar, sE, sH);
            // the left cell (this lane) and the right cell (the next lane, by DPP); a
            // non-reflecting ghost side receives nothing: the sending lane zeroes the right
            // cell's share, so the moves need no select on the receiving side
            const bool nrR = BND && (nrx1 || row_is_nr(q - 1, a.ny, a.bc[2], a.bc[3]));
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const T sub = nrR ? T(0) : wbar[3 + f], sdx = nrR ? T(0) : wbar[12 + f], sdy = nrR ? T(0) : wbar[15 + f];
                A1.ub[f] += (nr ? T(0) : wbar[f]) + from_left(sub);
                A1.dxb[f] += (nr ? T(0) : wbar[6 + f]) + from_left(sdx);
                A1.dyb[f] += (nr ? T(0) : wbar[9 + f]) + from_left(sdy);
                A1.div[f] += phi[f] - from_left(phi[f]);
            }
            A1.sE += sE + from_left(sE);
            A1.sH += sH + from_left(sH);
        }

        // y face between rows q-2 and q-1: inputs [UL UR dyL dxL dyR dxR]
        if (i >= 1) {
            const bool zl = pos_nr(q - 2), zr = pos_nr(q - 1);
            T w[18], ad[3];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                w[f] = zl ? T(0) : P2.u[f];
                w[3 + f] = zr ? T(0) : P1.u[f];
                w[6 + f] = zl ? T(0) : G2[3 + f];
                w[9 + f] = zl ? T(0) : G2[f];
                w[12 + f] = zr ? T(0) : G1[3 + f];
                w[15 + f] = zr ? T(0) : G1[f];
            }
            ad[0] = P2.mE * P2.l[0] - P1.mE * P1.l[0];
            ad[1] = P2.mH * P2.l[1] - P1.mH * P1.l[1];
            ad[2] = P2.mH * P2.l[2] - P1.mH * P1.l[2];
            T phi[3], wbar[18], sE, sH;
            face<PatTMy>(w, P2.mE + P1.mE, P2.mH + P1.mH, ad, scalar_ptr_after(a.ops + OPS0 + 1, G1[2]), phi, wbar, sE, sH);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                A2.ub[f] += zl ? T(0) : wbar[f];
                A2.dyb[f] += zl ? T(0) : wbar[6 + f];
                A2.dxb[f] += zl ? T(0) : wbar[9 + f];
                A2.div[f] += phi[f];
                A1.ub[f] += zr ? T(0) : wbar[3 + f];
                A1.dyb[f] += zr ? T(0) : wbar[12 + f];
                A1.dxb[f] += zr ? T(0) : wbar[15 + f];
                A1.div[f] -= phi[f];
            }
            A2.sE += sE;
            A2.sH += sH;
            A1.sE += sE;
            A1.sH += sH;
        }

        // finish row q-3: every face of it and of its four neighbours is known now
        const int r = q - 3;
        if (r >= R0 && r < R1) {
            T psi[3];
#pragma unroll
            for (int f = 0; f < 3; ++f)
                psi[f] = lf[f] - A3.ub[f] - from_left(A3.dxb[f]) + from_right(A3.dxb[f]) - A4.dyb[f] + A2.dyb[f];
            const double gE = -(double)lf[0] * (double)A3.div[0] - (double)A3.sE;
            const double gH = HM ? -((double)lf[1] * (double)A3.div[1] + (double)lf[2] * (double)A3.div[2]) - (double)A3.sH : 0.0;
            const bool ry = r >= 0 && r < a.ny;
            const bool own_y = (r >= -2 && r <= a.ny + 1) && ((r >= R0 && r < R1 && ry) || (!ry && (first_y || last_y)));
            if (own_x && own_y) {
                if (!gx && ry) {
                    const int64_t c = (int64_t)r * a.nx + x;
#pragma unroll
                    for (int f = 0; f < 3; ++f) a.lam_out[((int64_t)b * 3 + f) * ncell + c] = psi[f];
                    if (a.g_epsinv) a.g_epsinv[(int64_t)b * ncell + c] += gE;
                    if (a.g_muinv) a.g_muinv[(int64_t)b * ncell + c] += gH;
                } else {
                    const Ring2D pd{a.nx, a.ny};
                    const int64_t npos = pd.size(), pp = pd.idx(x, r);
#pragma unroll
                    for (int f = 0; f < 3; ++f) padpsi[((int64_t)b * 3 + f) * npos + pp] = psi[f];
                    padg[((int64_t)b * 2 + 0) * npos + pp] = gE;
                    padg[((int64_t)b * 2 + 1) * npos + pp] = gH;
                }
            }
        }
    }

    __device__ __forceinline__ void run() const
    {
        APos<T> P[4];
        AAcc<T> S[4];
        T G[2][6];
#pragma unroll
        for (int k = 0; k < 4; ++k) zero_acc(S[k]);
#pragma unroll
        for (int k = 0; k < 6; ++k) G[0][k] = G[1][k] = T(0);
        const int qs = R0 - 1;                 // the first step forms the differences of row R0-2
        load(qs - 3, P[1]);
        load(qs - 2, P[2]);
        load(qs - 1, P[3]);
        load(qs, P[0]);
        const int n = R1 - R0 + 4;             // the last step finishes row R1-1
        for (int i = 0; i < n; i += 4) {
            step<0>(i, qs, P, S, G);
            if (i + 1 >= n) break;
            step<1>(i + 1, qs, P, S, G);
            if (i + 2 >= n) break;
            step<2>(i + 2, qs, P, S, G);
            if (i + 3 >= n) break;
            step<3>(i + 3, qs, P, S, G);
        }
    }
};

template <typename T, bool HAS_EPS, bool HAS_MU, bool HM>
__global__ __launch_bounds__(ADJ_MARCH_BLOCK) void adj2d_march_kernel(Cart2DAdjArgs<T> a, T *padpsi, double *padg, int32_t ntx,
                                                                int32_t nty, int32_t tile_y)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = xcd_logical_block() * (ADJ_MARCH_BLOCK / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int per_b = ntx * nty;
    const int b = wave / per_b;
    if (b >= a.batch) return;
    const int rem = wave - b * per_b;
    const int ty = rem / ntx;
    const int tx = rem - ty * ntx;
    const int64_t ncell = (int64_t)a.nx * a.ny;
    const uint32_t fbytes = (uint32_t)(ncell * (int64_t)sizeof(T));
    const Rsrc rU = make_rsrc(a.U + (int64_t)b * 3 * ncell, 3ull * fbytes);
    const Rsrc rL = make_rsrc(a.lam + (int64_t)b * 3 * ncell, 3ull * fbytes);
    const Rsrc rE = make_rsrc(a.epsinv ? a.epsinv + (int64_t)b * ncell : a.U, fbytes);
    const Rsrc rM = make_rsrc(a.muinv ? a.muinv + (int64_t)b * ncell : a.U, fbytes);
    const int x0 = tx * (WAVE - 4) - 2, x = x0 + lane;
    const int y0 = ty * tile_y, y1 = min(y0 + tile_y, a.ny);
    const bool first_y = ty == 0, last_y = ty == nty - 1;
    const int R0 = first_y ? -2 : y0, R1 = last_y ? a.ny + 2 : y1;
    const bool interior = x0 >= 0 && x0 + WAVE - 1 <= a.nx - 1 && R0 - 4 >= 0 && R1 + 2 <= a.ny - 1;
    auto go = [&](auto bnd) {
        constexpr bool BND = decltype(bnd)::value;
        AdjStrip<T, HAS_EPS, HAS_MU, HM, BND> s{a, rU, rL, rE, rM, fbytes, lane, x, x0};
        bool mx, nrx;
        const int sx = map_axis(x, a.nx, a.bc[0], a.bc[1], mx, nrx);
        s.vx = (uint32_t)sx * (uint32_t)sizeof(T);
        s.sgx = mx ? T(-1) : T(1);
        s.gx = x < 0 || x >= a.nx;
        s.nrx = nrx;
        bool mx1, nrx1;
        map_axis(x + 1, a.nx, a.bc[0], a.bc[1], mx1, nrx1);
        s.nrx1 = nrx1;
        s.own_x = (x >= -2 && x <= a.nx + 1) &&
                  ((lane >= 2 && lane < WAVE - 2) || x < 0 || (x >= a.nx && tx == ntx - 1));
        s.R0 = R0;
        s.R1 = R1;
        s.first_y = first_y;
        s.last_y = last_y;
        s.ncell = ncell;
        s.b = b;
        s.padpsi = padpsi;
        s.padg = padg;
        s.run();
    };
    if (interior) go(std::integral_constant<bool, false>{});
    else go(std::integral_constant<bool, true>{});
}

// Cells within two cells of a side (the only ones a ghost position reads): the first and
// last two rows in full, then the first and last two columns of the rows between.
struct Band2D {
    int nx, ny, nrow, ncol;   // band rows (all rows if ny <= 4), band columns of the middle rows
    __host__ __device__ Band2D(int nx_, int ny_) : nx(nx_), ny(ny_), nrow(ny_ <= 4 ? ny_ : 4), ncol(nx_ <= 4 ? nx_ : 4) {}
    __host__ __device__ int64_t count() const { return (int64_t)nrow * nx + (int64_t)(ny > 4 ? ny - 4 : 0) * ncol; }
    // (both branches computed and selected, so that i and j stay in registers)
    __device__ __forceinline__ void cell(int t, int &i, int &j) const
    {
        const int top = nrow * nx;
        const bool inrow = t < top;
        const int r = t / nx, ci = t - r * nx;   // band rows
        const int u = inrow ? 0 : t - top;
        const int v = u / ncol, c = u - v * ncol; // band columns of the middle rows
        const int jr = (ny <= 4 || r < 2) ? r : ny - 4 + r;
        const int ic = (nx <= 4 || c < 2) ? c : nx - 4 + c;
        i = inrow ? ci : ic;
        j = inrow ? jr : 2 + v;
    }
};

// pad^T: each cell within two cells of a side gathers the ghost positions that read it.
template <typename T>
__global__ __launch_bounds__(ADJ_BLOCK) void adj2d_fold_kernel(Cart2DAdjArgs<T> a, const T *padpsi, const double *padg)
{
    const Ring2D pd{a.nx, a.ny};
    const int64_t npos = pd.size();
    const int64_t ncell = (int64_t)a.nx * a.ny;
    const int b = blockIdx.y;
    const Band2D band(a.nx, a.ny);
    const int64_t tb = (int64_t)blockIdx.x * ADJ_BLOCK + threadIdx.x;
    if (tb >= band.count()) return;
    int i, j;
    band.cell((int)tb, i, j);
    const int64_t t = (int64_t)j * a.nx + i;
    // candidate images along each axis: the ghost indices -2, -1, n, n+1 that map to this cell
    // (fixed-size, fully unrolled, so that they stay in registers and every gather below is
    // issued at once)
    const int gxs[4] = {-2, -1, a.nx, a.nx + 1}, gys[4] = {-2, -1, a.ny, a.ny + 1};
    bool hx[5], hy[5];
    T sx[5], sy[5];
    int cx[5], cy[5];
    hx[0] = hy[0] = true;
    sx[0] = sy[0] = T(1);
    cx[0] = i;
    cy[0] = j;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        bool m, nr;
        hx[q + 1] = map_axis(gxs[q], a.nx, a.bc[0], a.bc[1], m, nr) == i;
        sx[q + 1] = m ? T(-1) : T(1);
        cx[q + 1] = gxs[q];
        hy[q + 1] = map_axis(gys[q], a.ny, a.bc[2], a.bc[3], m, nr) == j;
        sy[q + 1] = m ? T(-1) : T(1);
        cy[q + 1] = gys[q];
    }
    // the cell's own values first, so that their loads overlap the gathers
    T own[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) own[f] = a.lam_out[((int64_t)b * 3 + f) * ncell + t];
    const double oE = a.g_epsinv ? a.g_epsinv[(int64_t)b * ncell + t] : 0.0;
    const double oH = a.g_muinv ? a.g_muinv[(int64_t)b * ncell + t] : 0.0;
    T add[3] = {T(0), T(0), T(0)};
    double gE = 0.0, gH = 0.0;
    // The 24 ghost candidates (u, v) != (0, 0), in two halves of 12.  A half's gathers are all
    // issued before any is used (a candidate that does not image this cell reads position 0 and
    // adds a selected zero; a select rather than a branch, so that the loads are not moved into
    // branches), so the kernel waits on memory twice rather than once per ghost that images the
    // cell; the sums keep the (u, v) order.
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        T vp[12][3];
        double vg[12][2];
        bool ok[12];
#pragma unroll
        for (int m = 0; m < 12; ++m) {
            const int k = 1 + 12 * half + m, u = k / 5, v = k % 5;
            ok[m] = hx[u] && hy[v];
            const int64_t p = ok[m] ? pd.idx(cx[u], cy[v]) : 0;
#pragma unroll
            for (int f = 0; f < 3; ++f) vp[m][f] = padpsi[((int64_t)b * 3 + f) * npos + p];
            vg[m][0] = padg[((int64_t)b * 2 + 0) * npos + p];
            vg[m][1] = padg[((int64_t)b * 2 + 1) * npos + p];
        }
#pragma unroll
        for (int m = 0; m < 12; ++m) {
            const int k = 1 + 12 * half + m, u = k / 5, v = k % 5;
            // signs: Ez odd in both mirrors, Hx odd in the x mirror, Hy odd in the y mirror
            add[0] += ok[m] ? sx[u] * sy[v] * vp[m][0] : T(0);
            add[1] += ok[m] ? sx[u] * vp[m][1] : T(0);
            add[2] += ok[m] ? sy[v] * vp[m][2] : T(0);
            gE += ok[m] ? vg[m][0] : 0.0;
            gH += ok[m] ? vg[m][1] : 0.0;
        }
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) a.lam_out[((int64_t)b * 3 + f) * ncell + t] = own[f] + add[f];
    if (a.g_epsinv) a.g_epsinv[(int64_t)b * ncell + t] = oE + gE;
    if (a.g_muinv) a.g_muinv[(int64_t)b * ncell + t] = oH + gH;
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

int64_t adjoint_ring_positions(int nx, int ny) { return Ring2D{nx, ny}.size(); }

// Scratch of the allocation-free adjoint step (gks_adjoint_step_noalloc): one array per GPU in
// the library's device data, shared by every call on that GPU.  Its address on each device is
// looked up once (with that device current) and kept; host code passes that address, never the
// array's name, to the kernels.
static __device__ __align__(256) unsigned char scratch[ADJ_STATIC_SCRATCH_BYTES];

int adjoint_static_scratch(void **ptr)
{
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static void *addr[MAXDEV] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= MAXDEV) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return 0;
}

// One launch of the march kernel variant: the tile height follows from the device's compute
// units and the waves one unit holds of this variant (its occupancy, looked up once).
template <typename T, bool HAS_EPS, bool HAS_MU, bool HM>
static void launch_march(const Cart2DAdjArgs<T> &a, T *padpsi, double *padg, hipStream_t s)
{
    static const int waves_per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adj2d_march_kernel<T, HAS_EPS, HAS_MU, HM>,
                                                         ADJ_MARCH_BLOCK, 0) != hipSuccess ||
            n <= 0)
            n = 8;
        return n * (ADJ_MARCH_BLOCK / WAVE);
    }();
    const int64_t slots = (int64_t)std::max(a.ncu, 1) * waves_per_cu;
    const int ty = adj_tile_rows(a.nx, a.ny, a.batch, slots);
    const int ntx = (a.nx + (WAVE - 4) - 1) / (WAVE - 4), nty = (a.ny + ty - 1) / ty;
    const int64_t waves = (int64_t)ntx * nty * a.batch;
    dim3 grid((unsigned)((waves + ADJ_MARCH_BLOCK / WAVE - 1) / (ADJ_MARCH_BLOCK / WAVE)));
    hipLaunchKernelGGL((adj2d_march_kernel<T, HAS_EPS, HAS_MU, HM>), grid, dim3(ADJ_MARCH_BLOCK), 0, s, a, padpsi, padg,
                       ntx, nty, ty);
}

template <typename T>
int launch_cart2d_adjoint(const Cart2DAdjArgs<T> &a, T *padpsi, double *padg, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (a.epsinv && a.muinv) launch_march<T, true, true, true>(a, padpsi, padg, s);
    else if (a.muinv) launch_march<T, false, true, true>(a, padpsi, padg, s);
    else if (a.g_muinv) {   // vacuum 1/mu, but its gradient is asked for
        if (a.epsinv) launch_march<T, true, false, true>(a, padpsi, padg, s);
        else launch_march<T, false, false, true>(a, padpsi, padg, s);
    } else if (a.epsinv) launch_march<T, true, false, false>(a, padpsi, padg, s);
    else launch_march<T, false, false, false>(a, padpsi, padg, s);
    const int64_t nband = Band2D(a.nx, a.ny).count();
    dim3 gband((unsigned)((nband + ADJ_BLOCK - 1) / ADJ_BLOCK), a.batch);
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

template int launch_cart2d_adjoint<float>(const Cart2DAdjArgs<float> &, float *, double *, void *);
template int launch_cart2d_adjoint<double>(const Cart2DAdjArgs<double> &, double *, double *, void *);
template int launch_adjoint_source<float>(const float *, double *, int64_t, int64_t, int32_t, const int64_t *,
                                          const double *, double, int32_t, void *);
template int launch_adjoint_source<double>(const double *, double *, int64_t, int64_t, int32_t, const int64_t *,
                                           const double *, double, int32_t, void *);

}  // namespace gks
