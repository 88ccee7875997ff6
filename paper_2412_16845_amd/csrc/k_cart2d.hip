// Fused GKS step on a 2D Cartesian grid, TM fields (Ez, Hx, Hy), or the TM fields of the
// perfectly hyperbolic Maxwell system with the divergence-cleaning potential psi (Sec. 2.1):
// (Ez, Hx, Hy, psi).  The field count NF is a template parameter; everything below applies
// to both.
//
// One wavefront owns a strip of 64 lanes x NC adjacent columns (NC = 2 for FP32, 1 for FP64,
// so that every lane moves 8 bytes per field and row); the two outermost columns on each side
// are halo, the rest are written.  The wave marches a tile of rows up or down (the host's tile
// table gives each tile row's batch item, rows and direction, in dispatch order).  Each field value is
// loaded once per strip row; neighbours along x come from the lane itself or from the adjacent
// lanes through DPP moves, so no LDS and no barriers are needed.  Per row the wave:
//   1. issues the loads of the row PF rows ahead (structure-of-arrays, 512 contiguous bytes
//      per field: coalesced), so that several rows of loads are in flight while it computes;
//   2. forms the Green-Gauss (central) differences of the middle row of its three-row window;
//   3. evaluates the GKS flux of the horizontal face below the middle row and of the vertical
//      face right of each column, as sparse linear forms of the stencil values (the
//      closed-form moments of Sec. 3.1 folded into coefficients on the host);
//   4. sums the face fluxes of each cell of the row it finishes in double precision (in FP32
//      mode the fluxes are widened first), adds the divergence and a single point source to the
//      old value in double precision and stores the result rounded once to the storage type
//      (longer source lists are added afterwards by a small scatter kernel, which keeps the
//      per-cell source tests out of the marching loop).
// The row loop is unrolled six times so that the rotating window (six row slots, two gradient
// slots, two flux slots) lives in fixed registers without copies.
// Strips that touch no domain side take a path without index mapping.  On the others, ghost
// rows/columns follow the boundary condition: non-reflecting sides give the ghost side of a
// boundary face no distribution (zero state and slopes) and the Green-Gauss gradient the cell's
// own value; PEC sides read mirror ghosts (Ez and the normal H odd, the tangential H even, psi
// even); periodic sides wrap.
#include "gks_device.h"

namespace gks {

constexpr int HALO = 2;
constexpr int PF = 3;   // rows loaded ahead of use: with the three-row window, six row slots
// Four waves (four horizontally adjacent strips) per workgroup: they share their halo columns
// in the compute unit's L1.  Measured on 4096^2 (fp32): 116.6 us, against 119.3 us with one wave
// and 121.8 us with four vertically adjacent tiles per workgroup.
constexpr int STEP2D_BLOCK = 256;

#ifndef GKS_FP32_COLS_PER_LANE
#define GKS_FP32_COLS_PER_LANE 2
#endif
template <typename T>
constexpr int cols_per_lane() { return sizeof(T) == 4 ? GKS_FP32_COLS_PER_LANE : 1; }
template <typename T>
constexpr int out_cols() { return WAVE * cols_per_lane<T>() - 2 * HALO; }

// The two field sets: sparsity tables and operator layout of the x- and y-faces.
template <int NF> struct Fields2D;
template <> struct Fields2D<3> {   // Ez, Hx, Hy
    using PX = PatTMx;
    using PY = PatTMy;
    template <typename T> using Op = FaceOpTM<T>;
};
template <> struct Fields2D<4> {   // Ez, Hx, Hy, psi
    using PX = PatTPx;
    using PY = PatTPy;
    template <typename T> using Op = FaceOpTP<T>;
};

template <typename T, int NC, int NF>
struct Row2D {
    T u[NC][NF];     // Ez, Hx, Hy (, psi) per column (mirror signs applied)
    T mE[NC], mH[NC];
    bool nr[NC];     // non-reflecting ghost (boundary strips only)
};

// NC consecutive values at byte offsets (voff + soff): one 8-byte access.
template <typename T, int NC>
__device__ __forceinline__ void load_cols(Rsrc r, uint32_t voff, uint32_t soff, T (&out)[NC])
{
    if constexpr (NC == 2) {
        const float2 v = buf_load_f2(r, voff, soff);
        out[0] = v.x;
        out[1] = v.y;
    } else {
        out[0] = buf_load<T>(r, voff, soff);
    }
}

template <typename T, int NC, int NF, bool HAS_EPS, bool HAS_MU, bool BND, bool LIM>
struct Strip2D {
    static_assert(!LIM || NF == 3, "the limited step is built for the TM fields only");
    using FS = Fields2D<NF>;
    using OpT = typename FS::template Op<T>;
    using Row = Row2D<T, NC, NF>;
    // coefficient chunk of the face operators: 8 for the fp64 PHM kernel (4096^2: 274.2 ->
    // 269.8 us), 12 elsewhere (the fastest there)
    static constexpr int CH2 = (sizeof(T) == 8 && NF == 4) ? 8 : 12;
    // vacuum 1/mu with the TM fields: the host folds the operators' 1/mu parts into K0 (the
    // second pair of operators), which saves five multiply-adds per face
    static constexpr bool HM = HAS_MU || NF != 3;
    static constexpr int OPS0 = HM ? 0 : 2;
    const Cart2DArgs<T> &a;
    Rsrc rU, rE, rM, rO;   // this batch item's fields, 1/eps, 1/mu, output fields
    uint32_t fbytes;       // bytes per field array
    uint32_t vlane;        // byte offset of this lane's first column inside the strip
    int x0;                // first column of the strip (uniform; -2 on the first strip)
    int gx0;               // first column of this lane
    uint32_t vx[NC];       // boundary strips: byte offset of the column each cell reads
    T sgx[NC];             // boundary strips: x-mirror sign of Ez and Hx
    bool nrx[NC];          // boundary strips: non-reflecting ghost column
    bool writer[NC];
    int y0, y1;

    __device__ __forceinline__ void load(int gy, Row &r) const
    {
        if constexpr (BND) {
            bool mir, nry;
            const int sy = map_axis(gy, a.ny, a.bc[2], a.bc[3], mir, nry);
            const uint32_t so = (uint32_t)sy * (uint32_t)a.nx * (uint32_t)sizeof(T);
            const T sgy = mir ? T(-1) : T(1);   // y mirror: Ez and Hy odd, Hx and psi even
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                r.u[k][0] = buf_load<T>(rU, vx[k], so) * (sgx[k] * sgy);
                r.u[k][1] = buf_load<T>(rU, vx[k], so + fbytes) * sgx[k];
                r.u[k][2] = buf_load<T>(rU, vx[k], so + 2 * fbytes) * sgy;
                if constexpr (NF == 4) r.u[k][3] = buf_load<T>(rU, vx[k], so + 3 * fbytes);
                r.mE[k] = HAS_EPS ? buf_load<T>(rE, vx[k], so) : T(1);
                r.mH[k] = HAS_MU ? buf_load<T>(rM, vx[k], so) : T(1);
                r.nr[k] = nry || nrx[k];
            }
        } else {
            const uint32_t so = ((uint32_t)gy * (uint32_t)a.nx + (uint32_t)x0) * (uint32_t)sizeof(T);
            T v[NC];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                load_cols<T, NC>(rU, vlane, so + f * fbytes, v);
#pragma unroll
                for (int k = 0; k < NC; ++k) r.u[k][f] = v[k];
            }
            if (HAS_EPS) load_cols<T, NC>(rE, vlane, so, r.mE);
            else
#pragma unroll
                for (int k = 0; k < NC; ++k) r.mE[k] = T(1);
            if (HAS_MU) load_cols<T, NC>(rM, vlane, so, r.mH);
            else
#pragma unroll
                for (int k = 0; k < NC; ++k) r.mH[k] = T(1);
#pragma unroll
            for (int k = 0; k < NC; ++k) r.nr[k] = false;
        }
    }

    // One row step number i of the march in direction s = +1 (upwards, DN false) or -1: the
    // window holds rows q-2s (Rs), q-s (Rc), q (Rn) with q = qs + s i; Rp receives row q+PF s.
    // fyP is the horizontal face computed one step earlier, fyN the one computed now.
    template <bool DN>
    __device__ __forceinline__ void body(int i, int qs, Row &Rs, Row &Rc, Row &Rn, Row &Rp, T (&Ds)[NC][2 * NF],
                                         T (&Dc)[NC][2 * NF], T (&fyP)[NC][NF], T (&fyN)[NC][NF]) const
    {
        constexpr int sd = DN ? -1 : 1;
        const int q = qs + sd * i;
        const OpT *ops = (const OpT *)a.ops;
        // coefficients of the horizontal faces: loaded after the previous row's divergence
        const auto opy = scalar_ptr_after(ops + OPS0 + 1, fyP[0][0]);
        // rows beyond the tile and its halo are not needed: re-read the last halo row instead
        // (already cached), which keeps the load unconditional so the loads in flight are
        // counted exactly
        load(DN ? max(q - PF, y0 - 2) : min(q + PF, y1 + 1), Rp);
        // central differences of row q-1: [d/dx x fields, d/dy x fields] times 2h
        T right[NC][NF], left[NC][NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T rnext = from_right(Rc.u[0][f]);       // first column of the next lane
            const T lprev = from_left(Rc.u[NC - 1][f]);   // last column of the previous lane
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                right[k][f] = (k + 1 < NC) ? Rc.u[k + 1 < NC ? k + 1 : 0][f] : rnext;
                left[k][f] = (k > 0) ? Rc.u[k > 0 ? k - 1 : 0][f] : lprev;
                Dc[k][f] = right[k][f] - left[k][f];
                Dc[k][NF + f] = DN ? Rs.u[k][f] - Rn.u[k][f] : Rn.u[k][f] - Rs.u[k][f];
            }
        }
        if constexpr (LIM) {
            // limited slopes: minmod of the one-sided differences of the variables that travel
            // along each axis (x: Ez +/- Hy, with Hx normal; y: Ez +/- Hx, with Hy normal)
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const T(&c)[NF] = Rc.u[k];
                const T(&up)[NF] = DN ? Rs.u[k] : Rn.u[k];   // the row above (larger y)
                const T(&dn)[NF] = DN ? Rn.u[k] : Rs.u[k];
                limit_pair(right[k][0] - c[0], right[k][2] - c[2], c[0] - left[k][0], c[2] - left[k][2], Dc[k][0],
                           Dc[k][2]);
                Dc[k][1] = T(2) * minmod(right[k][1] - c[1], c[1] - left[k][1]);
                limit_pair(up[0] - c[0], up[1] - c[1], c[0] - dn[0], c[1] - dn[1], Dc[k][NF + 0], Dc[k][NF + 1]);
                Dc[k][NF + 2] = T(2) * minmod(up[2] - c[2], c[2] - dn[2]);
            }
        }
        if (i < 1) return;

        // horizontal face between rows q-2s and q-s: inputs [UL UR dyL dxL dyR dxR] x fields,
        // L the lower row
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const Row &RL = DN ? Rc : Rs;
            const Row &RR = DN ? Rs : Rc;
            const T(&DL)[NC][2 * NF] = DN ? Dc : Ds;
            const T(&DR)[NC][2 * NF] = DN ? Ds : Dc;
            const bool zl = BND && RL.nr[k], zr = BND && RR.nr[k];
            T w[6 * NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                w[f] = zl ? T(0) : RL.u[k][f];
                w[NF + f] = zr ? T(0) : RR.u[k][f];
                w[2 * NF + f] = zl ? T(0) : DL[k][NF + f];
                w[3 * NF + f] = zl ? T(0) : DL[k][f];
                w[4 * NF + f] = zr ? T(0) : DR[k][NF + f];
                w[5 * NF + f] = zr ? T(0) : DR[k][f];
            }
            // face material: the two cells' values (a ghost reads its interior cell); the
            // operator applies their mean
            apply_op<typename FS::PY, CH2, HM>(w, RL.mE[k] + RR.mE[k], HM ? RL.mH[k] + RR.mH[k] : T(2), opy, fyN[k]);
        }
        if (i < 2) return;
        // coefficients of the vertical faces: loaded once the horizontal faces are done
        const auto opx = scalar_ptr_after(ops + OPS0, fyN[NC - 1][2]);

        // vertical faces right of each column, row q-2s: inputs [UL UR dxL dyL dxR dyR] x fields
        T ul[NC][NF], dl[NC][2 * NF];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const bool z = BND && Rs.nr[k];
#pragma unroll
            for (int f = 0; f < NF; ++f) ul[k][f] = z ? T(0) : Rs.u[k][f];
#pragma unroll
            for (int f = 0; f < 2 * NF; ++f) dl[k][f] = z ? T(0) : Ds[k][f];
        }
        T fx[NC][NF];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            constexpr int last = NC - 1;
            const int kr = (k + 1 < NC) ? k + 1 : 0;
            T v[6 * NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                v[f] = ul[k][f];
                v[NF + f] = (k < last) ? ul[kr][f] : from_right(ul[0][f]);
                v[2 * NF + f] = dl[k][f];
                v[3 * NF + f] = dl[k][NF + f];
                v[4 * NF + f] = (k < last) ? dl[kr][f] : from_right(dl[0][f]);
                v[5 * NF + f] = (k < last) ? dl[kr][NF + f] : from_right(dl[0][NF + f]);
            }
            const T mEr = (k < last) ? Rs.mE[kr] : from_right(Rs.mE[0]);
            const T mHr = !HM ? T(1) : (k < last) ? Rs.mH[kr] : from_right(Rs.mH[0]);
            apply_op<typename FS::PX, CH2, HM>(v, Rs.mE[k] + mEr, Rs.mH[k] + mHr, opx, fx[k]);
        }

        // update: the face fluxes (FP32 in FP32 mode) are widened to FP64, their divergence is
        // summed and added to the old value in FP64 with the explicit point source, and the
        // result is rounded once to the storage type (longer source lists are added by a
        // separate scatter kernel)
        const int row = q - 2 * sd;
        const uint32_t rowc = (uint32_t)row * (uint32_t)a.nx;
        T nv[NC][NF];
        double src[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) src[k] = (row == a.src_row && gx0 + k == a.src_col) ? a.src_amp : 0.0;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double fr = (double)fx[k][f];
                const double fl = (double)((k > 0) ? fx[k > 0 ? k - 1 : 0][f] : from_left(fx[NC - 1][f]));
                const double fu = (double)(DN ? fyP[k][f] : fyN[k][f]);   // upper face
                const double fd = (double)(DN ? fyN[k][f] : fyP[k][f]);   // lower face
                const double div = (fr - fl) + (fu - fd);
                // 1/eps scales Ez, 1/mu scales H; psi carries no material factor
                const double m = (f == 0) ? (double)Rs.mE[k] : (f < 3) ? (double)Rs.mH[k] : 1.0;
                const double add = (f == 0) ? src[k] : 0.0;
                nv[k][f] = (T)fma(m, add - div, (double)Rs.u[k][f]);
            }
        }
        if constexpr (!BND) {
            // interior strips: every lane but the two halo lanes writes all its columns
            if (writer[0]) {
                const uint32_t so = (rowc + (uint32_t)x0) * (uint32_t)sizeof(T);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    if constexpr (NC == 2) buf_store_f2(make_float2(nv[0][f], nv[1][f]), rO, vlane, so + f * fbytes);
                    else buf_store(nv[0][f], rO, vlane, so + f * fbytes);
                }
            }
        } else {
            // boundary strips (whose first columns may be ghosts): row start + own column
            const uint32_t so = rowc * (uint32_t)sizeof(T);
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (writer[k]) {
                    const uint32_t vo = (uint32_t)(gx0 + k) * (uint32_t)sizeof(T);
#pragma unroll
                    for (int f = 0; f < NF; ++f) buf_store(nv[k][f], rO, vo, so + f * fbytes);
                }
        }
    }

    // March the tile upwards (DN false: rows y0-2 .. y1+1) or downwards (rows y1+1 .. y0-2).
    template <bool DN>
    __device__ __forceinline__ void run() const
    {
        constexpr int sd = DN ? -1 : 1;
        Row R0, R1, R2, R3, R4, R5;
        T D0[NC][2 * NF], D1[NC][2 * NF];
        T F0[NC][NF], F1[NC][NF];
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int f = 0; f < NF; ++f) F0[k][f] = F1[k][f] = T(0);
        const int qs = DN ? y1 - 1 : y0;       // window head of the first step
        load(qs - 2 * sd, R0);
        load(qs - sd, R1);
        load(qs, R2);
        load(qs + sd, R3);
        load(qs + 2 * sd, R4);
        const int n = y1 - y0 + 2;             // steps: the head runs over y0..y1+1
        for (int i = 0; i < n; i += 6) {
            body<DN>(i, qs, R0, R1, R2, R5, D0, D1, F0, F1);
            if (i + 1 >= n) break;
            body<DN>(i + 1, qs, R1, R2, R3, R0, D1, D0, F1, F0);
            if (i + 2 >= n) break;
            body<DN>(i + 2, qs, R2, R3, R4, R1, D0, D1, F0, F1);
            if (i + 3 >= n) break;
            body<DN>(i + 3, qs, R3, R4, R5, R2, D1, D0, F1, F0);
            if (i + 4 >= n) break;
            body<DN>(i + 4, qs, R4, R5, R0, R3, D0, D1, F0, F1);
            if (i + 5 >= n) break;
            body<DN>(i + 5, qs, R5, R0, R1, R4, D1, D0, F1, F0);
        }
    }

    // Vertically adjacent tiles march in opposite directions, so that the two rows they share
    // at a tile edge are read by both at the same time (both at the start or both at the end
    // of their march) and the second read is served by the L2.
    __device__ __forceinline__ void run(bool down) const
    {
        if (down) run<true>();
        else run<false>();
    }
};

// ------------------------------------------------------------------ two steps per launch
// The paired kernel runs two consecutive steps of the TM fields (with or without psi, with or
// without the limiter) in one march, so that the fields are read and written once per two steps.
// Stage 1 is the march above over a strip with four halo columns and a tile widened by two rows
// on each side.  Every row it finishes (the state after the first step, rounded to the storage
// type as a stored state would be) enters stage 2, a second march of the same form that takes
// its rows from registers instead of memory and writes the state after the second step.  Both
// stages do the single-step kernel's arithmetic in its order, so the two kernels give the same
// results bit for bit.
// Ghost values of the intermediate state behind a non-reflecting or PEC side are formed from its
// own cells, as the loads form them for a stored state: along x from the boundary column held
// by another lane of the same wave, along y from the last two rows stage 1 finished (so a tile
// that touches the lower side marches down and one that touches the upper side marches up).
// Behind a periodic side stage 1 forms them itself, as the step of the cells they image (its
// inputs wrap, and the step is the same at every position).
constexpr int PAIR_HALO = 4;
// One column per lane in both precisions: the paired fp32 kernel with two columns per lane
// needs all 256 VGPRs (and spills); with one it takes 150.0 against 173.6 us per launch on the
// 4096^2 workload, for the wider halo (8 of 64 columns).
#ifndef GKS_PAIR_FP32_COLS
#define GKS_PAIR_FP32_COLS 1
#endif
template <typename T>
constexpr int pair_cols_per_lane() { return sizeof(T) == 4 ? GKS_PAIR_FP32_COLS : 1; }
template <typename T>
constexpr int pair_out_cols() { return WAVE * pair_cols_per_lane<T>() - 2 * PAIR_HALO; }

// v of the lane whose byte address (4 x lane) is given; all lanes take part (the asm keeps
// the move out of any branch, where lanes switched off would read as zero)
__device__ __forceinline__ float lane_fetch(float v, int addr)
{
    int r = __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v));
    asm volatile("" : "+v"(r));
    return __builtin_bit_cast(float, r);
}
__device__ __forceinline__ double lane_fetch(double v, int addr)
{
    const long long b = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffll));
    int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    asm volatile("" : "+v"(lo), "+v"(hi));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, int NC, int NF, bool HAS_EPS, bool HAS_MU, bool BND, bool PER, bool LIM>
struct Pair2D {
    using S = Strip2D<T, NC, NF, HAS_EPS, HAS_MU, BND, LIM>;
    using Row = Row2D<T, NC, NF>;
    using FS = Fields2D<NF>;
    using OpT = typename FS::template Op<T>;
    static constexpr int CH2 = S::CH2;
    static constexpr bool HM = S::HM;
    static constexpr int OPS0 = S::OPS0;
    S s;              // the strip: buffer resources, column maps, stage 1's loads, stage 2's writers
    int ylo, yhi;     // the rows stage 1 reads (its loads are clamped to them)
    bool yper;        // periodic y sides: rows beyond them wrap, and ghost rows are formed by stage 1
    int scol[NC];     // the column each lane's cells are (a periodic ghost: its image), for the source
    int gaddr[NC];    // boundary strips: the lane (byte address) holding each ghost column's image
    int gk[NC];       // ... and the column of that lane
    bool gcol[NC];    // a ghost column whose intermediate value stage 2 reads

    // the row a periodic y side wraps a row to (other rows unchanged)
    __device__ __forceinline__ int wrap_row(int y) const
    {
        if (!BND || !PER || !yper) return y;
        const int ny = s.a.ny;
        return ((y % ny) + ny) % ny;
    }
    // the row stage 1 loads for march row y: clamped to the rows it reads, wrapped on periodic sides
    __device__ __forceinline__ int stage1_row(int y) const
    {
        if constexpr (BND && PER) return wrap_row(min(max(y, ylo), yhi));
        else return min(max(y, ylo), yhi);
    }

    // One row step of a march whose window holds rows Rs = q-2s, Rc = q-s, Rn = q: the
    // differences of Rc, the horizontal face between Rs and Rc, and from the third step on the
    // vertical faces of Rs and its new values nv.  Returns whether nv was formed.
    template <bool DN>
    __device__ __forceinline__ bool stage(int i, int q, double amp, const Row &Rs, const Row &Rc, const Row &Rn,
                                          T (&Ds)[NC][2 * NF], T (&Dc)[NC][2 * NF], T (&fyP)[NC][NF],
                                          T (&fyN)[NC][NF], T (&nv)[NC][NF]) const
    {
        constexpr int sd = DN ? -1 : 1;
        const Cart2DArgs<T> &a = s.a;
        const OpT *ops = (const OpT *)a.ops;
        const auto opy = scalar_ptr_after(ops + OPS0 + 1, fyP[0][0]);
        T right[NC][NF], left[NC][NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T rnext = from_right(Rc.u[0][f]);
            const T lprev = from_left(Rc.u[NC - 1][f]);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                right[k][f] = (k + 1 < NC) ? Rc.u[k + 1 < NC ? k + 1 : 0][f] : rnext;
                left[k][f] = (k > 0) ? Rc.u[k > 0 ? k - 1 : 0][f] : lprev;
                Dc[k][f] = right[k][f] - left[k][f];
                Dc[k][NF + f] = DN ? Rs.u[k][f] - Rn.u[k][f] : Rn.u[k][f] - Rs.u[k][f];
            }
        }
        if constexpr (LIM) {
            // limited slopes, as in the single-step kernel
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const T(&c)[NF] = Rc.u[k];
                const T(&up)[NF] = DN ? Rs.u[k] : Rn.u[k];
                const T(&dn)[NF] = DN ? Rn.u[k] : Rs.u[k];
                limit_pair(right[k][0] - c[0], right[k][2] - c[2], c[0] - left[k][0], c[2] - left[k][2], Dc[k][0],
                           Dc[k][2]);
                Dc[k][1] = T(2) * minmod(right[k][1] - c[1], c[1] - left[k][1]);
                limit_pair(up[0] - c[0], up[1] - c[1], c[0] - dn[0], c[1] - dn[1], Dc[k][NF + 0], Dc[k][NF + 1]);
                Dc[k][NF + 2] = T(2) * minmod(up[2] - c[2], c[2] - dn[2]);
            }
        }
        if (i < 1) return false;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const Row &RL = DN ? Rc : Rs;
            const Row &RR = DN ? Rs : Rc;
            const T(&DL)[NC][2 * NF] = DN ? Dc : Ds;
            const T(&DR)[NC][2 * NF] = DN ? Ds : Dc;
            const bool zl = BND && RL.nr[k], zr = BND && RR.nr[k];
            T w[6 * NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                w[f] = zl ? T(0) : RL.u[k][f];
                w[NF + f] = zr ? T(0) : RR.u[k][f];
                w[2 * NF + f] = zl ? T(0) : DL[k][NF + f];
                w[3 * NF + f] = zl ? T(0) : DL[k][f];
                w[4 * NF + f] = zr ? T(0) : DR[k][NF + f];
                w[5 * NF + f] = zr ? T(0) : DR[k][f];
            }
            apply_op<typename FS::PY, CH2, HM>(w, RL.mE[k] + RR.mE[k], HM ? RL.mH[k] + RR.mH[k] : T(2), opy, fyN[k]);
        }
        if (i < 2) return false;
        const auto opx = scalar_ptr_after(ops + OPS0, fyN[NC - 1][2]);
        T ul[NC][NF], dl[NC][2 * NF];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const bool z = BND && Rs.nr[k];
#pragma unroll
            for (int f = 0; f < NF; ++f) ul[k][f] = z ? T(0) : Rs.u[k][f];
#pragma unroll
            for (int f = 0; f < 2 * NF; ++f) dl[k][f] = z ? T(0) : Ds[k][f];
        }
        T fx[NC][NF];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            constexpr int last = NC - 1;
            const int kr = (k + 1 < NC) ? k + 1 : 0;
            T v[6 * NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                v[f] = ul[k][f];
                v[NF + f] = (k < last) ? ul[kr][f] : from_right(ul[0][f]);
                v[2 * NF + f] = dl[k][f];
                v[3 * NF + f] = dl[k][NF + f];
                v[4 * NF + f] = (k < last) ? dl[kr][f] : from_right(dl[0][f]);
                v[5 * NF + f] = (k < last) ? dl[kr][NF + f] : from_right(dl[0][NF + f]);
            }
            const T mEr = (k < last) ? Rs.mE[kr] : from_right(Rs.mE[0]);
            const T mHr = !HM ? T(1) : (k < last) ? Rs.mH[kr] : from_right(Rs.mH[0]);
            apply_op<typename FS::PX, CH2, HM>(v, Rs.mE[k] + mEr, Rs.mH[k] + mHr, opx, fx[k]);
        }
        const int row = q - 2 * sd;
        double src[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            // boundary strips: a periodic ghost takes the source of the cell it images
            if constexpr (BND && PER) src[k] = (wrap_row(row) == a.src_row && scol[k] == a.src_col) ? amp : 0.0;
            else src[k] = (row == a.src_row && s.gx0 + k == a.src_col) ? amp : 0.0;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double fr = (double)fx[k][f];
                const double fl = (double)((k > 0) ? fx[k > 0 ? k - 1 : 0][f] : from_left(fx[NC - 1][f]));
                const double fu = (double)(DN ? fyP[k][f] : fyN[k][f]);
                const double fd = (double)(DN ? fyN[k][f] : fyP[k][f]);
                const double div = (fr - fl) + (fu - fd);
                // 1/eps scales Ez, 1/mu scales H; psi carries no material factor
                const double m = (f == 0) ? (double)Rs.mE[k] : (f < 3) ? (double)Rs.mH[k] : 1.0;
                const double add = (f == 0) ? src[k] : 0.0;
                nv[k][f] = (T)fma(m, add - div, (double)Rs.u[k][f]);
            }
        }
        return true;
    }

    __device__ __forceinline__ void store(int row, const T (&nv)[NC][NF]) const
    {
        const Cart2DArgs<T> &a = s.a;
        const uint32_t rowc = (uint32_t)row * (uint32_t)a.nx;
        if constexpr (!BND) {
            if (s.writer[0]) {
                const uint32_t so = (rowc + (uint32_t)s.x0) * (uint32_t)sizeof(T);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    if constexpr (NC == 2) buf_store_f2(make_float2(nv[0][f], nv[1][f]), s.rO, s.vlane, so + f * s.fbytes);
                    else buf_store(nv[0][f], s.rO, s.vlane, so + f * s.fbytes);
                }
            }
        } else {
            const uint32_t so = rowc * (uint32_t)sizeof(T);
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (s.writer[k]) {
                    const uint32_t vo = (uint32_t)(s.gx0 + k) * (uint32_t)sizeof(T);
#pragma unroll
                    for (int f = 0; f < NF; ++f) buf_store(nv[k][f], s.rO, vo, so + f * s.fbytes);
                }
        }
    }

    // Stage-1 step i (window head q = qs + s i) and, from i = 4 on, stage-2 step i - 4, whose
    // window (Bs, Bc, Bn) holds the intermediate rows formed at steps i - 2, i - 1 and i.
    // h0 and h1 hold the last two real intermediate rows (h0 the later one, row hrow).
    template <bool DN>
    __device__ __forceinline__ void pstep(int i, int qs, Row &Rs, Row &Rc, Row &Rn, Row &Rp, T (&Ds)[NC][2 * NF],
                                          T (&Dc)[NC][2 * NF], T (&fyP)[NC][NF], T (&fyN)[NC][NF], Row &Bs,
                                          Row &Bc, Row &Bn, T (&Es)[NC][2 * NF], T (&Ec)[NC][2 * NF],
                                          T (&gP)[NC][NF], T (&gN)[NC][NF], T (&h0)[NC][NF], T (&h1)[NC][NF],
                                          int &hrow) const
    {
        constexpr int sd = DN ? -1 : 1;
        const Cart2DArgs<T> &a = s.a;
        const int q = qs + sd * i;
        s.load(stage1_row(q + sd * PF), Rp);
        T nv[NC][NF];
        if (!stage<DN>(i, q, a.src_amp, Rs, Rc, Rn, Ds, Dc, fyP, fyN, nv)) return;
        const int r = q - 2 * sd;   // the intermediate row just formed
        if constexpr (BND) {
            // ghost columns: the (mirror) image of a column of the same row; x mirror: Ez and Hx
            // odd, Hy and psi even
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                T got[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    T from[NC];
#pragma unroll
                    for (int kk = 0; kk < NC; ++kk) from[kk] = lane_fetch(nv[kk][f], gaddr[k]);
                    T v = from[0];
#pragma unroll
                    for (int kk = 1; kk < NC; ++kk) v = (gk[k] == kk) ? from[kk] : v;
                    got[k] = (f < 2) ? v * s.sgx[k] : v;
                }
#pragma unroll
                for (int k = 0; k < NC; ++k) nv[k][f] = gcol[k] ? got[k] : nv[k][f];
            }
            if (!(PER && yper) && (r < 0 || r >= a.ny)) {
                // a ghost row: the (mirror) image of one of the last two real rows; y mirror: Ez and
                // Hy odd, Hx and psi even
                bool mir, nry;
                const int m = map_axis(r, a.ny, a.bc[2], a.bc[3], mir, nry);
                const bool last = m == hrow;
                const T sg = mir ? T(-1) : T(1);
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        const T v = last ? h0[k][f] : h1[k][f];
                        nv[k][f] = (f == 0 || f == 2) ? v * sg : v;
                    }
            } else {
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        h1[k][f] = h0[k][f];
                        h0[k][f] = nv[k][f];
                    }
                hrow = r;
            }
        }
        // the row enters stage 2 with the materials and ghost flags of its cells
#pragma unroll
        for (int k = 0; k < NC; ++k) {
#pragma unroll
            for (int f = 0; f < NF; ++f) Bn.u[k][f] = nv[k][f];
            Bn.mE[k] = Rs.mE[k];
            Bn.mH[k] = Rs.mH[k];
            Bn.nr[k] = Rs.nr[k];
        }
        if (i < 4) return;
        T nv2[NC][NF];
        if (!stage<DN>(i - 4, r, a.src_amp2, Bs, Bc, Bn, Es, Ec, gP, gN, nv2)) return;
        store(r - 2 * sd, nv2);
    }

    // March the tile (rows y0 .. y1-1 written): stage 1 forms the intermediate rows y0-2 ..
    // y1+1, upwards (DN false) or downwards.
    template <bool DN>
    __device__ __forceinline__ void run() const
    {
        constexpr int sd = DN ? -1 : 1;
        const int y0 = s.y0, y1 = s.y1;
        Row R0, R1, R2, R3, R4, R5, B0, B1, B2;
        T D0[NC][2 * NF], D1[NC][2 * NF], E0[NC][2 * NF], E1[NC][2 * NF];
        T F0[NC][NF], F1[NC][NF], G0[NC][NF], G1[NC][NF], H0[NC][NF], H1[NC][NF];
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int f = 0; f < NF; ++f) F0[k][f] = F1[k][f] = G0[k][f] = G1[k][f] = H0[k][f] = H1[k][f] = T(0);
        int hrow = -1000;
        const int Y0 = y0 - 2, Y1 = y1 + 2;          // intermediate rows formed: [Y0, Y1)
        const int qs = DN ? Y1 - 1 : Y0;
        auto ld = [&](int y, Row &R) { s.load(stage1_row(y), R); };
        ld(qs - 2 * sd, R0);
        ld(qs - sd, R1);
        ld(qs, R2);
        ld(qs + sd, R3);
        ld(qs + 2 * sd, R4);
        const int n = Y1 - Y0 + 2;
        for (int i = 0; i < n; i += 6) {
            pstep<DN>(i, qs, R0, R1, R2, R5, D0, D1, F0, F1, B1, B2, B0, E0, E1, G0, G1, H0, H1, hrow);
            if (i + 1 >= n) break;
            pstep<DN>(i + 1, qs, R1, R2, R3, R0, D1, D0, F1, F0, B2, B0, B1, E1, E0, G1, G0, H0, H1, hrow);
            if (i + 2 >= n) break;
            pstep<DN>(i + 2, qs, R2, R3, R4, R1, D0, D1, F0, F1, B0, B1, B2, E0, E1, G0, G1, H0, H1, hrow);
            if (i + 3 >= n) break;
            pstep<DN>(i + 3, qs, R3, R4, R5, R2, D1, D0, F1, F0, B1, B2, B0, E1, E0, G1, G0, H0, H1, hrow);
            if (i + 4 >= n) break;
            pstep<DN>(i + 4, qs, R4, R5, R0, R3, D0, D1, F0, F1, B2, B0, B1, E0, E1, G0, G1, H0, H1, hrow);
            if (i + 5 >= n) break;
            pstep<DN>(i + 5, qs, R5, R0, R1, R4, D1, D0, F1, F0, B0, B1, B2, E1, E0, G1, G0, H0, H1, hrow);
        }
    }
};

// Four waves per SIMD in fp32 (at most 128 VGPRs; the 1/eps kernel then spills 5 values): 143.7
// against 150.0 us per launch on the 4096^2 workload at the compiler's 134 VGPRs and three waves.
// The kernel with both material maps would spill 42 values and keeps three, as do the PHM fields
// (four per cell); fp64 needs two.
// PER: the grid has a periodic side (a separate instantiation keeps that bookkeeping out of the
// others: with it the 4096^2 non-reflecting launch took 164.3 against 144.1 us in fp32).  LIM:
// minmod-limited slopes (TM fields only).
template <typename T, int NF, bool HAS_EPS, bool HAS_MU, bool PER, bool LIM>
__global__ __launch_bounds__(STEP2D_BLOCK, sizeof(T) == 8 ? 2 : (NF == 4 || LIM || (HAS_EPS && HAS_MU)) ? 3 : 4) void
cart2d_pair_kernel(Cart2DArgs<T> a)
{
    constexpr int NC = pair_cols_per_lane<T>();
    const int lane = threadIdx.x & (WAVE - 1);
    const int band = blockIdx.x % NBANDS;
    const int wave = (blockIdx.x / NBANDS) * (STEP2D_BLOCK / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int tl = wave / a.ntx;
    if (tl >= a.nty) return;
    const int tx = wave - tl * a.ntx;
    const int t = band * a.nty + tl;
    const int b = __builtin_amdgcn_readfirstlane(a.tiles[4 * t]);
    if (b < 0) return;
    const int y0 = __builtin_amdgcn_readfirstlane(a.tiles[4 * t + 1]);
    const int y1 = __builtin_amdgcn_readfirstlane(a.tiles[4 * t + 2]);
    const bool down = __builtin_amdgcn_readfirstlane(a.tiles[4 * t + 3]) != 0;

    const int64_t ncell = (int64_t)a.nx * a.ny;
    const uint32_t fbytes = (uint32_t)(ncell * (int64_t)sizeof(T));
    const Rsrc rU = make_rsrc(a.U + (int64_t)b * NF * ncell, (uint64_t)NF * fbytes);
    const Rsrc rO = make_rsrc(a.Unew + (int64_t)b * NF * ncell, (uint64_t)NF * fbytes);
    const Rsrc rE = make_rsrc(HAS_EPS ? a.epsinv + (int64_t)b * ncell : a.U, fbytes);
    const Rsrc rM = make_rsrc(HAS_MU ? a.muinv + (int64_t)b * ncell : a.U, fbytes);

    const int x0 = tx * pair_out_cols<T>() - PAIR_HALO;
    const int gx0 = x0 + NC * lane;
    const uint32_t vlane = (uint32_t)(NC * lane) * (uint32_t)sizeof(T);
    // periodic y sides: rows beyond them wrap (stage 1 forms the intermediate ghost rows as the
    // step of the rows they image); other sides: the two ghost rows a load can form
    const bool yper = PER && a.bc[2] == GKS_BC_PERIODIC;
    const int ylo = yper ? y0 - 4 : max(y0 - 4, -2), yhi = yper ? y1 + 3 : min(y1 + 3, a.ny + 1);

    const bool interior = x0 >= 0 && x0 + WAVE * NC - 1 <= a.nx - 1 && y0 - 4 >= 0 && y1 + 3 <= a.ny - 1;
    if (interior) {
        Pair2D<T, NC, NF, HAS_EPS, HAS_MU, false, PER, LIM> p{{a, rU, rE, rM, rO, fbytes, vlane, x0, gx0}};
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            p.s.vx[k] = 0;
            p.s.sgx[k] = T(1);
            p.s.nrx[k] = false;
            p.s.writer[k] = NC * lane + k >= PAIR_HALO && NC * lane + k < WAVE * NC - PAIR_HALO;
            p.gaddr[k] = 0;
            p.gk[k] = 0;
            p.gcol[k] = false;
            p.scol[k] = gx0 + k;
        }
        p.yper = false;   // interior tiles never reach a side
        p.s.y0 = y0;
        p.s.y1 = y1;
        p.ylo = ylo;
        p.yhi = yhi;
        if (down) p.template run<true>();
        else p.template run<false>();
    } else {
        Pair2D<T, NC, NF, HAS_EPS, HAS_MU, true, PER, LIM> p{{a, rU, rE, rM, rO, fbytes, vlane, x0, gx0}};
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int g = gx0 + k;
            // periodic x sides: every column wraps (stage 1 forms the intermediate ghost columns as
            // the step of the columns they image); other sides: columns beyond the two ghost layers
            // feed only halo values that stage 2 never reads
            const bool xper = PER && a.bc[0] == GKS_BC_PERIODIC;
            const int gc = xper ? ((g % a.nx) + a.nx) % a.nx : min(max(g, -2), a.nx + 1);
            bool mirx, nrx;
            const int sx = map_axis(gc, a.nx, a.bc[0], a.bc[1], mirx, nrx);
            p.s.vx[k] = (uint32_t)sx * (uint32_t)sizeof(T);
            p.s.sgx[k] = mirx ? T(-1) : T(1);
            p.s.nrx[k] = nrx;
            p.s.writer[k] = NC * lane + k >= PAIR_HALO && NC * lane + k < WAVE * NC - PAIR_HALO && g >= 0 && g < a.nx;
            p.gcol[k] = !xper && (g == -2 || g == -1 || g == a.nx || g == a.nx + 1);
            p.scol[k] = xper ? sx : g;
            const int src = min(max(sx - x0, 0), WAVE * NC - 1);   // the image's place in the strip
            p.gaddr[k] = (src / NC) * 4;
            p.gk[k] = src % NC;
        }
        p.s.y0 = y0;
        p.s.y1 = y1;
        p.ylo = ylo;
        p.yhi = yhi;
        p.yper = yper;
        if (down) p.template run<true>();
        else p.template run<false>();
    }
}

// The fp32 four-field (PHM) kernel is held to three waves per SIMD: left alone the compiler
// takes 172 VGPRs, two waves fit, and the 4096^2 step takes 183 us; held to 168 it takes 155
// VGPRs and 165 us, with fewer scalar spills.
template <typename T, int NF, bool HAS_EPS, bool HAS_MU, bool LIM>
__global__ __launch_bounds__(STEP2D_BLOCK, (sizeof(T) == 4 && NF == 4) ? 3 : 1) void cart2d_step_kernel(Cart2DArgs<T> a)
{
    constexpr int NC = cols_per_lane<T>();
    const int lane = threadIdx.x & (WAVE - 1);
    // the wave's index inside the block is uniform: say so, so that everything derived from it
    // (tile, batch item, buffer resources, row offsets) lives in scalar registers
    // workgroup g runs on XCD g mod 8 and works on that XCD's band of tile rows, in order
    const int band = blockIdx.x % NBANDS;
    const int wave = (blockIdx.x / NBANDS) * (STEP2D_BLOCK / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int tl = wave / a.ntx;   // tile row within the band
    if (tl >= a.nty) return;
    const int tx = wave - tl * a.ntx;
    const int t = band * a.nty + tl;
    const int b = __builtin_amdgcn_readfirstlane(a.tiles[4 * t]);
    if (b < 0) return;   // padding of a shorter band
    const int y0 = __builtin_amdgcn_readfirstlane(a.tiles[4 * t + 1]);
    const int y1 = __builtin_amdgcn_readfirstlane(a.tiles[4 * t + 2]);   // rows [y0, y1) are written
    const bool down = __builtin_amdgcn_readfirstlane(a.tiles[4 * t + 3]) != 0;

    const int64_t ncell = (int64_t)a.nx * a.ny;
    const uint32_t fbytes = (uint32_t)(ncell * (int64_t)sizeof(T));
    const Rsrc rU = make_rsrc(a.U + (int64_t)b * NF * ncell, (uint64_t)NF * fbytes);
    const Rsrc rO = make_rsrc(a.Unew + (int64_t)b * NF * ncell, (uint64_t)NF * fbytes);
    const Rsrc rE = make_rsrc(HAS_EPS ? a.epsinv + (int64_t)b * ncell : a.U, fbytes);
    const Rsrc rM = make_rsrc(HAS_MU ? a.muinv + (int64_t)b * ncell : a.U, fbytes);

    const int x0 = tx * out_cols<T>() - HALO;
    const int gx0 = x0 + NC * lane;
    const uint32_t vlane = (uint32_t)(NC * lane) * (uint32_t)sizeof(T);

    const bool interior = x0 >= 0 && x0 + WAVE * NC - 1 <= a.nx - 1 && y0 - 2 >= 0 && y1 + 1 <= a.ny - 1;
    if (interior) {
        Strip2D<T, NC, NF, HAS_EPS, HAS_MU, false, LIM> s{a, rU, rE, rM, rO, fbytes, vlane, x0, gx0};
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            s.vx[k] = 0;
            s.sgx[k] = T(1);
            s.nrx[k] = false;
            s.writer[k] = NC * lane + k >= HALO && NC * lane + k < WAVE * NC - HALO;
        }
        s.y0 = y0;
        s.y1 = y1;
        s.run(down);
    } else {
        Strip2D<T, NC, NF, HAS_EPS, HAS_MU, true, LIM> s{a, rU, rE, rM, rO, fbytes, vlane, x0, gx0};
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            bool mirx, nrx;
            const int sx = map_axis(gx0 + k, a.nx, a.bc[0], a.bc[1], mirx, nrx);
            s.vx[k] = (uint32_t)sx * (uint32_t)sizeof(T);
            s.sgx[k] = mirx ? T(-1) : T(1);   // x mirror: Ez and Hx odd, Hy and psi even
            s.nrx[k] = nrx;
            s.writer[k] = NC * lane + k >= HALO && NC * lane + k < WAVE * NC - HALO && gx0 + k < a.nx;
        }
        s.y0 = y0;
        s.y1 = y1;
        s.run(down);
    }
}

template <typename T>
int launch_cart2d_step(const Cart2DArgs<T> &a, void *stream)
{
    static_assert(STEP2D_BLOCK / WAVE == CART2D_WAVES_PER_BLOCK, "the tile table pads bands to whole workgroups");
    const int waves = a.ntx * a.nty;   // per band: a whole number of workgroups (padded by the host)
    const int wpb = STEP2D_BLOCK / WAVE;
    dim3 grid(NBANDS * ((waves + wpb - 1) / wpb)), block(STEP2D_BLOCK);
    hipStream_t s = (hipStream_t)stream;
    if (a.nfields == 4) {   // TM with psi (never limited: the host refuses that combination)
        if (a.limiter) return (int)hipErrorInvalidValue;
        if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 4, true, true, false>), grid, block, 0, s, a);
        else if (a.epsinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 4, true, false, false>), grid, block, 0, s, a);
        else if (a.muinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 4, false, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((cart2d_step_kernel<T, 4, false, false, false>), grid, block, 0, s, a);
        return (int)hipGetLastError();
    }
    if (a.nfields != 3) return (int)hipErrorInvalidValue;
    if (a.limiter) {
        if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 3, true, true, true>), grid, block, 0, s, a);
        else if (a.epsinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 3, true, false, true>), grid, block, 0, s, a);
        else if (a.muinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 3, false, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((cart2d_step_kernel<T, 3, false, false, true>), grid, block, 0, s, a);
        return (int)hipGetLastError();
    }
    if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 3, true, true, false>), grid, block, 0, s, a);
    else if (a.epsinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 3, true, false, false>), grid, block, 0, s, a);
    else if (a.muinv) hipLaunchKernelGGL((cart2d_step_kernel<T, 3, false, true, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((cart2d_step_kernel<T, 3, false, false, false>), grid, block, 0, s, a);
    return (int)hipGetLastError();
}

template int launch_cart2d_step<float>(const Cart2DArgs<float> &, void *);
template int launch_cart2d_step<double>(const Cart2DArgs<double> &, void *);

template <typename T, bool PER, bool LIM>
static void launch_pair(const Cart2DArgs<T> &a, dim3 grid, dim3 block, hipStream_t s)
{
    if constexpr (!LIM) {
        if (a.nfields == 4) {
            if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart2d_pair_kernel<T, 4, true, true, PER, false>), grid, block, 0, s, a);
            else if (a.epsinv) hipLaunchKernelGGL((cart2d_pair_kernel<T, 4, true, false, PER, false>), grid, block, 0, s, a);
            else if (a.muinv) hipLaunchKernelGGL((cart2d_pair_kernel<T, 4, false, true, PER, false>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((cart2d_pair_kernel<T, 4, false, false, PER, false>), grid, block, 0, s, a);
            return;
        }
    }
    if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart2d_pair_kernel<T, 3, true, true, PER, LIM>), grid, block, 0, s, a);
    else if (a.epsinv) hipLaunchKernelGGL((cart2d_pair_kernel<T, 3, true, false, PER, LIM>), grid, block, 0, s, a);
    else if (a.muinv) hipLaunchKernelGGL((cart2d_pair_kernel<T, 3, false, true, PER, LIM>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((cart2d_pair_kernel<T, 3, false, false, PER, LIM>), grid, block, 0, s, a);
}

template <typename T>
int launch_cart2d_pair(const Cart2DArgs<T> &a, void *stream)
{
    if (a.nfields != 3 && a.nfields != 4) return (int)hipErrorInvalidValue;
    if (a.limiter && a.nfields != 3) return (int)hipErrorInvalidValue;   // the host refuses PHM + limiter
    const int waves = a.ntx * a.nty;
    const int wpb = STEP2D_BLOCK / WAVE;
    dim3 grid(NBANDS * ((waves + wpb - 1) / wpb)), block(STEP2D_BLOCK);
    hipStream_t s = (hipStream_t)stream;
    bool per = false;
    for (int i = 0; i < 4; ++i) per = per || a.bc[i] == GKS_BC_PERIODIC;
    if (a.limiter) {
        if (per) launch_pair<T, true, true>(a, grid, block, s);
        else launch_pair<T, false, true>(a, grid, block, s);
    } else {
        if (per) launch_pair<T, true, false>(a, grid, block, s);
        else launch_pair<T, false, false>(a, grid, block, s);
    }
    return (int)hipGetLastError();
}

template int launch_cart2d_pair<float>(const Cart2DArgs<float> &, void *);
template int launch_cart2d_pair<double>(const Cart2DArgs<double> &, void *);

int cart2d_tile_x(int precision) { return precision == GKS_FP64 ? out_cols<double>() : out_cols<float>(); }
int cart2d_pair_tile_x(int precision) { return precision == GKS_FP64 ? pair_out_cols<double>() : pair_out_cols<float>(); }

}  // namespace gks
