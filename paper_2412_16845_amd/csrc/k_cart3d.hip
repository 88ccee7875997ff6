// Fused GKS step on a 3D Cartesian grid, six fields (Ex, Ey, Ez, Hx, Hy, Hz), or the eight of
// the perfectly hyperbolic Maxwell system with its divergence-cleaning potentials (Ex .. Hz,
// phi, psi; Sec. 2.1).  The field count NF is a template parameter; everything below applies to
// both.
//
// A workgroup owns a tile of 64 columns (x) by ROWS rows (y) and marches it through a range of
// z planes.  Wave w holds row w of the tile, one column per lane; the two outermost columns and
// rows on each side are halo, the rest are written.  Per plane q the workgroup:
//   1. issues the loads of plane q+2 (each lane: six fields and the materials of its cell), so
//      one plane of loads is in flight while plane q is processed;
//   2. shares the fields of plane q through LDS and forms the Green-Gauss (central) differences
//      of plane q: along x from the neighbouring lanes (DPP row shifts), along y from the rows
//      above and below (LDS), along z from the planes q-1 and q+1 it holds in registers;
//   3. shares the differences and evaluates, as sparse linear forms of the face inputs (the
//      closed-form moments of Sec. 3.1 folded into coefficients on the host), the flux of the
//      face above each cell (y, with the upper row's data from LDS), right of it (x, with the
//      next lane's data by DPP) and below it in z (from the previous plane kept in registers);
//   4. shares the y fluxes and finishes the flux divergence of each cell of plane q-1, summed in
//      double precision (the FP32 face fluxes are widened first), adds it to the old value in
//      double precision and stores the result rounded once to the storage type.
// Each face is evaluated once; each field value is loaded once per workgroup.  In fp32 the
// fields are double-buffered by plane parity (the next plane's fields are written before the
// last barrier of the current one), which leaves two barriers per plane; in fp64 they are
// single-buffered and shared at the start of the plane (three barriers).  The differences and
// materials and the y fluxes are single-buffered, each slot's reads ordered before the next
// plane's write by a barrier.
// Boundaries follow the 2D kernel: ghost cells read the wrapped (periodic), mirrored (PEC:
// tangential E, normal H and phi odd) or clamped (non-reflecting) cell; the ghost side of a
// non-reflecting boundary face carries no distribution (zero state and slopes).
#include "gks_device.h"

namespace gks {

namespace {

// Rows (waves) per workgroup: the LDS tile below must fit the compute unit's 160 KiB.
template <typename T, int NF> constexpr int rows3d()
{
    return NF == 6 ? (sizeof(T) == 4 ? 16 : 8) : (sizeof(T) == 4 ? 12 : 7);
}
constexpr int OUT_X3 = WAVE - 4;

// Coefficient chunk of the face operators (apply_op): 5 for the fp64 six-field kernel (384^3:
// 4131 us with 12; 3, 4, 5, 6 and 8 give 4045, 3714, 3618, 3789 and 4328 us), 12 for the others,
// which are fastest with it.
template <typename T, int NF> constexpr int CH3() { return (sizeof(T) == 8 && NF == 6) ? 5 : 12; }

// Fields that change sign under a PEC mirror across an x-, y- or z-wall (tangential E, normal H,
// and phi, which follows div E; psi is even).
constexpr uint32_t ODD_X = (1u << 1) | (1u << 2) | (1u << 3) | (1u << 6);
constexpr uint32_t ODD_Y = (1u << 0) | (1u << 2) | (1u << 4) | (1u << 6);
constexpr uint32_t ODD_Z = (1u << 0) | (1u << 1) | (1u << 5) | (1u << 6);

// Face operators of the two field sets.
template <int NF> struct Fields3D;
// PXF.. and OpF: the operators with the 1/mu part folded into K0, stored after the three plain
// ones (six fields only; the eight-field kernel always applies KH).
template <> struct Fields3D<6> {
    using PX = PatEMx;
    using PY = PatEMy;
    using PZ = PatEMz;
    using PXF = PatEMxF;
    using PYF = PatEMyF;
    using PZF = PatEMzF;
    template <typename T> using Op = FaceOpEM<T>;
    template <typename T> using OpF = FaceOpEMF<T>;
};
template <> struct Fields3D<8> {
    using PX = PatEPx;
    using PY = PatEPy;
    using PZ = PatEPz;
    using PXF = PatEPx;
    using PYF = PatEPy;
    using PZF = PatEPz;
    template <typename T> using Op = FaceOpEP<T>;
    template <typename T> using OpF = FaceOpEP<T>;
};

template <typename T, int NF>
struct Plane3 {
    T u[NF];
    T mE, mH;
};

template <typename T, int NF>
struct Lds3 {
    static constexpr int R = rows3d<T, NF>();
    // fields of the current plane: double-buffered by plane parity in fp32 (one barrier per plane
    // fewer); single in fp64, whose registers cannot also hold the next plane's fields that long
    static constexpr int NU = sizeof(T) == 4 ? 2 : 1;
    T u[NU][NF][R][WAVE];
    T g[3 * NF + 2][R][WAVE];   // differences [x(NF) y(NF) z(NF)] and mE, mH
    T p[NF][R][WAVE];           // flux of the face above each cell (y)
};
static_assert(sizeof(Lds3<float, 6>) <= 160 * 1024 && sizeof(Lds3<double, 6>) <= 160 * 1024 &&
                  sizeof(Lds3<float, 8>) <= 160 * 1024 && sizeof(Lds3<double, 8>) <= 160 * 1024,
              "LDS tile above 160 KiB");

__device__ __forceinline__ bool side_nr(int g, int n, int bclo, int bchi)
{
    return (g < 0 && bclo == GKS_BC_NONREFLECT) || (g >= n && bchi == GKS_BC_NONREFLECT);
}

// Limited differences along axis K (times twice the cell width) from the fields of the cell (c)
// and of its neighbours above (up) and below (dn): minmod of the one-sided differences of the
// variables that travel along K (E_a +/- H_b, E_b +/- H_a, a and b the other axes) and of the
// normal components E_K, H_K.
template <int K, typename T>
__device__ __forceinline__ void limit_axis(const T (&up)[6], const T (&c)[6], const T (&dn)[6], T *out)
{
    constexpr int A = (K + 1) % 3, B = (K + 2) % 3;
    limit_pair(up[A] - c[A], up[3 + B] - c[3 + B], c[A] - dn[A], c[3 + B] - dn[3 + B], out[A], out[3 + B]);
    limit_pair(up[B] - c[B], up[3 + A] - c[3 + A], c[B] - dn[B], c[3 + A] - dn[3 + A], out[B], out[3 + A]);
    out[K] = T(2) * minmod(up[K] - c[K], c[K] - dn[K]);
    out[3 + K] = T(2) * minmod(up[3 + K] - c[3 + K], c[3 + K] - dn[3 + K]);
}

template <typename T, int NF, bool HAS_EPS, bool HAS_MU, bool BXY, bool LIM>
struct March3D {
    static_assert(!LIM || NF == 6, "the limited step is built for the six Maxwell fields only");
    static constexpr int R = rows3d<T, NF>();
    using OpT = typename Fields3D<NF>::template Op<T>;
    using Plane = Plane3<T, NF>;
    // vacuum 1/mu with the six fields: the folded operators, which save the KH products (about
    // ten multiply-adds per face)
    static constexpr bool HM = HAS_MU || NF != 6;
    using FS = Fields3D<NF>;
    using PX_ = typename std::conditional<HM, typename FS::PX, typename FS::PXF>::type;
    using PY_ = typename std::conditional<HM, typename FS::PY, typename FS::PYF>::type;
    using PZ_ = typename std::conditional<HM, typename FS::PZ, typename FS::PZF>::type;
    using OpU = typename std::conditional<HM, typename FS::template Op<T>, typename FS::template OpF<T>>::type;
    __device__ __forceinline__ const OpU *opsets() const
    {
        return HM ? (const OpU *)a.ops : (const OpU *)((const char *)a.ops + 3 * sizeof(OpT));
    }
    const Cart3DArgs<T> &a;
    Lds3<T, NF> &s;
    Rsrc rU, rE, rM, rO;
    uint32_t fbytes, pbytes;   // bytes per field, per plane
    uint32_t vcol;             // byte offset of the cell this lane reads, inside a plane
    uint32_t sgn;              // BXY: fields negated by the x/y mirror of this lane's cell
    bool nr_c, nr_x, nr_y;     // BXY: non-reflecting ghost at (x, y), (x+1, y), (x, y+1)
    bool writer;
    int lane, row, rowp, rowm, z0, z1;
    bool need_g, need_yf, need_all;   // wave roles by row

    __device__ __forceinline__ void load(int gz, Plane &p) const
    {
        bool mz, nrz;
        const int sz = map_axis(gz, a.nz, a.bc[4], a.bc[5], mz, nrz);
        const uint32_t so = (uint32_t)sz * pbytes;
#pragma unroll
        for (int f = 0; f < NF; ++f) p.u[f] = buf_load<T>(rU, vcol, so + f * fbytes);
        p.mE = HAS_EPS ? buf_load<T>(rE, vcol, so) : T(1);
        p.mH = HAS_MU ? buf_load<T>(rM, vcol, so) : T(1);
        if constexpr (BXY) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
                if ((sgn >> f) & 1u) p.u[f] = -p.u[f];
        }
        if (mz) {   // uniform: a mirrored ghost plane
#pragma unroll
            for (int f = 0; f < NF; ++f)
                if ((ODD_Z >> f) & 1u) p.u[f] = -p.u[f];
        }
    }

    __device__ __forceinline__ bool plane_nr(int gz) const { return side_nr(gz, a.nz, a.bc[4], a.bc[5]); }

    // The differences of plane q-1 for the z face below plane q: in fp32 they are read back
    // from the LDS slot this wave wrote them to in the previous step, which keeps them out of
    // the 128 registers of the 16-wave workgroup (with them in registers the double-precision
    // accumulator spilled: 384^3, 1528 -> 1378 us); so does the fp64 eight-field kernel, whose
    // registers spill (20.9 -> 17.0 ms); the fp64 six-field kernel keeps them in registers
    // (3604 us against 3770 us with the LDS reads).
    static constexpr bool GP_LDS = sizeof(T) == 4 || NF == 8;
    // fp64 with eight fields: values that would live across a barrier (the row above, this
    // plane's differences, the x and y fluxes) are read again from LDS or folded first, which
    // frees registers in a kernel that spills (384^3: 17.0 -> 15.9 ms; the six-field fp64
    // kernel, which does not spill, is slower with it: 3.45 -> 3.75 ms)
    static constexpr bool LEAN = sizeof(T) == 8 && NF == 8;
    // this plane's differences for the x and y faces, which come after the barrier that
    // publishes them: LEAN reads them back from this lane's LDS slot
    __device__ __forceinline__ T gown(const T (&G)[3 * NF], int k) const { return LEAN ? s.g[k][row][lane] : G[k]; }
    __device__ __forceinline__ T gprev(const T (&Gp)[3 * NF], int k) const { return GP_LDS ? s.g[k][row][lane] : Gp[k]; }

    // One march step with central plane q: A = q-1, B = q, C = q+1 (loaded), D receives q+2.
    // Gp / G: differences of planes q-1 / q.  acc: on entry the x and y divergence of plane
    // q-1 minus the flux of the z face below it, in double precision; on exit the same for
    // plane q.
    __device__ __forceinline__ void step(int q, Plane &A, Plane &B, Plane &C, Plane &D, T (&Gp)[3 * NF],
                                         T (&G)[3 * NF], double (&acc)[NF]) const
    {
        const OpU *ops = opsets();
        // plane q+2 (beyond the range: re-read the last halo plane, already cached, so that the
        // load stays unconditional)
        load(min(q + 2, z1 + 1), D);
        constexpr int NU = Lds3<T, NF>::NU;
        if constexpr (NU == 1) {
#pragma unroll
            for (int f = 0; f < NF; ++f) s.u[0][f][row][lane] = B.u[f];
            __syncthreads();
        }
        // (double-buffered: the fields of plane q were shared at the end of the previous step)
        const int cu = NU == 2 ? (q & 1) : 0;
        T uy[NF];   // fields of the row above (plane q)
        if (need_g) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                uy[f] = s.u[cu][f][rowp][lane];
                G[f] = from_right(B.u[f]) - from_left(B.u[f]);
                G[NF + f] = uy[f] - s.u[cu][f][rowm][lane];
                G[2 * NF + f] = C.u[f] - A.u[f];
            }
            if constexpr (LIM) {
                T xr[6], xl[6], ym[6];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    xr[f] = from_right(B.u[f]);
                    xl[f] = from_left(B.u[f]);
                    ym[f] = s.u[cu][f][rowm][lane];
                }
                limit_axis<0>(xr, B.u, xl, G);
                limit_axis<1>(uy, B.u, ym, G + NF);
                limit_axis<2>(C.u, B.u, A.u, G + 2 * NF);
            }
            // every face that reads the differences of a non-reflecting ghost zeroes them:
            // zero them at the source (the lane itself), so that the values neighbours receive
            // by DPP or LDS need no select on the receiving side
            if constexpr (BXY) {
#pragma unroll
                for (int k = 0; k < 3 * NF; ++k) G[k] = nr_c ? T(0) : G[k];
            }
        }
        // face below plane q, then the update of plane q-1, whose divergence it completes
        if (q >= z0 && need_all) {
            // inputs [UL UR dzL dxL dyL dzR dxR dyR] x fields, L plane q-1
            const bool zlu = plane_nr(q - 1), zru = plane_nr(q);   // uniform: a non-reflecting z side
            const auto opz = scalar_ptr_after(ops + 2, G[3 * NF - 1]);
            T Z[NF];
            // interior planes of interior tiles (the common case): no side is zeroed, so the
            // operator reads the registers directly (384^3 fp64: 4590 -> 4130 us, fp32: 1328 -> 1319
            // us; the eight-field fp64 kernel 15.9 -> 15.5 ms)
            if (!BXY && !zlu && !zru) {
                T w[8 * NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    w[f] = A.u[f];
                    w[NF + f] = B.u[f];
                    w[2 * NF + f] = gprev(Gp, 2 * NF + f);
                    w[3 * NF + f] = gprev(Gp, f);
                    w[4 * NF + f] = gprev(Gp, NF + f);
                    w[5 * NF + f] = G[2 * NF + f];
                    w[6 * NF + f] = G[f];
                    w[7 * NF + f] = G[NF + f];
                }
                apply_op<PZ_, CH3<T, NF>(), HM>(w, A.mE + B.mE, A.mH + B.mH, opz, Z);
            } else {
                const bool zl = zlu || (BXY && nr_c), zr = zru || (BXY && nr_c);
                T w[8 * NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    w[f] = zl ? T(0) : A.u[f];
                    w[NF + f] = zr ? T(0) : B.u[f];
                    w[2 * NF + f] = zl ? T(0) : gprev(Gp, 2 * NF + f);
                    w[3 * NF + f] = zl ? T(0) : gprev(Gp, f);
                    w[4 * NF + f] = zl ? T(0) : gprev(Gp, NF + f);
                    w[5 * NF + f] = zr ? T(0) : G[2 * NF + f];
                    w[6 * NF + f] = zr ? T(0) : G[f];
                    w[7 * NF + f] = zr ? T(0) : G[NF + f];
                }
                apply_op<PZ_, CH3<T, NF>(), HM>(w, A.mE + B.mE, A.mH + B.mH, opz, Z);
            }
            if (q - 1 >= z0) {
                const uint32_t so = (uint32_t)(q - 1) * pbytes;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    // the divergence and its addition to the old value in double precision,
                    // rounded once to the storage type on store
                    const double div = acc[f] + (double)Z[f];
                    // 1/eps scales E, 1/mu scales H; the potentials carry no material factor
                    const double m = (f < 3) ? (double)A.mE : (f < 6) ? (double)A.mH : 1.0;
                    const T nv = (T)fma(-m, div, (double)A.u[f]);
                    if (writer) buf_store(nv, rO, vcol, so + f * fbytes);
                }
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f] = -(double)Z[f];
        }
        if (need_g) {
#pragma unroll
            for (int k = 0; k < 3 * NF; ++k) s.g[k][row][lane] = G[k];
            s.g[3 * NF][row][lane] = B.mE;
            s.g[3 * NF + 1][row][lane] = B.mH;
        }
        __syncthreads();
        const bool outp = q >= z0 && q < z1;
        T px[NF], py[NF];
        // this cell's fields as a face side: zero on a non-reflecting ghost (the DPP moves
        // below then read them unconditionally: a move under a partial lane mask would read the
        // masked lanes as zero)
        T su[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) su[f] = (BXY && nr_c) ? T(0) : B.u[f];
        if (outp && need_yf) {
            // face above: inputs [UL UR dyL dxL dzL dyR dxR dzR] x fields, L this row, R the row above
            const bool zr = BXY && nr_y;
            const auto opy = scalar_ptr(ops + 1);
            T w[8 * NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                w[f] = su[f];
                w[NF + f] = zr ? T(0) : (LEAN ? s.u[cu][f][rowp][lane] : uy[f]);
                w[2 * NF + f] = gown(G, NF + f);
                w[3 * NF + f] = gown(G, f);
                w[4 * NF + f] = gown(G, 2 * NF + f);
                w[5 * NF + f] = s.g[NF + f][rowp][lane];
                w[6 * NF + f] = s.g[f][rowp][lane];
                w[7 * NF + f] = s.g[2 * NF + f][rowp][lane];
            }
            apply_op<PY_, CH3<T, NF>(), HM>(w, B.mE + s.g[3 * NF][rowp][lane], B.mH + s.g[3 * NF + 1][rowp][lane],
                                            opy, py);
#pragma unroll
            for (int f = 0; f < NF; ++f) s.p[f][row][lane] = py[f];
        }
        if (outp && need_all) {
            // face to the right: inputs [UL UR dxL dyL dzL dxR dyR dzR] x fields, R the next lane
            const auto opx = scalar_ptr_after(ops, py[NF - 1]);
            T w[8 * NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                w[f] = su[f];
                w[NF + f] = from_right(su[f]);
                w[2 * NF + f] = gown(G, f);
                w[3 * NF + f] = gown(G, NF + f);
                w[4 * NF + f] = gown(G, 2 * NF + f);
                w[5 * NF + f] = from_right(gown(G, f));
                w[6 * NF + f] = from_right(gown(G, NF + f));
                w[7 * NF + f] = from_right(gown(G, 2 * NF + f));
            }
            apply_op<PX_, CH3<T, NF>(), HM>(w, B.mE + from_right(B.mE), HM ? B.mH + from_right(B.mH) : T(2), opx, px);
        }
        // LEAN: the x part of the divergence now, so that px need not live across the barrier
        // (the y fluxes are read back from LDS after it): the same sums in the same order
        double tx[NF];
        if (LEAN && outp && need_all) {
#pragma unroll
            for (int f = 0; f < NF; ++f) tx[f] = (double)px[f] - (double)from_left(px[f]);
        }
        if constexpr (NU == 2) {
            // share the fields of plane q+1 in the other buffer (its last readers, in the
            // previous step, are all past this step's first barrier); the barrier below
            // publishes them with the y fluxes
#pragma unroll
            for (int f = 0; f < NF; ++f) s.u[cu ^ 1][f][row][lane] = C.u[f];
        }
        __syncthreads();
        if (outp && need_all) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double dx = LEAN ? tx[f] : (double)px[f] - (double)from_left(px[f]);
                const T pyf = LEAN ? s.p[f][row][lane] : py[f];
                acc[f] += dx + ((double)pyf - (double)s.p[f][rowm][lane]);
            }
        }
    }

    __device__ __forceinline__ void run() const
    {
        Plane P0, P1, P2, P3;
        T G0[3 * NF], G1[3 * NF];
        double acc[NF];   // flux divergence of the plane being finished, in double precision
#pragma unroll
        for (int k = 0; k < 3 * NF; ++k) G0[k] = G1[k] = T(0);
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = 0.0;
        const int qs = z0 - 1;
        load(qs - 1, P0);
        load(qs, P1);
        load(qs + 1, P2);
        if constexpr (Lds3<T, NF>::NU == 2) {
#pragma unroll
            for (int f = 0; f < NF; ++f) s.u[qs & 1][f][row][lane] = P1.u[f];
            __syncthreads();
        }
        const int n = z1 - z0 + 2;   // central planes z0-1 .. z1
        if constexpr (GP_LDS) {
            // one register set of differences: the previous plane's come from LDS
            for (int i = 0; i < n; i += 4) {
                step(qs + i, P0, P1, P2, P3, G0, G0, acc);
                if (i + 1 >= n) break;
                step(qs + i + 1, P1, P2, P3, P0, G0, G0, acc);
                if (i + 2 >= n) break;
                step(qs + i + 2, P2, P3, P0, P1, G0, G0, acc);
                if (i + 3 >= n) break;
                step(qs + i + 3, P3, P0, P1, P2, G0, G0, acc);
            }
        } else {
            for (int i = 0; i < n; i += 4) {
                step(qs + i, P0, P1, P2, P3, G1, G0, acc);
                if (i + 1 >= n) break;
                step(qs + i + 1, P1, P2, P3, P0, G0, G1, acc);
                if (i + 2 >= n) break;
                step(qs + i + 2, P2, P3, P0, P1, G1, G0, acc);
                if (i + 3 >= n) break;
                step(qs + i + 3, P3, P0, P1, P2, G0, G1, acc);
            }
        }
    }
};

template <typename T, int NF, bool HAS_EPS, bool HAS_MU, bool LIM>
__global__ __launch_bounds__((WAVE * rows3d<T, NF>())) void cart3d_step_kernel(Cart3DArgs<T> a)
{
    constexpr int R = rows3d<T, NF>();
    __shared__ Lds3<T, NF> lds;
    const int lane = threadIdx.x & (WAVE - 1);
    const int row = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    int t = xcd_logical_block();
    const int tx = t % a.ntx;
    t /= a.ntx;
    const int ty = t % a.nty;
    t /= a.nty;
    const int tz = t % a.ntz;
    const int b = t / a.ntz;

    const int64_t ncell = (int64_t)a.nx * a.ny * a.nz;
    const uint32_t fbytes = (uint32_t)(ncell * (int64_t)sizeof(T));
    const uint32_t pbytes = (uint32_t)((int64_t)a.nx * a.ny * (int64_t)sizeof(T));
    const Rsrc rU = make_rsrc(a.U + (int64_t)b * NF * ncell, (uint64_t)NF * fbytes);
    const Rsrc rO = make_rsrc(a.Unew + (int64_t)b * NF * ncell, (uint64_t)NF * fbytes);
    const Rsrc rE = make_rsrc(a.epsinv ? a.epsinv + (int64_t)b * ncell : a.U, fbytes);
    const Rsrc rM = make_rsrc(a.muinv ? a.muinv + (int64_t)b * ncell : a.U, fbytes);

    const int x0 = tx * OUT_X3 - 2, y0 = ty * (R - 4) - 2;
    const int x = x0 + lane, y = y0 + row;
    const int z0 = tz * a.tile_z, z1 = min(z0 + a.tile_z, a.nz);
    bool mx, nrx, my, nry, mx1, nrx1, my1, nry1;
    const int sx = map_axis(x, a.nx, a.bc[0], a.bc[1], mx, nrx);
    const int sy = map_axis(y, a.ny, a.bc[2], a.bc[3], my, nry);
    map_axis(x + 1, a.nx, a.bc[0], a.bc[1], mx1, nrx1);
    map_axis(y + 1, a.ny, a.bc[2], a.bc[3], my1, nry1);
    const bool bxy = x0 < 0 || x0 + WAVE > a.nx || y0 < 0 || y0 + R > a.ny;   // uniform

    auto go = [&](auto bnd) {
        constexpr bool BXY = decltype(bnd)::value;
        March3D<T, NF, HAS_EPS, HAS_MU, BXY, LIM> m{a, lds, rU, rE, rM, rO, fbytes, pbytes};
        m.vcol = (uint32_t)((int64_t)sy * a.nx + sx) * (uint32_t)sizeof(T);
        m.sgn = (mx ? ODD_X : 0u) ^ (my ? ODD_Y : 0u);
        m.nr_c = nrx || nry;
        m.nr_x = nrx1 || nry;
        m.nr_y = nrx || nry1;
        m.writer = lane >= 2 && lane < WAVE - 2 && row >= 2 && row < R - 2 && x < a.nx && y < a.ny;
        m.lane = lane;
        m.row = row;
        m.rowp = min(row + 1, R - 1);
        m.rowm = max(row - 1, 0);
        m.z0 = z0;
        m.z1 = z1;
        m.need_g = row >= 1 && row <= R - 2;
        m.need_yf = row >= 1 && row <= R - 3;
        m.need_all = row >= 2 && row <= R - 3;
        m.run();
    };
    if (bxy) go(std::integral_constant<bool, true>{});
    else go(std::integral_constant<bool, false>{});
}

}  // namespace

template <typename T>
int launch_cart3d_step(const Cart3DArgs<T> &a, void *stream)
{
    const unsigned blocks = (unsigned)(a.ntx * a.nty * a.ntz * a.batch);
    dim3 grid(blocks);
    hipStream_t s = (hipStream_t)stream;
    if (a.nfields == 8) {   // with the PHM potentials (never limited: the host refuses that)
        if (a.limiter) return (int)hipErrorInvalidValue;
        dim3 block(WAVE * rows3d<T, 8>());
        if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 8, true, true, false>), grid, block, 0, s, a);
        else if (a.epsinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 8, true, false, false>), grid, block, 0, s, a);
        else if (a.muinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 8, false, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((cart3d_step_kernel<T, 8, false, false, false>), grid, block, 0, s, a);
        return (int)hipGetLastError();
    }
    if (a.nfields != 6) return (int)hipErrorInvalidValue;
    dim3 block(WAVE * rows3d<T, 6>());
    if (a.limiter) {
        if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 6, true, true, true>), grid, block, 0, s, a);
        else if (a.epsinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 6, true, false, true>), grid, block, 0, s, a);
        else if (a.muinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 6, false, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((cart3d_step_kernel<T, 6, false, false, true>), grid, block, 0, s, a);
        return (int)hipGetLastError();
    }
    if (a.epsinv && a.muinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 6, true, true, false>), grid, block, 0, s, a);
    else if (a.epsinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 6, true, false, false>), grid, block, 0, s, a);
    else if (a.muinv) hipLaunchKernelGGL((cart3d_step_kernel<T, 6, false, true, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((cart3d_step_kernel<T, 6, false, false, false>), grid, block, 0, s, a);
    return (int)hipGetLastError();
}

template int launch_cart3d_step<float>(const Cart3DArgs<float> &, void *);
template int launch_cart3d_step<double>(const Cart3DArgs<double> &, void *);

int cart3d_tile_x(int) { return OUT_X3; }
int cart3d_tile_y(int precision, int nfields)
{
    if (nfields == 8) return precision == GKS_FP64 ? rows3d<double, 8>() - 4 : rows3d<float, 8>() - 4;
    return precision == GKS_FP64 ? rows3d<double, 6>() - 4 : rows3d<float, 6>() - 4;
}

}  // namespace gks
