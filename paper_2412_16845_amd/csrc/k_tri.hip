// GKS step on a triangle mesh, TM fields (Ez, Hx, Hy), or the TM fields of the perfectly
// hyperbolic Maxwell system with the divergence-cleaning potential psi (Ez, Hx, Hy, psi; Sec.
// 2.1).  The field count NF is a template parameter; psi is a scalar in the face frame and an
// even PEC ghost.
//
// Two kernels, one thread per cell (cells in Hilbert order, so the neighbours a thread gathers
// are mostly cached; consecutive blocks are renumbered onto one XCD, so that a block's
// neighbouring blocks share its L2):
//   1. cell gradients grad U_i = sum_s W_s (U_s - U_i) over the three faces, with host weights:
//      Green-Gauss (Sec. 3.1, W_s = n_s |l_s| / (2 |Omega_i|)) or the least-squares fit; the
//      ghost of a non-reflecting face equals the cell itself, the ghost of a PEC face is its
//      mirror image (Ez and the normal H odd);
//   2. the cell's three faces and its update: each face is reconstructed at its midpoint from
//      both sides, rotated into its frame (printed rotation of Sec. 3.1: local axes n and
//      (-n_y, n_x)), evaluated as a sparse linear form of the face-frame states and slopes (the
//      closed-form flux folded into coefficients on the host; both states taken relative to the
//      cell's own, which leaves the sum of the three fluxes unchanged), rotated back, and the
//      cell's divergence is summed and added to its old value in double precision, rounded once
//      on store.
// A face is evaluated by both of its cells, each from its own side: no face fluxes are stored
// and no atomics are needed.  Boundary faces: non-reflecting (the ghost side carries no
// distribution) or PEC (face-frame mirror of the state, the normal slope mirrored with the
// opposite sign).
#include <type_traits>

#include "gks_device.h"

namespace gks {

namespace {

// Threads per block: 256, except 128 for the fp64 PHM kernels (4.06M cells: 509.3 -> 496.6 us;
// 64 and 512 measured too, and 256 is the fastest for the other instances).
template <typename T, int NF> constexpr int tri_block() { return (sizeof(T) == 8 && NF == 4) ? 128 : 256; }

// The gradient scratch holds one record of 2 NF values per cell, [d/dx (fields), d/dy
// (fields)], so that the gradients of a gathered neighbour come from one or two cache lines.
template <typename T> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };

template <typename T, int NF>
__device__ __forceinline__ void load_grad(const T *G, int64_t c, T (&gx)[NF], T (&gy)[NF])
{
    using V = typename Pair<T>::type;
    const V *p = reinterpret_cast<const V *>(G + c * 2 * NF);
    T r[2 * NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        const V v = p[q];
        r[2 * q] = v.x;
        r[2 * q + 1] = v.y;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        gx[f] = r[f];
        gy[f] = r[NF + f];
    }
}

// Geometry vector p of cell c (x, y) with one load, and the |l_k| / |Omega| of slot k.
template <typename T>
__device__ __forceinline__ void geo_vec(const T *geo, int p, int64_t nc, int64_t c, T &x, T &y)
{
    using V = typename Pair<T>::type;
    const V v = reinterpret_cast<const V *>(geo)[(int64_t)p * nc + c];
    x = v.x;
    y = v.y;
}
template <typename T>
__device__ __forceinline__ T geo_lw(const T *geo, int k, int64_t nc, int64_t c)
{
    return geo[2 * (int64_t)TRI_GEO_PAIRS * nc + (int64_t)k * nc + c];
}

template <typename T, int NF>
__device__ __forceinline__ void store_grad(T *G, int64_t c, const T (&gx)[NF], const T (&gy)[NF])
{
    using V = typename Pair<T>::type;
    V *p = reinterpret_cast<V *>(G + c * 2 * NF);
    T r[2 * NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        r[f] = gx[f];
        r[NF + f] = gy[f];
    }
#pragma unroll
    for (int q = 0; q < NF; ++q) p[q] = V{r[2 * q], r[2 * q + 1]};
}

template <typename T, int NF>
__global__ __launch_bounds__((tri_block<T, NF>())) void tri_grad_kernel(TriArgs<T> a)
{
    const int64_t nc = a.ncell;
    const int64_t i = (int64_t)xcd_logical_block() * tri_block<T, NF>() + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= nc) return;
    const T *U = a.U + (int64_t)b * NF * nc;
    T u[NF], gx[NF], gy[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        u[f] = U[f * nc + i];
        gx[f] = gy[f] = T(0);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t nb = a.nb[k * nc + i];
        T wx, wy;
        geo_vec(a.geo, TGP_W + k, nc, i, wx, wy);
        T d[NF];   // U_k - U_i: the neighbour, or the ghost of a boundary face
        if (nb >= 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) d[f] = U[f * nc + nb] - u[f];
        } else if (nb == -(1 + GKS_BC_PEC)) {
            // mirror ghost: Ez and the normal H odd, the tangential H and psi even
            T nx, ny;
            geo_vec(a.geo, TGP_N + k, nc, i, nx, ny);
            const T hn = u[1] * nx + u[2] * ny;
            d[0] = T(-2) * u[0];
            d[1] = T(-2) * hn * nx;
            d[2] = T(-2) * hn * ny;
            if constexpr (NF == 4) d[3] = T(0);
        } else {   // non-reflecting: the ghost repeats the cell
#pragma unroll
            for (int f = 0; f < NF; ++f) d[f] = T(0);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            gx[f] = fma(wx, d[f], gx[f]);
            gy[f] = fma(wy, d[f], gy[f]);
        }
    }
    store_grad<T, NF>(a.grad + (int64_t)b * 2 * NF * nc, i, gx, gy);
}

// Face-frame form of a global vector (Ez, Hx, Hy[, psi]) for the normal n: (Ez, H.n, H.t[, psi]).
template <typename T, int NF>
__device__ __forceinline__ void to_face(const T (&v)[NF], T nx, T ny, T (&o)[NF])
{
    o[0] = v[0];
    o[1] = v[1] * nx + v[2] * ny;
    o[2] = v[2] * nx - v[1] * ny;
    if constexpr (NF == 4) o[3] = v[3];
}

template <typename T, int NF, bool HAS_EPS, bool HAS_MU>
__global__ __launch_bounds__((tri_block<T, NF>())) void tri_step_kernel(TriArgs<T> a)
{
    using P = typename std::conditional<NF == 4, PatTriP, PatTri>::type;
    using OpT = typename std::conditional<NF == 4, FaceOpTP<T>, FaceOpTM<T>>::type;
    const int64_t nc = a.ncell;
    const int64_t i = (int64_t)xcd_logical_block() * tri_block<T, NF>() + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= nc) return;
    const T *U = a.U + (int64_t)b * NF * nc;
    const T *Gr = a.grad + (int64_t)b * 2 * NF * nc;
    const T *E = HAS_EPS ? a.epsinv + (int64_t)b * nc : nullptr;
    const T *M = HAS_MU ? a.muinv + (int64_t)b * nc : nullptr;
    T u[NF], gx[NF], gy[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) u[f] = U[f * nc + i];
    load_grad<T, NF>(Gr, i, gx, gy);
    const T mE = HAS_EPS ? E[i] : T(1), mH = HAS_MU ? M[i] : T(1);
    double div[NF];   // sum of the face fluxes, in double precision
#pragma unroll
    for (int f = 0; f < NF; ++f) div[f] = 0.0;
    // midpoint offsets of slots 0 and 1; slot 2's is minus their sum
    T ax01[2], ay01[2];
    geo_vec(a.geo, TGP_A + 0, nc, i, ax01[0], ay01[0]);
    geo_vec(a.geo, TGP_A + 1, nc, i, ax01[1], ay01[1]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t nb = a.nb[k * nc + i];
        T nx, ny;
        geo_vec(a.geo, TGP_N + k, nc, i, nx, ny);
        const T lw = geo_lw(a.geo, k, nc, i);
        const T ax = k < 2 ? ax01[k < 2 ? k : 0] : -(ax01[0] + ax01[1]);
        const T ay = k < 2 ? ay01[k < 2 ? k : 0] : -(ay01[0] + ay01[1]);
        // The face operator is linear and, for a constant state on both sides, gives that
        // state's physical flux through the face, which the cell's three faces sum to zero
        // (sum_k |l_k| n_k = 0).  Both sides therefore enter relative to the cell's own state
        // (U_l - U_i, U_r - U_i): the result is the same, and the FP32 rounding of the stored
        // geometry then scales these differences instead of the state itself, so it does not
        // accumulate into a spurious source.  w = [Ul Ur s1l s2l s1r s2r] x fields, face frame.
        T w[6 * NF];
        T tu[NF];   // the cell's own state in the face frame
        to_face<T, NF>(u, nx, ny, tu);
        {
            T dl[NF], dn[NF], dt[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                dl[f] = gx[f] * ax + gy[f] * ay;   // U_l - U_i: the reconstruction offset
                dn[f] = gx[f] * nx + gy[f] * ny;
                dt[f] = gy[f] * nx - gx[f] * ny;
            }
            T o[NF];
            to_face<T, NF>(dl, nx, ny, o);
#pragma unroll
            for (int f = 0; f < NF; ++f) w[f] = o[f];
            to_face<T, NF>(dn, nx, ny, o);
#pragma unroll
            for (int f = 0; f < NF; ++f) w[2 * NF + f] = o[f];
            to_face<T, NF>(dt, nx, ny, o);
#pragma unroll
            for (int f = 0; f < NF; ++f) w[3 * NF + f] = o[f];
        }
        T mEs, mHs;
        if (nb >= 0) {
            T bx, by;
            geo_vec(a.geo, TGP_B + k, nc, i, bx, by);
            T dr[NF], dn[NF], dt[NF], hxs[NF], hys[NF];
            load_grad<T, NF>(Gr, nb, hxs, hys);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T v = U[f * nc + nb], hx = hxs[f], hy = hys[f];
                dr[f] = (v - u[f]) + (hx * bx + hy * by);   // U_r - U_i
                dn[f] = hx * nx + hy * ny;
                dt[f] = hy * nx - hx * ny;
            }
            T o[NF];
            to_face<T, NF>(dr, nx, ny, o);
#pragma unroll
            for (int f = 0; f < NF; ++f) w[NF + f] = o[f];
            to_face<T, NF>(dn, nx, ny, o);
#pragma unroll
            for (int f = 0; f < NF; ++f) w[4 * NF + f] = o[f];
            to_face<T, NF>(dt, nx, ny, o);
#pragma unroll
            for (int f = 0; f < NF; ++f) w[5 * NF + f] = o[f];
            mEs = mE + (HAS_EPS ? E[nb] : T(1));
            mHs = mH + (HAS_MU ? M[nb] : T(1));
        } else if (nb == -(1 + GKS_BC_PEC)) {
            // face-frame mirror P = diag(-1, -1, +1[, +1]) on (Ez, Hn, Ht[, psi]) of the left
            // state U_i + w_l: U_r - U_i = P w_l + (P - 1) U_i; normal slope -P, tangential slope P
            constexpr T PS[4] = {T(-1), T(-1), T(1), T(1)};
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                w[NF + f] = PS[f] * w[f] + (PS[f] - T(1)) * tu[f];
                w[4 * NF + f] = -PS[f] * w[2 * NF + f];
                w[5 * NF + f] = PS[f] * w[3 * NF + f];
            }
            mEs = mE + mE;
            mHs = mH + mH;
        } else {
            // non-reflecting: no distribution on the ghost side, U_r = 0, U_r - U_i = -U_i
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                w[NF + f] = -tu[f];
                w[4 * NF + f] = w[5 * NF + f] = T(0);
            }
            mEs = mE + mE;
            mHs = mH + mH;
        }
        T phi[NF];
        // coefficient chunk: 6 for the fp64 TM kernel (4.06M cells: 395.4 -> 390.7 us, no scalar
        // spills), 12 elsewhere
        apply_op<P, (sizeof(T) == 8 && NF == 3) ? 6 : 12>(w, mEs, mHs, scalar_ptr((const OpT *)a.op), phi);
        // back to the global frame, times |l| / |Omega| (the face's flux, in the storage type),
        // added to the divergence in double precision
        div[0] += (double)(lw * phi[0]);
        div[1] += (double)(lw * (phi[1] * nx - phi[2] * ny));
        div[2] += (double)(lw * (phi[1] * ny + phi[2] * nx));
        if constexpr (NF == 4) div[3] += (double)(lw * phi[3]);
    }
    T *O = a.Unew + (int64_t)b * NF * nc;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        // 1/eps scales Ez, 1/mu scales H; psi carries no material factor.  u - m div in double
        // precision, rounded once to the storage type
        const double m = (f == 0) ? (double)mE : (f < 3) ? (double)mH : 1.0;
        O[f * nc + i] = (T)fma(-m, div[f], (double)u[f]);
    }
}

}  // namespace

template <typename T>
int launch_tri_step(const TriArgs<T> &a, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (a.nfields == 4) {   // TM with psi
        constexpr int B = tri_block<T, 4>();
        const dim3 grid((unsigned)((a.ncell + B - 1) / B), a.batch), block(B);
        hipLaunchKernelGGL((tri_grad_kernel<T, 4>), grid, block, 0, s, a);
        if (a.epsinv && a.muinv) hipLaunchKernelGGL((tri_step_kernel<T, 4, true, true>), grid, block, 0, s, a);
        else if (a.epsinv) hipLaunchKernelGGL((tri_step_kernel<T, 4, true, false>), grid, block, 0, s, a);
        else if (a.muinv) hipLaunchKernelGGL((tri_step_kernel<T, 4, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((tri_step_kernel<T, 4, false, false>), grid, block, 0, s, a);
        return (int)hipGetLastError();
    }
    if (a.nfields != 3) return (int)hipErrorInvalidValue;
    constexpr int B = tri_block<T, 3>();
    const dim3 grid((unsigned)((a.ncell + B - 1) / B), a.batch), block(B);
    hipLaunchKernelGGL((tri_grad_kernel<T, 3>), grid, block, 0, s, a);
    if (a.epsinv && a.muinv) hipLaunchKernelGGL((tri_step_kernel<T, 3, true, true>), grid, block, 0, s, a);
    else if (a.epsinv) hipLaunchKernelGGL((tri_step_kernel<T, 3, true, false>), grid, block, 0, s, a);
    else if (a.muinv) hipLaunchKernelGGL((tri_step_kernel<T, 3, false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((tri_step_kernel<T, 3, false, false>), grid, block, 0, s, a);
    return (int)hipGetLastError();
}

template int launch_tri_step<float>(const TriArgs<float> &, void *);
template int launch_tri_step<double>(const TriArgs<double> &, void *);

}  // namespace gks
