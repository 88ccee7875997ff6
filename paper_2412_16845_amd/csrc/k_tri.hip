// GKS step on a triangle mesh, TM fields (Ez, Hx, Hy).
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
//      closed-form flux folded into coefficients on the host), rotated back, and the cell's
//      divergence is added to its old value in double precision.
// A face is evaluated by both of its cells, each from its own side: no face fluxes are stored
// and no atomics are needed.  Boundary faces: non-reflecting (the ghost side carries no
// distribution) or PEC (face-frame mirror of the state, the normal slope mirrored with the
// opposite sign).
#include "gks_device.h"

namespace gks {

namespace {

constexpr int TRI_BLOCK = 256;

// The gradient scratch holds one record of six values per cell, [d/dx (Ez Hx Hy), d/dy (Ez Hx
// Hy)], so that the gradients of a gathered neighbour come from one or two cache lines.
template <typename T> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ void load_grad(const T *G, int64_t c, T (&gx)[3], T (&gy)[3])
{
    using V = typename Pair<T>::type;
    const V *p = reinterpret_cast<const V *>(G + c * 6);
    const V v0 = p[0], v1 = p[1], v2 = p[2];
    gx[0] = v0.x;
    gx[1] = v0.y;
    gx[2] = v1.x;
    gy[0] = v1.y;
    gy[1] = v2.x;
    gy[2] = v2.y;
}

template <typename T>
__device__ __forceinline__ void store_grad(T *G, int64_t c, const T (&gx)[3], const T (&gy)[3])
{
    using V = typename Pair<T>::type;
    V *p = reinterpret_cast<V *>(G + c * 6);
    p[0] = V{gx[0], gx[1]};
    p[1] = V{gx[2], gy[0]};
    p[2] = V{gy[1], gy[2]};
}

template <typename T>
__global__ __launch_bounds__(TRI_BLOCK) void tri_grad_kernel(TriArgs<T> a)
{
    const int64_t nc = a.ncell;
    const int64_t i = (int64_t)xcd_logical_block() * TRI_BLOCK + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= nc) return;
    const T *U = a.U + (int64_t)b * 3 * nc;
    T u[3], gx[3] = {T(0), T(0), T(0)}, gy[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int f = 0; f < 3; ++f) u[f] = U[f * nc + i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t nb = a.nb[k * nc + i];
        const T wx = a.geo[(TG_WX + k) * nc + i], wy = a.geo[(TG_WY + k) * nc + i];
        T d[3];   // U_k - U_i: the neighbour, or the ghost of a boundary face
        if (nb >= 0) {
#pragma unroll
            for (int f = 0; f < 3; ++f) d[f] = U[f * nc + nb] - u[f];
        } else if (nb == -(1 + GKS_BC_PEC)) {
            // mirror ghost: Ez and the normal H odd, the tangential H even
            const T nx = a.geo[(TG_NX + k) * nc + i], ny = a.geo[(TG_NY + k) * nc + i];
            const T hn = u[1] * nx + u[2] * ny;
            d[0] = T(-2) * u[0];
            d[1] = T(-2) * hn * nx;
            d[2] = T(-2) * hn * ny;
        } else {   // non-reflecting: the ghost repeats the cell
#pragma unroll
            for (int f = 0; f < 3; ++f) d[f] = T(0);
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            gx[f] = fma(wx, d[f], gx[f]);
            gy[f] = fma(wy, d[f], gy[f]);
        }
    }
    store_grad(a.grad + (int64_t)b * 6 * nc, i, gx, gy);
}

// Face-frame form of a global TM vector (Ez, Hx, Hy) for the normal n: (Ez, H.n, H.t).
template <typename T>
__device__ __forceinline__ void to_face(const T (&v)[3], T nx, T ny, T (&o)[3])
{
    o[0] = v[0];
    o[1] = v[1] * nx + v[2] * ny;
    o[2] = v[2] * nx - v[1] * ny;
}

template <typename T, bool HAS_EPS, bool HAS_MU>
__global__ __launch_bounds__(TRI_BLOCK) void tri_step_kernel(TriArgs<T> a)
{
    const int64_t nc = a.ncell;
    const int64_t i = (int64_t)xcd_logical_block() * TRI_BLOCK + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= nc) return;
    const T *U = a.U + (int64_t)b * 3 * nc;
    const T *Gr = a.grad + (int64_t)b * 6 * nc;
    const T *E = HAS_EPS ? a.epsinv + (int64_t)b * nc : nullptr;
    const T *M = HAS_MU ? a.muinv + (int64_t)b * nc : nullptr;
    T u[3], gx[3], gy[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) u[f] = U[f * nc + i];
    load_grad(Gr, i, gx, gy);
    const T mE = HAS_EPS ? E[i] : T(1), mH = HAS_MU ? M[i] : T(1);
    T div[3] = {T(0), T(0), T(0)};
    // midpoint offsets of slots 0 and 1; slot 2's is minus their sum
    const T ax01[2] = {a.geo[(TG_AX + 0) * nc + i], a.geo[(TG_AX + 1) * nc + i]};
    const T ay01[2] = {a.geo[(TG_AY + 0) * nc + i], a.geo[(TG_AY + 1) * nc + i]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t nb = a.nb[k * nc + i];
        const T nx = a.geo[(TG_NX + k) * nc + i], ny = a.geo[(TG_NY + k) * nc + i];
        const T lw = a.geo[(TG_LW + k) * nc + i];
        const T ax = k < 2 ? ax01[k < 2 ? k : 0] : -(ax01[0] + ax01[1]);
        const T ay = k < 2 ? ay01[k < 2 ? k : 0] : -(ay01[0] + ay01[1]);
        // own side: reconstruction at the midpoint, slopes along n and t, all in the face frame
        T w[18];
        {
            T ul[3], dn[3], dt[3];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                ul[f] = u[f] + gx[f] * ax + gy[f] * ay;
                dn[f] = gx[f] * nx + gy[f] * ny;
                dt[f] = gy[f] * nx - gx[f] * ny;
            }
            T o[3];
            to_face(ul, nx, ny, o);
#pragma unroll
            for (int f = 0; f < 3; ++f) w[f] = o[f];
            to_face(dn, nx, ny, o);
#pragma unroll
            for (int f = 0; f < 3; ++f) w[6 + f] = o[f];
            to_face(dt, nx, ny, o);
#pragma unroll
            for (int f = 0; f < 3; ++f) w[9 + f] = o[f];
        }
        T mEs, mHs;
        if (nb >= 0) {
            const T bx = a.geo[(TG_BX + k) * nc + i], by = a.geo[(TG_BY + k) * nc + i];
            T ur[3], dn[3], dt[3], hxs[3], hys[3];
            load_grad(Gr, nb, hxs, hys);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const T v = U[f * nc + nb], hx = hxs[f], hy = hys[f];
                ur[f] = v + hx * bx + hy * by;
                dn[f] = hx * nx + hy * ny;
                dt[f] = hy * nx - hx * ny;
            }
            T o[3];
            to_face(ur, nx, ny, o);
#pragma unroll
            for (int f = 0; f < 3; ++f) w[3 + f] = o[f];
            to_face(dn, nx, ny, o);
#pragma unroll
            for (int f = 0; f < 3; ++f) w[12 + f] = o[f];
            to_face(dt, nx, ny, o);
#pragma unroll
            for (int f = 0; f < 3; ++f) w[15 + f] = o[f];
            mEs = mE + (HAS_EPS ? E[nb] : T(1));
            mHs = mH + (HAS_MU ? M[nb] : T(1));
        } else if (nb == -(1 + GKS_BC_PEC)) {
            // face-frame mirror P = diag(-1, -1, +1) on (Ez, Hn, Ht); normal slope -P, tangential P
            w[3] = -w[0];
            w[4] = -w[1];
            w[5] = w[2];
            w[12] = w[6];
            w[13] = w[7];
            w[14] = -w[8];
            w[15] = -w[9];
            w[16] = -w[10];
            w[17] = w[11];
            mEs = mE + mE;
            mHs = mH + mH;
        } else {
#pragma unroll
            for (int f = 0; f < 3; ++f) w[3 + f] = w[12 + f] = w[15 + f] = T(0);
            mEs = mE + mE;
            mHs = mH + mH;
        }
        T phi[3];
        apply_op<PatTri>(w, mEs, mHs, scalar_ptr(a.op), phi);
        // back to the global frame, times |l| / |Omega|
        div[0] = fma(lw, phi[0], div[0]);
        div[1] = fma(lw, phi[1] * nx - phi[2] * ny, div[1]);
        div[2] = fma(lw, phi[1] * ny + phi[2] * nx, div[2]);
    }
    T *O = a.Unew + (int64_t)b * 3 * nc;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const double m = (f == 0) ? (double)mE : (double)mH;
        O[f * nc + i] = (T)((double)u[f] - m * (double)div[f]);
    }
}

}  // namespace

template <typename T>
int launch_tri_step(const TriArgs<T> &a, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    dim3 grid((unsigned)((a.ncell + TRI_BLOCK - 1) / TRI_BLOCK), a.batch), block(TRI_BLOCK);
    hipLaunchKernelGGL(tri_grad_kernel<T>, grid, block, 0, s, a);
    if (a.epsinv && a.muinv) hipLaunchKernelGGL((tri_step_kernel<T, true, true>), grid, block, 0, s, a);
    else if (a.epsinv) hipLaunchKernelGGL((tri_step_kernel<T, true, false>), grid, block, 0, s, a);
    else if (a.muinv) hipLaunchKernelGGL((tri_step_kernel<T, false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((tri_step_kernel<T, false, false>), grid, block, 0, s, a);
    return (int)hipGetLastError();
}

template int launch_tri_step<float>(const TriArgs<float> &, void *);
template int launch_tri_step<double>(const TriArgs<double> &, void *);

}  // namespace gks
