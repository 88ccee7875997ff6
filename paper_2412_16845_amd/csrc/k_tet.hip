// GKS step on a tetrahedral mesh, six fields (Ex, Ey, Ez, Hx, Hy, Hz) (the unstructured 3D
// meshes of Sec. 5.5).
//
// Three kernels (cells in Morton order, faces ordered by owner, so gathered neighbours are
// mostly cached; blocks renumbered so that consecutive blocks share an XCD's L2):
//   1. cell gradients grad U_i = sum_k W_k (U_k - U_i) over the four faces (Green-Gauss, Sec.
//      3.1); the ghost of a non-reflecting face is the cell itself, that of a PEC face its
//      mirror image (tangential E and normal H odd);
//   2. one thread per face: both sides reconstructed at the face centroid, states and slopes
//      rotated into the face frame with the printed rotation T' (Sec. 3.1), the flux evaluated as
//      a sparse linear form (the closed-form moments folded into coefficients on the host),
//      rotated back and stored times |l|.  Each face is evaluated once, from its owner: the
//      D3Q4 lattice is chiral, so the other side's flux would differ;
//   3. one thread per cell: the four face fluxes with the sign of the cell's side, divided by
//      |Omega|, added to the old value in double precision and rounded once on store.
// Boundary faces: non-reflecting (the ghost side carries no distribution) or PEC (face-frame
// mirror of the state, the normal slope mirrored with the opposite sign).
#include "gks_device.h"

namespace gks {

namespace {

constexpr int TET_BLOCK = 256;

// Gradient records: 18 values per cell, [d/dx (6 fields) d/dy (6) d/dz (6)], as 9 pairs.
template <typename T> struct Pair3;
template <> struct Pair3<float> { using type = float2; };
template <> struct Pair3<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ void load_grad18(const T *G, int64_t c, T (&g)[3][6])
{
    using V = typename Pair3<T>::type;
    const V *p = reinterpret_cast<const V *>(G + c * 18);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const V v = p[q];
        g[(2 * q) / 6][(2 * q) % 6] = v.x;
        g[(2 * q + 1) / 6][(2 * q + 1) % 6] = v.y;
    }
}

template <typename T>
__global__ __launch_bounds__(TET_BLOCK) void tet_grad_kernel(TetArgs<T> a)
{
    const int64_t nc = a.ncell;
    const int64_t i = (int64_t)xcd_logical_block() * TET_BLOCK + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= nc) return;
    const T *U = a.U + (int64_t)b * 6 * nc;
    T u[6], g[3][6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        u[f] = U[f * nc + i];
        g[0][f] = g[1][f] = g[2][f] = T(0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t nb = a.nb[k * nc + i];
        T d[6];   // U_k - U_i: the neighbour, or the ghost of a boundary face
        if (nb >= 0) {
#pragma unroll
            for (int f = 0; f < 6; ++f) d[f] = U[f * nc + nb] - u[f];
        } else if (nb == -(1 + GKS_BC_PEC)) {
            // mirror ghost: E_g = 2 (E.n) n - E, H_g = H - 2 (H.n) n
            T n[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) n[q] = a.cgeo[(TC_N + 3 * k + q) * nc + i];
            const T en = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
            const T hn = u[3] * n[0] + u[4] * n[1] + u[5] * n[2];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                d[q] = T(2) * (en * n[q] - u[q]);
                d[3 + q] = T(-2) * hn * n[q];
            }
        } else {   // non-reflecting: the ghost repeats the cell
#pragma unroll
            for (int f = 0; f < 6; ++f) d[f] = T(0);
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const T w = a.cgeo[(TC_W + 3 * k + q) * nc + i];
#pragma unroll
            for (int f = 0; f < 6; ++f) g[q][f] = fma(w, d[f], g[q][f]);
        }
    }
    using V = typename Pair3<T>::type;
    V *p = reinterpret_cast<V *>(a.grad + ((int64_t)b * nc + i) * 18);
#pragma unroll
    for (int q = 0; q < 9; ++q)
        p[q] = V{g[(2 * q) / 6][(2 * q) % 6], g[(2 * q + 1) / 6][(2 * q + 1) % 6]};
}

// y = T' x on both (E, H) blocks of a six-vector.
template <typename T>
__device__ __forceinline__ void rot6(const T (&R)[3][3], const T (&x)[6], T (&y)[6])
{
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
        for (int r = 0; r < 3; ++r)
            y[3 * blk + r] = R[r][0] * x[3 * blk] + R[r][1] * x[3 * blk + 1] + R[r][2] * x[3 * blk + 2];
}

// One side of a face in the face frame: the state reconstructed at the face centroid and the
// slopes along the face axes, written to w[so + f] and w[sl + 6 j + f].
template <typename T>
__device__ __forceinline__ void face_side(const T *U, int64_t nc, int64_t c, const T (&g)[3][6], const T (&d)[3],
                                          const T (&R)[3][3], T *w, int so, int sl)
{
    T x[6], y[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) x[f] = U[f * nc + c] + g[0][f] * d[0] + g[1][f] * d[1] + g[2][f] * d[2];
    rot6(R, x, y);
#pragma unroll
    for (int f = 0; f < 6; ++f) w[so + f] = y[f];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // derivative along face axis j: sum_i T'_ji d_i U, then rotated like a state
#pragma unroll
        for (int f = 0; f < 6; ++f) x[f] = R[j][0] * g[0][f] + R[j][1] * g[1][f] + R[j][2] * g[2][f];
        rot6(R, x, y);
#pragma unroll
        for (int f = 0; f < 6; ++f) w[sl + 6 * j + f] = y[f];
    }
}

template <typename T, bool HAS_EPS, bool HAS_MU>
__global__ __launch_bounds__(TET_BLOCK) void tet_face_kernel(TetArgs<T> a)
{
    const int64_t nf = a.nface, nc = a.ncell;
    const int64_t s = (int64_t)xcd_logical_block() * TET_BLOCK + threadIdx.x;
    const int b = blockIdx.y;
    if (s >= nf) return;
    const T *U = a.U + (int64_t)b * 6 * nc;
    const T *Gr = a.grad + (int64_t)b * 18 * nc;
    const int32_t L = a.fc[2 * s], R = a.fc[2 * s + 1];
    const T n0 = a.fgeo[(TF_N + 0) * nf + s], n1 = a.fgeo[(TF_N + 1) * nf + s], n2 = a.fgeo[(TF_N + 2) * nf + s];
    const T A = a.fgeo[TF_A * nf + s], B = a.fgeo[TF_B * nf + s];
    // the printed rotation: rows n, (-n2, n1 + n3^2/q, -n2 n3/q), (-n3, -n2 n3/q, 1 - n3^2/q), q = 1 + n1
    const T Rm[3][3] = {{n0, n1, n2}, {-n1, n0 + A, -B}, {-n2, -B, T(1) - A}};
    T w[48];
    {
        T g[3][6];
        const T d[3] = {a.fgeo[(TF_DL + 0) * nf + s], a.fgeo[(TF_DL + 1) * nf + s], a.fgeo[(TF_DL + 2) * nf + s]};
        load_grad18(Gr, L, g);
        face_side(U, nc, L, g, d, Rm, w, 0, 12);
    }
    const T *E = HAS_EPS ? a.epsinv + (int64_t)b * nc : nullptr;
    const T *M = HAS_MU ? a.muinv + (int64_t)b * nc : nullptr;
    const T eL = HAS_EPS ? E[L] : T(1), mL = HAS_MU ? M[L] : T(1);
    T mEs, mHs;
    if (R >= 0) {
        T g[3][6];
        const T d[3] = {a.fgeo[(TF_DR + 0) * nf + s], a.fgeo[(TF_DR + 1) * nf + s], a.fgeo[(TF_DR + 2) * nf + s]};
        load_grad18(Gr, R, g);
        face_side(U, nc, R, g, d, Rm, w, 6, 30);
        mEs = eL + (HAS_EPS ? E[R] : T(1));
        mHs = mL + (HAS_MU ? M[R] : T(1));
    } else if (R == -(1 + GKS_BC_PEC)) {
        // face-frame mirror P = diag(+1, -1, -1 | -1, +1, +1); normal slope -P, tangential P
        constexpr T PS[6] = {T(1), T(-1), T(-1), T(-1), T(1), T(1)};
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            w[6 + f] = PS[f] * w[f];
            w[30 + f] = -PS[f] * w[12 + f];
            w[36 + f] = PS[f] * w[18 + f];
            w[42 + f] = PS[f] * w[24 + f];
        }
        mEs = eL + eL;
        mHs = mL + mL;
    } else {   // non-reflecting: no distribution from the ghost side
#pragma unroll
        for (int f = 0; f < 6; ++f) w[6 + f] = w[30 + f] = w[36 + f] = w[42 + f] = T(0);
        mEs = eL + eL;
        mHs = mL + mL;
    }
    T phi[6];
    apply_op<PatTet>(w, mEs, mHs, scalar_ptr((const FaceOpEM<T> *)a.op), phi);
    // back to the global frame (T'^T on both blocks), times |l|
    const T area = a.fgeo[TF_AREA * nf + s];
    T *out = a.flux + ((int64_t)b * nf + s) * 6;
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
        for (int r = 0; r < 3; ++r)
            out[3 * blk + r] =
                area * (Rm[0][r] * phi[3 * blk] + Rm[1][r] * phi[3 * blk + 1] + Rm[2][r] * phi[3 * blk + 2]);
}

template <typename T, bool HAS_EPS, bool HAS_MU>
__global__ __launch_bounds__(TET_BLOCK) void tet_update_kernel(TetArgs<T> a)
{
    const int64_t nc = a.ncell, nf = a.nface;
    const int64_t i = (int64_t)xcd_logical_block() * TET_BLOCK + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= nc) return;
    const T *Fl = a.flux + (int64_t)b * nf * 6;
    double div[6];   // sum of the four face fluxes, in double precision
#pragma unroll
    for (int f = 0; f < 6; ++f) div[f] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t cf = a.cf[k * nc + i];
        const int64_t s = (cf > 0 ? cf : -cf) - 1;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const double v = (double)Fl[s * 6 + f];
            div[f] = cf > 0 ? div[f] + v : div[f] - v;
        }
    }
    const double iv = (double)a.cgeo[TC_IVOL * nc + i];
    const T mE = HAS_EPS ? a.epsinv[(int64_t)b * nc + i] : T(1), mH = HAS_MU ? a.muinv[(int64_t)b * nc + i] : T(1);
    const T *U = a.U + (int64_t)b * 6 * nc;
    T *O = a.Unew + (int64_t)b * 6 * nc;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        // U - m div / |Omega| in double precision, rounded once to the storage type
        const double m = (f < 3) ? (double)mE : (double)mH;
        O[f * nc + i] = (T)fma(-m, div[f] * iv, (double)U[f * nc + i]);
    }
}

}  // namespace

template <typename T>
int launch_tet_step(const TetArgs<T> &a, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const dim3 block(TET_BLOCK);
    const dim3 gc((unsigned)((a.ncell + TET_BLOCK - 1) / TET_BLOCK), a.batch);
    const dim3 gf((unsigned)((a.nface + TET_BLOCK - 1) / TET_BLOCK), a.batch);
    hipLaunchKernelGGL(tet_grad_kernel<T>, gc, block, 0, s, a);
    if (a.epsinv && a.muinv) {
        hipLaunchKernelGGL((tet_face_kernel<T, true, true>), gf, block, 0, s, a);
        hipLaunchKernelGGL((tet_update_kernel<T, true, true>), gc, block, 0, s, a);
    } else if (a.epsinv) {
        hipLaunchKernelGGL((tet_face_kernel<T, true, false>), gf, block, 0, s, a);
        hipLaunchKernelGGL((tet_update_kernel<T, true, false>), gc, block, 0, s, a);
    } else if (a.muinv) {
        hipLaunchKernelGGL((tet_face_kernel<T, false, true>), gf, block, 0, s, a);
        hipLaunchKernelGGL((tet_update_kernel<T, false, true>), gc, block, 0, s, a);
    } else {
        hipLaunchKernelGGL((tet_face_kernel<T, false, false>), gf, block, 0, s, a);
        hipLaunchKernelGGL((tet_update_kernel<T, false, false>), gc, block, 0, s, a);
    }
    return (int)hipGetLastError();
}

template int launch_tet_step<float>(const TetArgs<float> &, void *);
template int launch_tet_step<double>(const TetArgs<double> &, void *);

}  // namespace gks
