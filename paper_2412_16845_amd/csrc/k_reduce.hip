// Diagnostics of the GKS state (double precision, deterministic order) and small helpers:
//   energy        W = 1/2 sum_i |Omega_i| (eps_i |E_i|^2 + mu_i |H_i|^2 + |potentials|^2) per batch item
//   probe energy  sum over a box of cells of |Omega| Ez^2, and its gradient 2 |Omega| Ez
//   source        explicit point-source scatter for long source lists
// Sums run in two passes: fixed per-block partial sums, then one block per batch item adds the
// partials in a fixed tree order, so results do not depend on scheduling.
#include "gks_device.h"

namespace gks {

constexpr int RBLOCK = 256;

__device__ __forceinline__ double block_sum(double v, double *lds)
{
    // wave reduction with fixed butterfly order, then across the 4 waves in LDS
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < RBLOCK / WAVE; ++i) s += lds[i];
    return s;   // valid on thread 0
}

// Fields [0, NE) are E, [NE, NE + NH) are H, the rest the PHM potentials.  Each thread takes
// four cells a block-stride apart per iteration, so that four cells' loads are in flight
// before any is used; the per-thread order of the sum is fixed.
template <typename T, int NF, int NE, int NH>
__global__ __launch_bounds__(RBLOCK) void energy_partial_kernel(const T *U, const T *epsinv, const T *muinv,
                                                                int64_t ncell, const double *vol, double uvol,
                                                                double *partial, int32_t nblk)
{
    constexpr int UN = 4;
    __shared__ double lds[RBLOCK / WAVE];
    const int b = blockIdx.y;
    const T *Ub = U + (int64_t)b * NF * ncell;
    const T *eb = epsinv ? epsinv + (int64_t)b * ncell : nullptr;
    const T *mb = muinv ? muinv + (int64_t)b * ncell : nullptr;
    const int64_t stride = (int64_t)nblk * RBLOCK;
    double acc = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * RBLOCK + threadIdx.x; i0 < ncell; i0 += UN * stride) {
        T v[UN][NF], e[UN], m[UN];
#pragma unroll
        for (int k = 0; k < UN; ++k) {
            const int64_t i = min(i0 + k * stride, ncell - 1);   // clamped reads; the sum skips them
#pragma unroll
            for (int f = 0; f < NF; ++f) v[k][f] = Ub[(int64_t)f * ncell + i];
            e[k] = eb ? eb[i] : T(1);
            m[k] = mb ? mb[i] : T(1);
        }
#pragma unroll
        for (int k = 0; k < UN; ++k) {
            const int64_t i = i0 + k * stride;
            if (i >= ncell) break;
            double e2 = 0.0, h2 = 0.0, p2 = 0.0;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double x = (double)v[k][f];
                if (f < NE) e2 += x * x;
                else if (f < NE + NH) h2 += x * x;
                else p2 += x * x;
            }
            const double w = vol ? vol[i] : uvol;
            acc += 0.5 * w * (e2 / (double)e[k] + h2 / (double)m[k] + p2);
        }
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[(int64_t)b * nblk + blockIdx.x] = s;
}

__global__ __launch_bounds__(RBLOCK) void final_sum_kernel(const double *partial, int32_t nblk, double *out)
{
    __shared__ double lds[RBLOCK / WAVE];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RBLOCK) acc += partial[(int64_t)b * nblk + i];
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) out[b] = s;
}

template <typename T>
int launch_energy(const T *U, const T *epsinv, const T *muinv, int64_t ncell, int32_t nfields, int32_t nE, int32_t nH,
                  int32_t batch, const double *vol, double uniform_vol, double *partial, int32_t nblk, double *out,
                  void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid(nblk, batch), block(RBLOCK);
    if (nfields == 3 && nE == 1 && nH == 2)
        hipLaunchKernelGGL((energy_partial_kernel<T, 3, 1, 2>), grid, block, 0, s, U, epsinv, muinv, ncell, vol,
                           uniform_vol, partial, nblk);
    else if (nfields == 4 && nE == 1 && nH == 2)
        hipLaunchKernelGGL((energy_partial_kernel<T, 4, 1, 2>), grid, block, 0, s, U, epsinv, muinv, ncell, vol,
                           uniform_vol, partial, nblk);
    else if (nfields == 6 && nE == 3 && nH == 3)
        hipLaunchKernelGGL((energy_partial_kernel<T, 6, 3, 3>), grid, block, 0, s, U, epsinv, muinv, ncell, vol,
                           uniform_vol, partial, nblk);
    else if (nfields == 8 && nE == 3 && nH == 3)
        hipLaunchKernelGGL((energy_partial_kernel<T, 8, 3, 3>), grid, block, 0, s, U, epsinv, muinv, ncell, vol,
                           uniform_vol, partial, nblk);
    else
        return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(final_sum_kernel, dim3(batch), dim3(RBLOCK), 0, s, partial, nblk, out);
    return (int)hipGetLastError();
}

struct Box {
    int64_t i0, i1, j0, j1, k0, k1;
};

template <typename T>
__global__ __launch_bounds__(RBLOCK) void probe_partial_kernel(const T *U, int64_t nx, int64_t ny, int64_t nz,
                                                               int32_t nfields, int32_t ezf, Box bx, double vol,
                                                               double *partial, int32_t nblk)
{
    __shared__ double lds[RBLOCK / WAVE];
    const int b = blockIdx.y;
    const int64_t ncell = nx * ny * nz;
    const T *Ez = U + ((int64_t)b * nfields + ezf) * ncell;
    const int64_t sx = bx.i1 - bx.i0, sy = bx.j1 - bx.j0, sz = bx.k1 - bx.k0;
    const int64_t n = sx * sy * sz;
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * RBLOCK + threadIdx.x; t < n; t += (int64_t)nblk * RBLOCK) {
        const int64_t i = bx.i0 + t % sx, j = bx.j0 + (t / sx) % sy, k = bx.k0 + t / (sx * sy);
        const double v = (double)Ez[(k * ny + j) * nx + i];
        acc += vol * v * v;
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[(int64_t)b * nblk + blockIdx.x] = s;
}

template <typename T>
int launch_probe_energy(const T *U, int64_t nx, int64_t ny, int64_t nz, int32_t nfields, int32_t ez_field,
                        int32_t batch, const int64_t box[6], double vol, double *partial, int32_t nblk, double *out,
                        void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Box bx{box[0], box[1], box[2], box[3], box[4], box[5]};
    hipLaunchKernelGGL(probe_partial_kernel<T>, dim3(nblk, batch), dim3(RBLOCK), 0, s, U, nx, ny, nz, nfields,
                       ez_field, bx, vol, partial, nblk);
    hipLaunchKernelGGL(final_sum_kernel, dim3(batch), dim3(RBLOCK), 0, s, partial, nblk, out);
    return (int)hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(RBLOCK) void probe_grad_kernel(const T *U, T *lam, int64_t nx, int64_t ny, int64_t nz,
                                                            int32_t nfields, int32_t ezf, Box bx, double vol,
                                                            int64_t total)
{
    const int64_t ncell = nx * ny * nz;
    for (int64_t t = (int64_t)blockIdx.x * RBLOCK + threadIdx.x; t < total; t += (int64_t)gridDim.x * RBLOCK) {
        const int64_t c = t % ncell;
        const int64_t f = (t / ncell) % nfields;
        T v = T(0);
        if (f == ezf) {
            const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
            if (i >= bx.i0 && i < bx.i1 && j >= bx.j0 && j < bx.j1 && k >= bx.k0 && k < bx.k1)
                v = (T)(2.0 * vol * (double)U[t]);
        }
        lam[t] = v;
    }
}

template <typename T>
int launch_probe_grad(const T *U, T *lam, int64_t nx, int64_t ny, int64_t nz, int32_t nfields, int32_t ez_field,
                      int32_t batch, const int64_t box[6], double vol, void *stream)
{
    const int64_t total = nx * ny * nz * nfields * (int64_t)batch;
    int64_t blocks = (total + RBLOCK - 1) / RBLOCK;
    if (blocks > 65536) blocks = 65536;
    Box bx{box[0], box[1], box[2], box[3], box[4], box[5]};
    hipLaunchKernelGGL(probe_grad_kernel<T>, dim3((unsigned)blocks), dim3(RBLOCK), 0, (hipStream_t)stream, U, lam,
                       nx, ny, nz, nfields, ez_field, bx, vol, total);
    return (int)hipGetLastError();
}

template <typename T>
__global__ void source_scatter_kernel(T *U, const T *epsinv, int64_t ncell, int64_t fstride, int32_t field,
                                      const int64_t *cells, const double *weight, double amp, int32_t n)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (s >= n) return;
    const int64_t c = cells[s];
    const double m = epsinv ? (double)epsinv[(int64_t)b * ncell + c] : 1.0;
    T *p = U + (int64_t)b * fstride + (int64_t)field * ncell + c;
    *p = (T)((double)*p + m * (amp * weight[s]));
}

template <typename T>
int launch_source_scatter(T *U, const T *epsinv, int64_t ncell, int64_t fstride, int32_t batch, int32_t field,
                          const int64_t *cells, const double *weight, double amp, int32_t n, void *stream)
{
    hipLaunchKernelGGL(source_scatter_kernel<T>, dim3((n + 255) / 256, batch), dim3(256), 0, (hipStream_t)stream, U,
                       epsinv, ncell, fstride, field, cells, weight, amp, n);
    return (int)hipGetLastError();
}

#define GKS_INST(T)                                                                                                  \
    template int launch_energy<T>(const T *, const T *, const T *, int64_t, int32_t, int32_t, int32_t, int32_t,    \
                                  const double *, double, double *, int32_t, double *, void *);                    \
    template int launch_probe_energy<T>(const T *, int64_t, int64_t, int64_t, int32_t, int32_t, int32_t,            \
                                        const int64_t[6], double, double *, int32_t, double *, void *);             \
    template int launch_probe_grad<T>(const T *, T *, int64_t, int64_t, int64_t, int32_t, int32_t, int32_t,         \
                                      const int64_t[6], double, void *);                                            \
    template int launch_source_scatter<T>(T *, const T *, int64_t, int64_t, int32_t, int32_t, const int64_t *,      \
                                          const double *, double, int32_t, void *);
GKS_INST(float)
GKS_INST(double)

}  // namespace gks
