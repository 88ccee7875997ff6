// Device helpers shared by the kernels of libgks (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "gks_internal.h"
#include "gks_pattern.h"

namespace gks {

constexpr int WAVE = 64;

// ------------------------------------------------------------------ cross-lane moves (DPP)
// from_right(v): lane i receives lane i+1 (wave_shl:1); from_left(v): lane i receives lane i-1
// (wave_shr:1).  The end lanes receive 0 (only halo lanes read them).
__device__ __forceinline__ float from_right(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ double from_right(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_left(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------------------ boundary index maps
// Maps a ghost-extended index g in [-2, n+1] of one axis to the cell it reads.  mirror: the
// value is the PEC mirror image; nr: a non-reflecting ghost (the clamped value feeds the
// neighbour's zero-gradient Green-Gauss ghost; the face flux sees an empty ghost side).
__device__ __forceinline__ int map_axis(int g, int n, int bclo, int bchi, bool &mirror, bool &nr)
{
    mirror = false;
    nr = false;
    g = g < -2 ? -2 : (g > n + 1 ? n + 1 : g);
    if (g < 0) {
        if (bclo == GKS_BC_PERIODIC) return g + n;
        if (bclo == GKS_BC_PEC) { mirror = true; return -1 - g; }
        nr = true;
        return 0;
    }
    if (g >= n) {
        if (bchi == GKS_BC_PERIODIC) return g - n;
        if (bchi == GKS_BC_PEC) { mirror = true; return 2 * n - 1 - g; }
        nr = true;
        return n - 1;
    }
    return g;
}

// ------------------------------------------------------------------ sparse face operators
// phi = K0 w + mE KE w + mH KH w using the compile-time sparsity tables.
template <typename T>
__device__ __forceinline__ void apply_tm(const T (&w)[18], T mE, T mH, const FaceOpTM<T> &K, T (&phi)[3])
{
    T a[3] = {T(0), T(0), T(0)}, e[3] = {T(0), T(0), T(0)}, h[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < TM_N0; ++q) a[TM_R0[q]] = fma(K.k0[q], w[TM_C0[q]], a[TM_R0[q]]);
#pragma unroll
    for (int q = 0; q < TM_NE; ++q) e[TM_RE[q]] = fma(K.ke[q], w[TM_CE[q]], e[TM_RE[q]]);
#pragma unroll
    for (int q = 0; q < TM_NH; ++q) h[TM_RH[q]] = fma(K.kh[q], w[TM_CH[q]], h[TM_RH[q]]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        T v = a[r];
        if (TM_EROWS >> r & 1u) v = fma(mE, e[r], v);
        if (TM_HROWS >> r & 1u) v = fma(mH, h[r], v);
        phi[r] = v;
    }
}

// Transpose: wbar += K(mE, mH)^T abar.
template <typename T>
__device__ __forceinline__ void apply_tm_transpose(const T (&abar)[3], T mE, T mH, const FaceOpTM<T> &K,
                                                   T (&wbar)[18])
{
    T ae[3], ah[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        ae[r] = mE * abar[r];
        ah[r] = mH * abar[r];
    }
#pragma unroll
    for (int q = 0; q < TM_N0; ++q) wbar[TM_C0[q]] = fma(K.k0[q], abar[TM_R0[q]], wbar[TM_C0[q]]);
#pragma unroll
    for (int q = 0; q < TM_NE; ++q) wbar[TM_CE[q]] = fma(K.ke[q], ae[TM_RE[q]], wbar[TM_CE[q]]);
#pragma unroll
    for (int q = 0; q < TM_NH; ++q) wbar[TM_CH[q]] = fma(K.kh[q], ah[TM_RH[q]], wbar[TM_CH[q]]);
}

// abar . (KE w) and abar . (KH w): the derivatives of abar . phi with respect to mE and mH.
template <typename T>
__device__ __forceinline__ void material_sens_tm(const T (&abar)[3], const T (&w)[18], const FaceOpTM<T> &K,
                                                 T &dE, T &dH)
{
    T e = T(0), h = T(0);
#pragma unroll
    for (int q = 0; q < TM_NE; ++q) e = fma(K.ke[q] * abar[TM_RE[q]], w[TM_CE[q]], e);
#pragma unroll
    for (int q = 0; q < TM_NH; ++q) h = fma(K.kh[q] * abar[TM_RH[q]], w[TM_CH[q]], h);
    dE = e;
    dH = h;
}

}  // namespace gks
