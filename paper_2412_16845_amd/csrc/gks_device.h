// Device helpers shared by the kernels of libgks (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "gks_internal.h"
#include "gks_pattern.h"

namespace gks {

constexpr int WAVE = 64;

// ------------------------------------------------------------------ cross-lane moves (DPP)
// from_right(v): lane i receives lane i+1 (wave_shl:1); from_left(v): lane i receives lane i-1
// (wave_shr:1).  bound_ctrl makes the end lane (which has no source) receive 0; only halo lanes
// read it.
__device__ __forceinline__ int dpp_shl1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_shr1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }

__device__ __forceinline__ float from_right(float v)
{
    return __builtin_bit_cast(float, dpp_shl1(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float from_left(float v)
{
    return __builtin_bit_cast(float, dpp_shr1(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double from_right(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_shl1((int)(b & 0xffffffffll));
    const int hi = dpp_shl1((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_left(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_shr1((int)(b & 0xffffffffll));
    const int hi = dpp_shr1((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------------------ buffer memory access
// Raw buffer loads/stores: a 128-bit resource (base, size) in scalar registers, a per-lane
// 32-bit byte offset in a vector register and a uniform 32-bit byte offset in a scalar
// register, so the per-row address arithmetic runs on the scalar unit.  Accesses at or beyond
// the resource size read 0 / are dropped by the hardware.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int RSRC_DWORD3 = 0x00020000;   // 32-bit data format, raw (stride 0) buffer

__device__ __forceinline__ Rsrc make_rsrc(const void *p, uint64_t bytes)
{
    const uint32_t n = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, RSRC_DWORD3);
}

template <typename T> __device__ __forceinline__ T buf_load(Rsrc r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float buf_load<float>(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ double buf_load<double>(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// Two adjacent floats (one 8-byte access per lane).
__device__ __forceinline__ float2 buf_load_f2(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

#ifndef GKS_STORE_AUX
#define GKS_STORE_AUX 0
#endif
__device__ __forceinline__ void buf_store(float v, Rsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, voff, soff, GKS_STORE_AUX);
}
__device__ __forceinline__ void buf_store(double v, Rsrc r, uint32_t voff, uint32_t soff)
{
    using v2u = __attribute__((ext_vector_type(2))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, voff, soff, GKS_STORE_AUX);
}

__device__ __forceinline__ void buf_store_f2(float2 v, Rsrc r, uint32_t voff, uint32_t soff)
{
    using v2u = __attribute__((ext_vector_type(2))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, voff, soff, GKS_STORE_AUX);
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

// ------------------------------------------------------------------ coefficient access
// Face-operator coefficients live in a small device buffer of the context.  They are read
// through the constant address space (scalar loads into SGPRs, served by the scalar cache)
// right where a face is evaluated: the empty asm hides the pointer's loop invariance so the
// loads are not hoisted into a register set that would not fit the SGPR file.
template <typename Op>
using ConstPtr = const __attribute__((address_space(4))) Op *;

template <typename Op>
__device__ __forceinline__ ConstPtr<Op> scalar_ptr(const Op *p)
{
    ConstPtr<Op> q = (ConstPtr<Op>)p;
    asm volatile("" : "+s"(q));
    return q;
}

// The same, but the pointer (hence the coefficient loads) only becomes available once `after`
// has been computed: keeps the coefficient sets of consecutive faces from being live together.
template <typename Op, typename V>
__device__ __forceinline__ ConstPtr<Op> scalar_ptr_after(const Op *p, V after)
{
    ConstPtr<Op> q = (ConstPtr<Op>)p;
    asm volatile("" : "+s"(q) : "v"(after));
    return q;
}

// ------------------------------------------------------------------ slope limiter
// minmod: the argument of smaller magnitude when both have the same sign, else zero (a tie
// returns b).
template <typename T>
__device__ __forceinline__ T minmod(T a, T b)
{
    if (a > T(0) && b > T(0)) return a < b ? a : b;
    if (a < T(0) && b < T(0)) return a > b ? a : b;
    return T(0);
}

// Limited difference of a pair (p, q) of fields that travel along one axis as p + q and p - q:
// with forward differences fp, fq and backward differences bp, bq (each times the cell width),
// the limited central differences (times twice the cell width) are S + R and S - R, where
// S = minmod(fp + fq, bp + bq) and R = minmod(fp - fq, bp - bq).
template <typename T>
__device__ __forceinline__ void limit_pair(T fp, T fq, T bp, T bq, T &dp, T &dq)
{
    const T S = minmod(fp + fq, bp + bq), Rr = minmod(fp - fq, bp - bq);
    dp = S + Rr;
    dq = S - Rr;
}

// ------------------------------------------------------------------ sparse face operators
// phi = K0 w + mE KE w + mH KH w for the face orientation described by the table struct P
// (callers pass mE, mH as the SUM of the two cells' 1/eps, 1/mu: the host halves KE, KH)
// (gks_pattern.h); the loops unroll into straight-line FMAs on the structural non-zeros.
// K points to the coefficients (a ConstPtr from scalar_ptr).
// K0 is applied in chunks of CH entries: the coefficients of a chunk are loaded only once the
// previous chunk has started, so at most two chunks' scalar registers are live.  12 suits most
// kernels; a kernel whose scalar registers spill with 12 passes a smaller chunk (FP64 takes two
// scalar registers per coefficient).
// HM = false: the operator's KH part is folded into K0 on the host (every face has 1/mu = 1), so
// the KH products and their scaling are skipped and mH is unused.
template <typename P, int CH = 12, bool HM = true, typename T, int NF, int NIN, typename Op>
__device__ __forceinline__ void apply_op(const T (&w)[NIN], T mE, T mH, Op K, T (&phi)[NF])
{
    T a[NF], e[NF], h[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) a[r] = e[r] = h[r] = T(0);
#pragma unroll
    for (int q = 0; q < P::N0; ++q) {
        if (q % CH == 1 && q + CH - 1 < P::N0) asm volatile("" : "+s"(K) : "v"(a[P::R0[q - 1]]));
        a[P::R0[q]] = fma(K->k0[q], w[P::C0[q]], a[P::R0[q]]);
    }
    // the material parts' coefficients are loaded once K0's have been used
    asm volatile("" : "+s"(K) : "v"(a[P::R0[P::N0 - 1]]));
#pragma unroll
    for (int q = 0; q < P::NE; ++q) e[P::RE[q]] = fma(K->ke[q], w[P::CE[q]], e[P::RE[q]]);
    if constexpr (HM) {
#pragma unroll
        for (int q = 0; q < P::NH; ++q) h[P::RH[q]] = fma(K->kh[q], w[P::CH[q]], h[P::RH[q]]);
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        T v = a[r];
        if ((P::EROWS >> r) & 1u) v = fma(mE, e[r], v);
        if (HM && ((P::HROWS >> r) & 1u)) v = fma(mH, h[r], v);
        phi[r] = v;
    }
}

// As apply_op, and also returns the material parts e = KE w and h = KH w (per output row; the
// rows outside EROWS / HROWS are zero): phi = K0 w + mE e + mH h.
template <typename P, int CH = 12, bool HM = true, typename T, int NF, int NIN, typename Op>
__device__ __forceinline__ void apply_op_parts(const T (&w)[NIN], T mE, T mH, Op K, T (&phi)[NF], T (&e)[NF],
                                               T (&h)[NF])
{
    T a[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) a[r] = e[r] = h[r] = T(0);
#pragma unroll
    for (int q = 0; q < P::N0; ++q) {
        if (q % CH == 1 && q + CH - 1 < P::N0) asm volatile("" : "+s"(K) : "v"(a[P::R0[q - 1]]));
        a[P::R0[q]] = fma(K->k0[q], w[P::C0[q]], a[P::R0[q]]);
    }
    asm volatile("" : "+s"(K) : "v"(a[P::R0[P::N0 - 1]]));
#pragma unroll
    for (int q = 0; q < P::NE; ++q) e[P::RE[q]] = fma(K->ke[q], w[P::CE[q]], e[P::RE[q]]);
    if constexpr (HM) {
#pragma unroll
        for (int q = 0; q < P::NH; ++q) h[P::RH[q]] = fma(K->kh[q], w[P::CH[q]], h[P::RH[q]]);
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        T v = a[r];
        if ((P::EROWS >> r) & 1u) v = fma(mE, e[r], v);
        if (HM && ((P::HROWS >> r) & 1u)) v = fma(mH, h[r], v);
        phi[r] = v;
    }
}

// Transpose: wbar += K(mE, mH)^T abar (HM = false: KH folded into K0, as in apply_op).
template <typename P, int CH = 12, bool HM = true, typename T, int NF, int NIN, typename Op>
__device__ __forceinline__ void apply_op_transpose(const T (&abar)[NF], T mE, T mH, Op K, T (&wbar)[NIN])
{
    T ae[NF], ah[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        ae[r] = mE * abar[r];
        ah[r] = mH * abar[r];
    }
#pragma unroll
    for (int q = 0; q < P::N0; ++q) {
        if (q % CH == 1 && q + CH - 1 < P::N0) asm volatile("" : "+s"(K) : "v"(wbar[P::C0[q - 1]]));
        wbar[P::C0[q]] = fma(K->k0[q], abar[P::R0[q]], wbar[P::C0[q]]);
    }
    asm volatile("" : "+s"(K) : "v"(wbar[P::C0[P::N0 - 1]]));
#pragma unroll
    for (int q = 0; q < P::NE; ++q) wbar[P::CE[q]] = fma(K->ke[q], ae[P::RE[q]], wbar[P::CE[q]]);
    if constexpr (HM) {
#pragma unroll
        for (int q = 0; q < P::NH; ++q) wbar[P::CH[q]] = fma(K->kh[q], ah[P::RH[q]], wbar[P::CH[q]]);
    }
}

// apply_op_parts and apply_op_transpose in one pass over the coefficients: every coefficient is
// loaded once and used for both products (phi = K0 w + mE e + mH h with its parts e, h; and
// wbar += K(mE, mH)^T abar), which halves the scalar loads of a face that needs both.
template <typename P, int CH = 12, bool HM = true, typename T, int NF, int NIN, typename Op>
__device__ __forceinline__ void apply_op_both(const T (&w)[NIN], const T (&abar)[NF], T mE, T mH, Op K, T (&phi)[NF],
                                              T (&e)[NF], T (&h)[NF], T (&wbar)[NIN])
{
    T a[NF], ae[NF], ah[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        a[r] = e[r] = h[r] = T(0);
        ae[r] = mE * abar[r];
        ah[r] = mH * abar[r];
    }
#pragma unroll
    for (int q = 0; q < P::N0; ++q) {
        if (q % CH == 1 && q + CH - 1 < P::N0) asm volatile("" : "+s"(K) : "v"(a[P::R0[q - 1]]));
        const T k = K->k0[q];
        a[P::R0[q]] = fma(k, w[P::C0[q]], a[P::R0[q]]);
        wbar[P::C0[q]] = fma(k, abar[P::R0[q]], wbar[P::C0[q]]);
    }
    asm volatile("" : "+s"(K) : "v"(a[P::R0[P::N0 - 1]]));
#pragma unroll
    for (int q = 0; q < P::NE; ++q) {
        const T k = K->ke[q];
        e[P::RE[q]] = fma(k, w[P::CE[q]], e[P::RE[q]]);
        wbar[P::CE[q]] = fma(k, ae[P::RE[q]], wbar[P::CE[q]]);
    }
    if constexpr (HM) {
#pragma unroll
        for (int q = 0; q < P::NH; ++q) {
            const T k = K->kh[q];
            h[P::RH[q]] = fma(k, w[P::CH[q]], h[P::RH[q]]);
            wbar[P::CH[q]] = fma(k, ah[P::RH[q]], wbar[P::CH[q]]);
        }
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        T v = a[r];
        if ((P::EROWS >> r) & 1u) v = fma(mE, e[r], v);
        if (HM && ((P::HROWS >> r) & 1u)) v = fma(mH, h[r], v);
        phi[r] = v;
    }
}

// abar . (KE w) and abar . (KH w): derivatives of abar . phi with respect to mE and mH.
template <typename P, typename T, int NF, int NIN, typename Op>
__device__ __forceinline__ void material_sens(const T (&abar)[NF], const T (&w)[NIN], Op K, T &dE, T &dH)
{
    T e = T(0), h = T(0);
#pragma unroll
    for (int q = 0; q < P::NE; ++q) e = fma(K->ke[q] * abar[P::RE[q]], w[P::CE[q]], e);
#pragma unroll
    for (int q = 0; q < P::NH; ++q) h = fma(K->kh[q] * abar[P::RH[q]], w[P::CH[q]], h);
    dE = e;
    dH = h;
}

// Work distribution: workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that every XCD receives one contiguous range of logical workgroups,
// i.e. a contiguous band of tiles whose shared halo rows and columns stay in that XCD's L2.
__device__ __forceinline__ int xcd_logical_block()
{
    const int nb = gridDim.x, bid = blockIdx.x;
    const int x = bid % 8, per = nb / 8, rem = nb % 8;
    return x * per + min(x, rem) + bid / 8;
}

}  // namespace gks
