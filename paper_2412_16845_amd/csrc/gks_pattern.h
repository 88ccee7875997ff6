// Sparsity tables of the face operators (host and device), one struct per face orientation.
// Cartesian faces take global-frame inputs
//   TM (18): [UL UR dnL dtL dnR dtR] x (Ez, Hx, Hy)
//   TP (24): [UL UR dnL dtL dnR dtR] x (Ez, Hx, Hy, psi)   (TM with the PHM potential psi)
//   EM (48): [UL UR dnL dt1L dt2L dnR dt1R dt2R] x (Ex, Ey, Ez, Hx, Hy, Hz)
//   EP (64): [UL UR dnL dt1L dt2L dnR dt1R dt2R] x (Ex, Ey, Ez, Hx, Hy, Hz, phi, psi)   (PHM)
// with dn the central difference along the face normal and dt1, dt2 along the other axes in
// increasing order; rows are the global output components.  PatTri takes face-frame inputs
// [Ul Ur s1l s2l s1r s2r] x (Ez, Hn, Ht) (triangle faces).  N0/NE/NH count the entries of K0,
// KE (times 1/eps) and KH (times 1/mu); EROWS/HROWS flag the rows KE/KH reach.  Context
// creation probes the closed-form flux and verifies that every other entry is exactly zero.
#pragma once
#include <cstdint>

#include "gks_internal.h"

namespace gks {

struct PatTMx {
    static constexpr int N0 = 24;
    static constexpr uint8_t R0[24] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2};
    static constexpr uint8_t C0[24] = {0, 2, 3, 5, 6, 8, 10, 12, 14, 16, 1, 4, 7, 9, 13, 15, 0, 2, 3, 5, 6, 8, 12, 14};
    static constexpr int NE = 6;
    static constexpr uint8_t RE[6] = {2, 2, 2, 2, 2, 2};
    static constexpr uint8_t CE[6] = {6, 8, 10, 12, 14, 16};
    static constexpr uint32_t EROWS = 0x4u;
    static constexpr int NH = 4;
    static constexpr uint8_t RH[4] = {0, 0, 0, 0};
    static constexpr uint8_t CH[4] = {6, 8, 12, 14};
    static constexpr uint32_t HROWS = 0x1u;
};

struct PatTMy {
    static constexpr int N0 = 24;
    static constexpr uint8_t R0[24] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2};
    static constexpr uint8_t C0[24] = {0, 1, 3, 4, 6, 7, 11, 12, 13, 17, 0, 1, 3, 4, 6, 7, 12, 13, 2, 5, 8, 9, 14, 15};
    static constexpr int NE = 6;
    static constexpr uint8_t RE[6] = {1, 1, 1, 1, 1, 1};
    static constexpr uint8_t CE[6] = {6, 7, 11, 12, 13, 17};
    static constexpr uint32_t EROWS = 0x2u;
    static constexpr int NH = 4;
    static constexpr uint8_t RH[4] = {0, 0, 0, 0};
    static constexpr uint8_t CH[4] = {6, 7, 12, 13};
    static constexpr uint32_t HROWS = 0x1u;
};

struct PatTPx {
    static constexpr int N0 = 42;
    static constexpr uint8_t R0[42] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3};
    static constexpr uint8_t C0[42] = {0, 2, 4, 6, 8, 10, 13, 16, 18, 21, 1, 3, 5, 7, 9, 11, 12, 14, 17, 19, 20, 22, 0, 2, 4, 6, 8, 10, 15, 16, 18, 23, 1, 3, 5, 7, 9, 11, 14, 17, 19, 22};
    static constexpr int NE = 8;
    static constexpr uint8_t RE[8] = {2, 2, 2, 2, 2, 2, 2, 2};
    static constexpr uint8_t CE[8] = {8, 10, 13, 15, 16, 18, 21, 23};
    static constexpr uint32_t EROWS = 0x4u;
    static constexpr int NH = 16;
    static constexpr uint8_t RH[16] = {0, 0, 0, 0, 0, 0, 0, 0, 3, 3, 3, 3, 3, 3, 3, 3};
    static constexpr uint8_t CH[16] = {8, 10, 13, 15, 16, 18, 21, 23, 9, 11, 12, 14, 17, 19, 20, 22};
    static constexpr uint32_t HROWS = 0x9u;
};

struct PatTPy {
    static constexpr int N0 = 42;
    static constexpr uint8_t R0[42] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3};
    static constexpr uint8_t C0[42] = {0, 1, 4, 5, 8, 9, 14, 16, 17, 22, 0, 1, 4, 5, 8, 9, 15, 16, 17, 23, 2, 3, 6, 7, 10, 11, 12, 13, 18, 19, 20, 21, 2, 3, 6, 7, 10, 11, 13, 18, 19, 21};
    static constexpr int NE = 8;
    static constexpr uint8_t RE[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr uint8_t CE[8] = {8, 9, 14, 15, 16, 17, 22, 23};
    static constexpr uint32_t EROWS = 0x2u;
    static constexpr int NH = 16;
    static constexpr uint8_t RH[16] = {0, 0, 0, 0, 0, 0, 0, 0, 3, 3, 3, 3, 3, 3, 3, 3};
    static constexpr uint8_t CH[16] = {8, 9, 14, 15, 16, 17, 22, 23, 10, 11, 12, 13, 18, 19, 20, 21};
    static constexpr uint32_t HROWS = 0x9u;
};

struct PatEMx {
    static constexpr int N0 = 80;
    static constexpr uint8_t R0[80] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5};
    static constexpr uint8_t C0[80] = {0, 6, 12, 20, 22, 23, 25, 28, 29, 30, 38, 40, 41, 43, 46, 47, 1, 5, 7, 11, 13, 17, 21, 27, 31, 35, 39, 45, 2, 4, 8, 10, 14, 16, 21, 27, 32, 34, 39, 45, 3, 9, 15, 19, 20, 23, 25, 26, 28, 33, 37, 38, 41, 43, 44, 46, 2, 4, 8, 10, 14, 16, 18, 24, 32, 34, 36, 42, 1, 5, 7, 11, 13, 17, 18, 24, 31, 35, 36, 42};
    static constexpr int NE = 12;
    static constexpr uint8_t RE[12] = {4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5};
    static constexpr uint8_t CE[12] = {14, 16, 21, 32, 34, 39, 13, 17, 27, 31, 35, 45};
    static constexpr uint32_t EROWS = 0x30u;
    static constexpr int NH = 12;
    static constexpr uint8_t RH[12] = {1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2};
    static constexpr uint8_t CH[12] = {13, 17, 18, 31, 35, 36, 14, 16, 24, 32, 34, 42};
    static constexpr uint32_t HROWS = 0x6u;
};

struct PatEMy {
    static constexpr int N0 = 80;
    static constexpr uint8_t R0[80] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5};
    static constexpr uint8_t C0[80] = {0, 5, 6, 11, 12, 17, 22, 28, 30, 35, 40, 46, 1, 7, 13, 20, 21, 23, 24, 27, 29, 31, 38, 39, 41, 42, 45, 47, 2, 3, 8, 9, 14, 15, 22, 28, 32, 33, 40, 46, 2, 3, 8, 9, 14, 15, 19, 25, 32, 33, 37, 43, 4, 10, 16, 18, 20, 23, 24, 26, 27, 34, 36, 38, 41, 42, 44, 45, 0, 5, 6, 11, 12, 17, 19, 25, 30, 35, 37, 43};
    static constexpr int NE = 12;
    static constexpr uint8_t RE[12] = {3, 3, 3, 3, 3, 3, 5, 5, 5, 5, 5, 5};
    static constexpr uint8_t CE[12] = {14, 15, 22, 32, 33, 40, 12, 17, 28, 30, 35, 46};
    static constexpr uint32_t EROWS = 0x28u;
    static constexpr int NH = 12;
    static constexpr uint8_t RH[12] = {0, 0, 0, 0, 0, 0, 2, 2, 2, 2, 2, 2};
    static constexpr uint8_t CH[12] = {12, 17, 19, 30, 35, 37, 14, 15, 25, 32, 33, 43};
    static constexpr uint32_t HROWS = 0x5u;
};

struct PatEMz {
    static constexpr int N0 = 80;
    static constexpr uint8_t R0[80] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5};
    static constexpr uint8_t C0[80] = {0, 4, 6, 10, 12, 16, 23, 29, 30, 34, 41, 47, 1, 3, 7, 9, 13, 15, 23, 29, 31, 33, 41, 47, 2, 8, 14, 19, 21, 22, 24, 27, 28, 32, 37, 39, 40, 42, 45, 46, 1, 3, 7, 9, 13, 15, 20, 26, 31, 33, 38, 44, 0, 4, 6, 10, 12, 16, 20, 26, 30, 34, 38, 44, 5, 11, 17, 18, 19, 22, 24, 25, 27, 35, 36, 37, 40, 42, 43, 45};
    static constexpr int NE = 12;
    static constexpr uint8_t RE[12] = {3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4};
    static constexpr uint8_t CE[12] = {13, 15, 23, 31, 33, 41, 12, 16, 29, 30, 34, 47};
    static constexpr uint32_t EROWS = 0x18u;
    static constexpr int NH = 12;
    static constexpr uint8_t RH[12] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1};
    static constexpr uint8_t CH[12] = {12, 16, 20, 30, 34, 38, 13, 15, 26, 31, 33, 44};
    static constexpr uint32_t HROWS = 0x3u;
};

struct PatEPx {
    static constexpr int N0 = 168;
    static constexpr uint8_t R0[168] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7};
    static constexpr uint8_t C0[168] = {0, 6, 8, 14, 16, 22, 25, 26, 28, 29, 33, 34, 36, 37, 40, 46, 49, 50, 52, 53, 57, 58, 60, 61, 1, 5, 9, 13, 17, 21, 27, 30, 31, 32, 35, 38, 41, 45, 51, 54, 55, 56, 59, 62, 2, 4, 10, 12, 18, 20, 24, 27, 30, 35, 38, 39, 42, 44, 48, 51, 54, 59, 62, 63, 3, 7, 11, 15, 19, 23, 25, 26, 28, 29, 33, 34, 36, 37, 43, 47, 49, 50, 52, 53, 57, 58, 60, 61, 2, 4, 10, 12, 18, 20, 24, 30, 31, 32, 35, 39, 42, 44, 48, 54, 55, 56, 59, 63, 1, 5, 9, 13, 17, 21, 24, 27, 31, 32, 38, 39, 41, 45, 48, 51, 55, 56, 62, 63, 0, 6, 8, 14, 16, 22, 25, 26, 28, 33, 34, 37, 40, 46, 49, 50, 52, 57, 58, 61, 3, 7, 11, 15, 19, 23, 25, 28, 29, 34, 36, 37, 43, 47, 49, 52, 53, 58, 60, 61};
    static constexpr int NE = 36;
    static constexpr uint8_t RE[36] = {4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6};
    static constexpr uint8_t CE[36] = {18, 20, 27, 31, 32, 38, 42, 44, 51, 55, 56, 62, 17, 21, 24, 30, 35, 39, 41, 45, 48, 54, 59, 63, 16, 22, 25, 29, 34, 36, 40, 46, 49, 53, 58, 60};
    static constexpr uint32_t EROWS = 0x70u;
    static constexpr int NH = 36;
    static constexpr uint8_t RH[36] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7};
    static constexpr uint8_t CH[36] = {17, 21, 24, 30, 35, 39, 41, 45, 48, 54, 59, 63, 18, 20, 27, 31, 32, 38, 42, 44, 51, 55, 56, 62, 19, 23, 26, 28, 33, 37, 43, 47, 50, 52, 57, 61};
    static constexpr uint32_t HROWS = 0x86u;
};

struct PatEPy {
    static constexpr int N0 = 168;
    static constexpr uint8_t R0[168] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7};
    static constexpr uint8_t C0[168] = {0, 5, 8, 13, 16, 21, 28, 30, 31, 33, 36, 38, 40, 45, 52, 54, 55, 57, 60, 62, 1, 6, 9, 14, 17, 22, 24, 26, 27, 29, 32, 34, 35, 37, 41, 46, 48, 50, 51, 53, 56, 58, 59, 61, 2, 3, 10, 11, 18, 19, 25, 28, 30, 36, 38, 39, 42, 43, 49, 52, 54, 60, 62, 63, 2, 3, 10, 11, 18, 19, 25, 30, 31, 33, 36, 39, 42, 43, 49, 54, 55, 57, 60, 63, 4, 7, 12, 15, 20, 23, 24, 26, 27, 29, 32, 34, 35, 37, 44, 47, 48, 50, 51, 53, 56, 58, 59, 61, 0, 5, 8, 13, 16, 21, 25, 28, 31, 33, 38, 39, 40, 45, 49, 52, 55, 57, 62, 63, 1, 6, 9, 14, 17, 22, 24, 26, 27, 32, 34, 37, 41, 46, 48, 50, 51, 56, 58, 61, 4, 7, 12, 15, 20, 23, 24, 27, 29, 34, 35, 37, 44, 47, 48, 51, 53, 58, 59, 61};
    static constexpr int NE = 36;
    static constexpr uint8_t RE[36] = {3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6};
    static constexpr uint8_t CE[36] = {18, 19, 28, 31, 33, 38, 42, 43, 52, 55, 57, 62, 16, 21, 25, 30, 36, 39, 40, 45, 49, 54, 60, 63, 17, 22, 24, 29, 34, 35, 41, 46, 48, 53, 58, 59};
    static constexpr uint32_t EROWS = 0x68u;
    static constexpr int NH = 36;
    static constexpr uint8_t RH[36] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7};
    static constexpr uint8_t CH[36] = {16, 21, 25, 30, 36, 39, 40, 45, 49, 54, 60, 63, 18, 19, 28, 31, 33, 38, 42, 43, 52, 55, 57, 62, 20, 23, 26, 27, 32, 37, 44, 47, 50, 51, 56, 61};
    static constexpr uint32_t HROWS = 0x85u;
};

struct PatEPz {
    static constexpr int N0 = 168;
    static constexpr uint8_t R0[168] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7};
    static constexpr uint8_t C0[168] = {0, 4, 8, 12, 16, 20, 29, 30, 31, 34, 37, 38, 40, 44, 53, 54, 55, 58, 61, 62, 1, 3, 9, 11, 17, 19, 26, 29, 30, 37, 38, 39, 41, 43, 50, 53, 54, 61, 62, 63, 2, 6, 10, 14, 18, 22, 24, 25, 27, 28, 32, 33, 35, 36, 42, 46, 48, 49, 51, 52, 56, 57, 59, 60, 1, 3, 9, 11, 17, 19, 26, 30, 31, 34, 37, 39, 41, 43, 50, 54, 55, 58, 61, 63, 0, 4, 8, 12, 16, 20, 26, 29, 31, 34, 38, 39, 40, 44, 50, 53, 55, 58, 62, 63, 5, 7, 13, 15, 21, 23, 24, 25, 27, 28, 32, 33, 35, 36, 45, 47, 48, 49, 51, 52, 56, 57, 59, 60, 2, 6, 10, 14, 18, 22, 24, 25, 27, 32, 33, 36, 42, 46, 48, 49, 51, 56, 57, 60, 5, 7, 13, 15, 21, 23, 24, 27, 28, 33, 35, 36, 45, 47, 48, 51, 52, 57, 59, 60};
    static constexpr int NE = 36;
    static constexpr uint8_t RE[36] = {3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6};
    static constexpr uint8_t CE[36] = {17, 19, 29, 31, 34, 38, 41, 43, 53, 55, 58, 62, 16, 20, 26, 30, 37, 39, 40, 44, 50, 54, 61, 63, 18, 22, 24, 28, 33, 35, 42, 46, 48, 52, 57, 59};
    static constexpr uint32_t EROWS = 0x58u;
    static constexpr int NH = 36;
    static constexpr uint8_t RH[36] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7, 7};
    static constexpr uint8_t CH[36] = {16, 20, 26, 30, 37, 39, 40, 44, 50, 54, 61, 63, 17, 19, 29, 31, 34, 38, 41, 43, 53, 55, 58, 62, 21, 23, 25, 27, 32, 36, 45, 47, 49, 51, 56, 60};
    static constexpr uint32_t HROWS = 0x83u;
};

struct PatTri {
    static constexpr int N0 = 24;
    static constexpr uint8_t R0[24] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2};
    static constexpr uint8_t C0[24] = {0, 2, 3, 5, 6, 8, 10, 12, 14, 16, 1, 4, 7, 9, 13, 15, 0, 2, 3, 5, 6, 8, 12, 14};
    static constexpr int NE = 6;
    static constexpr uint8_t RE[6] = {2, 2, 2, 2, 2, 2};
    static constexpr uint8_t CE[6] = {6, 8, 10, 12, 14, 16};
    static constexpr uint32_t EROWS = 0x4u;
    static constexpr int NH = 4;
    static constexpr uint8_t RH[4] = {0, 0, 0, 0};
    static constexpr uint8_t CH[4] = {6, 8, 12, 14};
    static constexpr uint32_t HROWS = 0x1u;
};

// The EM tables with the 1/mu part folded into K0, for vacuum 1/mu: K0's entries, then those of
// KH that K0 does not have (the host adds KH onto K0 there); KE unchanged.
struct PatEMxF {
    static constexpr int N0 = 84;
    static constexpr uint8_t R0[84] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 1, 1, 2, 2};
    static constexpr uint8_t C0[84] = {0, 6, 12, 20, 22, 23, 25, 28, 29, 30, 38, 40, 41, 43, 46, 47, 1, 5, 7, 11, 13, 17, 21, 27, 31, 35, 39, 45, 2, 4, 8, 10, 14, 16, 21, 27, 32, 34, 39, 45, 3, 9, 15, 19, 20, 23, 25, 26, 28, 33, 37, 38, 41, 43, 44, 46, 2, 4, 8, 10, 14, 16, 18, 24, 32, 34, 36, 42, 1, 5, 7, 11, 13, 17, 18, 24, 31, 35, 36, 42, 18, 36, 24, 42};
    static constexpr int NE = PatEMx::NE;
    static constexpr uint8_t RE[12] = {4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5};
    static constexpr uint8_t CE[12] = {14, 16, 21, 32, 34, 39, 13, 17, 27, 31, 35, 45};
    static constexpr uint32_t EROWS = PatEMx::EROWS;
    static constexpr int NH = 0;
    static constexpr uint8_t RH[1] = {0};
    static constexpr uint8_t CH[1] = {0};
    static constexpr uint32_t HROWS = 0;
};

struct PatEMyF {
    static constexpr int N0 = 84;
    static constexpr uint8_t R0[84] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 0, 0, 2, 2};
    static constexpr uint8_t C0[84] = {0, 5, 6, 11, 12, 17, 22, 28, 30, 35, 40, 46, 1, 7, 13, 20, 21, 23, 24, 27, 29, 31, 38, 39, 41, 42, 45, 47, 2, 3, 8, 9, 14, 15, 22, 28, 32, 33, 40, 46, 2, 3, 8, 9, 14, 15, 19, 25, 32, 33, 37, 43, 4, 10, 16, 18, 20, 23, 24, 26, 27, 34, 36, 38, 41, 42, 44, 45, 0, 5, 6, 11, 12, 17, 19, 25, 30, 35, 37, 43, 19, 37, 25, 43};
    static constexpr int NE = PatEMy::NE;
    static constexpr uint8_t RE[12] = {3, 3, 3, 3, 3, 3, 5, 5, 5, 5, 5, 5};
    static constexpr uint8_t CE[12] = {14, 15, 22, 32, 33, 40, 12, 17, 28, 30, 35, 46};
    static constexpr uint32_t EROWS = PatEMy::EROWS;
    static constexpr int NH = 0;
    static constexpr uint8_t RH[1] = {0};
    static constexpr uint8_t CH[1] = {0};
    static constexpr uint32_t HROWS = 0;
};

struct PatEMzF {
    static constexpr int N0 = 84;
    static constexpr uint8_t R0[84] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 0, 0, 1, 1};
    static constexpr uint8_t C0[84] = {0, 4, 6, 10, 12, 16, 23, 29, 30, 34, 41, 47, 1, 3, 7, 9, 13, 15, 23, 29, 31, 33, 41, 47, 2, 8, 14, 19, 21, 22, 24, 27, 28, 32, 37, 39, 40, 42, 45, 46, 1, 3, 7, 9, 13, 15, 20, 26, 31, 33, 38, 44, 0, 4, 6, 10, 12, 16, 20, 26, 30, 34, 38, 44, 5, 11, 17, 18, 19, 22, 24, 25, 27, 35, 36, 37, 40, 42, 43, 45, 20, 38, 26, 44};
    static constexpr int NE = PatEMz::NE;
    static constexpr uint8_t RE[12] = {3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4};
    static constexpr uint8_t CE[12] = {13, 15, 23, 31, 33, 41, 12, 16, 29, 30, 34, 47};
    static constexpr uint32_t EROWS = PatEMz::EROWS;
    static constexpr int NH = 0;
    static constexpr uint8_t RH[1] = {0};
    static constexpr uint8_t CH[1] = {0};
    static constexpr uint32_t HROWS = 0;
};

// Tetrahedral faces: face-frame inputs [Ul Ur s1l s2l s3l s1r s2r s3r] x (Ex .. Hz) have the
// sparsity of the Cartesian x-face table.
using PatTet = PatEMx;

// Triangle faces with the PHM potential psi: face-frame inputs [Ul Ur s1l s2l s1r s2r] x (Ez, Hn,
// Ht, psi) have the sparsity of the Cartesian x-face table (as PatTri has that of PatTMx).
using PatTriP = PatTPx;

static_assert(PatTMx::N0 == TM_N0 && PatTMx::NE == TM_NE && PatTMx::NH == TM_NH, "TM table size");
static_assert(PatTMy::N0 == TM_N0 && PatTMy::NE == TM_NE && PatTMy::NH == TM_NH, "TM table size");
static_assert(PatTri::N0 == TM_N0 && PatTri::NE == TM_NE && PatTri::NH == TM_NH, "TM table size");
static_assert(PatTPx::N0 == TP_N0 && PatTPx::NE == TP_NE && PatTPx::NH == TP_NH, "TP table size");
static_assert(PatTPy::N0 == TP_N0 && PatTPy::NE == TP_NE && PatTPy::NH == TP_NH, "TP table size");
static_assert(PatEPx::N0 == EP_N0 && PatEPx::NE == EP_NE && PatEPx::NH == EP_NH, "EP table size");
static_assert(PatEPy::N0 == EP_N0 && PatEPy::NE == EP_NE && PatEPy::NH == EP_NH, "EP table size");
static_assert(PatEPz::N0 == EP_N0 && PatEPz::NE == EP_NE && PatEPz::NH == EP_NH, "EP table size");
static_assert(PatEMx::N0 == EM_N0 && PatEMx::NE == EM_NE && PatEMx::NH == EM_NH, "EM table size");
static_assert(PatEMy::N0 == EM_N0 && PatEMy::NE == EM_NE && PatEMy::NH == EM_NH, "EM table size");
static_assert(PatEMz::N0 == EM_N0 && PatEMz::NE == EM_NE && PatEMz::NH == EM_NH, "EM table size");
static_assert(PatEMxF::N0 == EMF_N0 && PatEMyF::N0 == EMF_N0 && PatEMzF::N0 == EMF_N0, "folded EM table size");

}  // namespace gks
