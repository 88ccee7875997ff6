// Sparsity tables of the Cartesian face operators (host and device).  Inputs, local frame:
//   TM2D (18): [UL UR d1L d2L d1R d2R] x (Ez, Hx, Hy)
//   EM3D (48): [UL UR d1L d2L d3L d1R d2R d3R] x (Ex, Ey, Ez, Hx, Hy, Hz)
// Rows are the output components.  The same TM tables serve the triangle face operator
// (inputs [Ul Ur s1l s2l s1r s2r]).  Context creation verifies that every entry of the probed
// operators outside these tables is exactly zero.
#pragma once
#include <cstdint>

#include "gks_internal.h"

namespace gks {

constexpr uint8_t TM_R0[TM_N0] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2};
constexpr uint8_t TM_C0[TM_N0] = {0, 2, 3, 5, 6, 8, 10, 12, 14, 16, 1, 4, 7, 9, 13, 15, 0, 2, 3, 5, 6, 8, 12, 14};
constexpr uint8_t TM_RE[TM_NE] = {2, 2, 2, 2, 2, 2};
constexpr uint8_t TM_CE[TM_NE] = {6, 8, 10, 12, 14, 16};
constexpr uint8_t TM_RH[TM_NH] = {0, 0, 0, 0};
constexpr uint8_t TM_CH[TM_NH] = {6, 8, 12, 14};

constexpr uint8_t EM_R0[EM_N0] = {
    0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2,
    3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5};
constexpr uint8_t EM_C0[EM_N0] = {
    0,  6,  12, 20, 22, 23, 25, 28, 29, 30, 38, 40, 41, 43, 46, 47, 1,  5,  7,  11, 13, 17, 21, 27, 31, 35, 39, 45,
    2,  4,  8,  10, 14, 16, 21, 27, 32, 34, 39, 45, 3,  9,  15, 19, 20, 23, 25, 26, 28, 33, 37, 38, 41, 43, 44, 46,
    2,  4,  8,  10, 14, 16, 18, 24, 32, 34, 36, 42, 1,  5,  7,  11, 13, 17, 18, 24, 31, 35, 36, 42};
constexpr uint8_t EM_RE[EM_NE] = {4, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5};
constexpr uint8_t EM_CE[EM_NE] = {14, 16, 21, 32, 34, 39, 13, 17, 27, 31, 35, 45};
constexpr uint8_t EM_RH[EM_NH] = {1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2};
constexpr uint8_t EM_CH[EM_NH] = {13, 17, 18, 31, 35, 36, 14, 16, 24, 32, 34, 42};

// Output rows reached by KE / KH (bit r set = row r has entries).
constexpr uint32_t TM_EROWS = 1u << 2, TM_HROWS = 1u << 0;
constexpr uint32_t EM_EROWS = (1u << 4) | (1u << 5), EM_HROWS = (1u << 1) | (1u << 2);

}  // namespace gks
