// Internal declarations shared by the host runtime and the kernels of libgks.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/gks.h"

namespace gks {

// ------------------------------------------------------------------ sparse face operators
// Structurally non-zero entries (row = output component, col = input index) of the face
// operators K0 (material independent), KE (times 1/eps_s) and KH (times 1/mu_s).
struct Pattern {
    int n0, nE, nH;
    const uint8_t *r0, *c0, *rE, *cE, *rH, *cH;
};
const Pattern &pattern_cart(int model, int axis);
const Pattern &pattern_cart_em_folded(int axis);
const Pattern &pattern_tri(int model);

constexpr int TM_N0 = 24, TM_NE = 6, TM_NH = 4;
constexpr int TP_N0 = 42, TP_NE = 8, TP_NH = 16;
constexpr int EM_N0 = 80, EM_NE = 12, EM_NH = 12;
constexpr int EP_N0 = 168, EP_NE = 36, EP_NH = 36;
constexpr int EMF_N0 = 84;   // EM with the 1/mu part folded into K0 (vacuum 1/mu)

void flux_coefficients(double dt, double tau, double C[5]);
// Face operator of an axis-aligned Cartesian face (normal +e_axis), global-frame inputs whose
// differences are dfac * h * slope; output (dt/h_axis) * F.  chi, gamma: PHM couplings.
bool cart_face_operator(int model, int axis, double c, double chi, double gamma, const double C[5],
                        const double h[3], double dfac, double *k0, double *ke, double *kh, char *err,
                        size_t errlen);
bool tri_face_operator(int model, double c, double chi, double gamma, const double C[5], double *k0, double *ke,
                       double *kh, char *err, size_t errlen);
// Face operator of a tetrahedral face: face-frame inputs [Ul Ur s1l s2l s3l s1r s2r s3r] x (Ex .. Hz),
// physical slopes along the face axes (PatTet); output dt * F~.
bool tet_face_operator(double c, const double C[5], double *k0, double *ke, double *kh, char *err, size_t errlen);
const Pattern &pattern_tet();

// Coefficients of one face orientation, in the storage precision T.
template <typename T, int N0, int NE, int NH>
struct FaceOp {
    T k0[N0];
    T ke[NE];
    T kh[NH];
};
template <typename T> using FaceOpTM = FaceOp<T, TM_N0, TM_NE, TM_NH>;
template <typename T> using FaceOpTP = FaceOp<T, TP_N0, TP_NE, TP_NH>;
template <typename T> using FaceOpEM = FaceOp<T, EM_N0, EM_NE, EM_NH>;
template <typename T> using FaceOpEP = FaceOp<T, EP_N0, EP_NE, EP_NH>;
template <typename T> using FaceOpEMF = FaceOp<T, EMF_N0, EM_NE, EM_NH>;



// Arguments of the Cartesian 2D TM step kernel.
template <typename T>
struct Cart2DArgs {
    const T *U;
    T *Unew;
    const T *epsinv;      // nullable: vacuum
    const T *muinv;       // nullable: vacuum
    int32_t nx, ny;
    int32_t batch;
    int32_t bc[4];        // x-, x+, y-, y+
    int32_t ntx, nty;     // strips per row; tile rows per band (one band per XCD)
    const int32_t *tiles; // device [NBANDS][nty][4]: batch item (-1: none), first row, end row,
                          // march downwards
    int32_t nfields;      // 3: (Ez, Hx, Hy); 4: (Ez, Hx, Hy, psi)
    const void *ops;      // device: x-face and y-face operators (FaceOpTM<T> or FaceOpTP<T>)
    int32_t src_row, src_col; // one point source applied inside the step (src_row < 0: none)
    double src_amp;           // its dt * S_z = -dt * J_z(t^n) (before the 1/eps factor)
    int32_t limiter;          // 0: central differences, 1: minmod-limited slopes
    double src_amp2;          // the paired kernel: the source amplitude of its second step
};

// Arguments of the Cartesian 3D (six-field) step kernel.
template <typename T>
struct Cart3DArgs {
    const T *U;
    T *Unew;
    const T *epsinv;      // nullable: vacuum
    const T *muinv;       // nullable: vacuum
    int32_t nx, ny, nz;
    int32_t batch;
    int32_t bc[6];        // x-, x+, y-, y+, z-, z+
    int32_t ntx, nty, ntz;   // workgroup tiles along x, y and z
    int32_t tile_z;          // planes per z tile
    int32_t nfields;         // 6: (Ex .. Hz); 8: (Ex .. Hz, phi, psi)
    const void *ops;         // device: x-, y- and z-face operators (FaceOpEM<T> or FaceOpEP<T>)
    int32_t limiter;         // 0: central differences, 1: minmod-limited slopes
};

// Triangle meshes: per cell the neighbour of each of its three face slots (-(1 + bc) on a
// boundary face) and TRI_GEO_ROWS rows of geometry, each an [ncell] array:
//   TG_NX + k, TG_NY + k   outward unit normal of slot k, k = 0..2 (the two cells of a face store
//                          exact negatives)
//   TG_LW + k              |l_k| / |Omega|
//   TG_AX + k, TG_AY + k   x_s - x_i, the midpoint of slot k minus the cell's centroid, k = 0, 1
//                          (slot 2: minus their sum, as the three offsets of a triangle add to zero)
//   TG_BX + k, TG_BY + k   x_s - x_nb, the midpoint minus the neighbour's centroid (0 on boundary
//                          faces), k = 0..2
//   TG_WX + k, TG_WY + k   gradient weight of slot k: grad U_i = sum_k W_k (U_k - U_i), with U_k
//                          the neighbour or the boundary ghost (Green-Gauss: W_k = n_k |l_k| /
//                          (2 |Omega|); least squares: W_k = M^-1 d_k, M = sum_k d_k d_k^T, d_k the
//                          neighbour's centroid or the centroid's mirror image minus x_i)
constexpr int TG_NX = 0, TG_NY = 3, TG_LW = 6, TG_AX = 9, TG_AY = 11, TG_BX = 13, TG_BY = 16, TG_WX = 19, TG_WY = 22;
constexpr int TRI_GEO_ROWS = 25;
// On the device the same values are stored with the x and y components of each vector side by
// side, so that a lane reads a vector with one 8-byte (16-byte in fp64) load: TRI_GEO_PAIRS
// arrays [pair][ncell][2] (TGP_N + k: normal of slot k; TGP_A + k: x_s - x_i of slot k = 0, 1;
// TGP_B + k: x_s - x_nb; TGP_W + k: gradient weight), then the three |l_k| / |Omega| arrays
// [k][ncell] at element offset 2 TRI_GEO_PAIRS ncell.
constexpr int TGP_N = 0, TGP_A = 3, TGP_B = 5, TGP_W = 8, TRI_GEO_PAIRS = 11;
struct TriGeometry {
    int64_t ncell = 0;
    std::vector<int32_t> nb;     // [3][ncell]
    std::vector<double> geo;     // [TRI_GEO_ROWS][ncell]
    std::vector<double> area;    // [ncell]
    double rmin = 0;             // smallest inradius 2|Omega| / perimeter
};
bool build_tri_geometry(const gks_mesh_desc *m, int gradient, TriGeometry &g, char *err, size_t errlen);

// Tetrahedral meshes (kind GKS_TET3D, six fields).  Per cell, [row][ncell]:
//   TC_W + 3k + d   Green-Gauss weight of face slot k, component d: n_k |l_k| / (2 |Omega|)
//   TC_N + 3k + d   outward unit normal of slot k
//   TC_IVOL         1 / |Omega|
// and int32 [4][ncell]: nb (neighbour or -(1 + bc)), cf (face id + 1, negative on the
// neighbour's side).  Per face, [row][nface]:
//   TF_N + d        unit normal owner -> neighbour
//   TF_A, TF_B      n3^2 / (1 + n1), n2 n3 / (1 + n1) (0, 0 when n1 = -1): T' follows from n, a, b
//   TF_AREA         |l|
//   TF_DL + d       x_s - x_L;  TF_DR + d  x_s - x_R (0 on boundary faces)
// and int32 [2][nface]: owner, neighbour or -(1 + bc).
constexpr int TC_W = 0, TC_N = 12, TC_IVOL = 24, TET_CGEO_ROWS = 25;
constexpr int TF_N = 0, TF_A = 3, TF_B = 4, TF_AREA = 5, TF_DL = 6, TF_DR = 9, TET_FGEO_ROWS = 12;
struct TetGeometry {
    int64_t ncell = 0, nface = 0;
    std::vector<int32_t> nb, cf;   // [4][ncell]
    std::vector<int32_t> fc;       // [2][nface] interleaved: owner, neighbour per face
    std::vector<double> cgeo;      // [TET_CGEO_ROWS][ncell]
    std::vector<double> fgeo;      // [TET_FGEO_ROWS][nface]
    std::vector<double> vol;       // [ncell]
    double rmin = 0;               // smallest inradius 3|Omega| / surface
};
bool build_tet_geometry(const gks_mesh_desc *m, TetGeometry &g, char *err, size_t errlen);

template <typename T>
struct TetArgs {
    const T *U;
    T *Unew;
    const T *epsinv;      // nullable: vacuum
    const T *muinv;       // nullable: vacuum
    T *grad;              // scratch [batch][ncell][18]: d/dx, d/dy, d/dz of the six fields per cell
    T *flux;              // scratch [batch][nface][6]: |l| F of each face (global frame, owner -> neighbour)
    int32_t ncell, nface, batch;
    const int32_t *nb;    // device [4][ncell]
    const int32_t *cf;    // device [4][ncell]
    const int32_t *fc;    // device [nface][2]
    const T *cgeo;        // device [TET_CGEO_ROWS][ncell]
    const T *fgeo;        // device [TET_FGEO_ROWS][nface]
    const void *op;       // device: FaceOpEM<T> (face-frame inputs, PatTet)
};
template <typename T> int launch_tet_step(const TetArgs<T> &a, void *stream);

template <typename T>
struct TriArgs {
    const T *U;
    T *Unew;
    const T *epsinv;      // nullable: vacuum
    const T *muinv;       // nullable: vacuum
    T *grad;              // scratch [batch][ncell][2 nfields]: d/dx (fields), d/dy (fields) per cell
    int32_t ncell, batch;
    int32_t nfields;      // 3: (Ez, Hx, Hy); 4: (Ez, Hx, Hy, psi)
    const int32_t *nb;    // device [3][ncell]
    const T *geo;         // device: the paired layout above (TRI_GEO_PAIRS pairs, then |l_k| / |Omega|)
    const void *op;       // device: the face operator (face-frame inputs; FaceOpTM<T> or FaceOpTP<T>)
};
template <typename T> int launch_tri_step(const TriArgs<T> &a, void *stream);

// Arguments of the Cartesian 2D TM adjoint kernels.
template <typename T>
struct Cart2DAdjArgs {
    const T *U;           // state the forward step started from
    const T *lam;         // lambda^{n+1}
    T *lam_out;           // lambda^n
    double *g_epsinv;     // nullable, accumulated
    double *g_muinv;      // nullable, accumulated
    const T *epsinv;      // nullable: vacuum
    const T *muinv;       // nullable: vacuum
    int32_t nx, ny, batch;
    int32_t bc[4];
    int32_t ncu;              // compute units of the device (sizes the march's tiles)
    const FaceOpTM<T> *ops;   // device: x-face and y-face operators
};

// Launchers (defined in the .hip files).  Return a hipError_t as int.
template <typename T> int launch_cart2d_step(const Cart2DArgs<T> &a, void *stream);
// Two steps in one launch (TM fields with or without psi or the limiter, at most one source cell;
// a.tiles from cart2d_pair_tile_table, a.ntx from cart2d_pair_tile_x).
template <typename T> int launch_cart2d_pair(const Cart2DArgs<T> &a, void *stream);
// Adjoint of one 2D step.  Scratch (device), over the npos = adjoint_ring_positions(nx, ny)
// ghost positions around the grid: padpsi [batch][3][npos] of T and padg [batch][2][npos]
// doubles; every entry is written by the step's first kernel before its second reads it, so
// the scratch needs no clearing between calls.
template <typename T> int launch_cart2d_adjoint(const Cart2DAdjArgs<T> &a, T *padpsi, double *padg, void *stream);
int64_t adjoint_ring_positions(int nx, int ny);
// The allocation-free adjoint's scratch: a static device array of ADJ_STATIC_SCRATCH_BYTES per
// GPU.  adjoint_static_scratch returns its address on the current device (looked up once per
// device, then cached); a hipError_t as int.
constexpr size_t ADJ_STATIC_SCRATCH_BYTES = size_t(16) << 20;
int adjoint_static_scratch(void **ptr);
// g_epsinv[b][cells[s]] += lam[b][Ez][cells[s]] * amp * weight[s]  (1/eps gradient of the source)
template <typename T> int launch_adjoint_source(const T *lam, double *g_epsinv, int64_t ncell, int64_t fstride,
                                                int32_t batch, const int64_t *cells, const double *weight,
                                                double amp, int32_t n, void *stream);
// U[b][field][cells[s]] += (1/eps) * amp * weight[s]  (explicit point source after a step)
template <typename T> int launch_source_scatter(T *U, const T *epsinv, int64_t ncell, int64_t fstride,
                                                int32_t batch, int32_t field, const int64_t *cells,
                                                const double *weight, double amp, int32_t n, void *stream);
template <typename T> int launch_cart3d_step(const Cart3DArgs<T> &a, void *stream);
// Output columns / rows per 3D workgroup tile (depend on the element size and field count).
int cart3d_tile_x(int precision);
int cart3d_tile_y(int precision, int nfields);
// Planes per 3D z tile for an nx x ny x nz x batch grid on ncu compute units.
int cart3d_pick_tile_z(int nx, int ny, int nz, int batch, int ncu, int precision, int nfields);
// Columns written per wave strip (depends on the element size).
int cart2d_tile_x(int precision);
// Tile rows of the 2D step, four ints each (batch item or -1, first row, end row, march
// downwards), NBANDS bands of tiles_per_band entries, one band per XCD: see gks_host.cpp.
constexpr int NBANDS = 8;
constexpr int CART2D_WAVES_PER_BLOCK = 4;
std::vector<int32_t> cart2d_tile_table(int ny, int batch, int precision, int ntx, int32_t &tiles_per_band);
// Output columns per strip of the paired kernel, and its tile table (same layout as above): the
// first tile row of every batch item marches down and the last up, and every tile keeps two
// rows away from a side it does not touch.  Empty when the grid is too small for it.
int cart2d_pair_tile_x(int precision);
std::vector<int32_t> cart2d_pair_tile_table(int ny, int batch, int precision, int ntx, int32_t &tiles_per_band);

// Energy: partial sums per (batch, block) then a fixed-order final sum; all FP64.
// Fields [0, nE) are E (weight eps), [nE, nE + nH) are H (weight mu), the rest potentials (1).
template <typename T>
int launch_energy(const T *U, const T *epsinv, const T *muinv, int64_t ncell, int32_t nfields, int32_t nE,
                  int32_t nH, int32_t batch, const double *vol /*nullable: uniform*/, double uniform_vol,
                  double *partial, int32_t nblk, double *out, void *stream);
template <typename T>
int launch_probe_energy(const T *U, int64_t nx, int64_t ny, int64_t nz, int32_t nfields, int32_t ez_field,
                        int32_t batch, const int64_t box[6], double vol, double *partial, int32_t nblk, double *out,
                        void *stream);
template <typename T>
int launch_probe_grad(const T *U, T *lam, int64_t nx, int64_t ny, int64_t nz, int32_t nfields, int32_t ez_field,
                      int32_t batch, const int64_t box[6], double vol, void *stream);

}  // namespace gks
