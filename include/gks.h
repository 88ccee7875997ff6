/*
 * libgks: the gas-kinetic scheme (GKS) time step for Maxwell's equations on one AMD MI355X GPU.
 *
 * The method is the discrete-velocity GKS of "A Gas-Kinetic Scheme for Maxwell Equations"
 * (Pu, Long, Xu): a finite-volume update of cell averages (Sec. 3.1, cell-average update)
 * whose interface fluxes are the time averages over one step of the integral solution of the
 * vector BGK model (Sec. 3.1, numerical flux with coefficients C1..C5), built from the
 * D2Q4 / D3Q4 lattice equilibria (Sec. 2.2) in the face-local frame.
 *
 * Conventions for every entry point
 *   - Plain C ABI: pointers and sizes only.  Every call returns a gks_status; 0 is success,
 *     a negative value an error whose text gks_last_error() returns.  No call throws, exits
 *     or aborts.
 *   - Pointers documented as "device" must be device memory of the GPU the context was
 *     created on; "host" pointers are ordinary CPU memory.
 *   - Field arrays are structure-of-arrays, [batch][field][cell], x fastest on Cartesian
 *     grids (cell = ix + nx*(iy + ny*iz)).  Fields: TM2D (Ez, Hx, Hy); TM2D_PHM (Ez, Hx, Hy,
 *     psi); EM3D (Ex, Ey, Ez, Hx, Hy, Hz); EM3D_PHM (Ex, Ey, Ez, Hx, Hy, Hz, phi, psi).  Units
 *     have c = eps0 = mu0 = 1 (Sec. 5), so H and B coincide in vacuum.
 *   - The element type is double for GKS_FP64 contexts and float for GKS_FP32 contexts
 *     (in FP32 the fields are stored and the face fluxes computed in single precision; each
 *     cell sums its face fluxes and adds them to its old value in double precision, rounding
 *     once to single precision on store; the host computes the flux coefficients, and the
 *     diagnostics sum, in double precision).
 *   - All GPU work is enqueued on the stream given to gks_init_mesh and runs asynchronously,
 *     except the calls that return host values (gks_energy, gks_probe_energy, gks_run with an
 *     energy buffer), which synchronise that stream.
 *   - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef GKS_H
#define GKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gks_ctx gks_ctx;

typedef enum {
    GKS_OK = 0,
    GKS_EINVAL = -1,      /* bad argument (checked on the host before any launch) */
    GKS_ENOMEM = -2,      /* device or host allocation failed */
    GKS_EDEVICE = -3,     /* a HIP call failed */
    GKS_EUNSTABLE = -4,   /* energy grew beyond the stability threshold */
    GKS_ENONFINITE = -5,  /* energy is NaN or infinite */
    GKS_ESTATE = -6       /* call not valid in the context's state */
} gks_status;

typedef enum { GKS_CART2D = 0, GKS_CART3D = 1, GKS_TRI2D = 2, GKS_TET3D = 3 } gks_mesh_kind;
/* The perfectly hyperbolic Maxwell (PHM) system (Sec. 2.1) adds the divergence-cleaning
 * potentials phi and psi, coupled through chi and gamma (gks_params), to the fields:
 *   GKS_TM2D_PHM: the TM fields with psi (dpsi/dt + gamma c^2 div H = 0, dH/dt += -gamma
 *   grad psi): (Ez, Hx, Hy, psi).  phi follows div E, which TM fields do not have, so it stays
 *   zero and is not stored.
 *   GKS_EM3D_PHM: all eight, (Ex, Ey, Ez, Hx, Hy, Hz, phi, psi), with dphi/dt + chi div E = 0
 *   and dE/dt += -chi c^2 grad phi. */
typedef enum { GKS_TM2D = 0, GKS_EM3D = 1, GKS_TM2D_PHM = 2, GKS_EM3D_PHM = 3 } gks_model;
typedef enum { GKS_BC_PERIODIC = 0, GKS_BC_NONREFLECT = 1, GKS_BC_PEC = 2 } gks_bc;
typedef enum { GKS_FP64 = 0, GKS_FP32 = 1 } gks_precision;
typedef enum { GKS_GRAD_GREEN_GAUSS = 0, GKS_GRAD_LSQ = 1 } gks_gradient;
typedef enum { GKS_LIMITER_NONE = 0, GKS_LIMITER_MINMOD = 1 } gks_limiter;

/*
 * Mesh description (host memory; copied by gks_init_mesh, not retained).
 *   Cartesian (GKS_CART2D with GKS_TM2D or GKS_TM2D_PHM, GKS_CART3D with GKS_EM3D or GKS_EM3D_PHM):
 *   n[3] cells per axis
 *   (n[2] = 1 in 2D), box [lo, hi], bc[6] = x-, x+, y-, y+, z-, z+ sides (the z entries are
 *   ignored in 2D).  A periodic axis must be periodic on both sides.
 *   Triangles (GKS_TRI2D with GKS_TM2D or GKS_TM2D_PHM): nverts vertices vert_xy[2*v], ncells triangles
 *   cell_verts[3*c], nfaces edges face_cells[2*s] = (owner, neighbour) with neighbour < 0
 *   meaning a boundary edge of type -(1 + gks_bc) (non-reflecting or PEC), and
 *   face_verts[2*s] = the edge's two vertices.  Every cell must be a side of exactly three
 *   faces, and a face's vertices an edge of its cells (checked: GKS_EINVAL).  Cells ordered
 *   along a space-filling curve keep the neighbour reads of the kernels in cache.
 *   batch: number of independent problems sharing the mesh (fields and materials carry a
 *   leading batch axis).
 *   Tetrahedra (GKS_TET3D with GKS_EM3D; the unstructured 3D meshes of Sec. 5.5): vert_xy holds
 *   3 coordinates per vertex, cell_verts 4 vertices per cell, face_verts 3 vertices per face,
 *   face_cells as for triangles.  Each face's flux is evaluated once, from its owner
 *   face_cells[2s] (the D3Q4 lattice is chiral: the other side would give a different flux);
 *   meshes from a generator that makes the owner the lower cell index match the oracle's
 *   convention.  Green-Gauss gradients only (least squares grows on such meshes: GKS_EINVAL).
 */
typedef struct {
    int32_t kind, model, precision;
    int64_t batch;
    int64_t n[3];
    double lo[3], hi[3];
    int32_t bc[6];
    int64_t ncells, nfaces, nverts;
    const double *vert_xy;
    const int32_t *cell_verts;
    const int32_t *face_cells;
    const int32_t *face_verts;
} gks_mesh_desc;

/*
 * Scheme parameters (host memory, copied).
 *   c:            lattice speed = speed of light (> 0).
 *   cfl, dt:      dt > 0 is used as given; otherwise dt = cfl * h / c with h the smallest
 *                 cell width (Cartesian) or the smallest inradius 2|Omega|/perimeter
 *                 (triangles).  c dt / h above the stability limit is rejected (GKS_EINVAL):
 *                 0.5 on 2D grids and triangle meshes, 1/3 on 3D Cartesian grids (the D3Q4
 *                 step grows above it: at 1/2 a Fourier mode gains about 10% per step).
 *                 With the PHM potentials coupled the Cartesian limits are lower: 0.42 on 2D
 *                 grids with gamma > 0 (at 0.5 and gamma = 1 a mode gains 11% per step) and
 *                 0.3 on 3D grids with chi or gamma > 0 (2.6% per step at 1/3).
 *                 Tetrahedral meshes take c dt / (smallest inradius 3|Omega|/surface) <= 0.5.
 *                 The limits are those of tau -> 0.  On 3D grids tau shrinks the stable range
 *                 (the free-transport part of the D3Q4 flux has no transverse terms): at
 *                 tau = 0.01 dt the Maxwell step is stable to 0.32 (at 1/3 a mode gains 2e-5
 *                 per step, under 1% in 500 steps); at 0.3 a mode gains 1e-4 per step at
 *                 tau = 0.03 dt and 6e-3 as tau -> infinity.  unstable_growth guards such runs.
 *   tau_over_dt:  collision time tau = tau_over_dt * dt (>= 0; +INFINITY = collisionless).
 *   energy_every: gks_run records the energy every this many steps (0 = never).
 *   unstable_growth: gks_run fails with GKS_EUNSTABLE when a recorded energy exceeds this
 *                 factor times the first recorded one (0 = no check).
 *   gradient:     cell gradients of the reconstruction (Sec. 3.1 uses Green-Gauss and allows
 *                 others).  GKS_GRAD_GREEN_GAUSS: (1/|Omega_i|) sum_s (U_nb - U_i)/2 n_s |l_s|.
 *                 GKS_GRAD_LSQ: the least-squares fit to the face neighbours, each boundary
 *                 ghost (the same ghost state) placed at the mirror image of the cell centroid
 *                 across the face; it is exact for linear fields on any triangle mesh.  On
 *                 Cartesian grids both give the central difference, and both values are
 *                 accepted.  Other values: GKS_EINVAL.
 *   limiter:      slope limiter for discontinuous data (Sec. 5, Riemann problem: the paper's
 *                 step limits its slopes there and does not name the limiter).
 *                 GKS_LIMITER_MINMOD: along each axis, minmod of the two one-sided
 *                 differences of the variables that travel along that axis (E_a +/- H_b,
 *                 E_b +/- H_a, with a and b the other axes) and of the normal components, in
 *                 place of the central difference.  Cartesian grids only (GKS_EINVAL on a
 *                 triangle mesh).  The limited step is nonlinear: gks_adjoint_step refuses a
 *                 limited context (GKS_ESTATE).  Not available with the PHM models
 *                 (GKS_EINVAL).  Other values: GKS_EINVAL.
 *   chi, gamma:   couplings of the PHM potentials phi and psi (Sec. 2.1); divergence errors
 *                 of E and H travel at chi c and gamma c.  PHM models only: both in [0, 1],
 *                 so that no wave outruns the lattice speed c (chi has no effect on TM fields).
 *                 Other models: both must be 0 (GKS_EINVAL otherwise).  The potentials carry
 *                 no material factor: 1/eps scales E and 1/mu scales H only.
 */
typedef struct {
    double c;
    double cfl;
    double dt;
    double tau_over_dt;
    int32_t energy_every;
    double unstable_growth;
    int32_t gradient;
    int32_t limiter;
    double chi;
    double gamma;
} gks_params;

/* Creates a context on the current HIP device.  hip_stream: a hipStream_t (NULL = the null
 * stream) on which every later call enqueues its work.  *out receives the context; on error
 * *out is NULL. */
gks_status gks_init_mesh(const gks_mesh_desc *mesh, const gks_params *params, void *hip_stream,
                         gks_ctx **out);

/* Releases the context and everything it owns (NULL is accepted). */
gks_status gks_destroy(gks_ctx *ctx);

/* Text of the last error on this context (or of the last failed gks_init_mesh when ctx is
 * NULL).  Owned by the library, valid until the next call on the context. */
const char *gks_last_error(const gks_ctx *ctx);

/* The time step in use and the five coefficients C1..C5 of the time-integrated flux
 * (Sec. 3.1) as computed in double precision on the host. */
gks_status gks_get_dt(const gks_ctx *ctx, double *dt_out);
gks_status gks_flux_coefficients(double dt, double tau, double C_out[5]);

/*
 * Per-cell material maps (device, element type of the context, [batch][ncells]):
 * epsinv = 1/eps, muinv = 1/mu; NULL means 1 (vacuum).  The pointers are retained and read
 * by every later step until the next call: the caller keeps the memory alive.
 * Materials are absent from the paper; the library scales the cell update by 1/eps, 1/mu
 * and the equilibrium time derivative at a face by the face average of 1/eps, 1/mu.
 */
gks_status gks_set_material(gks_ctx *ctx, const void *epsinv, const void *muinv);

/*
 * Point current source (Sec. 2.1 source term S = (-J, 0)): on each listed cell (host
 * arrays cells[n], weight[n]) J_z(t) = weight * J0 * exp(-((t - t0)/sigma_t)^2), applied
 * explicitly at t^n in every batch item.  n = 0 removes the source.  At most 4096 cells.
 */
gks_status gks_set_point_source(gks_ctx *ctx, int64_t n, const int64_t *cells, const double *weight,
                                double J0, double t0, double sigma_t);

/*
 * One explicit step from time t_n (Sec. 3.1): U_out = Phi(U_in).  U_in, U_out: device,
 * [batch][nfields][ncells], must not overlap (GKS_EINVAL otherwise).
 */
gks_status gks_step(gks_ctx *ctx, const void *U_in, void *U_out, double t_n);

/*
 * nsteps steps in place on U (device) starting at t0 (t^n = t0 + n dt), ping-ponging with a
 * library-owned buffer.  energy_host: NULL, or host memory for (nsteps / energy_every) x batch
 * doubles receiving W = 1/2 sum |Omega| (eps |E|^2 + mu |H|^2) after every energy_every-th
 * step.  When given, each record is checked while the next energy_every steps run: a NaN/Inf
 * energy returns GKS_ENONFINITE and growth beyond unstable_growth times the first record returns
 * GKS_EUNSTABLE.  The run then stops early: U holds the state after the record that followed
 * the failing one (at most energy_every steps past it), the records up to that one are written
 * and the later entries of energy_host are left untouched; the error text names the batch item
 * and the step of the failing record.
 * On 2D Cartesian grids (GKS_TM2D, with or without the limiter, or GKS_TM2D_PHM) with at most
 * one source cell, gks_run advances two steps per kernel launch (the fields are read and
 * written once for both); the result equals that of nsteps gks_step calls at the same times,
 * bit for bit.
 */
gks_status gks_run(gks_ctx *ctx, void *U, int64_t nsteps, double t0, double *energy_host);

/*
 * Reverse-mode adjoint of one gks_step (the step is linear in U for fixed materials):
 *   lam_n   = (dPhi/dU)^T lam_np1                  (device, field type, [batch][nf][ncells])
 *   g_epsinv += (dPhi/d epsinv)^T lam_np1           (device, double, [batch][ncells]; nullable)
 *   g_muinv  += (dPhi/d muinv)^T lam_np1            (device, double, [batch][ncells]; nullable)
 * U_n is the state the forward step started from (device, field type).  lam_n must not
 * overlap lam_np1 or U_n.  Cartesian 2D TM contexts without the slope limiter only (GKS_ESTATE
 * otherwise: the limited step is nonlinear, and the PHM model has no adjoint kernel).  The
 * co-states and material gradients of the ghost positions around the grid go through a scratch
 * buffer of batch x (4 (nx + ny) + 16) x (16 + 3 x element size) bytes, which the context
 * allocates on its first adjoint call (GKS_ENOMEM if that fails) and keeps.
 */
gks_status gks_adjoint_step(gks_ctx *ctx, const void *U_n, const void *lam_np1, void *lam_n,
                            double *g_epsinv, double *g_muinv, double t_n);

/*
 * gks_adjoint_step for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same operation, arguments,
 * results and errors, but its scratch is a static device array of 16 MiB per GPU that the
 * library holds until the process ends, so the call itself allocates nothing.  A grid and batch
 * needing more scratch than that (see gks_adjoint_step) are refused with GKS_EINVAL before any
 * launch.  The array is shared by every call on one GPU, across contexts: calls that overlap on
 * one GPU (concurrent streams, threads) race and must be serialised by the caller.  Each call
 * writes every scratch entry it reads, so nothing carries over from earlier calls.
 */
gks_status gks_adjoint_step_noalloc(gks_ctx *ctx, const void *U_n, const void *lam_np1, void *lam_n,
                                    double *g_epsinv, double *g_muinv, double t_n);

/* Energy W = 1/2 sum_i |Omega_i| (eps_i |E_i|^2 + mu_i |H_i|^2) of each batch item (plus
 * 1/2 sum_i |Omega_i| (phi_i^2 + psi_i^2) with the PHM models), summed in double precision in
 * a fixed order; out_host: host, [batch].  Synchronises the stream. */
gks_status gks_energy(gks_ctx *ctx, const void *U, double *out_host);

/* Probe-box field energy sum_{cells in box} |Omega| Ez^2 of each batch item (Cartesian only;
 * box = [i0, i1) x [j0, j1) x [k0, k1) cell indices, host int64[6]); out_host: host, [batch]. */
gks_status gks_probe_energy(gks_ctx *ctx, const void *U, const int64_t *box, double *out_host);

/* Gradient of gks_probe_energy with respect to U: lam = 2 |Omega| Ez on the box cells, 0
 * elsewhere (device, field type, [batch][nf][ncells]); the seed of an adjoint sweep. */
gks_status gks_probe_energy_grad(gks_ctx *ctx, const void *U, const int64_t *box, void *lam);

#ifdef __cplusplus
}
#endif
#endif /* GKS_H */
