/*
 * Plain FP64 CPU oracle of the discrete-velocity gas-kinetic scheme (GKS) step for
 * Maxwell's equations.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this code.  It shares nothing with the HIP library: no headers, no
 * helpers, no tables.  It is deliberately slow and literal: every interface flux is formed by
 * summing over the four discrete velocities of the lattice in the face-local frame, exactly in
 * the order the paper builds it (Sec. 3.1), with no closed forms, no blocking and no fusion.
 *
 * State: eight components per cell, U = (Ex, Ey, Ez, Hx, Hy, Hz, phi, psi) of the perfectly
 * hyperbolic Maxwell (PHM) system (Sec. 2.1), array-of-structures U[8*i + f], with B read as
 * H.  phi and psi are the divergence-cleaning potentials, coupled through chi and gamma; with
 * chi = gamma = 0 (the paper's experiments) they decouple and stay zero.  Two-dimensional TM
 * problems use components (Ez, Hx, Hy) (and psi with PHM) with the D2Q4 lattice; the others
 * stay identically zero.
 *
 * Mesh: a general face-based finite-volume mesh (Sec. 3.1): cells with volume |Omega_i|,
 * faces with owner L, neighbour R (or a boundary code), unit normal n pointing L -> R, area
 * |l_s| and the offsets x_s - x_L, x_s - x_R from the cell centroids to the face centre
 * (periodic wrap is encoded in those offsets).
 *
 * Readings of the paper taken where it is silent (each is listed in the design notes):
 *  - Coefficients C1..C5 are computed by the caller (in high precision) from the paper's
 *    time integrals (Sec. 3.1, numerical flux), with the exponent signs of c4, c5 read as
 *    e^{-t/tau} (the printed C4, C5 are the integrals of that reading).
 *  - Cell gradients: Green-Gauss with the arithmetic face value (Sec. 3.1); ghost values
 *    for the gradient: non-reflecting -> the cell's own value, PEC -> the mirror state.
 *    Optionally least squares over the face neighbours (Sec. 3.1 allows other gradients), with
 *    each boundary ghost placed at the mirror image of the cell centroid across the face.
 *  - Limiter (Sec. 5, Riemann problem; its type is not given): optionally minmod of the two
 *    one-sided differences per axis, applied to the characteristic variables along that axis
 *    (E_a +/- H_b, E_b +/- H_a and the normal components), on Cartesian grids.
 *  - Non-reflecting boundary (Sec. 3.1, last paragraph): the ghost-side distributions are
 *    zero, i.e. the right state and its slopes vanish in the face frame.
 *  - PEC boundary (Sec. 5.5 conditions): mirror ghost in the face frame, even normal E and
 *    tangential H, odd tangential E and normal H; the slopes are mirrored.  The potentials
 *    follow the parity that keeps the PHM system invariant under the mirror: phi odd (it
 *    tracks div E), psi even (it tracks div H).
 *  - Materials (absent from the paper): the kinetic flux uses the vacuum lattice; the cell
 *    update is scaled by M_i^{-1} = diag(1/eps_i, 1/mu_i, 1, 1) and the time derivative of the
 *    interface equilibrium by the face average of M^{-1}.
 *  - Sources: the current density J only; the charge density of the phi equation is zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NC 8 /* components carried per cell */

enum { BC_NONREFLECT = 1, BC_PEC = 2 };

typedef struct {
    int32_t dim;              /* 2: D2Q4 in the xy plane, 3: D3Q4 */
    int64_t ncells, nfaces;
    const double *vol;        /* [ncells] */
    const int64_t *face_L;    /* [nfaces] owner */
    const int64_t *face_R;    /* [nfaces] neighbour, or -(1+bc) on a boundary face */
    const double *normal;     /* [3*nfaces] unit normal L -> R */
    const double *area;       /* [nfaces] */
    const double *dL;         /* [3*nfaces] x_s - x_L */
    const double *dR;         /* [3*nfaces] x_s - x_R (unused on boundary faces) */
    const int64_t *cf_ptr;    /* [ncells+1] CSR: faces of each cell */
    const int64_t *cf_idx;    /* [cf_ptr[ncells]] */
} orc_mesh;

typedef struct {
    double c;      /* lattice speed = speed of light */
    double dt;     /* time step */
    double C[5];   /* time-integrated coefficients C1..C5 */
    int32_t gradient; /* 0: Green-Gauss (the paper's), 1: least squares */
    int32_t limiter;  /* 0: none, 1: minmod slopes (Cartesian meshes only) */
    double chi;       /* PHM coupling of phi (E divergence), 0 for plain Maxwell */
    double gamma;     /* PHM coupling of psi (H divergence), 0 for plain Maxwell */
} orc_params;

/* ---------------------------------------------------------------- physics (Sec. 2.1) */

/* Directional flux F_j(U) = A_j U of the PHM system (Sec. 2.1, flux functions): the curl
 * terms of Maxwell's equations, plus chi c^2 phi in E_j, gamma psi in B_j, chi E_j in phi and
 * gamma c^2 B_j in psi. */
static void flux_dir(int j, const double *U, double c, double chi, double gam, double *F)
{
    const double c2 = c * c;
    const double Ex = U[0], Ey = U[1], Ez = U[2], Bx = U[3], By = U[4], Bz = U[5];
    const double phi = U[6], psi = U[7];
    if (j == 0) {
        F[0] = 0.0;      F[1] = c2 * Bz;  F[2] = -c2 * By;
        F[3] = 0.0;      F[4] = -Ez;      F[5] = Ey;
    } else if (j == 1) {
        F[0] = -c2 * Bz; F[1] = 0.0;      F[2] = c2 * Bx;
        F[3] = Ez;       F[4] = 0.0;      F[5] = -Ex;
    } else {
        F[0] = c2 * By;  F[1] = -c2 * Bx; F[2] = 0.0;
        F[3] = -Ey;      F[4] = Ex;       F[5] = 0.0;
    }
    F[j] += chi * c2 * phi;
    F[3 + j] += gam * psi;
    F[6] = chi * U[j];
    F[7] = gam * c2 * U[3 + j];
}

/* ---------------------------------------------------------------- lattice (Sec. 2.2) */

/* Discrete velocities u_k in the face-local frame: D3Q4 (Sec. 2.2, kinetic velocities in 3D)
 * and its degeneration D2Q4 in 2D (the z component dropped). */
static void lattice(int dim, double c, double u[4][3])
{
    static const double d3[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
    for (int k = 0; k < 4; ++k)
        for (int m = 0; m < 3; ++m)
            u[k][m] = c * d3[k][m] * ((dim == 2 && m == 2) ? 0.0 : 1.0);
}

/* Local-equilibrium distribution g_k(V) = V/4 + sum_m F_m(V) u_k^m / (4 c^2)  (Sec. 2.2). */
static void equilibrium(const double u[4][3], double c, double chi, double gam, const double *V,
                        double g[4][NC])
{
    double F[3][NC];
    const double w = 1.0 / (4.0 * c * c);
    for (int m = 0; m < 3; ++m) flux_dir(m, V, c, chi, gam, F[m]);
    for (int k = 0; k < 4; ++k)
        for (int f = 0; f < NC; ++f) {
            double s = 0.25 * V[f];
            for (int m = 0; m < 3; ++m) s += F[m][f] * u[k][m] * w;
            g[k][f] = s;
        }
}

/* ---------------------------------------------------------------- face frame (Sec. 3.1) */

/* Rotation T' taking the face normal to the local x axis, exactly as printed, with
 * T' = diag(-1,-1,1) when n1 = -1. */
static void rotation(const double *n, double T[3][3])
{
    const double n1 = n[0], n2 = n[1], n3 = n[2];
    if (n1 == -1.0) {
        memset(T, 0, 9 * sizeof(double));
        T[0][0] = -1.0; T[1][1] = -1.0; T[2][2] = 1.0;
        return;
    }
    const double q = 1.0 + n1;
    T[0][0] = n1;  T[0][1] = n2;                  T[0][2] = n3;
    T[1][0] = -n2; T[1][1] = n1 + n3 * n3 / q;    T[1][2] = -n2 * n3 / q;
    T[2][0] = -n3; T[2][1] = -n2 * n3 / q;        T[2][2] = 1.0 - n3 * n3 / q;
}

/* T = diag(T', T', 1, 1) acting on (E, H, phi, psi); forward (global -> local) and inverse
 * (= transpose).  The potentials are scalars. */
static void rot_fwd(const double T[3][3], const double *a, double *b)
{
    for (int blk = 0; blk < 2; ++blk)
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += T[r][q] * a[3 * blk + q];
            b[3 * blk + r] = s;
        }
    b[6] = a[6];
    b[7] = a[7];
}
static void rot_inv(const double T[3][3], const double *a, double *b)
{
    for (int blk = 0; blk < 2; ++blk)
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += T[q][r] * a[3 * blk + q];
            b[3 * blk + r] = s;
        }
    b[6] = a[6];
    b[7] = a[7];
}

/* Mirror of a state in the face frame for a perfect electric conductor: the normal E and the
 * tangential H are even, the tangential E and the normal H are odd; phi (div E) is odd and psi
 * (div H) even, the parities under which the mirrored PHM fields solve the same system. */
static void pec_mirror(const double *a, double *b)
{
    static const double P[NC] = {+1, -1, -1, -1, +1, +1, -1, +1};
    for (int f = 0; f < NC; ++f) b[f] = P[f] * a[f];
}

/* ---------------------------------------------------------------- interface flux (Sec. 3.1) */

/*
 * Time-averaged GKS interface flux in the face-local frame (normal along local x).
 * Inputs: reconstructed left/right states Ul, Ur and their slopes dUl[j], dUr[j] along the
 * local axes j; the face material factors minvE = 1/eps_s, minvH = 1/mu_s.
 * Every moment is a literal sum over the four discrete velocities; half-moments select the
 * sign of the normal velocity component.
 */
static void gks_face_flux(int dim, const orc_params *p, const double *Ul, const double *Ur,
                          double dUl[3][NC], double dUr[3][NC], double minvE, double minvH,
                          double *Fout)
{
    const double c = p->c, chi = p->chi, gam = p->gamma;
    double u[4][3];
    lattice(dim, c, u);

    /* equilibria of the two reconstructed states and of their slopes */
    double gl[4][NC], gr[4][NC], dgl[3][4][NC], dgr[3][4][NC];
    equilibrium(u, c, chi, gam, Ul, gl);
    equilibrium(u, c, chi, gam, Ur, gr);
    for (int j = 0; j < 3; ++j) {
        equilibrium(u, c, chi, gam, dUl[j], dgl[j]);
        equilibrium(u, c, chi, gam, dUr[j], dgr[j]);
    }

    /* interface equilibrium state: <g0> = <g^l>_{>0} + <g^r>_{<0} */
    double U0[NC] = {0}, dU0[3][NC];
    memset(dU0, 0, sizeof dU0);
    for (int k = 0; k < 4; ++k)
        for (int f = 0; f < NC; ++f) {
            if (u[k][0] > 0) U0[f] += gl[k][f];
            else             U0[f] += gr[k][f];
        }
    /* its spatial derivative: <grad g0> = <grad g^l>_{>0} + <grad g^r>_{<0} */
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 4; ++k)
            for (int f = 0; f < NC; ++f) {
                if (u[k][0] > 0) dU0[j][f] += dgl[j][k][f];
                else             dU0[j][f] += dgr[j][k][f];
            }

    double g0[4][NC], dg0[3][4][NC];
    equilibrium(u, c, chi, gam, U0, g0);
    for (int j = 0; j < 3; ++j) equilibrium(u, c, chi, gam, dU0[j], dg0[j]);

    /* time derivative from the compatibility condition <g_t + u . grad g0> = 0,
     * scaled by the face material factor */
    double Ut[NC] = {0};
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 3; ++j)
            for (int f = 0; f < NC; ++f) Ut[f] -= u[k][j] * dg0[j][k][f];
    for (int f = 0; f < 3; ++f) Ut[f] *= minvE;
    for (int f = 3; f < 6; ++f) Ut[f] *= minvH;
    double gt[4][NC];
    equilibrium(u, c, chi, gam, Ut, gt);

    /* the five moments of the time-integrated flux */
    double m1[NC] = {0}, m2[NC] = {0}, m3[NC] = {0}, m4[NC] = {0}, m5[NC] = {0};
    for (int k = 0; k < 4; ++k) {
        const double un = u[k][0];
        for (int f = 0; f < NC; ++f) {
            double tg0 = 0.0, tgl = 0.0, tgr = 0.0;   /* u_k . grad g */
            for (int j = 0; j < 3; ++j) {
                tg0 += u[k][j] * dg0[j][k][f];
                tgl += u[k][j] * dgl[j][k][f];
                tgr += u[k][j] * dgr[j][k][f];
            }
            m1[f] += un * g0[k][f];
            m2[f] += un * tg0;
            m3[f] += un * gt[k][f];
            if (un > 0) { m4[f] += un * gl[k][f]; m5[f] += un * tgl; }
            else        { m4[f] += un * gr[k][f]; m5[f] += un * tgr; }
        }
    }
    for (int f = 0; f < NC; ++f)
        Fout[f] = (p->C[0] * m1[f] + p->C[1] * m2[f] + p->C[2] * m3[f] + p->C[3] * m4[f]
                   - p->C[4] * m5[f]) / p->dt;
}

/* ---------------------------------------------------------------- mesh-level pieces */

static void ghost_state(int bc, const double *n, const double *Ui, double *Ug)
{
    if (bc == BC_PEC) {
        double T[3][3], loc[NC], mir[NC];
        rotation(n, T);
        rot_fwd(T, Ui, loc);
        pec_mirror(loc, mir);
        rot_inv(T, mir, Ug);
    } else {
        for (int f = 0; f < NC; ++f) Ug[f] = Ui[f];
    }
}

/* Green-Gauss cell gradients: grad U_i = (1/|Omega_i|) sum_s (U_nb - U_i)/2 n_out |l_s|,
 * the arithmetic face value form (Sec. 3.1).  grad[(i*3 + d)*8 + f]. */
static void gradients(const orc_mesh *m, const double *U, double *grad)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->ncells; ++i) {
        double acc[3][NC];
        memset(acc, 0, sizeof acc);
        for (int64_t q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; ++q) {
            const int64_t s = m->cf_idx[q];
            const double *n = m->normal + 3 * s;
            double nout[3], Unb[NC];
            const int64_t L = m->face_L[s], R = m->face_R[s];
            if (L == i) {
                for (int d = 0; d < 3; ++d) nout[d] = n[d];
                if (R >= 0) memcpy(Unb, U + NC * R, sizeof Unb);
                else        ghost_state((int)(-R - 1), n, U + NC * i, Unb);
            } else {
                for (int d = 0; d < 3; ++d) nout[d] = -n[d];
                memcpy(Unb, U + NC * L, sizeof Unb);
            }
            for (int d = 0; d < 3; ++d)
                for (int f = 0; f < NC; ++f)
                    acc[d][f] += 0.5 * (Unb[f] - U[NC * i + f]) * nout[d] * m->area[s];
        }
        for (int d = 0; d < 3; ++d)
            for (int f = 0; f < NC; ++f) grad[(i * 3 + d) * NC + f] = acc[d][f] / m->vol[i];
    }
}

/* Least-squares cell gradients, the "other" reconstruction gradient Sec. 3.1 allows: grad U_i
 * minimises sum_j |U_i + grad U_i . d_j - U_j|^2 over the face neighbours j of cell i, with
 * d_j = x_j - x_i.  A boundary face contributes its ghost state (the same ghost as for
 * Green-Gauss) placed at the mirror image of x_i across the face, d = 2 ((x_s - x_i) . n) n.
 * The normal equations (sum_j d_j d_j^T) g = sum_j d_j (U_j - U_i) are solved by Cramer's rule,
 * in the xy plane on 2D meshes.  grad[(i*3 + d)*8 + f]. */
static void gradients_lsq(const orc_mesh *m, const double *U, double *grad)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->ncells; ++i) {
        double M[3][3], b[3][NC];
        memset(M, 0, sizeof M);
        memset(b, 0, sizeof b);
        for (int64_t q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; ++q) {
            const int64_t s = m->cf_idx[q];
            const double *n = m->normal + 3 * s, *dL = m->dL + 3 * s, *dR = m->dR + 3 * s;
            const int64_t L = m->face_L[s], R = m->face_R[s];
            double d[3], Unb[NC];
            if (L == i && R >= 0) {          /* neighbour across the face: x_R - x_i */
                for (int k = 0; k < 3; ++k) d[k] = dL[k] - dR[k];
                memcpy(Unb, U + NC * R, sizeof Unb);
            } else if (L == i) {             /* boundary: the ghost at the mirror point */
                const double h = dL[0] * n[0] + dL[1] * n[1] + dL[2] * n[2];
                for (int k = 0; k < 3; ++k) d[k] = 2.0 * h * n[k];
                ghost_state((int)(-R - 1), n, U + NC * i, Unb);
            } else {                         /* this cell is the face's neighbour: x_L - x_i */
                for (int k = 0; k < 3; ++k) d[k] = dR[k] - dL[k];
                memcpy(Unb, U + NC * L, sizeof Unb);
            }
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c) M[r][c] += d[r] * d[c];
                for (int f = 0; f < NC; ++f) b[r][f] += d[r] * (Unb[f] - U[NC * i + f]);
            }
        }
        double g[3][NC];
        memset(g, 0, sizeof g);
        if (m->dim == 2) {
            const double det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
            for (int f = 0; f < NC; ++f) {
                g[0][f] = (b[0][f] * M[1][1] - M[0][1] * b[1][f]) / det;
                g[1][f] = (M[0][0] * b[1][f] - b[0][f] * M[1][0]) / det;
            }
        } else {
            const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                               M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                               M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
            for (int f = 0; f < NC; ++f)
                for (int k = 0; k < 3; ++k) {   /* Cramer: column k replaced by b */
                    double A[3][3];
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 3; ++c) A[r][c] = (c == k) ? b[r][f] : M[r][c];
                    g[k][f] = (A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                               A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0])) / det;
                }
        }
        for (int k = 0; k < 3; ++k)
            for (int f = 0; f < NC; ++f) grad[(i * 3 + k) * NC + f] = g[k][f];
    }
}

static double minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}

/* Limited slopes (Sec. 5, Riemann problem: the limiter is not named; this is minmod on the
 * characteristic variables): along each axis d the one-sided slopes (U_+ - U_i)/h_+ and
 * (U_i - U_-)/h_-, with U_+ and U_- the values across the faces whose outward normals are +e_d
 * and -e_d (the neighbour, or the boundary ghost placed at the mirror image of x_i, h its
 * centroid distance), are limited by minmod in the variables that travel along d.  Only meshes
 * whose every cell has one face per axis direction qualify (Cartesian grids); returns -1
 * otherwise. */
static int gradients_limited(const orc_mesh *m, const double *U, double *grad)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < m->ncells; ++i) {
        double up[3][NC], um[3][NC], hp[3] = {0, 0, 0}, hm[3] = {0, 0, 0};
        int np[3] = {0, 0, 0}, nm[3] = {0, 0, 0};
        for (int64_t q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; ++q) {
            const int64_t s = m->cf_idx[q];
            const double *n = m->normal + 3 * s, *dL = m->dL + 3 * s, *dR = m->dR + 3 * s;
            const int64_t L = m->face_L[s], R = m->face_R[s];
            double nout[3], d[3], Unb[NC];
            if (L == i && R >= 0) {
                for (int k = 0; k < 3; ++k) { nout[k] = n[k]; d[k] = dL[k] - dR[k]; }
                memcpy(Unb, U + NC * R, sizeof Unb);
            } else if (L == i) {
                const double h = dL[0] * n[0] + dL[1] * n[1] + dL[2] * n[2];
                for (int k = 0; k < 3; ++k) { nout[k] = n[k]; d[k] = 2.0 * h * n[k]; }
                ghost_state((int)(-R - 1), n, U + NC * i, Unb);
            } else {
                for (int k = 0; k < 3; ++k) { nout[k] = -n[k]; d[k] = dR[k] - dL[k]; }
                memcpy(Unb, U + NC * L, sizeof Unb);
            }
            int ax = 0;
            for (int k = 1; k < 3; ++k)
                if (fabs(nout[k]) > fabs(nout[ax])) ax = k;
            const double dist = fabs(d[ax]);
            if (nout[ax] > 0) { memcpy(up[ax], Unb, sizeof Unb); hp[ax] = dist; ++np[ax]; }
            else              { memcpy(um[ax], Unb, sizeof Unb); hm[ax] = dist; ++nm[ax]; }
        }
        for (int k = 0; k < 3; ++k) {
            const int present = np[k] + nm[k];
            if (present && (np[k] != 1 || nm[k] != 1)) bad = 1;
            double *g = grad + (i * 3 + k) * NC;
            if (present != 2) {
                for (int f = 0; f < NC; ++f) g[f] = 0.0;
                continue;
            }
            double sp[NC], sm[NC];   /* one-sided slopes */
            for (int f = 0; f < NC; ++f) {
                sp[f] = (up[k][f] - U[NC * i + f]) / hp[k];
                sm[f] = (U[NC * i + f] - um[k][f]) / hm[k];
            }
            /* along axis k Maxwell's equations pair E_a with H_b and E_b with H_a (a, b the
             * other two axes) into waves E_a +/- H_b, E_b +/- H_a at the speed of light; the
             * normal components E_k, H_k pair with phi and psi (waves at chi c and gamma c under
             * PHM; without it they do not move and the potentials are zero).  Limit those
             * characteristic variables. */
            const int a = (k + 1) % 3, b = (k + 2) % 3;
            const int pe[4] = {a, b, k, 3 + k}, ph[4] = {3 + b, 3 + a, 6, 7};
            for (int q = 0; q < 4; ++q) {
                const int e = pe[q], h = ph[q];
                const double s = minmod(sp[e] + sp[h], sm[e] + sm[h]);
                const double r = minmod(sp[e] - sp[h], sm[e] - sm[h]);
                g[e] = 0.5 * (s + r);
                g[h] = 0.5 * (s - r);
            }
        }
    }
    return bad ? -1 : 0;
}

/* Numerical flux of every face in the global frame (normal flux along n, L -> R). */
static void face_fluxes(const orc_mesh *m, const orc_params *p, const double *U, const double *grad,
                        const double *epsinv, const double *muinv, double *flux)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < m->nfaces; ++s) {
        const int64_t L = m->face_L[s], R = m->face_R[s];
        const double *n = m->normal + 3 * s;
        const double *gL = grad + L * 3 * NC;
        double T[3][3];
        rotation(n, T);

        /* left state reconstructed at the face centre: U^l = U_L + grad U_L . (x_s - x_L) */
        double UlG[NC], Ul[NC], dUl[3][NC], dUr[3][NC], Ur[NC];
        for (int f = 0; f < NC; ++f) {
            UlG[f] = U[NC * L + f];
            for (int d = 0; d < 3; ++d) UlG[f] += gL[d * NC + f] * m->dL[3 * s + d];
        }
        rot_fwd(T, UlG, Ul);
        /* slopes along the local axes: d~_j U~ = sum_i T'_ji T d_i U */
        for (int j = 0; j < 3; ++j) {
            double gj[NC] = {0}, tmp[NC];
            for (int i = 0; i < 3; ++i)
                for (int f = 0; f < NC; ++f) gj[f] += T[j][i] * gL[i * NC + f];
            rot_fwd(T, gj, tmp);
            memcpy(dUl[j], tmp, sizeof tmp);
        }

        double minvE, minvH;
        if (R >= 0) {
            const double *gR = grad + R * 3 * NC;
            double UrG[NC];
            for (int f = 0; f < NC; ++f) {
                UrG[f] = U[NC * R + f];
                for (int d = 0; d < 3; ++d) UrG[f] += gR[d * NC + f] * m->dR[3 * s + d];
            }
            rot_fwd(T, UrG, Ur);
            for (int j = 0; j < 3; ++j) {
                double gj[NC] = {0}, tmp[NC];
                for (int i = 0; i < 3; ++i)
                    for (int f = 0; f < NC; ++f) gj[f] += T[j][i] * gR[i * NC + f];
                rot_fwd(T, gj, tmp);
                memcpy(dUr[j], tmp, sizeof tmp);
            }
            minvE = 0.5 * (epsinv[L] + epsinv[R]);
            minvH = 0.5 * (muinv[L] + muinv[R]);
        } else {
            const int bc = (int)(-R - 1);
            if (bc == BC_PEC) {
                pec_mirror(Ul, Ur);
                double tmp[NC];
                pec_mirror(dUl[0], tmp);
                for (int f = 0; f < NC; ++f) dUr[0][f] = -tmp[f];
                pec_mirror(dUl[1], dUr[1]);
                pec_mirror(dUl[2], dUr[2]);
            } else { /* non-reflecting: no distribution enters from the ghost side */
                memset(Ur, 0, sizeof Ur);
                memset(dUr, 0, sizeof dUr);
            }
            minvE = epsinv[L];
            minvH = muinv[L];
        }

        double Floc[NC];
        gks_face_flux(m->dim, p, Ul, Ur, dUl, dUr, minvE, minvH, Floc);
        rot_inv(T, Floc, flux + NC * s);
    }
}

/* ---------------------------------------------------------------- public entry points */

/*
 * One explicit step (Sec. 3.1, finite-volume update):
 *   U_i^{n+1} = U_i^n - dt/|Omega_i| M_i^{-1} sum_s sigma_is |l_s| F_s + dt M_i^{-1} S_i^n,
 * sigma = +1 on the owner, -1 on the neighbour.  S = (-J, 0) (Sec. 2.1 source term);
 * J is [3*ncells] (current density at t^n) or NULL.
 * Returns 0, -1 when a work buffer cannot be allocated, or -2 when the limiter is asked for on a
 * mesh that is not Cartesian.
 */
int orc_step(const orc_mesh *m, const orc_params *p, const double *U, double *Unew,
             const double *epsinv, const double *muinv, const double *J)
{
    double *grad = malloc(sizeof(double) * (size_t)m->ncells * 3 * NC);
    double *flux = malloc(sizeof(double) * (size_t)m->nfaces * NC);
    if (!grad || !flux) { free(grad); free(flux); return -1; }
    if (p->limiter) {
        if (gradients_limited(m, U, grad) != 0) { free(grad); free(flux); return -2; }
    } else if (p->gradient == 1) gradients_lsq(m, U, grad);
    else gradients(m, U, grad);
    face_fluxes(m, p, U, grad, epsinv, muinv, flux);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->ncells; ++i) {
        double acc[NC] = {0};
        for (int64_t q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; ++q) {
            const int64_t s = m->cf_idx[q];
            const double sigma = (m->face_L[s] == i) ? 1.0 : -1.0;
            for (int f = 0; f < NC; ++f) acc[f] += sigma * m->area[s] * flux[NC * s + f];
        }
        for (int f = 0; f < NC; ++f) {
            const double minv = (f < 3) ? epsinv[i] : (f < 6) ? muinv[i] : 1.0;
            double src = 0.0;
            if (J && f < 3) src = -J[3 * i + f];
            Unew[NC * i + f] = U[NC * i + f] - p->dt / m->vol[i] * minv * acc[f] + p->dt * minv * src;
        }
    }
    free(grad);
    free(flux);
    return 0;
}

/* Exposes the face flux for the unit tests: states and slopes already in the local frame. */
void orc_face_flux(int dim, const orc_params *p, const double *Ul, const double *Ur,
                   const double *dUl, const double *dUr, double minvE, double minvH, double *F)
{
    double a[3][NC], b[3][NC];
    memcpy(a, dUl, sizeof a);
    memcpy(b, dUr, sizeof b);
    gks_face_flux(dim, p, Ul, Ur, a, b, minvE, minvH, F);
}

/* Exposes the equilibrium and the rotation for the unit tests. */
void orc_equilibrium(int dim, double c, double chi, double gam, const double *V, double *g /*[4*8]*/)
{
    double u[4][3], gg[4][NC];
    lattice(dim, c, u);
    equilibrium(u, c, chi, gam, V, gg);
    memcpy(g, gg, sizeof gg);
}
void orc_lattice(int dim, double c, double *u /*[12]*/)
{
    double uu[4][3];
    lattice(dim, c, uu);
    memcpy(u, uu, sizeof uu);
}
void orc_rotation(const double *n, double *T /*[9]*/)
{
    double TT[3][3];
    rotation(n, TT);
    memcpy(T, TT, sizeof TT);
}
void orc_gradients(const orc_mesh *m, const double *U, double *grad) { gradients(m, U, grad); }
void orc_gradients_lsq(const orc_mesh *m, const double *U, double *grad) { gradients_lsq(m, U, grad); }
int orc_gradients_limited(const orc_mesh *m, const double *U, double *grad) { return gradients_limited(m, U, grad); }
