// Host-side coefficient algebra of the GKS interface flux.
//
// The kernels never evaluate the kinetic moments.  The interface flux of Sec. 3.1 is linear in
// the left/right face states and slopes for a fixed face material, so for a Cartesian face it
// is a sparse linear form of the stencil values:
//     Phi = K0 w + (1/eps_s) KE w + (1/mu_s) KH w,      Phi = (dt/h_n) * F~   (local frame)
// with w the left/right cell values and their central half-differences along the local axes
// (TM: 18 inputs, TM with the PHM potential psi: 24, EM: 48 inputs).  This file evaluates the closed-form moments of the D2Q4 /
// D3Q4 lattices in double precision and probes them with unit vectors to obtain K0, KE, KH.
// The kernels carry only the structurally non-zero entries (the tables in gks_pattern.h); the
// probe checks that every other entry is exactly zero, so a wrong table cannot go unnoticed.
#include "gks_internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

namespace gks {

// ------------------------------------------------------------------ C1..C5 (Sec. 3.1)
// C1 = dt - tau(1-e), C2 = tau(-dt + 2 tau (1-e) - dt e), C3 = dt^2/2 - tau dt + tau^2 (1-e),
// C4 = tau (1-e), C5 = tau^2 (1-e) - tau dt e, e = exp(-dt/tau).  For x = dt/tau < 1 the
// closed forms cancel badly, so their power series in x are summed instead.
void flux_coefficients(double dt, double tau, double C[5])
{
    if (tau == 0.0) {
        C[0] = dt; C[1] = 0.0; C[2] = 0.5 * dt * dt; C[3] = 0.0; C[4] = 0.0;
        return;
    }
    if (std::isinf(tau)) {
        C[0] = 0.0; C[1] = 0.0; C[2] = 0.0; C[3] = dt; C[4] = 0.5 * dt * dt;
        return;
    }
    const double x = dt / tau, d2 = dt * dt;
    if (x >= 1.0) {
        const double em1 = -std::expm1(-x), e = std::exp(-x);
        C[0] = dt * (1.0 - em1 / x);
        C[1] = d2 * ((2.0 * em1 - x * (1.0 + e)) / (x * x));
        C[2] = d2 * (0.5 - 1.0 / x + em1 / (x * x));
        C[3] = dt * (em1 / x);
        C[4] = d2 * ((em1 - x * e) / (x * x));
        return;
    }
    // series in x (m >= 0, f1 = (m+1)!, f2 = (m+2)!):
    //   C1/dt  = sum_{m>=1} (-1)^{m+1} x^m / f1     C4/dt  = sum_{m>=0} (-1)^m x^m / f1
    //   C3/dt2 = sum_{m>=1} (-1)^{m+1} x^m / f2     C5/dt2 = sum_{m>=0} (-1)^m (m+1) x^m / f2
    //   C2/dt2 = sum_{m>=1} (-1)^m m x^m / f2
    double s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
    double xm = 1.0, f1 = 1.0, f2 = 2.0;
    for (int m = 0; m <= 40; ++m) {
        if (m > 0) { xm *= x; f1 *= (m + 1); f2 *= (m + 2); }
        const double sg = (m % 2 == 0) ? 1.0 : -1.0;
        s4 += sg * xm / f1;
        s5 += sg * (m + 1) * xm / f2;
        if (m >= 1) {
            s1 -= sg * xm / f1;
            s3 -= sg * xm / f2;
            s2 += sg * m * xm / f2;
        }
    }
    C[0] = dt * s1; C[1] = d2 * s2; C[2] = d2 * s3; C[3] = dt * s4; C[4] = d2 * s5;
}

// ------------------------------------------------------------------ closed-form moments
// Directional fluxes of the perfectly hyperbolic Maxwell system (Sec. 2.1) on eight components
// (Ex, Ey, Ez, Hx, Hy, Hz, phi, psi): the curl terms, plus chi c^2 phi in E_j, gamma psi in
// H_j, chi E_j in phi and gamma c^2 H_j in psi.  chi = gamma = 0 is Maxwell's system.
constexpr int NV = 8;
struct Phm {
    double chi, gam;
};
static void Fdir(int j, const double *V, double c, Phm q, double *o)
{
    const double c2 = c * c;
    if (j == 0) {
        o[0] = 0; o[1] = c2 * V[5]; o[2] = -c2 * V[4]; o[3] = 0; o[4] = -V[2]; o[5] = V[1];
    } else if (j == 1) {
        o[0] = -c2 * V[5]; o[1] = 0; o[2] = c2 * V[3]; o[3] = V[2]; o[4] = 0; o[5] = -V[0];
    } else {
        o[0] = c2 * V[4]; o[1] = -c2 * V[3]; o[2] = 0; o[3] = -V[1]; o[4] = V[0]; o[5] = 0;
    }
    o[j] += q.chi * c2 * V[6];
    o[3 + j] += q.gam * V[7];
    o[6] = q.chi * V[j];
    o[7] = q.gam * c2 * V[3 + j];
}

// Closed-form GKS flux dt*F~ in the face frame (normal = local axis 1) from the reconstructed
// states Ul, Ur and the physical slopes sl[j], sr[j] along the local axes, for the D2Q4
// (dim 2; sl[2], sr[2] ignored) or D3Q4 (dim 3) lattice:
//   half moments      <g(V)>_{+-} = V/2 +- F1(V)/(2c),   <u1 g(V)>_{+-} = +-cV/2 + F1(V)/2
//   slope moments     Q(s)  = <u1 u.grad g> = c^2 s1 (+ c [F3(s2) + F2(s3)] on D3Q4)
//                     Q+-(s) = c^2 s1/2 +- c F1(s1)/2 +- c F2(s2)/2           (D2Q4)
//                     Q+(s) = c^2 s1/2 + c F1(s1)/2 + c [F2(s2)+F3(s2)+F2(s3)+F3(s3)]/2
//                     Q-(s) = c^2 s1/2 - c F1(s1)/2 + c [F3(s2)-F2(s2)+F2(s3)-F3(s3)]/2   (D3Q4)
//   dt F~ = C1 F1(U0) + C2 Q(grad U0) + C3 F1(U_t) + C4 [<u1 g^l>_+ + <u1 g^r>_-]
//           - C5 [Q+(grad U^l) + Q-(grad U^r)]
// with U0 = <g^l>_+ + <g^r>_-, grad U0 likewise, U_t = -M_s^{-1} sum_j F_j(d_j U0).
static void closed_flux(int dim, double c, Phm ph, const double C[5], const double *Ul, const double *Ur,
                        const double sl[3][NV], const double sr[3][NV], double mE, double mH, double *out)
{
    auto F1 = [&](const double *V, double, double *o) { Fdir(0, V, c, ph, o); };
    auto F2 = [&](const double *V, double, double *o) { Fdir(1, V, c, ph, o); };
    auto F3 = [&](const double *V, double, double *o) { Fdir(2, V, c, ph, o); };
    double a[NV], b[NV], U0[NV], s0[3][NV];
    F1(Ul, c, a);
    F1(Ur, c, b);
    for (int f = 0; f < NV; ++f) U0[f] = 0.5 * (Ul[f] + Ur[f]) + (a[f] - b[f]) / (2 * c);
    const int nd = dim;
    for (int j = 0; j < 3; ++j) {
        if (j >= nd) { std::memset(s0[j], 0, sizeof s0[j]); continue; }
        F1(sl[j], c, a);
        F1(sr[j], c, b);
        for (int f = 0; f < NV; ++f) s0[j][f] = 0.5 * (sl[j][f] + sr[j][f]) + (a[f] - b[f]) / (2 * c);
    }
    auto Q = [&](const double s[3][NV], int half, double *o) {
        double p1[NV], p2[NV], p3[NV], q2[NV], q3[NV];
        F1(s[0], c, p1);
        F2(s[1], c, p2);
        F3(s[1], c, p3);
        F2(s[2], c, q2);
        F3(s[2], c, q3);
        for (int f = 0; f < NV; ++f) {
            if (half == 0) {
                o[f] = c * c * s[0][f] + (nd == 3 ? c * (p3[f] + q2[f]) : 0.0);
            } else {
                const double h = (half > 0) ? 1.0 : -1.0;
                double v = 0.5 * c * c * s[0][f] + h * 0.5 * c * p1[f];
                if (nd == 2) v += h * 0.5 * c * p2[f];
                else if (half > 0) v += 0.5 * c * (p2[f] + p3[f] + q2[f] + q3[f]);
                else v += 0.5 * c * (p3[f] - p2[f] + q2[f] - q3[f]);
                o[f] = v;
            }
        }
    };
    double Ut[NV] = {0}, Fj[NV];
    F1(s0[0], c, Fj);
    for (int f = 0; f < NV; ++f) Ut[f] -= Fj[f];
    F2(s0[1], c, Fj);
    for (int f = 0; f < NV; ++f) Ut[f] -= Fj[f];
    if (nd == 3) {
        F3(s0[2], c, Fj);
        for (int f = 0; f < NV; ++f) Ut[f] -= Fj[f];
    }
    // material factors on E and H; the potentials carry none
    for (int f = 0; f < 3; ++f) Ut[f] *= mE;
    for (int f = 3; f < 6; ++f) Ut[f] *= mH;

    double m1[NV], m2[NV], m3[NV], ql[NV], qr[NV];
    F1(U0, c, m1);
    Q(s0, 0, m2);
    F1(Ut, c, m3);
    Q(sl, +1, ql);
    Q(sr, -1, qr);
    F1(Ul, c, a);
    F1(Ur, c, b);
    for (int f = 0; f < NV; ++f) {
        const double m4 = 0.5 * c * (Ul[f] - Ur[f]) + 0.5 * (a[f] + b[f]);
        out[f] = C[0] * m1[f] + C[1] * m2[f] + C[2] * m3[f] + C[3] * m4 - C[4] * (ql[f] + qr[f]);
    }
}

// ------------------------------------------------------------------ Cartesian face operators
// Rotation T' of Sec. 3.1 for a unit normal n: its rows are the local axes in global
// coordinates (local x along n), with T' = diag(-1, -1, 1) when n1 = -1.
static void face_rotation(const double n[3], double T[3][3])
{
    if (n[0] == -1.0) {
        std::memset(T, 0, 9 * sizeof(double));
        T[0][0] = -1.0; T[1][1] = -1.0; T[2][2] = 1.0;
        return;
    }
    const double q = 1.0 + n[0];
    T[0][0] = n[0];  T[0][1] = n[1];                      T[0][2] = n[2];
    T[1][0] = -n[1]; T[1][1] = n[0] + n[2] * n[2] / q;    T[1][2] = -n[1] * n[2] / q;
    T[2][0] = -n[2]; T[2][1] = -n[1] * n[2] / q;          T[2][2] = 1.0 - n[2] * n[2] / q;
}

// diag(T', T', 1, 1) on (E, H, phi, psi): the potentials are scalars
static void rotate_fields(const double T[3][3], const double *a, double *b, bool inverse)
{
    for (int blk = 0; blk < 2; ++blk)
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += (inverse ? T[k][r] : T[r][k]) * a[3 * blk + k];
            b[3 * blk + r] = s;
        }
    b[6] = a[6];
    b[7] = a[7];
}

// Position of field q of a model inside (Ex, Ey, Ez, Hx, Hy, Hz, phi, psi).
static int model_fields(int model)
{
    return model == GKS_TM2D ? 3 : model == GKS_TM2D_PHM ? 4 : model == GKS_EM3D ? 6 : 8;
}
static bool model_3d(int model) { return model == GKS_EM3D || model == GKS_EM3D_PHM; }
static int model_component(int model, int q)
{
    if (model == GKS_TM2D) return 2 + q;                  // Ez, Hx, Hy
    if (model == GKS_TM2D_PHM) return q < 3 ? 2 + q : 7;  // Ez, Hx, Hy, psi
    return q;                                             // Ex .. Hz (, phi, psi)
}

// Axis-aligned Cartesian face with normal +e_ax; inputs and outputs in the global frame:
//   w = [UL UR dnL dt1L (dt2L) dnR dt1R (dt2R)] x fields,
// d = dfac * h * (central slope) along the face normal (dn) and the remaining axes in increasing
// order (dt1, dt2).  Reconstruction (Sec. 3.1): U^l = U_L + (h_n/2) dU_L/dn, U^r = U_R - (h_n/2)
// dU_R/dn; states and slopes are rotated into the face frame (d~_j U~ = sum_i T'_ji T d_i U),
// the closed-form flux is evaluated there and rotated back.  Output phi = (dt/h_n) F (global).
static void cart_flux_eval(int model, int ax, double c, Phm ph, const double C[5], const double h[3], double dfac,
                           const double *w, double mE, double mH, double *phi)
{
    const int nf = model_fields(model);
    const int nd = model_3d(model) ? 3 : 2;
    int axes[3] = {ax, 0, 0};
    for (int i = 0, k = 1; i < nd; ++i)
        if (i != ax) axes[k++] = i;
    double UL[NV] = {0}, UR[NV] = {0}, gL[3][NV] = {{0}}, gR[3][NV] = {{0}};
    for (int q = 0; q < nf; ++q) {
        const int f = model_component(model, q);
        UL[f] = w[q];
        UR[f] = w[nf + q];
        for (int j = 0; j < nd; ++j) {
            const int i = axes[j];
            gL[i][f] = w[2 * nf + j * nf + q] / (dfac * h[i]);
            gR[i][f] = w[2 * nf + nd * nf + j * nf + q] / (dfac * h[i]);
        }
    }
    double n[3] = {0, 0, 0};
    n[ax] = 1.0;
    double T[3][3];
    face_rotation(n, T);
    double Ugl[NV], Ugr[NV], Ul[NV], Ur[NV], sl[3][NV], sr[3][NV];
    for (int f = 0; f < NV; ++f) {
        Ugl[f] = UL[f] + 0.5 * h[ax] * gL[ax][f];
        Ugr[f] = UR[f] - 0.5 * h[ax] * gR[ax][f];
    }
    rotate_fields(T, Ugl, Ul, false);
    rotate_fields(T, Ugr, Ur, false);
    for (int j = 0; j < 3; ++j) {
        double al[NV] = {0}, ar[NV] = {0};
        for (int i = 0; i < 3; ++i)
            for (int f = 0; f < NV; ++f) {
                al[f] += T[j][i] * gL[i][f];
                ar[f] += T[j][i] * gR[i][f];
            }
        rotate_fields(T, al, sl[j], false);
        rotate_fields(T, ar, sr[j], false);
    }
    double out[NV], Fg[NV];
    closed_flux(nd, c, ph, C, Ul, Ur, sl, sr, mE, mH, out);
    rotate_fields(T, out, Fg, true);
    for (int q = 0; q < nf; ++q) phi[q] = Fg[model_component(model, q)] / h[ax];
}

// Face operator on reconstructed states (triangles): inputs [Ul Ur s1l s2l s1r s2r] x the
// model's fields in the face frame (TM: Ez, Hn, Ht; with PHM also psi), physical slopes;
// output dt * F~ (the caller scales by |l_s|/|Omega_i|).
static void face_flux_eval(int model, double c, Phm ph, const double C[5], const double *w, double mE, double mH,
                           double *phi)
{
    const int nf = model_fields(model);
    double Ul[NV] = {0}, Ur[NV] = {0}, sl[3][NV] = {{0}}, sr[3][NV] = {{0}};
    for (int q = 0; q < nf; ++q) {
        const int f = model_component(model, q);
        Ul[f] = w[q];
        Ur[f] = w[nf + q];
        sl[0][f] = w[2 * nf + q];
        sl[1][f] = w[3 * nf + q];
        sr[0][f] = w[4 * nf + q];
        sr[1][f] = w[5 * nf + q];
    }
    double out[NV];
    closed_flux(2, c, ph, C, Ul, Ur, sl, sr, mE, mH, out);
    for (int q = 0; q < nf; ++q) phi[q] = out[model_component(model, q)];
}

// Face operator on reconstructed states in 3D (tetrahedra): inputs [Ul Ur s1l s2l s3l s1r s2r s3r]
// x (Ex, Ey, Ez, Hx, Hy, Hz) in the face frame, physical slopes along the face axes; output
// dt * F~ in the face frame.
static void tet_flux_eval(double c, const double C[5], const double *w, double mE, double mH, double *phi)
{
    double Ul[NV] = {0}, Ur[NV] = {0}, sl[3][NV] = {{0}}, sr[3][NV] = {{0}};
    for (int q = 0; q < 6; ++q) {
        Ul[q] = w[q];
        Ur[q] = w[6 + q];
        for (int j = 0; j < 3; ++j) {
            sl[j][q] = w[12 + 6 * j + q];
            sr[j][q] = w[30 + 6 * j + q];
        }
    }
    double out[NV];
    closed_flux(3, c, Phm{0.0, 0.0}, C, Ul, Ur, sl, sr, mE, mH, out);
    for (int q = 0; q < 6; ++q) phi[q] = out[q];
}

// Probe a linear evaluator into dense K0/KE/KH and compress to the pattern tables.
template <typename Eval>
static bool probe(int nout, int nin, Eval ev, const Pattern &pat, double *k0, double *ke, double *kh,
                  char *err, size_t errlen)
{
    std::vector<double> D0(nout * nin), DE(nout * nin), DH(nout * nin);
    std::vector<double> w(nin, 0.0), phi(nout);
    for (int i = 0; i < nin; ++i) {
        w.assign(nin, 0.0);
        w[i] = 1.0;
        ev(w.data(), 0.0, 0.0, phi.data());
        for (int r = 0; r < nout; ++r) D0[r * nin + i] = phi[r];
        ev(w.data(), 1.0, 0.0, phi.data());
        for (int r = 0; r < nout; ++r) DE[r * nin + i] = phi[r] - D0[r * nin + i];
        ev(w.data(), 0.0, 1.0, phi.data());
        for (int r = 0; r < nout; ++r) DH[r * nin + i] = phi[r] - D0[r * nin + i];
    }
    auto compress = [&](std::vector<double> &D, int nnz, const uint8_t *row, const uint8_t *col,
                        double *k, const char *name) {
        for (int q = 0; q < nnz; ++q) {
            k[q] = D[row[q] * nin + col[q]];
            D[row[q] * nin + col[q]] = 0.0;
        }
        for (int e = 0; e < nout * nin; ++e)
            if (D[e] != 0.0) {
                std::snprintf(err, errlen, "internal: %s entry (%d,%d) = %g outside the sparsity table",
                              name, e / nin, e % nin, D[e]);
                return false;
            }
        return true;
    };
    return compress(D0, pat.n0, pat.r0, pat.c0, k0, "K0") && compress(DE, pat.nE, pat.rE, pat.cE, ke, "KE") &&
           compress(DH, pat.nH, pat.rH, pat.cH, kh, "KH");
}

bool cart_face_operator(int model, int axis, double c, double chi, double gamma, const double C[5],
                        const double h[3], double dfac, double *k0, double *ke, double *kh, char *err, size_t errlen)
{
    const int nf = model_fields(model);
    const int nin = (model_3d(model) ? 8 : 6) * nf;
    auto ev = [&](const double *w, double mE, double mH, double *phi) {
        cart_flux_eval(model, axis, c, Phm{chi, gamma}, C, h, dfac, w, mE, mH, phi);
    };
    return probe(nf, nin, ev, pattern_cart(model, axis), k0, ke, kh, err, errlen);
}

bool tri_face_operator(int model, double c, double chi, double gamma, const double C[5], double *k0, double *ke,
                       double *kh, char *err, size_t errlen)
{
    const int nf = model_fields(model);
    auto ev = [&](const double *w, double mE, double mH, double *phi) {
        face_flux_eval(model, c, Phm{chi, gamma}, C, w, mE, mH, phi);
    };
    return probe(nf, 6 * nf, ev, pattern_tri(model), k0, ke, kh, err, errlen);
}

bool tet_face_operator(double c, const double C[5], double *k0, double *ke, double *kh, char *err, size_t errlen)
{
    auto ev = [&](const double *w, double mE, double mH, double *phi) { tet_flux_eval(c, C, w, mE, mH, phi); };
    return probe(6, 48, ev, pattern_tet(), k0, ke, kh, err, errlen);
}

}  // namespace gks

extern "C" gks_status gks_flux_coefficients(double dt, double tau, double C_out[5])
{
    if (!C_out || !(dt > 0.0) || !std::isfinite(dt) || !(tau >= 0.0)) return GKS_EINVAL;
    gks::flux_coefficients(dt, tau, C_out);
    return GKS_OK;
}
