"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: Maxwell's curl equations,
the exact BGK characteristic solution (ODE integration), the eigen-decomposition of the flux
Jacobian (Sec. 3.3 / Sec. 4.1 equivalence), the textbook Fromm scheme, the von Neumann symbol of
the whole step written independently from the closed-form lattice moments, exact solutions, mirror
and rotation symmetries, and the error tables printed in the paper (Sec. 5.1, Sec. 5.2).
"""
import os

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

from oracle import exact as X

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(1234)


def curl_operator(k, c=1.0):
    """sum_j k_j A_j from Maxwell's equations: dE/dt = c^2 curl B, dB/dt = -curl E, written
    as dU/dt + sum_j d_j (A_j U) = 0, i.e. sum_j k_j A_j U = (-c^2 k x B, k x E)."""
    A = np.zeros((6, 6))
    for q in range(6):
        U = np.zeros(6)
        U[q] = 1.0
        A[:3, q] = -c * c * np.cross(k, U[3:])
        A[3:, q] = np.cross(k, U[:3])
    return A


# ------------------------------------------------------------------ lattice and equilibrium
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("c", [1.0, 1.7])
def test_lattice_moments(oracle, dim, c):
    u = oracle.lattice(dim, c)
    nd = dim
    assert np.allclose(u.sum(0), 0, atol=1e-15)
    M2 = np.einsum("ki,kj->ij", u[:, :nd], u[:, :nd])
    assert np.allclose(M2, 4 * c * c * np.eye(nd), atol=1e-14)
    M3 = np.einsum("ki,kj,km->ijm", u, u, u)
    if dim == 3:
        # D3Q4: the only third moments are u^1 u^2 u^3 = 4 c^3 (all permutations)
        expect = np.zeros((3, 3, 3))
        for p in [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]:
            expect[p] = 4 * c ** 3
        assert np.allclose(M3, expect, atol=1e-13)
    else:
        assert np.allclose(M3, 0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_compatibility(oracle, dim):
    """sum_k g_k = U and sum_k u_k^j g_k = F_j(U), with F_j pinned to Maxwell's curl equations."""
    c = 1.3
    u = oracle.lattice(dim, c)
    A = np.zeros((3, 6, 6))
    for q in range(6):
        e = np.zeros(6)
        e[q] = 1.0
        g = oracle.equilibrium(dim, e, c)
        assert np.allclose(g.sum(0), e, atol=1e-15)
        for j in range(3):
            A[j, :, q] = (u[:, j][:, None] * g).sum(0)
    for _ in range(5):
        k = RNG.normal(size=3)
        if dim == 2:
            k[2] = 0.0
        assert np.allclose(np.einsum("j,jab->ab", k, A), curl_operator(k, c), atol=1e-14)


# ------------------------------------------------------------------ face frame
def test_rotation_matrix(oracle):
    for _ in range(50):
        n = RNG.normal(size=3)
        n /= np.linalg.norm(n)
        T = oracle.rotation(n)
        # the printed formula divides by 1 + n1: rounding grows as n1 -> -1
        tol = 1e-15 / (1.0 + n[0])
        assert np.allclose(T @ T.T, np.eye(3), atol=tol)
        assert abs(np.linalg.det(T) - 1) < tol
        assert np.allclose(T @ n, [1, 0, 0], atol=tol)
    T = oracle.rotation(np.array([-1.0, 0, 0]))
    assert np.array_equal(T, np.diag([-1.0, -1.0, 1.0]))
    # Cartesian face frames: x-face (x, y, z), y-face (y, -x, z), z-face (z, y, -x)
    assert np.allclose(oracle.rotation(np.array([0, 1.0, 0])), [[0, 1, 0], [-1, 0, 0], [0, 0, 1]])
    assert np.allclose(oracle.rotation(np.array([0, 0, 1.0])), [[0, 0, 1], [0, 1, 0], [-1, 0, 0]])


# ------------------------------------------------------------------ time-integrated coefficients
@pytest.mark.parametrize("tau_hat", [1e-3, 0.01, 0.3, 1.0, 7.0, 100.0])
def test_coefficients_match_bgk_characteristic_solution(oracle, tau_hat):
    """The flux coefficients reproduce the time average of the exact solution of the BGK
    equation df/dt + u df/dx = (g - f)/tau at x = 0, with the linear equilibrium
    g(x, t) = g0 + sg x + gt t and the linear initial distribution f(x, 0) = f0 + sf x,
    obtained here by integrating the ODE along the characteristic x(t') = -u (t - t')."""
    dt = 0.37
    tau = tau_hat * dt
    C = oracle.coefficients(dt, tau)
    g0, sg, gt, f0, sf, u = 0.7, -1.3, 0.45, -0.2, 2.1, 0.8

    def f_at(t):
        if t == 0.0:
            return f0
        rhs = lambda tp, F: [((g0 + sg * (-u * (t - tp)) + gt * tp) - F[0]) / tau]
        sol = solve_ivp(rhs, (0.0, t), [f0 + sf * (-u * t)], rtol=1e-12, atol=1e-14, method="DOP853")
        return sol.y[0, -1]

    avg = quad(f_at, 0.0, dt, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    pred = C[0] * g0 + C[1] * u * sg + C[2] * gt + C[3] * f0 - C[4] * u * sf
    assert abs(avg - pred) < 2e-10 * max(1.0, abs(avg))


def test_coefficient_limits(oracle):
    dt = 0.01
    C0 = oracle.coefficients(dt, 0.0)
    Ci = oracle.coefficients(dt, np.inf)
    assert np.allclose(C0, [dt, 0, dt * dt / 2, 0, 0], rtol=0, atol=1e-18)
    assert np.allclose(Ci, [0, 0, 0, dt, dt * dt / 2], rtol=0, atol=1e-18)
    Cs = oracle.coefficients(dt, 1e-9 * dt)
    Cl = oracle.coefficients(dt, 1e9 * dt)
    scale = np.array([dt, dt * dt, dt * dt, dt, dt * dt])
    assert np.allclose(np.array(Cs) / scale, np.array(C0) / scale, rtol=0, atol=1e-8)
    assert np.allclose(np.array(Cl) / scale, np.array(Ci) / scale, rtol=0, atol=1e-8)
    for th in (1e-4, 0.01, 1, 1e4):
        C = oracle.coefficients(dt, th * dt)
        assert abs(C[0] + C[3] - dt) < 1e-16
        assert abs((C[1] - C[4]) - (C[2] - dt * dt / 2)) < 1e-19


# ------------------------------------------------------------------ the interface flux
def split_jacobian(c=1.0):
    A1 = curl_operator(np.array([1.0, 0, 0]), c)
    lam, R = np.linalg.eig(A1)
    lam, R = lam.real, R.real
    Rinv = np.linalg.inv(R)
    Ap = R @ np.diag(np.maximum(lam, 0)) @ Rinv
    Am = R @ np.diag(np.minimum(lam, 0)) @ Rinv
    return Ap, Am


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("tau", [0.0, np.inf])
def test_flux_without_slopes_is_upwind_splitting(oracle, dim, tau):
    """With zero slopes, tau = 0 gives the equilibrium flux of the interface state, which is
    the upwind flux A+ U_L + A- U_R (A+- from the eigen-decomposition of the x Jacobian,
    Sec. 3.3).  tau -> inf gives kinetic flux-vector splitting, equal to A+ U_L + A- U_R on
    the propagating components (Sec. 4.1); the normal components (Ex, Hx), which Maxwell's
    flux does not transport, are moved by the lattice at +-c: F = c (U_L - U_R) / 2."""
    c = 1.0
    Ap, Am = split_jacobian(c)
    z = np.zeros((3, 6))
    normal = [0, 3]
    for _ in range(5):
        UL, UR = RNG.normal(size=6), RNG.normal(size=6)
        if dim == 2:
            UL[[0, 1, 5]] = 0
            UR[[0, 1, 5]] = 0
        for ur in (UR, np.zeros(6)):        # second case: non-reflecting side, F = A+ U_L
            F = oracle.face_flux(dim, 0.1, tau, UL, ur, z, z, c=c)
            ref = Ap @ UL + Am @ ur
            if np.isinf(tau):
                ref[normal] = 0.5 * c * (UL[normal] - ur[normal])
            assert np.allclose(F, ref, atol=1e-14)


@pytest.mark.parametrize("tau_hat", [0.0, 0.3, np.inf])
def test_face_flux_equals_d3q4_closed_forms(oracle, tau_hat):
    """The oracle's literal sums over the four D3Q4 velocities equal the closed-form moments of
    the lattice (third moment 4 c^3 |eps_1jm|): with F_j = A_j from Maxwell's curl equations,
    U0 = (Ul + Ur)/2 + (F1 Ul - F1 Ur)/(2c), Q(s) = c^2 s1 + c [F3 s2 + F2 s3],
    Q+(s) = c^2 s1/2 + c F1 s1/2 + c [F2 s2 + F3 s2 + F3 s3 + F2 s3]/2,
    Q-(s) = c^2 s1/2 - c F1 s1/2 - c [F2 s2 - F3 s2 + F3 s3 - F2 s3]/2,
    U_t = -M^-1 sum_j F_j s0_j, and dt F = C1 F1 U0 + C2 Q(s0) + C3 F1 U_t
    + C4 [c (Ul - Ur)/2 + (F1 Ul + F1 Ur)/2] - C5 [Q+(sl) + Q-(sr)]."""
    c, dt = 1.4, 0.03
    A = [curl_operator(np.eye(3)[j], c) for j in range(3)]
    C = oracle.coefficients(dt, tau_hat * dt)
    for _ in range(4):
        Ul, Ur = RNG.normal(size=6), RNG.normal(size=6)
        sl, sr = RNG.normal(size=(3, 6)), RNG.normal(size=(3, 6))
        mE, mH = RNG.uniform(0.3, 1.0, 2)
        U0 = 0.5 * (Ul + Ur) + (A[0] @ Ul - A[0] @ Ur) / (2 * c)
        s0 = [0.5 * (sl[j] + sr[j]) + (A[0] @ sl[j] - A[0] @ sr[j]) / (2 * c) for j in range(3)]
        Q = c * c * s0[0] + c * (A[2] @ s0[1] + A[1] @ s0[2])
        Qp = 0.5 * c * c * sl[0] + 0.5 * c * (A[0] @ sl[0]) + 0.5 * c * (A[1] @ sl[1] + A[2] @ sl[1] + A[2] @ sl[2]
                                                                          + A[1] @ sl[2])
        Qm = 0.5 * c * c * sr[0] - 0.5 * c * (A[0] @ sr[0]) - 0.5 * c * (A[1] @ sr[1] - A[2] @ sr[1] + A[2] @ sr[2]
                                                                          - A[1] @ sr[2])
        Ut = -sum(A[j] @ s0[j] for j in range(3))
        Ut[:3] *= mE
        Ut[3:] *= mH
        dtF = (C[0] * (A[0] @ U0) + C[1] * Q + C[2] * (A[0] @ Ut)
               + C[3] * (0.5 * c * (Ul - Ur) + 0.5 * (A[0] @ Ul + A[0] @ Ur)) - C[4] * (Qp + Qm))
        F = oracle.face_flux(3, dt, tau_hat * dt, Ul, Ur, sl, sr, mE, mH, c=c)
        assert np.allclose(F, dtF / dt, rtol=0, atol=1e-13 * max(1.0, np.abs(dtF / dt).max())), (F, dtF / dt)


def fromm_step(w, nu):
    """Fromm's method for w_t + a w_x = 0, a > 0, Courant number nu (average of Lax-Wendroff
    and Beam-Warming; periodic)."""
    wm1, wm2, wp1 = np.roll(w, 1), np.roll(w, 2), np.roll(w, -1)
    return w - nu * (w - wm1) - 0.25 * nu * (1 - nu) * (wp1 - w - wm1 + wm2)


@pytest.mark.parametrize("tau_hat", [0.0, 0.01, 1.0, np.inf])
@pytest.mark.parametrize("axis", [0, 1])
def test_one_dimensional_data_gives_fromm_2d(oracle, tau_hat, axis):
    """Data varying along one axis only: each characteristic pair follows Fromm's scheme."""
    N, nu = 24, 0.43
    mesh = oracle.cart2d(N, 3) if axis == 0 else oracle.cart2d(3, N)
    s = mesh.centroid[:, axis]
    a = np.sin(2 * np.pi * s) + 0.3 * np.cos(6 * np.pi * s)     # right-going invariant
    b = np.cos(4 * np.pi * s) - 0.2 * np.sin(2 * np.pi * s)    # left-going invariant
    U = np.zeros((mesh.ncells, 6))
    # along x: Ez - Hy moves +x, Ez + Hy moves -x; along y: Ez + Hx moves +y, Ez - Hx moves -y
    ht = 4 if axis == 0 else 3
    sgn = -1.0 if axis == 0 else 1.0
    U[:, 2] = 0.5 * (a + b)
    U[:, ht] = sgn * 0.5 * (a - b)
    dt = nu / N
    V = oracle.step(mesh, U, dt, tau_hat * dt)
    ap = V[:, 2] + sgn * V[:, ht]
    bm = V[:, 2] - sgn * V[:, ht]
    shape = (3, N) if axis == 0 else (N, 3)
    A = a.reshape(shape)
    B = b.reshape(shape)
    if axis == 1:
        A, B = A.T, B.T
    ref_a = np.stack([fromm_step(r, nu) for r in A])
    ref_b = np.stack([fromm_step(r[::-1], nu)[::-1] for r in B])
    got_a, got_b = ap.reshape(shape), bm.reshape(shape)
    if axis == 1:
        got_a, got_b = got_a.T, got_b.T
    assert np.max(np.abs(got_a - ref_a)) < 1e-14
    assert np.max(np.abs(got_b - ref_b)) < 1e-14
    # the normal magnetic component stays zero
    assert np.max(np.abs(V[:, 3 if axis == 0 else 4])) < 1e-15


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_one_dimensional_data_gives_fromm_3d(oracle, axis):
    """3D grid, data along one axis: (E_t, H_t) pairs follow Fromm's scheme on every face frame."""
    N, nu = 20, 0.3
    n = [2, 2, 2]
    n[axis] = N
    mesh = oracle.cart3d(*n)
    s = mesh.centroid[:, axis]
    e = np.zeros(3)
    e[axis] = 1.0
    # transverse E along t1, H along t2 = e x t1
    t1 = np.roll(e, 1)
    t2 = np.cross(e, t1)
    a = np.sin(2 * np.pi * s) + 0.2 * np.cos(4 * np.pi * s)
    b = np.cos(2 * np.pi * s)
    # right-going: H = e x E ; left-going: H = -e x E
    U = np.zeros((mesh.ncells, 6))
    U[:, :3] = np.outer(0.5 * (a + b), t1)
    U[:, 3:] = np.outer(0.5 * (a - b), t2)
    dt = nu / N
    V = oracle.step(mesh, U, dt, 0.01 * dt)
    Et, Ht = V[:, :3] @ t1, V[:, 3:] @ t2
    shape = [n[2], n[1], n[0]]
    got_a = np.moveaxis((Et + Ht).reshape(shape), 2 - axis, -1).reshape(-1, N)
    got_b = np.moveaxis((Et - Ht).reshape(shape), 2 - axis, -1).reshape(-1, N)
    A = np.moveaxis(a.reshape(shape), 2 - axis, -1).reshape(-1, N)
    B = np.moveaxis(b.reshape(shape), 2 - axis, -1).reshape(-1, N)
    assert np.max(np.abs(got_a - np.stack([fromm_step(r, nu) for r in A]))) < 1e-14
    assert np.max(np.abs(got_b - np.stack([fromm_step(r[::-1], nu)[::-1] for r in B]))) < 1e-14


# ------------------------------------------------------------------ symmetries and boundaries
def smooth_field(xy, seed):
    r = np.random.default_rng(seed)
    out = np.zeros(xy.shape[0])
    for _ in range(4):
        kx, ky = r.integers(-3, 4, size=2)
        out += r.normal() * np.cos(2 * np.pi * (kx * xy[:, 0] + ky * xy[:, 1]) + r.uniform(0, 6.3))
    return out


def test_rotation_invariance_2d(oracle):
    """A 90-degree rotation of a periodic problem (with a material map) commutes with the step."""
    N = 16
    mesh = oracle.cart2d(N, N)
    xy = mesh.centroid[:, :2]
    U = np.zeros((mesh.ncells, 6))
    for q, s in zip((2, 3, 4), (1, 2, 3)):
        U[:, q] = smooth_field(xy, s)
    epsinv = 1.0 / (1.5 + 0.5 * np.sin(2 * np.pi * xy[:, 0]) * np.cos(2 * np.pi * xy[:, 1]))
    dt = 0.4 / N

    def rot(V, einv):   # (x, y) -> (y, 1 - x); (Hx, Hy) -> (Hy, -Hx)
        W = np.zeros_like(V)
        Vg = V.reshape(N, N, 6)         # [j][i]
        Wg = W.reshape(N, N, 6)
        Wg[:, :, :] = np.rot90(Vg, k=1, axes=(0, 1))
        hx, hy = Wg[:, :, 3].copy(), Wg[:, :, 4].copy()
        Wg[:, :, 3], Wg[:, :, 4] = hy, -hx
        e = np.rot90(einv.reshape(N, N), k=1, axes=(0, 1)).reshape(-1)
        return W, e

    A = oracle.step(mesh, U, dt, 0.01 * dt, epsinv=epsinv)
    Ur, er = rot(U, epsinv)
    B = oracle.step(mesh, Ur, dt, 0.01 * dt, epsinv=er)
    Ar, _ = rot(A, epsinv)
    assert np.max(np.abs(Ar - B)) < 1e-14 * np.max(np.abs(A))


def test_gradient_is_central_difference_on_cartesian(oracle):
    N = 12
    mesh = oracle.cart2d(N, N, bc=(0, 0, 0, 0))
    U = RNG.normal(size=(mesh.ncells, 6))
    g = oracle.gradients(mesh, U)
    Ug = U.reshape(N, N, 6)
    gx = (np.roll(Ug, -1, axis=1) - np.roll(Ug, 1, axis=1)) / (2.0 / N)
    gy = (np.roll(Ug, -1, axis=0) - np.roll(Ug, 1, axis=0)) / (2.0 / N)
    assert np.allclose(g[:, 0, :].reshape(N, N, 6), gx, atol=1e-12)
    assert np.allclose(g[:, 1, :].reshape(N, N, 6), gy, atol=1e-12)
    assert np.all(g[:, 2, :] == 0)


def test_pec_box_equals_mirrored_periodic_run(oracle):
    """PEC walls on [0,1]^2 equal the periodic run on [-1,1]^2 of the mirror extension
    (Ez odd, normal H odd, tangential H even across each wall)."""
    N, nsteps = 12, 6
    box = oracle.cart2d(N, N, bc=(2, 2, 2, 2))
    big = oracle.cart2d(2 * N, 2 * N, lo=(-1, -1), hi=(1, 1))
    xy = box.centroid[:, :2]
    ez = smooth_field(xy, 7).reshape(N, N)
    hx = smooth_field(xy, 8).reshape(N, N)
    hy = smooth_field(xy, 9).reshape(N, N)

    def extend(f, sx, sy):   # [j][i] on [0,1]^2 -> [-1,1]^2 with parities sx (x-mirror), sy
        top = np.concatenate([sx * f[:, ::-1], f], axis=1)
        return np.concatenate([sy * top[::-1, :], top], axis=0)

    Ub = np.zeros((box.ncells, 6))
    Ub[:, 2], Ub[:, 3], Ub[:, 4] = ez.ravel(), hx.ravel(), hy.ravel()
    Ug = np.zeros((big.ncells, 6))
    Ug[:, 2] = extend(ez, -1, -1).ravel()
    Ug[:, 3] = extend(hx, -1, +1).ravel()
    Ug[:, 4] = extend(hy, +1, -1).ravel()
    dt = 0.5 / N
    A = oracle.run(box, Ub, nsteps, dt, 0.01 * dt)
    B = oracle.run(big, Ug, nsteps, dt, 0.01 * dt)
    Bq = B.reshape(2 * N, 2 * N, 6)[N:, N:, :].reshape(-1, 6)
    assert np.max(np.abs(A - Bq)) < 1e-13 * np.max(np.abs(A))


def test_pec_walls_3d_equal_mirrored_periodic_run(oracle):
    """3D: PEC on z-, z+ (tangential E odd, normal H odd) equals the mirrored periodic run over
    one step.  (The D3Q4 tetrahedron is not mirror-symmetric, so the doubled periodic run
    itself does not stay a mirror image beyond the first step.)"""
    n, nz, nsteps = 6, 4, 1
    box = oracle.cart3d(n, n, nz, bc=(0, 0, 0, 0, 2, 2))
    big = oracle.cart3d(n, n, 2 * nz, lo=(0, 0, -1), hi=(1, 1, 1))
    r = np.random.default_rng(5)
    F = r.normal(size=(nz, n, n, 6))
    par = np.array([-1, -1, +1, +1, +1, -1])   # Ex, Ey tangential (odd); Ez normal (even); Hz normal (odd)
    Fb = np.concatenate([F[::-1] * par, F], axis=0)
    dt = 0.25 / n
    A = oracle.run(box, F.reshape(-1, 6), nsteps, dt, 0.01 * dt)
    B = oracle.run(big, Fb.reshape(-1, 6), nsteps, dt, 0.01 * dt)
    assert np.max(np.abs(A - B.reshape(2 * nz, n, n, 6)[nz:].reshape(-1, 6))) < 1e-13 * np.max(np.abs(A))


def test_nonreflecting_normal_incidence_is_exact(oracle):
    """A right-going pulse leaves through a non-reflecting side without any left-going wave."""
    N = 64
    mesh = oracle.cart2d(N, 2, bc=(1, 1, 0, 0))
    x = mesh.centroid[:, 0]
    a = np.exp(-((x - 0.6) / 0.08) ** 2)
    U = np.zeros((mesh.ncells, 6))
    U[:, 2], U[:, 4] = 0.5 * a, -0.5 * a            # Ez - Hy = a, Ez + Hy = 0
    dt = 0.5 / N
    for _ in range(6):
        U = oracle.run(mesh, U, 20, dt, 0.01 * dt)
        assert np.max(np.abs(U[:, 2] + U[:, 4])) < 1e-15
    assert np.max(np.abs(U)) < 1e-6                   # the pulse has left


def test_nonreflecting_oblique_reflection_is_reported(oracle):
    """Oblique incidence has no exact statement in the paper: the kinetic non-reflecting side
    zeroes the incoming distributions, which is exact for waves along the normal only.  The
    reflection of a localized pulse (Gaussian Ez with H for propagation along (1, 1); it also
    radiates in every other direction) is measured against the same run on a 3x larger domain
    whose sides the waves have not reached; its size is reported (parity unpinned) and bounded
    loosely."""
    N = 64
    small = oracle.cart2d(N, N, bc=(1, 1, 1, 1))
    big = oracle.cart2d(3 * N, 3 * N, lo=(-1, -1), hi=(2, 2), bc=(1, 1, 1, 1))

    def pulse(m):
        xy = m.centroid[:, :2]
        g = np.exp(-((xy[:, 0] - 0.5) ** 2 + (xy[:, 1] - 0.5) ** 2) / (2 * 0.06 ** 2))
        U = np.zeros((m.ncells, 6))
        U[:, 2], U[:, 3], U[:, 4] = g, g / np.sqrt(2), -g / np.sqrt(2)
        return U

    dt = 0.5 / N
    n = int(round(0.7 / dt))
    U0 = pulse(small)
    A = oracle.run(small, U0, n, dt, 0.01 * dt)
    B = oracle.run(big, pulse(big), n, dt, 0.01 * dt).reshape(3 * N, 3 * N, 6)[N:2 * N, N:2 * N].reshape(-1, 6)
    refl = np.linalg.norm(A - B) / np.linalg.norm(U0)
    print(f"oblique non-reflecting side: reflected L2 = {refl:.3e} of the initial pulse (64^2, t = 0.7)")
    assert 1e-3 < refl < 0.1


def test_conservation_and_source_sign(oracle):
    N = 10
    mesh = oracle.cart2d(N, N)
    U = np.zeros((mesh.ncells, 6))
    U[:, 2:5] = RNG.normal(size=(mesh.ncells, 3))
    dt = 0.05
    V = oracle.step(mesh, U, dt, 0.01 * dt)
    assert np.allclose(V.sum(0), U.sum(0), rtol=0, atol=1e-13)
    # Ampere's law with a current: dEz/dt = -J_z / eps
    J = np.zeros((mesh.ncells, 3))
    J[37, 2] = 2.5
    epsinv = np.full(mesh.ncells, 0.25)
    W = oracle.step(mesh, np.zeros((mesh.ncells, 6)), dt, 0.01 * dt, epsinv=epsinv, J=J)
    expect = np.zeros((mesh.ncells, 6))
    expect[37, 2] = -dt * 0.25 * 2.5
    assert np.array_equal(W, expect)


def test_energy_does_not_grow_where_the_step_is_contractive(oracle):
    N = 24
    mesh = oracle.cart2d(N, N)
    xy = mesh.centroid[:, :2]
    U = np.zeros((mesh.ncells, 6))
    for q, s in zip((2, 3, 4), (11, 12, 13)):
        U[:, q] = smooth_field(xy, s)
    dt = 0.25 / N
    W0 = oracle.energy(mesh, U)
    for _ in range(30):
        U = oracle.step(mesh, U, dt, 0.05 * dt)
        W1 = oracle.energy(mesh, U)
        assert W1 <= W0 * (1 + 1e-13)
        W0 = W1


def _tm_symbol(theta_x, theta_y, nu, C, dt, c=1.0):
    """Amplification matrix G of one 2D TM step (U = (Ez, Hx, Hy)) for the Fourier mode
    U_j = U_hat exp(i (theta_x j_x + theta_y j_y)) on a periodic grid of width h = c dt / nu,
    written independently of the oracle from the closed-form moments of the D2Q4 lattice:
    half moments V/2 +- F1(V)/(2c), interface state U0 = (Ul + Ur)/2 + (F1(Ul) - F1(Ur))/(2c),
    second moments Q = c^2 d1 V and Q+- = c^2 d1 V / 2 +- c (F1(d1 V) + F2(d2 V)) / 2,
    dt F = C1 F1(U0) + C2 Q(grad U0) + C3 F1(Ut) + C4 [c (Ul - Ur)/2 + (F1(Ul) + F1(Ur))/2]
           - C5 [Q+(grad Ul) + Q-(grad Ur)],  Ut = -F1(d1 U0) - F2(d2 U0);
    the y face in the local frame (y, -x) (H~ = (Hy, -Hx)), rotated back."""
    h = c * dt / nu
    c2 = c * c
    F1 = lambda V: np.array([-c2 * V[2], 0.0 * V[0], -V[0]])     # local x flux of (Ez, H1, H2)
    F2 = lambda V: np.array([c2 * V[1], V[0], 0.0 * V[0]])       # local y flux
    G = np.zeros((3, 3), dtype=complex)
    for q in range(3):
        e = np.zeros(3, dtype=complex)
        e[q] = 1.0
        total = np.zeros(3, dtype=complex)
        for axis in (0, 1):
            th_n, th_t = (theta_x, theta_y) if axis == 0 else (theta_y, theta_x)
            # local frame: Ez, H along the normal, H along the second local axis
            if axis == 0:
                to = lambda V: np.array([V[0], V[1], V[2]])
                back = lambda V: np.array([V[0], V[1], V[2]])
                s_t = 1.0
            else:
                to = lambda V: np.array([V[0], V[2], -V[1]])
                back = lambda V: np.array([V[0], -V[2], V[1]])
                s_t = -1.0                                       # local axis 2 is -x
            UL = to(e)
            UR = to(e) * np.exp(1j * th_n)
            dnL = to(e) * 1j * np.sin(th_n) / h                  # central differences
            dtL = s_t * to(e) * 1j * np.sin(th_t) / h
            dnR, dtR = dnL * np.exp(1j * th_n), dtL * np.exp(1j * th_n)
            Ul, Ur = UL + 0.5 * h * dnL, UR - 0.5 * h * dnR
            U0 = 0.5 * (Ul + Ur) + (F1(Ul) - F1(Ur)) / (2 * c)
            d1 = 0.5 * (dnL + dnR) + (F1(dnL) - F1(dnR)) / (2 * c)
            d2 = 0.5 * (dtL + dtR) + (F1(dtL) - F1(dtR)) / (2 * c)
            Ut = -F1(d1) - F2(d2)
            Qp = 0.5 * c2 * dnL + 0.5 * c * (F1(dnL) + F2(dtL))
            Qm = 0.5 * c2 * dnR - 0.5 * c * (F1(dnR) + F2(dtR))
            dtF = (C[0] * F1(U0) + C[1] * c2 * d1 + C[2] * F1(Ut)
                   + C[3] * (0.5 * c * (Ul - Ur) + 0.5 * (F1(Ul) + F1(Ur))) - C[4] * (Qp + Qm))
            Fp = back(dtF)                                       # face on the + side of the cell
            total += (Fp - Fp * np.exp(-1j * th_n)) / h
        G[:, q] = e - total
    return G


@pytest.mark.parametrize("tau_hat", [0.0, 0.05, np.inf])
def test_von_neumann_symbol_matches_one_step(oracle, tau_hat):
    """One oracle step on a single Fourier mode equals G(theta) times the mode (2D TM, periodic)."""
    N, nu = 16, 0.5
    mesh = oracle.cart2d(N, N)
    dt = nu / N
    C = oracle.coefficients(dt, tau_hat * dt)
    ix, iy = np.arange(N * N) % N, np.arange(N * N) // N
    for mx, my in ((1, 0), (0, 3), (2, 5), (7, 7), (5, 2)):
        tx, ty = 2 * np.pi * mx / N, 2 * np.pi * my / N
        G = _tm_symbol(tx, ty, nu, C, dt)
        for q in range(3):
            for part in (np.real, np.imag):     # the step is real: apply it to both parts
                U = np.zeros((N * N, 6))
                U[:, 2 + q] = part(np.exp(1j * (tx * ix + ty * iy)))
                V = oracle.step(mesh, U, dt, tau_hat * dt)
                for r in range(3):
                    ref = part(G[r, q] * np.exp(1j * (tx * ix + ty * iy)))
                    assert np.max(np.abs(V[:, 2 + r] - ref)) < 1e-13, (mx, my, q, r)


# ------------------------------------------------------------------ accuracy against exact solutions
def run_tm(oracle, mesh, fields, T, nu, tau_hat=0.01, bc_eps=None):
    N = mesh.shape[0]
    dt = nu / N
    n = int(np.floor(T / dt + 1e-9))
    U = np.zeros((mesh.ncells, 6))
    U[:, 2:5] = np.stack(fields, axis=1)
    U = oracle.run(mesh, U, n, dt, tau_hat * dt, epsinv=bc_eps)
    rem = T - n * dt
    if rem > 1e-12:
        U = oracle.step(mesh, U, rem, tau_hat * dt, epsinv=bc_eps)
    return U


def test_second_order_plane_wave_oblique(oracle):
    errs = []
    for N in (24, 48, 96):
        mesh = oracle.cart2d(N, N)
        x, y = mesh.centroid[:, 0], mesh.centroid[:, 1]
        U = run_tm(oracle, mesh, X.plane_wave_tm(x, y, 0, 1, 1), 0.5, 0.5)
        errs.append(X.error_norms(U[:, 2], X.plane_wave_tm(x, y, 0.5, 1, 1)[0])[1])
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.9) & (orders < 2.3)), (errs, orders)


def test_second_order_periodic_gaussian(oracle):
    errs = []
    xc, yc = 0.41, 0.57
    for N in (32, 64, 128):
        mesh = oracle.cart2d(N, N)
        x, y = mesh.centroid[:, 0], mesh.centroid[:, 1]
        U = run_tm(oracle, mesh, X.gaussian_tm(x, y, 0.0, xc, yc), 0.25, 0.5)
        ref = X.gaussian_tm(x, y, 0.25, xc, yc)
        errs.append(np.sqrt(np.mean((U[:, 2:5] - np.stack(ref, 1)) ** 2)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), (errs, orders)


@pytest.mark.parametrize("tau_hat,order", [(0.0, 2.0), (0.1, 1.0)])
def test_material_plane_wave_speed(oracle, tau_hat, order):
    """Uniform eps = 4: the wave travels at v = 1/2 with H = -sqrt(eps/mu) E.  With tau = 0
    the step is second order.  The lattice speed c exceeds v, so a collision time tau > 0
    leaves a viscosity tau (c^2 - v^2) on the propagating pair: first order in dt when tau is
    a fixed fraction of dt."""
    errs = []
    for N in (64, 128, 256):
        mesh = oracle.cart2d(N, 2)
        x = mesh.centroid[:, 0]
        ph = lambda t: np.cos(2 * np.pi * (x - 0.5 * t))
        U = np.zeros((mesh.ncells, 6))
        U[:, 2], U[:, 4] = ph(0), -2.0 * ph(0)
        dt = 0.5 / N
        n = int(round(1.0 / dt))
        U = oracle.run(mesh, U, n, dt, tau_hat * dt, epsinv=np.full(mesh.ncells, 0.25))
        errs.append(X.error_norms(U[:, 2], ph(n * dt))[1])
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - order) < 0.25), (errs, orders)


def test_fresnel_reflection_at_normal_incidence(oracle):
    """Vacuum -> eps2 = 4 half-space: reflected amplitude (1 - sqrt(eps2))/(1 + sqrt(eps2)) = -1/3."""
    N = 800
    mesh = oracle.cart2d(N, 1 + 1, bc=(1, 1, 0, 0))
    x = mesh.centroid[:, 0]
    epsinv = np.where(x > 0.5, 0.25, 1.0)
    a = np.exp(-((x - 0.25) / 0.03) ** 2)
    U = np.zeros((mesh.ncells, 6))
    U[:, 2], U[:, 4] = a, -a                            # right-going, amplitude 1
    dt = 0.5 / N
    U = oracle.run(mesh, U, int(0.45 / dt), dt, 0.01 * dt, epsinv=epsinv)
    refl = U[:, 2][x < 0.45]
    R = refl[np.argmax(np.abs(refl))]
    assert abs(R - (-1.0 / 3.0)) < 1e-2


# ------------------------------------------------------------------ the paper's tables (soft pins)
def load_table(name):
    rows = [l.split() for l in open(os.path.join(GOLD, name)) if l.strip() and not l.startswith("#")]
    return {int(r[0]): tuple(float(v) for v in r[1:]) for r in rows}


def test_paper_plane_wave_table(oracle):
    """Sec. 5.1 table, read with dt = (1/12) dx / c (the reading under which the 3D table
    reproduces); data vary along x only, so N x 2 x 2 periodic grids carry the N^3 problem."""
    tab = load_table("paper_gks_plane_wave.txt")
    for N in (40, 80, 160):
        mesh = oracle.cart3d(N, 2, 2)
        x = mesh.centroid[:, 0]
        U = np.zeros((mesh.ncells, 6))
        U[:, 2], U[:, 4] = np.cos(2 * np.pi * x), -np.cos(2 * np.pi * x)
        dt = (1.0 / 12.0) / N
        n = int(round(1.0 / dt))
        U = oracle.run(mesh, U, n, dt, 0.01 * dt)
        got = X.error_norms(U[:, 2], np.cos(2 * np.pi * (x - n * dt)))
        for g, p in zip(got, tab[N]):
            assert abs(g / p - 1) < 0.03, (N, got, tab[N])


@pytest.mark.slow
def test_paper_cavity_table(oracle):
    """Sec. 5.2 table at N = 200 (errors along the cell row nearest y = 0.3125), CFL 0.5,
    small collision time; coarser grids are reported by the paper with larger deviations."""
    tab = load_table("paper_tm_cavity.txt")
    N = 200
    mesh = oracle.cart2d(N, N, bc=(2, 2, 2, 2))
    x, y = mesh.centroid[:, 0], mesh.centroid[:, 1]
    U = run_tm(oracle, mesh, X.cavity_tm(x, y, 0.0), 1.775, 0.5, tau_hat=1e-4)
    ez = X.cavity_tm(x, y, 1.775)[0].reshape(N, N)
    row = int(np.argmin(np.abs(y.reshape(N, N)[:, 0] - 0.3125)))
    got = X.error_norms(U[:, 2].reshape(N, N)[row], ez[row])
    for g, p in zip(got, tab[N]):
        assert abs(g / p - 1) < 0.06, (got, tab[N])
