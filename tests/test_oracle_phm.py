"""Pins of the oracle's perfectly hyperbolic Maxwell (PHM) system (CPU).

Sec. 2.1 adds two potentials to Maxwell's equations: phi, driven by the divergence of E and
fed back into E through chi, and psi, driven by the divergence of H (B) and fed back through
gamma; divergence errors then travel at chi c and gamma c.  The oracle carries the eight
components (Ex, Ey, Ez, Hx, Hy, Hz, phi, psi).  The pins:

  * wave speeds: the flux Jacobian that the oracle's equilibrium moments define along any
    direction k has the eigenvalues +-c|k| (twice), +-chi c|k| and +-gamma c|k|;
  * one-dimensional data: the pairs (Hx, psi) and (Ex, phi) split into the scalar invariants
    psi +- c Hx and phi +- Ex / c moving at +-gamma c and +-chi c; one oracle step equals the
    kinetic scheme for a scalar of speed a written out from the lattice moments (the lattice
    speed c, the interface state, its slope and the five C-terms), in 2D and 3D and for every
    tau;
  * exact solutions: a longitudinal wave (H along k, with psi) on an oblique periodic grid
    converges at second order to its exact travelling solution at speed gamma c; with a uniform
    1/mu it moves at gamma c sqrt(1/mu) (the potentials carry no material factor);
  * transverse data: an axis-aligned TM plane wave has no discrete divergence, so the
    potentials stay zero and the step is the plain Maxwell step;
  * PEC: a PEC box equals the periodic run of the mirror extension in which phi is odd and
    psi even (the parities that keep the PHM system invariant under the mirror);
  * cleaning: in a non-reflecting box, a divergent H bump leaves with gamma = 1 and stays with
    gamma = 0;
  * conservation of every component on a periodic grid.
"""
import numpy as np
import pytest

from oracle import gks_oracle as O
from tests.test_oracle_pins import smooth_field

RNG = np.random.default_rng(77)


def kinetic_scalar_step(w, a, c, h, dt, C):
    """One step of the lattice scheme for w_t + a w_x = 0 on a periodic row of cells, from the
    closed-form moments of the D2Q4 / D3Q4 lattices restricted to data along the face normal:
    central slopes s; face states w^l = w_i + h s_i / 2, w^r = w_{i+1} - h s_{i+1} / 2;
    half moments <g>_{+-} = v/2 +- a v/(2c), so the interface state and slope are
    w0 = (w^l + w^r)/2 + a (w^l - w^r)/(2c) and s0 likewise; w_t = -a s0;
    dt F = C1 a w0 + C2 c^2 s0 + C3 a w_t + C4 [c (w^l - w^r)/2 + a (w^l + w^r)/2]
           - C5 [c^2 (s^l + s^r)/2 + c a (s^l - s^r)/2]."""
    s = (np.roll(w, -1) - np.roll(w, 1)) / (2 * h)
    wl, wr = w + 0.5 * h * s, np.roll(w, -1) - 0.5 * h * np.roll(s, -1)
    sl, sr = s, np.roll(s, -1)
    w0 = 0.5 * (wl + wr) + a * (wl - wr) / (2 * c)
    s0 = 0.5 * (sl + sr) + a * (sl - sr) / (2 * c)
    wt = -a * s0
    F = (C[0] * a * w0 + C[1] * c * c * s0 + C[2] * a * wt + C[3] * (0.5 * c * (wl - wr) + 0.5 * a * (wl + wr))
         - C[4] * (0.5 * c * c * (sl + sr) + 0.5 * c * a * (sl - sr))) / dt
    return w - dt / h * (F - np.roll(F, 1))


@pytest.mark.parametrize("dim", [2, 3])
def test_phm_wave_speeds(oracle, dim):
    c, chi, gam = 1.3, 0.45, 0.8
    u = O.lattice(dim, c)
    A = np.zeros((3, 8, 8))
    for q in range(8):
        e = np.zeros(8)
        e[q] = 1.0
        g = O.equilibrium(dim, e, c, chi, gam)
        assert np.allclose(g.sum(0), e, atol=1e-15)
        A[:, :, q] = np.einsum("kj,kf->jf", u, g)       # first moments: the columns of A_j
    for _ in range(4):
        k = RNG.normal(size=3)
        if dim == 2:
            k[2] = 0.0
        K = np.einsum("j,jab->ab", k, A)
        lam = np.sort(np.linalg.eigvals(K).real)
        kk = np.linalg.norm(k)
        want = np.sort([c * kk, c * kk, -c * kk, -c * kk, chi * c * kk, -chi * c * kk, gam * c * kk, -gam * c * kk])
        if dim == 2:
            # the D2Q4 lattice has no z velocity, so A_3 is not represented; k has no z part
            assert np.max(np.abs(A[2])) == 0.0
        assert np.allclose(lam, want, atol=1e-12), (lam, want)


@pytest.mark.parametrize("tau_hat", [0.0, 0.01, 1.0, np.inf])
@pytest.mark.parametrize("c", [1.0, 1.6])
def test_phm_one_dimensional_pairs_2d(oracle, tau_hat, c):
    """Data along x on a 2D grid: psi +- c Hx and phi +- Ex/c follow the scalar kinetic scheme."""
    N, chi, gam = 24, 0.55, 0.8
    h = 1.0 / N
    dt = 0.4 * h / c
    mesh = O.cart2d(N, 3)
    x = mesh.centroid[:, 0]
    U = np.zeros((mesh.ncells, 8))
    wp, wm = np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x), np.cos(4 * np.pi * x)
    vp, vm = np.cos(2 * np.pi * x) - 0.4 * np.sin(4 * np.pi * x), 0.5 * np.sin(6 * np.pi * x)
    U[:, 7], U[:, 3] = 0.5 * (wp + wm), 0.5 * (wp - wm) / c        # psi, Hx
    U[:, 6], U[:, 0] = 0.5 * (vp + vm), 0.5 * (vp - vm) * c        # phi, Ex
    C = O.coefficients(dt, tau_hat * dt)
    V = O.step(mesh, U, dt, tau_hat * dt, c=c, chi=chi, gamma=gam)
    rows = lambda f: f.reshape(3, N)
    for got, w, a in ((V[:, 7] + c * V[:, 3], wp, gam * c), (V[:, 7] - c * V[:, 3], wm, -gam * c),
                      (V[:, 6] + V[:, 0] / c, vp, chi * c), (V[:, 6] - V[:, 0] / c, vm, -chi * c)):
        ref = np.stack([kinetic_scalar_step(r, a, c, h, dt, C) for r in rows(w)])
        assert np.max(np.abs(rows(got) - ref)) < 1e-14, a
    # nothing else moves
    assert np.max(np.abs(V[:, [1, 2, 4, 5]])) < 1e-15


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_phm_one_dimensional_pairs_3d(oracle, axis):
    """Data along one axis of a 3D grid: the normal E and H pair with phi and psi."""
    N, c, chi, gam = 20, 1.0, 0.7, 0.35
    n = [2, 2, 2]
    n[axis] = N
    mesh = O.cart3d(*n)
    s = mesh.centroid[:, axis]
    h = 1.0 / N
    dt = 0.3 * h
    U = np.zeros((mesh.ncells, 8))
    wp, wm = np.sin(2 * np.pi * s), 0.5 * np.cos(4 * np.pi * s) + 0.2
    vp, vm = np.cos(2 * np.pi * s) + 0.1 * np.sin(6 * np.pi * s), -np.sin(4 * np.pi * s)
    U[:, 7], U[:, 3 + axis] = 0.5 * (wp + wm), 0.5 * (wp - wm)
    U[:, 6], U[:, axis] = 0.5 * (vp + vm), 0.5 * (vp - vm)
    C = O.coefficients(dt, 0.01 * dt)
    V = O.step(mesh, U, dt, 0.01 * dt, chi=chi, gamma=gam)
    shape = [n[2], n[1], n[0]]
    lines = lambda f: np.moveaxis(f.reshape(shape), 2 - axis, -1).reshape(-1, N)
    for got, w, a in ((V[:, 7] + V[:, 3 + axis], wp, gam), (V[:, 7] - V[:, 3 + axis], wm, -gam),
                      (V[:, 6] + V[:, axis], vp, chi), (V[:, 6] - V[:, axis], vm, -chi)):
        ref = np.stack([kinetic_scalar_step(r, a, c, h, dt, C) for r in lines(w)])
        assert np.max(np.abs(lines(got) - ref)) < 1e-14, a
    others = [f for f in range(6) if f not in (axis, 3 + axis)]
    assert np.max(np.abs(V[:, others])) < 1e-15


def _longitudinal(xy, t, k, speed):
    """H along k and psi, the right-moving invariant only: Hx, Hy, psi."""
    kk = np.linalg.norm(k)
    ph = np.cos(xy @ k - speed * kk * t)
    return ph * k[0] / kk, ph * k[1] / kk, ph


@pytest.mark.parametrize("muinv", [1.0, 0.5])
def test_phm_longitudinal_wave_converges(oracle, muinv):
    """H parallel to k = 2 pi (1, 1) with psi: a divergence wave of speed gamma c sqrt(1/mu)."""
    gam = 0.8
    speed = gam * np.sqrt(muinv)
    k = 2 * np.pi * np.array([1.0, 1.0])
    errs = []
    for N in (16, 32, 64):
        mesh = O.cart2d(N, N)
        xy = mesh.centroid[:, :2]
        U = np.zeros((mesh.ncells, 8))
        hx, hy, psi = _longitudinal(xy, 0.0, k, speed)
        # the invariant of (H along k, psi) moving at gamma sqrt(1/mu) is psi + sqrt(mu) H_l
        U[:, 3], U[:, 4], U[:, 7] = hx * np.sqrt(muinv), hy * np.sqrt(muinv), psi
        dt = 0.5 / N
        nsteps = int(round(0.5 / dt))
        V = O.run(mesh, U, nsteps, dt, 0.01 * dt, muinv=np.full(mesh.ncells, muinv), gamma=gam)
        hx1, hy1, psi1 = _longitudinal(xy, nsteps * dt, k, speed)
        e = np.concatenate([V[:, 3] - hx1 * np.sqrt(muinv), V[:, 4] - hy1 * np.sqrt(muinv), V[:, 7] - psi1])
        errs.append(np.sqrt(np.mean(e ** 2)))
        assert np.max(np.abs(V[:, [0, 1, 2, 5, 6]])) < 1e-12     # no transverse field appears
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 2e-2 and rates.min() >= 1.8, (errs, rates)


@pytest.mark.parametrize("axis", [0, 1])
def test_phm_leaves_transverse_plane_waves_alone(oracle, axis):
    N, chi, gam = 20, 0.9, 0.6
    mesh = O.cart2d(N, N, bc=(1, 2, 0, 0) if axis == 0 else (0, 0, 1, 2))
    xy = mesh.centroid[:, :2]
    s = xy[:, axis]
    U = np.zeros((mesh.ncells, 8))
    U[:, 2] = np.sin(2 * np.pi * s) + 0.2 * np.cos(6 * np.pi * s)
    U[:, 4 if axis == 0 else 3] = (-1.0 if axis == 0 else 1.0) * np.cos(2 * np.pi * s)
    dt = 0.5 / N
    A = O.run(mesh, U, 5, dt, 0.01 * dt, chi=chi, gamma=gam)
    B = O.run(mesh, U[:, :6], 5, dt, 0.01 * dt)
    assert np.max(np.abs(A[:, 6:])) == 0.0
    assert np.max(np.abs(A[:, :6] - B)) == 0.0


def test_phm_pec_box_equals_mirrored_periodic_run(oracle):
    """All eight components in 2D (TM and TE parts), PEC on every side."""
    N, nsteps, chi, gam = 12, 6, 0.7, 0.9
    box = O.cart2d(N, N, bc=(2, 2, 2, 2))
    big = O.cart2d(2 * N, 2 * N, lo=(-1, -1), hi=(1, 1))
    xy = box.centroid[:, :2]
    F = [smooth_field(xy, 20 + f).reshape(N, N) for f in range(8)]
    # mirror parities across x = 0 and y = 0: E normal even, E tangential odd, H normal odd,
    # H tangential even, phi odd, psi even
    sx = (+1, -1, -1, -1, +1, +1, -1, +1)
    sy = (-1, +1, -1, +1, -1, +1, -1, +1)

    def extend(f, ax, ay):
        top = np.concatenate([ax * f[:, ::-1], f], axis=1)
        return np.concatenate([ay * top[::-1, :], top], axis=0)

    Ub = np.stack([f.ravel() for f in F], axis=1)
    Ug = np.stack([extend(F[q], sx[q], sy[q]).ravel() for q in range(8)], axis=1)
    dt = 0.5 / N
    A = O.run(box, Ub, nsteps, dt, 0.01 * dt, chi=chi, gamma=gam)
    B = O.run(big, Ug, nsteps, dt, 0.01 * dt, chi=chi, gamma=gam)
    Bq = B.reshape(2 * N, 2 * N, 8)[N:, N:, :].reshape(-1, 8)
    assert np.max(np.abs(A - Bq)) < 1e-13 * np.max(np.abs(A))
    # the opposite parity of psi does not match
    Ug[:, 7] = extend(F[7], -1, -1).ravel()
    B = O.run(big, Ug, nsteps, dt, 0.01 * dt, chi=chi, gamma=gam)
    Bq = B.reshape(2 * N, 2 * N, 8)[N:, N:, :].reshape(-1, 8)
    assert np.max(np.abs(A - Bq)) > 1e-3


def _div_h(U, N):
    hx, hy = U[:, 3].reshape(N, N), U[:, 4].reshape(N, N)
    d = (hx[1:-1, 2:] - hx[1:-1, :-2] + hy[2:, 1:-1] - hy[:-2, 1:-1]) * (N / 2.0)
    return np.sqrt(np.mean(d ** 2))


def test_phm_cleans_a_divergent_field(oracle):
    N = 48
    mesh = O.cart2d(N, N, bc=(1, 1, 1, 1))
    xy = mesh.centroid[:, :2]
    U = np.zeros((mesh.ncells, 8))
    U[:, 3] = np.exp(-((xy[:, 0] - 0.5) ** 2 + (xy[:, 1] - 0.5) ** 2) / (2 * 0.08 ** 2))
    dt = 0.5 / N
    nsteps = int(round(2.4 / dt))    # the 2D wave's wake has passed the sides by then
    d0 = _div_h(U, N)
    kept = _div_h(O.run(mesh, U, nsteps, dt, 0.01 * dt), N)
    V = O.run(mesh, U, nsteps, dt, 0.01 * dt, gamma=1.0)
    cleaned = _div_h(V, N)
    assert kept > 0.5 * d0, (kept, d0)              # without PHM the divergence stays
    assert cleaned < 0.05 * kept, (cleaned, kept)   # with gamma = 1 it travels out of the box


def test_phm_conservation(oracle):
    N = 16
    mesh = O.cart2d(N, N)
    xy = mesh.centroid[:, :2]
    U = np.stack([smooth_field(xy, 40 + f) + 0.3 * f for f in range(8)], axis=1)
    dt = 0.5 / N
    V = O.run(mesh, U, 7, dt, 0.01 * dt, chi=0.6, gamma=0.9, epsinv=RNG.uniform(0.3, 1.0, mesh.ncells))
    # E is scaled by 1/eps per cell, so its sum is not conserved; H, phi and psi are
    for f in (3, 4, 5, 6, 7):
        assert abs(V[:, f].sum() - U[:, f].sum()) < 1e-12 * np.abs(U[:, f]).sum(), f


def test_six_component_state_refuses_phm_couplings(oracle):
    mesh = O.cart2d(4, 4)
    with pytest.raises(ValueError):
        O.step(mesh, np.zeros((16, 6)), 0.01, 0.0001, gamma=0.5)
