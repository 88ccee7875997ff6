"""Pins of the oracle's limited step (CPU).

The paper's Riemann problem (Sec. 5) uses a limiter that keeps second order in smooth regions and
drops to first order at discontinuities, without naming it.  The reading: minmod of the two
one-sided differences along each axis of a Cartesian grid, applied to the variables that travel
along that axis (E_a +/- H_b, E_b +/- H_a, with a, b the other axes) and to the normal
components.

  * definition: minmod picks the smaller one-sided slope when both have the same sign and zero
    otherwise (hand-computed three-cell data of a normal component), and equals the central slope
    on linear data;
  * the paper's one-dimensional Riemann problem against its exact solution (characteristics
    Ey +/- Hz and Ez -/+ Hy at the speed of light), on a doubled periodic domain: no value
    leaves the range of the exact solution (the unlimited step overshoots), and the L1 error
    falls under refinement;
  * smooth data keep a high order (plane wave);
  * PEC walls: the limited run in a PEC box equals the limited periodic run of the mirror
    extension, which fixes the ghost slopes.
"""
import numpy as np
import pytest

from oracle import exact as X
from oracle import gks_oracle as O
from tests.test_oracle_pins import smooth_field

LIM = O.LIMITER_MINMOD

# the Riemann problem of Sec. 5: (Ex, Ey, Ez, Hx, Hy, Hz) left and right of x = 0.5
RP_L = np.array([0.0, 1.0, 0.0, 1.0, -0.75, 0.0])
RP_R = np.array([0.0, -1.0, 0.0, 1.0, 0.75, 0.0])


def riemann_exact(x, t, x0=0.5):
    """Maxwell along x (dE/dt = curl H, dH/dt = -curl E, c = 1): Ey + Hz and Ez - Hy move with
    +c, Ey - Hz and Ez + Hy with -c; Ex and Hx do not change."""
    sL = lambda xx: np.where(xx[:, None] < x0, RP_L[None], RP_R[None])
    a, b = sL(x - t), sL(x + t)    # states carried by the right- and left-moving families
    U = np.zeros((x.size, 6))
    w1, w2 = a[:, 1] + a[:, 5], b[:, 1] - b[:, 5]     # Ey + Hz (right), Ey - Hz (left)
    w4, w3 = a[:, 2] - a[:, 4], b[:, 2] + b[:, 4]     # Ez - Hy (right), Ez + Hy (left)
    U[:, 1], U[:, 5] = 0.5 * (w1 + w2), 0.5 * (w1 - w2)
    U[:, 2], U[:, 4] = 0.5 * (w3 + w4), 0.5 * (w3 - w4)
    U[:, 0], U[:, 3] = RP_L[0], RP_L[3]
    return U


def riemann_run(nx, limiter, t=0.25, cfl=1.0 / 3.0):
    """nx cells on [0, 1]: an nx x 2 x 2 grid (periodic y and z) doubled to [0, 2] periodic in x,
    with the reverse jump at x = 1.5.  Up to t = 0.25 the waves of the two jumps do not meet,
    so [0, 1] holds the single-jump solution (a non-reflecting side would feed zero
    distributions into the nonzero far field of this problem).  The six fields need the 3D
    lattice, whose step is stable up to CFL 1/3 (the paper's 0.5 is for its one-dimensional
    runs).  Returns x and the state there."""
    h = 1.0 / nx
    mesh = O.cart3d(2 * nx, 2, 2, hi=(2.0, 2 * h, 2 * h))
    x = mesh.centroid[:, 0]
    left = (x < 0.5) | (x >= 1.5)
    U = np.where(left[:, None], RP_L[None], RP_R[None]).astype(np.float64)
    nsteps = int(round(t / (cfl * h)))
    V = O.run(mesh, U, nsteps, cfl * h, 0.01 * cfl * h, limiter=limiter)
    keep = x < 1.0
    return x[keep], V[keep]


def test_minmod_definition_on_three_cells(oracle):
    mesh = O.cart2d(3, 2, bc=(1, 1, 0, 0))
    h = 1.0 / 3
    for vals, want in (([0.0, 1.0, 0.5], 0.0),          # a local maximum: no slope
                       ([0.0, 1.0, 3.0], 1.0 / h),      # monotone: the smaller one-sided slope
                       ([3.0, 1.0, 0.0], -1.0 / h),
                       ([2.0, 2.0, 5.0], 0.0)):         # one flat side: no slope
        U = np.zeros((6, 6))
        U[:, 3] = np.tile(vals, 2)                       # Hx: the normal component along x
        g = O.gradients(mesh, U, limiter=LIM)
        assert abs(g[1, 0, 3] - want) <= 1e-13 * max(1.0, abs(want)), (vals, g[1, 0, 3])
        # Ez alone along x: the pair (Ez + Hy, Ez - Hy) both carry the data, same result
        U = np.zeros((6, 6))
        U[:, 2] = np.tile(vals, 2)
        g = O.gradients(mesh, U, limiter=LIM)
        assert abs(g[1, 0, 2] - want) <= 1e-13 * max(1.0, abs(want)), (vals, g[1, 0, 2])
    # a pair with opposite trends: Ez rises, Hy falls by the same amount -> Ez - Hy carries
    # twice the slope, Ez + Hy none; minmod acts on those, not on Ez and Hy separately
    U = np.zeros((6, 6))
    U[:, 2] = np.tile([0.0, 1.0, 3.0], 2)
    U[:, 4] = -U[:, 2]
    g = O.gradients(mesh, U, limiter=LIM)
    assert abs(g[1, 0, 2] - 1.0 / h) <= 1e-13 / h and abs(g[1, 0, 4] + 1.0 / h) <= 1e-13 / h


def test_limited_slope_is_central_on_linear_data(oracle):
    nx, ny = 12, 10
    mesh = O.cart2d(nx, ny, bc=(1, 2, 1, 2))
    xy = mesh.centroid[:, :2]
    U = np.zeros((mesh.ncells, 6))
    U[:, 2] = 0.3 + 1.7 * xy[:, 0] - 0.9 * xy[:, 1]
    U[:, 3] = -0.4 + 0.5 * xy[:, 0] + 2.1 * xy[:, 1]
    U[:, 4] = 1.1 - 1.3 * xy[:, 0] + 0.2 * xy[:, 1]
    i, j = np.arange(mesh.ncells) % nx, np.arange(mesh.ncells) // nx
    inner = (i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1)
    a = O.gradients(mesh, U, limiter=LIM)
    b = O.gradients(mesh, U)
    assert np.max(np.abs(a[inner] - b[inner])) <= 1e-12
    assert abs(a[inner, 0, 2] - 1.7).max() <= 1e-11 and abs(a[inner, 1, 4] - 0.2).max() <= 1e-11


def test_limiter_needs_a_cartesian_mesh(oracle):
    from tests.test_oracle_tri import square_tri_mesh
    mesh = O.tri_mesh(*square_tri_mesh(3))
    with pytest.raises(ValueError):
        O.step(mesh, np.zeros((mesh.ncells, 6)), 0.01, 0.0001, limiter=LIM)


def test_riemann_problem_bounded_and_converging(oracle):
    errs = []
    for nx in (100, 200, 400):
        x, V = riemann_run(nx, LIM)
        ref = riemann_exact(x, 0.25)
        lo, hi = ref.min(axis=0), ref.max(axis=0)
        assert np.all(V >= lo - 1e-12) and np.all(V <= hi + 1e-12), nx    # no new extrema
        errs.append(np.mean(np.abs(V - ref), axis=0))
    errs = np.array(errs)
    # the moving components: Ey, Ez, Hy, Hz; Ex and Hx stay exact
    assert np.max(errs[:, [0, 3]]) <= 1e-14
    moving = errs[:, [1, 2, 4, 5]].sum(axis=1)
    rates = np.log2(moving[:-1] / moving[1:])
    assert moving[0] < 0.15 and rates.min() >= 0.55, (moving, rates)   # sum over the four moving fields
    # the same problem without the limiter overshoots
    x, V = riemann_run(100, O.LIMITER_NONE)
    ref = riemann_exact(x, 0.25)
    assert max(np.max(V - ref.max(axis=0)), np.max(ref.min(axis=0) - V)) > 1e-2


def test_limited_plane_wave_order(oracle):
    errs = []
    for N in (32, 64, 128):
        mesh = O.cart2d(N, 4, hi=(1.0, 4.0 / N))
        xy = mesh.centroid[:, :2]
        U = np.zeros((mesh.ncells, 6))
        U[:, 2], U[:, 3], U[:, 4] = X.plane_wave_tm(xy[:, 0], xy[:, 1], 0.0)
        dt = 0.5 / N
        nsteps = int(round(0.5 / dt))
        V = O.run(mesh, U, nsteps, dt, 0.01 * dt, limiter=LIM)
        ez, _, _ = X.plane_wave_tm(xy[:, 0], xy[:, 1], nsteps * dt)
        errs.append(np.mean(np.abs(V[:, 2] - ez)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() >= 1.4, (errs, rates)


def test_limited_pec_box_equals_mirrored_periodic_run(oracle):
    N, nsteps = 12, 6
    box = O.cart2d(N, N, bc=(2, 2, 2, 2))
    big = O.cart2d(2 * N, 2 * N, lo=(-1, -1), hi=(1, 1))
    xy = box.centroid[:, :2]
    ez, hx, hy = (smooth_field(xy, s).reshape(N, N) for s in (7, 8, 9))
    ez = ez + (xy[:, 0] > 0.6).reshape(N, N)    # a jump, so that the limiter acts

    def extend(f, sx, sy):
        top = np.concatenate([sx * f[:, ::-1], f], axis=1)
        return np.concatenate([sy * top[::-1, :], top], axis=0)

    Ub = np.zeros((box.ncells, 6))
    Ub[:, 2], Ub[:, 3], Ub[:, 4] = ez.ravel(), hx.ravel(), hy.ravel()
    Ug = np.zeros((big.ncells, 6))
    Ug[:, 2], Ug[:, 3], Ug[:, 4] = extend(ez, -1, -1).ravel(), extend(hx, -1, 1).ravel(), extend(hy, 1, -1).ravel()
    dt = 0.5 / N
    A = O.run(box, Ub, nsteps, dt, 0.01 * dt, limiter=LIM)
    B = O.run(big, Ug, nsteps, dt, 0.01 * dt, limiter=LIM)
    Bq = B.reshape(2 * N, 2 * N, 6)[N:, N:, :].reshape(-1, 6)
    assert np.max(np.abs(A - Bq)) < 1e-13 * np.max(np.abs(A))
    # and the limiter changed the result
    C = O.run(box, Ub, nsteps, dt, 0.01 * dt)
    assert np.max(np.abs(A - C)) > 1e-4
