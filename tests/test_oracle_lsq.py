"""Pins of the oracle's least-squares cell gradients (CPU).

Sec. 3.1 allows Green-Gauss "or other" cell gradients; the least-squares option fits grad U_i to
the face neighbours, with each boundary ghost placed at the mirror image of the cell centroid.

  * exactness: the fit reproduces a linear field exactly on every cell away from the boundary
    (Green-Gauss with arithmetic face values does not on an irregular mesh);
  * ghosts: at a wall whose ghost rule is consistent with a linear field (PEC: Ez and the normal
    H odd, the tangential H even; non-reflecting: the cell's own value, so a field constant
    along the normal), boundary cells are exact too, which fixes the mirror-point offset;
  * uniform grids: with the four (six) axis neighbours and the ghosts one cell width away, least
    squares and Green-Gauss both give the central difference, including at PEC and
    non-reflecting sides, in 2D and 3D;
  * rotation invariance and second-order convergence of whole steps, as for Green-Gauss.
"""
import numpy as np
import pytest

from oracle import exact as X
from oracle import gks_oracle as O
from paper_2412_16845_amd import inputs as I
from tests.test_oracle_tri import _rotate_mesh, square_tri_mesh

LSQ, GG = O.GRAD_LSQ, O.GRAD_GREEN_GAUSS
A = np.array([[0.3, 1.7, -0.9], [-0.4, 0.5, 2.1], [1.1, -1.3, 0.2]])   # (Ez, Hx, Hy) = a0 + a1 x + a2 y


def _linear_state(cen):
    U = np.zeros((cen.shape[0], 6))
    for r, f in enumerate((2, 3, 4)):
        U[:, f] = A[r, 0] + A[r, 1] * cen[:, 0] + A[r, 2] * cen[:, 1]
    return U


def _boundary_cells(fc):
    return set(fc[fc[:, 1] < 0, 0].tolist())


def test_lsq_exact_for_linear_fields_away_from_the_boundary(oracle):
    verts, tris, fc, fv = I.tri_ellipse_mesh(0.05, seed=11, cache=False)
    mesh = O.tri_mesh(verts, tris, fc, fv)
    cen = verts[tris].mean(axis=1)
    U = _linear_state(cen)
    inner = np.array(sorted(set(range(tris.shape[0])) - _boundary_cells(fc)))
    g = O.gradients(mesh, U, LSQ)
    gg = O.gradients(mesh, U, GG)
    for r, f in enumerate((2, 3, 4)):
        assert np.max(np.abs(g[inner, 0, f] - A[r, 1])) <= 1e-11
        assert np.max(np.abs(g[inner, 1, f] - A[r, 2])) <= 1e-11
    assert np.max(np.abs(g[:, 2, :])) == 0.0                      # no z derivative on a 2D mesh
    # the pin discriminates: Green-Gauss is off on the jittered mesh
    assert np.max(np.abs(gg[inner, 0, 2] - A[0, 1])) > 1e-3


@pytest.mark.parametrize("bc", [O.BC_PEC, O.BC_NONREFLECT])
def test_lsq_exact_at_walls_consistent_with_the_ghost(oracle, bc):
    N = 14
    verts, tris, fc, fv = square_tri_mesh(N)
    fc = fc.copy()
    fc[fc[:, 1] < 0, 1] = -(1 + bc)
    mesh = O.tri_mesh(verts, tris, fc, fv)
    cen = verts[tris].mean(axis=1)
    U = np.zeros((tris.shape[0], 6))
    if bc == O.BC_PEC:   # across x = 0: Ez and Hx (normal) odd, Hy (tangential) even
        U[:, 2], U[:, 3], U[:, 4] = 1.3 * cen[:, 0], -0.7 * cen[:, 0], 0.4 + 2.0 * cen[:, 1]
        want = {(0, 2): 1.3, (1, 2): 0.0, (0, 3): -0.7, (1, 3): 0.0, (0, 4): 0.0, (1, 4): 2.0}
    else:                # the ghost repeats the cell: any field constant along x
        U[:, 2], U[:, 3], U[:, 4] = 2.0 * cen[:, 1], -1.0 * cen[:, 1], 0.5 + 3.0 * cen[:, 1]
        want = {(0, 2): 0.0, (1, 2): 2.0, (0, 3): 0.0, (1, 3): -1.0, (0, 4): 0.0, (1, 4): 3.0}
    # cells whose boundary faces all lie on the wall x = 0 (and that have at least one)
    mid = verts[fv].mean(axis=1)
    on_wall = {}
    for s in np.nonzero(fc[:, 1] < 0)[0]:
        on_wall.setdefault(int(fc[s, 0]), []).append(abs(mid[s, 0]) < 1e-12)
    cells = np.array(sorted(c for c, flags in on_wall.items() if all(flags)))
    assert cells.size >= N - 2
    g = O.gradients(mesh, U, LSQ)
    for (d, f), v in want.items():
        assert np.max(np.abs(g[cells, d, f] - v)) <= 1e-12, (d, f)
    # the same cells with the ghost at the cell (not at its mirror image) would be off
    gg = O.gradients(mesh, U, GG)
    assert max(np.max(np.abs(gg[cells, d, f] - v)) for (d, f), v in want.items()) > 1e-3


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 2, 2, 1)])
def test_lsq_equals_green_gauss_on_uniform_grids_2d(oracle, bc):
    mesh = O.cart2d(13, 9, hi=(1.3, 0.9), bc=bc)
    U = np.random.default_rng(5).standard_normal((mesh.ncells, 6))
    U[:, [0, 1, 5]] = 0.0
    a, b = O.gradients(mesh, U, LSQ), O.gradients(mesh, U, GG)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("bc", [(0,) * 6, (1, 1, 1, 1, 2, 2)])
def test_lsq_equals_green_gauss_on_uniform_grids_3d(oracle, bc):
    mesh = O.cart3d(6, 5, 4, hi=(0.6, 0.5, 0.4), bc=bc)
    U = np.random.default_rng(6).standard_normal((mesh.ncells, 6))
    a, b = O.gradients(mesh, U, LSQ), O.gradients(mesh, U, GG)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_lsq_step_rotation_invariance(oracle):
    verts, tris, fc, fv = I.tri_ellipse_mesh(0.06, seed=3, cache=False)
    rng = np.random.default_rng(4)
    nc = tris.shape[0]
    U = np.zeros((nc, 6))
    U[:, 2:5] = rng.standard_normal((nc, 3))
    ei = rng.uniform(0.3, 1.0, nc)
    dt = 0.004
    Aref = O.run(O.tri_mesh(verts, tris, fc, fv), U, 3, dt, 0.01 * dt, epsinv=ei, gradient=LSQ)
    vr, R = _rotate_mesh(verts, 0.7371)
    Ur = U.copy()
    Ur[:, 3:5] = U[:, 3:5] @ R.T
    B = O.run(O.tri_mesh(vr, tris, fc, fv), Ur, 3, dt, 0.01 * dt, epsinv=ei, gradient=LSQ)
    B[:, 3:5] = B[:, 3:5] @ R
    assert np.max(np.abs(B - Aref)) <= 1e-13 * np.max(np.abs(Aref))
    # and the option changes the result (the two gradients differ on this mesh)
    G = O.run(O.tri_mesh(verts, tris, fc, fv), U, 3, dt, 0.01 * dt, epsinv=ei)
    assert np.max(np.abs(G - Aref)) > 1e-6


def test_lsq_pec_square_cavity_convergence(oracle):
    """The standing mode of the Green-Gauss test, with least-squares gradients."""
    a = 2 * np.pi
    errs = []
    for N in (12, 24, 48):
        verts, tris, fc, fv = square_tri_mesh(N)
        mesh = O.tri_mesh(verts, tris, fc, fv)
        cen = verts[tris].mean(axis=1)
        ez, hx, hy = X.cavity_tm(cen[:, 0], cen[:, 1], 0.0, a)
        U = np.zeros((mesh.ncells, 6))
        U[:, 2], U[:, 3], U[:, 4] = ez, hx, hy
        dt0 = 0.5 * (1.0 / N) / (2 + np.sqrt(2))
        nsteps = int(np.ceil(0.25 / dt0))
        dt = 0.25 / nsteps
        V = O.run(mesh, U, nsteps, dt, 0.01 * dt, gradient=LSQ)
        ez1, _, _ = X.cavity_tm(cen[:, 0], cen[:, 1], 0.25, a)
        errs.append(np.sqrt(np.mean((V[:, 2] - ez1) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 0.05 and rates.min() >= 1.5, (errs, rates)
