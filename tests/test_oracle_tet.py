"""Pins of the oracle on tetrahedral meshes (CPU).

The paper runs its scheme on unstructured 3D meshes (Sec. 5.5); the oracle's face-based step
applies to them unchanged, with the printed rotation T' for arbitrary face normals.  Each face
is evaluated once, from its owner (the lower cell index): the D3Q4 lattice is chiral, so the
flux of a face seen from its other side would differ.  The pins:

  * geometry of the generated meshes: positive volumes, closed cells (sum of n |l| = 0), four
    faces per cell, the total volume of the box minus the removed sphere;
  * a constant state stays constant in every cell away from the boundary (the fluxes of a
    closed cell cancel), for every tau;
  * least-squares gradients are exact for linear fields at interior cells (the face offsets);
  * the PEC cavity mode of the unit cube (exact standing wave) is approached with order > 1.1
    under refinement of jittered meshes, with Green-Gauss gradients;
  * a PEC wall face of the removed sphere reflects: the energy stays bounded and decays slowly.
"""
import numpy as np
import pytest

from oracle import exact as X
from oracle import gks_oracle as O
from paper_2412_16845_amd import inputs as I


def _inradius(m):
    S = np.zeros(m.ncells)
    np.add.at(S, m.face_L, m.area)
    inn = m.face_R >= 0
    np.add.at(S, m.face_R[inn], m.area[inn])
    return 3.0 * m.vol / S


def test_tet_mesh_geometry(oracle):
    v, T, fc, fv = I.tet_box_mesh(7, seed=2, sphere=((0.5, 0.5, 0.5), 0.2))
    m = O.tet_mesh(v, T, fc, fv)
    assert m.vol.min() > 0
    acc = np.zeros((m.ncells, 3))
    np.add.at(acc, m.face_L, m.normal * m.area[:, None])
    inn = m.face_R >= 0
    np.add.at(acc, m.face_R[inn], -(m.normal * m.area[:, None])[inn])
    assert np.abs(acc).max() < 1e-15
    cnt = np.bincount(np.concatenate([m.face_L, m.face_R[inn]]), minlength=m.ncells)
    assert cnt.min() == 4 and cnt.max() == 4
    assert np.all(fc[inn, 0] < fc[inn, 1])                      # owner = lower index
    # the removed tetrahedra approximate the sphere's volume
    assert abs((1.0 - m.vol.sum()) - 4.0 / 3.0 * np.pi * 0.2 ** 3) < 0.15 * 4.0 / 3.0 * np.pi * 0.2 ** 3
    # normals point away from the owner
    assert np.all(np.einsum("ij,ij->i", m.normal, m.dL) > 0)


@pytest.mark.parametrize("tau_hat", [0.0, 0.01, np.inf])
def test_tet_constant_state_is_kept_away_from_walls(oracle, tau_hat):
    v, T, fc, fv = I.tet_box_mesh(5, seed=3, bc=("pec", "nonreflecting") * 3)
    m = O.tet_mesh(v, T, fc, fv)
    Uc = np.array([0.3, -1.2, 0.7, 0.5, 2.0, -0.4])
    U = np.tile(Uc, (m.ncells, 1))
    dt = 0.5 * _inradius(m).min()
    V = O.step(m, U, dt, tau_hat * dt)
    touch = np.zeros(m.ncells, dtype=bool)
    touch[m.face_L[m.face_R < 0]] = True
    # cells sharing a face with a boundary cell see its non-zero gradient
    nb = np.zeros(m.ncells, dtype=bool)
    inn = m.face_R >= 0
    for a, b in ((m.face_L[inn], m.face_R[inn]), (m.face_R[inn], m.face_L[inn])):
        nb[a[touch[b]]] = True
    far = ~(touch | nb)
    assert far.sum() > 20
    assert np.max(np.abs(V[far] - U[far])) < 1e-14


def test_tet_lsq_gradients_exact_for_linear_fields(oracle):
    v, T, fc, fv = I.tet_box_mesh(6, seed=4)
    m = O.tet_mesh(v, T, fc, fv)
    A = np.random.default_rng(5).standard_normal((6, 4))
    c = m.centroid
    U = A[:, 0][None] + c @ A[:, 1:].T
    g = O.gradients(m, U, O.GRAD_LSQ)
    inner = np.ones(m.ncells, dtype=bool)
    inner[m.face_L[m.face_R < 0]] = False
    for d in range(3):
        assert np.max(np.abs(g[inner, d, :] - A[None, :, 1 + d])) < 1e-11
    # Green-Gauss is not exact on these meshes (the pin discriminates)
    gg = O.gradients(m, U)
    assert np.max(np.abs(gg[inner, 0, :] - A[None, :, 1])) > 1e-3


def test_tet_pec_cavity_mode_converges(oracle):
    a, tf = np.pi, 0.25
    errs = []
    for N in (4, 8, 16):
        v, T, fc, fv = I.tet_box_mesh(N, seed=1, bc=("pec",) * 6)
        m = O.tet_mesh(v, T, fc, fv)
        c = m.centroid
        ez, hx, hy = X.cavity_tm(c[:, 0], c[:, 1], 0.0, a)
        U = np.zeros((m.ncells, 6))
        U[:, 2], U[:, 3], U[:, 4] = ez, hx, hy
        ns = int(np.ceil(tf / (0.5 * _inradius(m).min())))
        dt = tf / ns
        V = O.run(m, U, ns, dt, 0.01 * dt)
        ez1, _, _ = X.cavity_tm(c[:, 0], c[:, 1], tf, a)
        errs.append(np.sqrt(np.sum(m.vol * (V[:, 2] - ez1) ** 2) / m.vol.sum()))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 6e-3 and rates.min() > 1.1, (errs, rates)


def test_tet_sphere_walls_keep_energy_bounded(oracle):
    v, T, fc, fv = I.tet_box_mesh(6, seed=6, sphere=((0.5, 0.5, 0.5), 0.22), bc=("pec",) * 6)
    m = O.tet_mesh(v, T, fc, fv)
    U = np.random.default_rng(7).standard_normal((m.ncells, 6))
    dt = 0.5 * _inradius(m).min()
    _, hist = O.run(m, U, 200, dt, 0.01 * dt, energy_every=20)
    W0 = O.energy(m, U)
    assert max(hist) <= W0 and hist[-1] > 1e-3 * W0
