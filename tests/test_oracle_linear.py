"""Pins of the probed-linear-map oracle (oracle/gks_linear.py) against the literal oracle.

The map is only a faster way to apply the literal step: each of its runs must equal the literal
run up to rounding order, on every mesh kind and boundary, with materials and sources, and its
adjoint must equal the adjoint written out from the definition (oracle/gks_adjoint.py).  The
two checks built into the probing (one probed cell per colour and region; no response outside
the regions) must fire when their assumption is broken.
"""
import numpy as np
import pytest

from oracle import gks_adjoint as OA
from oracle import gks_linear as GL
from oracle import gks_oracle as O
from paper_2412_16845_amd import inputs as I


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def tm_state(rng, nc):
    U = np.zeros((nc, 6))
    U[:, list(O.TM)] = rng.standard_normal((nc, 3))
    return U


@pytest.mark.parametrize("bc,tau_hat", [((1, 2, 1, 1), 0.01), ((2, 2, 2, 1), 0.0), ((1, 1, 1, 1), np.inf)])
def test_map_equals_literal_2d(bc, tau_hat):
    rng = np.random.default_rng(11)
    nx, ny = 27, 19
    nc = nx * ny
    mesh = O.cart2d(nx, ny, bc=bc)
    ei, mi = rng.uniform(0.25, 1.0, nc), rng.uniform(0.5, 1.0, nc)
    src = (np.array([4 * nx + 5, 12 * nx + 20]), np.array([1.0, -0.5]), 2.0, 0.05, 0.03)
    dt = 0.5 / nx
    U0 = tm_state(rng, nc)
    L = GL.LinearStep(mesh, dt, tau_hat * dt, epsinv=ei, muinv=mi, source=src)
    got = L.run(U0, 40, t0=0.01)
    ref = O.run(mesh, U0, 40, dt, tau_hat * dt, epsinv=ei, muinv=mi, source=src, t0=0.01)
    assert rel(got, ref) <= 1e-13


def test_map_equals_literal_periodic_greedy_colours():
    """Periodic axes whose length breaks the linear colouring take the greedy one."""
    rng = np.random.default_rng(12)
    nx, ny = 20, 15
    mesh = O.cart2d(nx, ny, bc=(0, 0, 1, 2))
    U0 = tm_state(rng, nx * ny)
    L = GL.LinearStep(mesh, 0.5 / nx, 0.3 * 0.5 / nx)
    assert np.unique(L.colors).shape[0] > 13
    assert rel(L.run(U0, 30), O.run(mesh, U0, 30, 0.5 / nx, 0.3 * 0.5 / nx)) <= 1e-13


def test_map_equals_literal_3d():
    rng = np.random.default_rng(13)
    n = (13, 11, 9)
    nc = int(np.prod(n))
    mesh = O.cart3d(*n, bc=(1, 1, 2, 1, 2, 2))
    ei = rng.uniform(0.25, 1.0, nc)
    dt = (1.0 / 3.0) / 13
    U0 = rng.standard_normal((nc, 6))
    src = (np.array([nc // 2]), np.array([1.0]), 1.0, 0.02, 0.02)
    L = GL.LinearStep(mesh, dt, 0.01 * dt, epsinv=ei, source=src)
    assert rel(L.run(U0, 25), O.run(mesh, U0, 25, dt, 0.01 * dt, epsinv=ei, source=src)) <= 1e-13


@pytest.mark.parametrize("gradient", [O.GRAD_GREEN_GAUSS, O.GRAD_LSQ])
def test_map_equals_literal_triangles(gradient):
    rng = np.random.default_rng(14)
    mesh4 = I.tri_ellipse_mesh(0.04, seed=3, cache=False)
    mesh = O.tri_mesh(*mesh4)
    nc = mesh.ncells
    ei = rng.uniform(0.25, 1.0, nc)
    U0 = tm_state(rng, nc)
    dt = 2e-3
    L = GL.LinearStep(mesh, dt, 0.01 * dt, epsinv=ei, gradient=gradient)
    ref = O.run(mesh, U0, 30, dt, 0.01 * dt, epsinv=ei, gradient=gradient)
    assert rel(L.run(U0, 30), ref) <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_map_equals_literal_phm(dim):
    """The PHM system (chi, gamma > 0, eight-component state): the map's runs equal the literal
    runs, in 2D on (Ez, Hx, Hy, psi) and in 3D on all eight components, with a source and a
    dielectric map."""
    rng = np.random.default_rng(16 + dim)
    if dim == 2:
        mesh = O.cart2d(23, 17, bc=(1, 2, 2, 1))
        comps, dt, steps = O.TM_PHM, 0.5 / 23, 30
    else:
        mesh = O.cart3d(11, 9, 8, bc=(1, 2, 1, 1, 2, 2))
        comps, dt, steps = tuple(range(8)), (1.0 / 3.0) / 11, 20
    nc = mesh.ncells
    U0 = np.zeros((nc, 8))
    U0[:, list(comps)] = rng.standard_normal((nc, len(comps)))
    ei = rng.uniform(0.25, 1.0, nc)
    src = (np.array([nc // 3]), np.array([1.0]), 1.5, 0.02, 0.02)
    phm = (0.7, 0.9)
    L = GL.LinearStep(mesh, dt, 0.01 * dt, epsinv=ei, source=src, phm=phm)
    assert L.comps == tuple(comps)
    ref = O.run(mesh, U0, steps, dt, 0.01 * dt, epsinv=ei, source=src, chi=phm[0], gamma=phm[1])
    got = L.run(U0, steps)
    assert got.shape == (nc, 8)
    assert rel(got, ref) <= 1e-13


def test_map_equals_literal_tetrahedra():
    """Tetrahedral meshes (greedy colours on the face graph): the map's run equals the literal run
    on a jittered box around a PEC sphere, with non-reflecting outer faces."""
    rng = np.random.default_rng(18)
    wl = I.tet_sphere_workload(n=5, seed=1, nsteps=10)
    ex = wl.extra
    mesh = O.tet_mesh(ex["verts"], ex["tets"], ex["face_cells"], ex["face_verts"])
    nc = mesh.ncells
    U0 = rng.standard_normal((nc, 6))
    dt = 2e-3
    L = GL.LinearStep(mesh, dt, 0.01 * dt)
    ref = O.run(mesh, U0, 10, dt, 0.01 * dt)
    assert rel(L.run(U0, 10), ref) <= 1e-13


def test_invalid_colouring_is_refused():
    mesh = O.cart2d(10, 9, bc=(1, 1, 1, 1))
    with pytest.raises(ValueError, match="twice"):
        GL.LinearStep(mesh, 0.05, 0.0005, colors=np.arange(90) % 5)


def test_reach_check_fires(monkeypatch):
    """Planted mistake: regions one hop wide (the step reaches two) must be detected."""
    monkeypatch.setattr(GL, "regions", GL._adjacency)
    mesh = O.cart2d(12, 10, bc=(1, 1, 1, 1))
    with pytest.raises(ValueError):
        GL.LinearStep(mesh, 0.5 / 12, 0.005 / 12)


@pytest.mark.parametrize("bc", [(1, 2, 1, 1), (2, 2, 2, 2)])
def test_adjoint_equals_definition(bc):
    """LinearAdjoint against gks_adjoint.run_gradients (Jacobian by unit vectors, material
    derivatives cell by cell), with a source and both materials."""
    rng = np.random.default_rng(15)
    nx, ny = 13, 11
    nc = nx * ny
    mesh = O.cart2d(nx, ny, bc=bc)
    ei, mi = rng.uniform(0.25, 1.0, nc), rng.uniform(0.5, 1.0, nc)
    dt = 0.5 / nx
    tau = 0.01 * dt
    src = (np.array([3 * nx + 4]), np.array([1.0]), 2.0, 0.05, 0.05)
    probe = np.array([i + nx * j for j in range(4, 8) for i in range(6, 10)])
    U0 = tm_state(rng, nc)
    loss, lam0, gE, gH = OA.run_gradients(mesh, U0, 7, dt, tau, 1.0, ei, mi, src, 0.0, probe)
    adj = GL.LinearAdjoint(GL.LinearStep(mesh, dt, tau, epsinv=ei, muinv=mi, source=src), materials=("eps", "mu"))
    states = adj.run(U0, 7)
    assert abs(OA.probe_energy(mesh, states[-1], probe) - loss) <= 1e-13 * loss
    lam, g = adj.gradients(states, OA.probe_energy_grad(mesh, states[-1], probe))
    assert rel(lam, lam0) <= 1e-13
    assert rel(g["eps"], gE) <= 1e-13
    assert rel(g["mu"], gH) <= 1e-13


@pytest.mark.slow
def test_geometry_rounding_sensitivity_of_the_triangle_workload():
    """How much FP32 rounding of the mesh geometry alone moves the FP64 scheme over the
    triangle workload's 2000 steps (h = 0.01): the oracle with its volumes, normals, face
    lengths and centroid offsets rounded to FP32 against the exact geometry.  The GPU's FP32
    mode stores its per-cell geometry in FP32, so its max-abs error on this workload is bounded
    below by effects of this size; the run is recorded and bounded loosely (the L2 part stays near
    1e-5, single cells move by up to a few 1e-4)."""
    wl = I.tri_ellipse_workload(h=0.01, seed=0, nsteps=2000)
    ex = wl.extra
    mesh4 = (ex["verts"], ex["tris"], ex["face_cells"], ex["face_verts"])
    mesh = O.tri_mesh(*mesh4)
    dt = 1e-3
    U0 = O.from_soa(wl.U0[0], "tm2d")
    ref = GL.LinearStep(mesh, dt, 0.01 * dt).run(U0, 2000)
    m32 = O.tri_mesh(*mesh4)
    for a in ("vol", "normal", "area", "dL", "dR"):
        setattr(m32, a, np.ascontiguousarray(getattr(m32, a).astype(np.float32).astype(np.float64)))
    out = GL.LinearStep(m32, dt, 0.01 * dt).run(U0, 2000)
    l2 = rel(out, ref)
    mx = float(np.abs(out - ref).max() / np.abs(ref).max())
    print(f"geometry rounded to FP32, 2000 steps: rel L2 {l2:.2e}, max-abs {mx:.2e}")
    assert 1e-7 < l2 < 1e-4 and mx < 3e-3
