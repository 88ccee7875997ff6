"""GPU parity of the triangle-mesh TM step (libgks through its C ABI) against the FP64 oracle.

Tolerances (relative L2 over all fields, cells and batch items, after the stated steps):
FP64 1e-12, FP32 1e-5 (FP32 storage and flux arithmetic, FP64 accumulation).
"""
import numpy as np
import pytest

from oracle import gks_oracle as O
from paper_2412_16845_amd import inputs as I
from tests.gks_helpers import rel_l2
from tests.test_oracle_tri import square_tri_mesh

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
SRC = (2.0, 0.01, 0.01)   # J0, t0, sigma_t


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def dev(torch, a, precision):
    if a is None:
        return None
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64 if precision == "fp64" else torch.float32,
                        device="cuda")


def solver(torch, mesh4, precision, batch, tau_hat, ei=None, mi=None, cells=(), w=(), gradient="green_gauss"):
    from paper_2412_16845_amd.gks import Solver
    s = Solver("tri2d", tri=mesh4, precision=precision, batch=batch, cfl=0.5, tau_over_dt=tau_hat,
               gradient=gradient)
    s.set_material(dev(torch, ei, precision), dev(torch, mi, precision))
    if len(cells):
        s.set_point_source(cells, w, *SRC)
    return s


def oracle_tri(mesh4, U0, nsteps, dt, tau, ei=None, mi=None, source=None, t0=0.0, gradient=O.GRAD_GREEN_GAUSS):
    mesh = O.tri_mesh(*mesh4)
    out = []
    for b in range(U0.shape[0]):
        U = O.from_soa(U0[b], "tm2d")
        e = None if ei is None else ei[b]
        m = None if mi is None else mi[b]
        out.append(O.to_soa(O.run(mesh, U, nsteps, dt, tau, epsinv=e, muinv=m, source=source, t0=t0,
                                  gradient=gradient), "tm2d"))
    return np.stack(out)


def _one_triangle(bc):
    verts = np.array([[0.0, 0.0], [1.0, 0.1], [0.3, 0.8]])
    tris = np.array([[0, 1, 2]])
    fv = np.array([[0, 1], [1, 2], [2, 0]])
    fc = np.array([[0, -(1 + bc)]] * 3)
    return verts, tris, fc, fv


CASES = {
    # name: (mesh, batch, tau_hat, eps, mu, sources, steps, gradient)
    "ellipse_eps_mu_src": (lambda: I.tri_ellipse_mesh(0.03, seed=1, cache=False), 2, 0.01, True, True, 2, 30, "green_gauss"),
    "ellipse_vacuum_tau0": (lambda: I.tri_ellipse_mesh(0.035, seed=2, cache=False), 1, 0.0, False, False, 0, 25, "green_gauss"),
    "ellipse_tau_inf": (lambda: I.tri_ellipse_mesh(0.035, seed=4, cache=False), 1, np.inf, True, False, 1, 25, "green_gauss"),
    "pec_square_mu": (lambda: square_tri_mesh(17), 1, 1.0, False, True, 0, 20, "green_gauss"),
    # least-squares gradients: the same meshes (PEC ellipse, non-reflecting outer square)
    "ellipse_lsq_eps_mu_src": (lambda: I.tri_ellipse_mesh(0.03, seed=5, cache=False), 2, 0.01, True, True, 2, 30, "lsq"),
    "pec_square_lsq": (lambda: square_tri_mesh(15), 1, np.inf, True, False, 0, 20, "lsq"),
    # the smallest meshes: one triangle with three boundary faces, and two triangles
    "one_triangle_pec": (lambda: _one_triangle(O.BC_PEC), 2, 0.01, True, True, 0, 6, "green_gauss"),
    "one_triangle_nr_lsq": (lambda: _one_triangle(O.BC_NONREFLECT), 1, 0.01, True, False, 1, 6, "lsq"),
    "two_triangles": (lambda: square_tri_mesh(1), 1, 1.0, False, True, 0, 6, "green_gauss"),
    "two_triangles_lsq": (lambda: square_tri_mesh(1), 1, 0.0, True, True, 0, 6, "lsq"),
}
GRAD = {"green_gauss": O.GRAD_GREEN_GAUSS, "lsq": O.GRAD_LSQ}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_tri_parity(torch, name, precision):
    make, batch, tau_hat, eps, mu, nsrc, nsteps, gradient = CASES[name]
    mesh4 = make()
    nc = mesh4[1].shape[0]
    rng = np.random.default_rng(len(name))
    U0 = rng.standard_normal((batch, 3, nc))
    ei = rng.uniform(0.25, 1.0, (batch, nc)) if eps else None
    mi = rng.uniform(0.5, 1.0, (batch, nc)) if mu else None
    cells = np.sort(rng.choice(nc, nsrc, replace=False)) if nsrc else np.zeros(0, dtype=np.int64)
    w = rng.uniform(0.5, 1.5, nsrc)
    s = solver(torch, mesh4, precision, batch, tau_hat, ei, mi, cells, w, gradient)
    U = dev(torch, U0, precision)
    s.run(U, nsteps)
    src = (cells, w) + SRC if nsrc else None
    ref = oracle_tri(mesh4, U0, nsteps, s.dt, tau_hat * s.dt, ei, mi, src, gradient=GRAD[gradient])
    err = rel_l2(U.cpu().numpy(), ref)
    print(f"{name} {precision}: rel L2 = {err:.3e} ({nc} cells, {nsteps} steps, dt {s.dt:.3e})")
    assert err <= TOL[precision]


def test_tri_energy_matches_oracle_definition(torch):
    mesh4 = I.tri_ellipse_mesh(0.04, seed=7, cache=False)
    nc = mesh4[1].shape[0]
    rng = np.random.default_rng(8)
    U0 = rng.standard_normal((1, 3, nc))
    ei = rng.uniform(0.25, 1.0, (1, nc))
    s = solver(torch, mesh4, "fp64", 1, 0.01, ei)
    W = s.energy(dev(torch, U0, "fp64"))[0]
    mesh = O.tri_mesh(*mesh4)
    ref = O.energy(mesh, O.from_soa(U0[0], "tm2d"), eps=1.0 / ei[0])
    assert abs(W - ref) <= 1e-13 * ref


def test_tri_bad_topology(torch):
    from paper_2412_16845_amd.gks import GKSError, Solver
    verts, tris, fc, fv = square_tri_mesh(4)
    bad = fc.copy()
    bad[0, 1] = -1            # periodic boundary code on a triangle mesh
    with pytest.raises(GKSError, match="EINVAL"):
        Solver("tri2d", tri=(verts, tris, bad, fv))
    bad = fc.copy()
    bad[3, 0] = tris.shape[0]  # owner out of range
    with pytest.raises(GKSError, match="EINVAL"):
        Solver("tri2d", tri=(verts, tris, bad, fv))
    with pytest.raises(GKSError, match="EINVAL"):
        Solver("tri2d", tri=(verts, tris, fc[1:], fv[1:]))   # a cell with two faces


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_ellipse_mesh(torch, precision):
    """The ~4M-triangle workload (square with an elliptical PEC hole, non-reflecting outer
    square, Gaussian pulse), 2000 steps; the last 2 steps are re-done by the oracle on the whole
    mesh from the GPU's state, and the energy does not grow."""
    wl = I.tri_ellipse_workload(h=6.8e-4, seed=0, nsteps=2000)
    ex = wl.extra
    mesh4 = (ex["verts"], ex["tris"], ex["face_cells"], ex["face_verts"])
    nc = mesh4[1].shape[0]
    assert 3.9e6 < nc < 4.2e6
    s = solver(torch, mesh4, precision, 1, wl.tau_over_dt)
    U = dev(torch, wl.U0, precision)
    W0 = s.energy(U)[0]
    K = 2
    s.run(U, wl.nsteps - K)
    start = U.cpu().numpy().astype(np.float64)
    s.run(U, K, t0=(wl.nsteps - K) * s.dt)
    end = U.cpu().numpy()
    W1 = s.energy(U)[0]
    assert np.isfinite(end).all() and W1 <= W0 * (1 + 1e-9)
    ref = oracle_tri(mesh4, start, K, s.dt, wl.tau_over_dt * s.dt, t0=(wl.nsteps - K) * s.dt)
    err = rel_l2(end, ref)
    print(f"{nc} triangles {precision}: last {K} steps rel L2 = {err:.3e}; energy {W0:.4e} -> {W1:.4e}")
    assert err <= TOL[precision]
