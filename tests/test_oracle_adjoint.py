"""Pins of the oracle adjoint (CPU).

The oracle adjoint assembles the step's Jacobian from steps of unit vectors and transposes it;
these tests pin it to facts that do not go through that assembly:
  * discrete reciprocity (2D): the flux Jacobians of Maxwell's equations are symmetric and odd under
    S = diag(1, 1, 1, -1, -1, -1) (E even, H odd), the central differences are skew on periodic
    and mirror-ghost grids and the lattice dissipation is symmetric and even under S, so in
    vacuum the step matrix satisfies A^T = S A S: the adjoint of a co-state is S Phi(S lam');
  * with materials and tau = inf the equilibrium time derivative (the only place a face-average
    material enters) drops out, A = I + M^{-1} K with K^T = S K S, hence A^T = M S A S M^{-1};
  * on non-reflecting grids, with materials and a source: <A^T lam', dU> = <lam', Phi(dU)>;
  * material gradients: the step is quadratic along any material direction, so the central
    difference of <lam', U'> along a random joint (1/eps, 1/mu) direction is exact;
  * gradients of a multi-step probe-energy loss against finite differences of the forward run.
"""
import numpy as np
import pytest

from oracle import gks_adjoint as OA
from oracle import gks_oracle as O

PER, NR, PEC = O.BC_PERIODIC, O.BC_NONREFLECT, O.BC_PEC


def _rand_state(rng, nc, comps):
    U = np.zeros((nc, 6))
    U[:, list(comps)] = rng.standard_normal((nc, len(comps)))
    return U


def _S(U):
    V = np.array(U, dtype=np.float64)
    V[:, 3:] *= -1.0
    return V


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("bc", [(PER,) * 4, (PEC,) * 4, (PER, PER, PEC, PEC)])
@pytest.mark.parametrize("tau_hat", [0.0, 0.01, 1.0, np.inf])
def test_reciprocity_vacuum_2d(oracle, bc, tau_hat):
    nx, ny = 9, 7
    mesh = O.cart2d(nx, ny, bc=bc)
    dt = 0.45 / nx
    tau = tau_hat * dt
    rng = np.random.default_rng(3)
    lamp = _rand_state(rng, mesh.ncells, O.TM)
    A = OA.step_matrix(mesh, dt, tau)
    lam = OA.adjoint_state(mesh, lamp, A)
    expect = _S(O.step(mesh, _S(lamp), dt, tau))
    assert _rel(lam[:, list(O.TM)], expect[:, list(O.TM)]) < 1e-14


def test_transpose_identity_3d(oracle):
    """3D: the D3Q4 lattice is chiral (its half-lattice third moment u_x u_y u_z does not
    vanish), so the upwind second-order terms are not S-symmetric and only the transposition
    identity applies."""
    mesh = O.cart3d(4, 4, 3, bc=(PER, PER, NR, NR, PEC, PEC))
    dt = 0.3 / 4
    tau = 0.01 * dt
    rng = np.random.default_rng(5)
    A = OA.step_matrix(mesh, dt, tau)
    for _ in range(2):
        lamp = rng.standard_normal((mesh.ncells, 6))
        dU = rng.standard_normal((mesh.ncells, 6))
        lhs = np.sum(OA.adjoint_state(mesh, lamp, A) * dU)
        rhs = np.sum(lamp * O.step(mesh, dU, dt, tau))
        assert abs(lhs - rhs) <= 1e-13 * np.abs(lamp).sum() * np.abs(dU).max()


@pytest.mark.parametrize("bc", [(PER,) * 4, (PEC, PEC, PER, PER)])
def test_weighted_reciprocity_materials_kfvs(oracle, bc):
    nx, ny = 8, 7
    mesh = O.cart2d(nx, ny, bc=bc)
    dt = 0.45 / nx
    rng = np.random.default_rng(7)
    ei = rng.uniform(0.25, 1.0, mesh.ncells)
    mi = rng.uniform(0.5, 1.0, mesh.ncells)
    lamp = _rand_state(rng, mesh.ncells, O.TM)
    A = OA.step_matrix(mesh, dt, np.inf, epsinv=ei, muinv=mi)
    lam = OA.adjoint_state(mesh, lamp, A)
    # A^T lam' = M S Phi(S M^{-1} lam'), M = diag(eps, mu)
    minv = np.concatenate([np.repeat(ei[:, None], 3, 1), np.repeat(mi[:, None], 3, 1)], axis=1)
    expect = _S(O.step(mesh, _S(lamp * minv), dt, np.inf, 1.0, ei, mi)) / minv
    assert _rel(lam[:, list(O.TM)], expect[:, list(O.TM)]) < 1e-14
    # the weighting matters: the plain S-conjugate differs
    plain = _S(O.step(mesh, _S(lamp), dt, np.inf, 1.0, ei, mi))
    assert _rel(lam[:, list(O.TM)], plain[:, list(O.TM)]) > 1e-3


@pytest.mark.parametrize("bc", [(NR,) * 4, (NR, PEC, PER, PER), (PEC, NR, NR, PEC)])
def test_transpose_identity_nr_materials(oracle, bc):
    nx, ny = 9, 8
    mesh = O.cart2d(nx, ny, bc=bc)
    dt = 0.5 / nx
    tau = 0.01 * dt
    rng = np.random.default_rng(11)
    ei = rng.uniform(0.25, 1.0, mesh.ncells)
    mi = rng.uniform(0.5, 1.0, mesh.ncells)
    A = OA.step_matrix(mesh, dt, tau, epsinv=ei, muinv=mi)
    for _ in range(3):
        lamp = _rand_state(rng, mesh.ncells, O.TM)
        dU = _rand_state(rng, mesh.ncells, O.TM)
        lam = OA.adjoint_state(mesh, lamp, A)
        lhs = np.sum(lam * dU)
        rhs = np.sum(lamp * O.step(mesh, dU, dt, tau, 1.0, ei, mi))
        assert abs(lhs - rhs) <= 1e-13 * (np.abs(lam).sum() * np.abs(dU).max())
    # a transposed operand is caught: A lam' differs from A^T lam'
    lamp = _rand_state(rng, mesh.ncells, O.TM)
    wrong = O.step(mesh, lamp, dt, tau, 1.0, ei, mi)
    assert _rel(OA.adjoint_state(mesh, lamp, A), wrong) > 1e-2


@pytest.mark.parametrize("tau_hat", [0.0, 0.01, np.inf])
def test_material_gradient_directional(oracle, tau_hat):
    nx, ny = 8, 7
    mesh = O.cart2d(nx, ny, bc=(NR, PEC, PER, PER))
    dt = 0.5 / nx
    tau = tau_hat * dt
    rng = np.random.default_rng(13)
    ei = rng.uniform(0.25, 1.0, mesh.ncells)
    mi = rng.uniform(0.5, 1.0, mesh.ncells)
    U = _rand_state(rng, mesh.ncells, O.TM)
    lamp = _rand_state(rng, mesh.ncells, O.TM)
    J = np.zeros((mesh.ncells, 3))
    J[[5, 20], 2] = [0.7, -1.3]
    gE, gH = OA.material_gradients(mesh, U, lamp, dt, tau, 1.0, ei, mi, J)
    de = rng.standard_normal(mesh.ncells) * 0.1
    dm = rng.standard_normal(mesh.ncells) * 0.1

    def Jv(s):
        return np.sum(lamp * O.step(mesh, U, dt, tau, 1.0, ei + s * de, mi + s * dm, J))

    fd = (Jv(1.0) - Jv(-1.0)) / 2.0
    an = np.dot(gE, de) + np.dot(gH, dm)
    assert abs(fd - an) <= 1e-12 * max(abs(fd), np.abs(gE).sum() * 0.1)
    # the source enters the 1/eps gradient of its cells: -dt J lam'_Ez on top of the flux part
    gE0, _ = OA.material_gradients(mesh, U, lamp, dt, tau, 1.0, ei, mi, None)
    d = gE - gE0
    expect = np.zeros(mesh.ncells)
    expect[[5, 20]] = -dt * np.array([0.7, -1.3]) * lamp[[5, 20], 2]
    assert np.allclose(d, expect, rtol=1e-12, atol=1e-14)


def test_run_gradients_against_finite_differences(oracle):
    nx, ny = 10, 8
    mesh = O.cart2d(nx, ny, bc=(NR, NR, PEC, NR))
    dt = 0.5 / nx
    tau = 0.01 * dt
    K = 3
    rng = np.random.default_rng(17)
    ei = rng.uniform(0.25, 1.0, mesh.ncells)
    mi = rng.uniform(0.5, 1.0, mesh.ncells)
    U0 = _rand_state(rng, mesh.ncells, O.TM)
    source = (np.array([33]), np.array([1.0]), 2.0, 0.05, 0.04)
    probe = np.array([i + nx * j for j in range(3, 6) for i in range(5, 9)])
    loss, lam0, gE, gH = OA.run_gradients(mesh, U0, K, dt, tau, 1.0, ei, mi, source, 0.0, probe)

    def L(U, e, m):
        V = U
        for n in range(K):
            V = O.step(mesh, V, dt, tau, 1.0, e, m, OA.source_field(mesh, source, n * dt))
        return OA.probe_energy(mesh, V, probe)

    assert abs(L(U0, ei, mi) - loss) <= 1e-15 * abs(loss)
    # quadratic in U0: the central difference is exact
    dU = _rand_state(rng, mesh.ncells, O.TM)
    fd = (L(U0 + dU, ei, mi) - L(U0 - dU, ei, mi)) / 2.0
    assert abs(fd - np.sum(lam0 * dU)) <= 1e-12 * abs(fd)
    # materials: fourth-order central difference
    de = rng.standard_normal(mesh.ncells)
    dm = rng.standard_normal(mesh.ncells)
    s = 1e-3

    def Lm(t):
        return L(U0, ei + t * de, mi + t * dm)

    fd = (8 * (Lm(s) - Lm(-s)) - (Lm(2 * s) - Lm(-2 * s))) / (12 * s)
    an = np.dot(gE, de) + np.dot(gH, dm)
    assert abs(fd - an) <= 1e-8 * abs(an)
