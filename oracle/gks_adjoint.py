"""FP64 CPU oracle of the reverse-mode adjoint of the GKS step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may import this
module.  It uses nothing but the oracle step of ``gks_oracle`` (Sec. 3.1) and writes the
adjoint out from its definition:

  * For fixed materials the step U' = Phi(U) + s (s: the explicit source) is linear in U, so
    its Jacobian A is the matrix whose column j is Phi(e_j).  ``step_matrix`` assembles A by
    stepping every unit vector, and the adjoint of a co-state lam' is A^T lam'.
  * For one cell c the step is a quadratic polynomial in 1/eps_c (and in 1/mu_c): the cell's
    own update is scaled by it and the face fluxes of its faces are linear in it (through the
    face-average material of the equilibrium time derivative).  A central difference of
    J(m) = <lam', U'(m)> with any step therefore gives dJ/dm_c exactly, up to rounding.

Nothing here is blocked, fused or reordered: it is the definition, slowly.

States are (ncells, 6) arrays as in ``gks_oracle`` (2D TM problems use the columns Ez, Hx, Hy).
"""
from __future__ import annotations

import numpy as np

from . import gks_oracle as O

ALL = (0, 1, 2, 3, 4, 5)


def default_comps(mesh) -> tuple:
    return O.TM if mesh.dim == 2 else ALL


def step_matrix(mesh, dt, tau, c=1.0, epsinv=None, muinv=None, comps=None) -> np.ndarray:
    """Jacobian of one step with respect to the components ``comps`` (field-major order:
    index f * ncells + cell), assembled column by column from steps of unit vectors."""
    comps = default_comps(mesh) if comps is None else tuple(comps)
    nc = mesh.ncells
    n = nc * len(comps)
    C = O.coefficients(dt, tau)
    A = np.zeros((n, n))
    for f, comp in enumerate(comps):
        for j in range(nc):
            e = np.zeros((nc, 6))
            e[j, comp] = 1.0
            out = O.step(mesh, e, dt, tau, c, epsinv, muinv, None, C)
            A[:, f * nc + j] = out[:, list(comps)].T.reshape(-1)
    return A


def _flat(U, comps):
    return np.asarray(U, dtype=np.float64)[:, list(comps)].T.reshape(-1)


def _unflat(v, nc, comps):
    U = np.zeros((nc, 6))
    U[:, list(comps)] = v.reshape(len(comps), nc).T
    return U


def adjoint_state(mesh, lam_next, A, comps=None) -> np.ndarray:
    """lam = A^T lam' (the co-state one step earlier)."""
    comps = default_comps(mesh) if comps is None else tuple(comps)
    return _unflat(A.T @ _flat(lam_next, comps), mesh.ncells, comps)


def material_gradients(mesh, U, lam_next, dt, tau, c=1.0, epsinv=None, muinv=None, J=None, comps=None):
    """(dJ/d(1/eps), dJ/d(1/mu)) per cell of J = <lam', step(U)>, including the source term,
    by exact central differences of the quadratic dependence on each cell's value."""
    comps = default_comps(mesh) if comps is None else tuple(comps)
    nc = mesh.ncells
    C = O.coefficients(dt, tau)
    ei = np.ones(nc) if epsinv is None else np.array(epsinv, dtype=np.float64)
    mi = np.ones(nc) if muinv is None else np.array(muinv, dtype=np.float64)
    lam = np.asarray(lam_next, dtype=np.float64)[:, list(comps)]

    def Jval(e, m):
        out = O.step(mesh, U, dt, tau, c, e, m, J, C)
        return out[:, list(comps)]

    gE = np.zeros(nc)
    gH = np.zeros(nc)
    for cell in range(nc):
        for which, g in ((0, gE), (1, gH)):
            base = ei if which == 0 else mi
            h = 0.5 * max(1.0, abs(base[cell]))
            up = base.copy()
            dn = base.copy()
            up[cell] += h
            dn[cell] -= h
            if which == 0:
                d = Jval(up, mi) - Jval(dn, mi)
            else:
                d = Jval(ei, up) - Jval(ei, dn)
            g[cell] = float(np.sum(lam * d)) / (2.0 * h)
    return gE, gH


def adjoint_step(mesh, U, lam_next, dt, tau, c=1.0, epsinv=None, muinv=None, J=None, comps=None, A=None):
    """Adjoint of one step from state U (ncells, 6) with source J (ncells, 3) or None:
    returns (lam, g_epsinv, g_muinv)."""
    if A is None:
        A = step_matrix(mesh, dt, tau, c, epsinv, muinv, comps)
    lam = adjoint_state(mesh, lam_next, A, comps)
    gE, gH = material_gradients(mesh, U, lam_next, dt, tau, c, epsinv, muinv, J, comps)
    return lam, gE, gH


def source_field(mesh, source, tn):
    """J (ncells, 3) of a point source (cells, weights, J0, tc, sigma_t) at time tn."""
    if source is None:
        return None
    cells, w, J0, tc, sg = source
    J = np.zeros((mesh.ncells, 3))
    J[np.asarray(cells), 2] = np.asarray(w) * O.gaussian_pulse(tn, J0, tc, sg)
    return J


def probe_energy(mesh, U, cells) -> float:
    """P = sum over the probe cells of |Omega| Ez^2."""
    U = np.asarray(U)
    cells = np.asarray(cells)
    return float(np.sum(mesh.vol[cells] * U[cells, 2] ** 2))


def probe_energy_grad(mesh, U, cells) -> np.ndarray:
    """dP/dU: 2 |Omega| Ez on the probe cells."""
    g = np.zeros((mesh.ncells, 6))
    cells = np.asarray(cells)
    g[cells, 2] = 2.0 * mesh.vol[cells] * np.asarray(U)[cells, 2]
    return g


def run_gradients(mesh, U0, nsteps, dt, tau, c=1.0, epsinv=None, muinv=None, source=None, t0=0.0,
                  probe_cells=None, comps=None):
    """Loss P(U^N) (probe energy) after nsteps steps from U0 and its gradients with respect to
    U0, 1/eps and 1/mu: the forward states are kept and the adjoint steps run backwards."""
    comps = default_comps(mesh) if comps is None else tuple(comps)
    C = O.coefficients(dt, tau)
    states = [np.asarray(U0, dtype=np.float64).reshape(mesh.ncells, 6)]
    for n in range(nsteps):
        J = source_field(mesh, source, t0 + n * dt)
        states.append(O.step(mesh, states[-1], dt, tau, c, epsinv, muinv, J, C))
    loss = probe_energy(mesh, states[-1], probe_cells)
    lam = probe_energy_grad(mesh, states[-1], probe_cells)
    A = step_matrix(mesh, dt, tau, c, epsinv, muinv, comps)
    gE = np.zeros(mesh.ncells)
    gH = np.zeros(mesh.ncells)
    for n in reversed(range(nsteps)):
        J = source_field(mesh, source, t0 + n * dt)
        e, h = material_gradients(mesh, states[n], lam, dt, tau, c, epsinv, muinv, J, comps)
        gE += e
        gH += h
        lam = adjoint_state(mesh, lam, A, comps)
    return loss, lam, gE, gH
