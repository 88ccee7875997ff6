"""The GKS step as a probed linear map -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may use this module (like the rest of ``oracle/``).  It adds no scheme
arithmetic of its own: every number in the map comes from steps of the literal oracle
(``gks_oracle.step``).

For fixed materials (and without the slope limiter) the step of Sec. 3.1 is affine in the
state: U' = A U + s(t), where s(t) = dt M^-1 S(t^n) is the explicit source, itself linear in the
current density J.  A therefore has column j equal to the step of the unit vector e_j, which is
what ``gks_adjoint.step_matrix`` computes one column at a time.  Here the columns are probed
many at once: the output of cell o depends only on the cells of its region R(o) (the cells at
most two face-neighbour hops away: one hop for the cell gradients, one for the faces of o), so
the unit vectors of cells that never share a region can be stepped together and each response
assigned to the one probed cell inside R(o).  The assignment is checked, not assumed: every
output outside the probed cells' regions must be exactly zero.

Runs then cost one sparse product per step instead of one literal step, which lets the oracle
follow the configurations over their full step counts on grids of a few hundred thousand cells.
The literal run and this one differ only in rounding order (checked in
``tests/test_oracle_linear.py``).

States are (ncells, 6) arrays as in ``gks_oracle`` ((ncells, 8) for the PHM system); the map acts
on the components ``comps`` (default: Ez, Hx, Hy in 2D, all six in 3D; with PHM also psi in 2D
and all eight in 3D), field-major: index f * ncells + cell.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import gks_oracle as O

ALL = (0, 1, 2, 3, 4, 5)


def _adjacency(mesh) -> sp.csr_matrix:
    """Cell adjacency through interior faces (periodic faces included), with the diagonal."""
    L, R = mesh.face_L, mesh.face_R
    inner = R >= 0
    nc = mesh.ncells
    i = np.concatenate([L[inner], R[inner], np.arange(nc)])
    j = np.concatenate([R[inner], L[inner], np.arange(nc)])
    A = sp.csr_matrix((np.ones(i.shape[0]), (i, j)), shape=(nc, nc))
    A.data[:] = 1.0
    return A


def regions(mesh) -> sp.csr_matrix:
    """R[o, p] = 1 when cell p is within two face-neighbour hops of cell o."""
    A = _adjacency(mesh)
    R = (A @ A).tocsr()
    R.data[:] = 1.0
    return R


def _cart_colors(mesh):
    """Linear colouring of a Cartesian grid: two cells of one colour are at least five face hops
    apart, so that no region holds two of them (2D: (i + 5 j) mod 13, 3D: (i + 4 j + 10 k) mod
    27).  None when a periodic axis would break it."""
    nx, ny, nz = mesh.shape
    M, a, b = (13, 5, 0) if mesh.dim == 2 else (27, 4, 10)
    periodic = np.zeros(3, dtype=bool)
    L, R = mesh.face_L, mesh.face_R
    inner = R >= 0
    d = np.abs(R[inner] - L[inner])
    periodic[0] = np.any(d == nx - 1) and nx > 2
    periodic[1] = np.any(d == nx * (ny - 1)) and ny > 2
    periodic[2] = mesh.dim == 3 and np.any(d == nx * ny * (nz - 1)) and nz > 2
    if (periodic[0] and nx % M) or (periodic[1] and (a * ny) % M) or (periodic[2] and (b * nz) % M):
        return None
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + a * j + b * k) % M).reshape(-1)


def greedy_colors(R: sp.csr_matrix) -> np.ndarray:
    """Greedy colouring of the cells such that no region holds two cells of one colour (cells p
    and q conflict when some region holds both, i.e. (R R)[p, q] != 0)."""
    C = (R @ R).tocsr()
    nc = R.shape[0]
    col = np.full(nc, -1, dtype=np.int64)
    for p in range(nc):
        nb = C.indices[C.indptr[p]:C.indptr[p + 1]]
        used = set(col[nb][col[nb] >= 0].tolist())
        c = 0
        while c in used:
            c += 1
        col[p] = c
    return col


class LinearStep:
    """The affine step U' = A U + pulse(t^n) b of one mesh, materials and time step, probed from
    the literal oracle."""

    def __init__(self, mesh, dt, tau, c=1.0, epsinv=None, muinv=None, source=None, comps=None, colors=None,
                 gradient=O.GRAD_GREEN_GAUSS, phm=None):
        self.mesh = mesh
        # phm = (chi, gamma): the eight-component PHM state (Sec. 2.1); the TM components then
        # include psi (column 7), and the 3D ones all eight
        self.chi, self.gamma = (0.0, 0.0) if phm is None else (float(phm[0]), float(phm[1]))
        self.width = 6 if phm is None else 8
        if comps is None:
            if phm is None:
                comps = O.TM if mesh.dim == 2 else ALL
            else:
                comps = O.TM_PHM if mesh.dim == 2 else tuple(range(8))
        self.comps = tuple(comps)
        self.dt, self.tau, self.c = dt, tau, c
        self.epsinv, self.muinv, self.gradient = epsinv, muinv, gradient
        self.C = O.coefficients(dt, tau)
        nc = mesh.ncells
        R = regions(mesh)
        if colors is None:
            colors = _cart_colors(mesh) if hasattr(mesh, "shape") else None
            if colors is None:
                colors = greedy_colors(R)
        self.colors = np.asarray(colors)
        self.A = self._probe(R, self.colors)
        self.source = source
        self.b = None
        if source is not None:
            cells, w, J0, tc, sg = source
            J = np.zeros((nc, 3))
            J[np.asarray(cells), 2] = np.asarray(w, dtype=np.float64)   # unit pulse amplitude
            out = O.step(mesh, np.zeros((nc, self.width)), dt, tau, c, epsinv, muinv, J, self.C, gradient,
                         chi=self.chi, gamma=self.gamma)
            self.b = out[:, list(self.comps)].T.reshape(-1).copy()

    def _probe(self, R, colors) -> sp.csr_matrix:
        mesh, comps = self.mesh, self.comps
        nc, nk = mesh.ncells, len(comps)
        Rc = R.tocoo()
        o_all, p_all = Rc.row, Rc.col
        rows, cols, vals = [], [], []
        for col in np.unique(colors):
            sel = colors[p_all] == col
            o, p = o_all[sel], p_all[sel]
            if np.unique(o).shape[0] != o.shape[0]:
                raise ValueError(f"colour {col} occurs twice in one region: the colouring is not valid")
            outside = np.ones(nc, dtype=bool)
            outside[o] = False
            probe_cells = np.nonzero(colors == col)[0]
            for f, comp in enumerate(comps):
                U = np.zeros((nc, self.width))
                U[probe_cells, comp] = 1.0
                out = O.step(mesh, U, self.dt, self.tau, self.c, self.epsinv, self.muinv, None, self.C,
                             self.gradient, chi=self.chi, gamma=self.gamma)[:, list(comps)]
                if np.any(out[outside] != 0.0):
                    raise ValueError("a cell responds to a probe outside its region: the step reaches further "
                                     "than two face hops")
                for g in range(nk):
                    v = out[o, g]
                    nz = v != 0.0
                    rows.append(g * nc + o[nz])
                    cols.append(f * nc + p[nz])
                    vals.append(v[nz])
        n = nc * nk
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))

    def flat(self, U) -> np.ndarray:
        return np.asarray(U, dtype=np.float64)[:, list(self.comps)].T.reshape(-1).copy()

    def unflat(self, v) -> np.ndarray:
        U = np.zeros((self.mesh.ncells, self.width))
        U[:, list(self.comps)] = np.asarray(v).reshape(len(self.comps), -1).T
        return U

    def run(self, U0, nsteps, t0=0.0) -> np.ndarray:
        """nsteps steps from time t0 (t^n = t0 + n dt) of the state U0 (ncells, 6; 8 with PHM)."""
        v = self.flat(U0)
        for n in range(nsteps):
            v = self.A @ v
            if self.b is not None:
                _, _, J0, tc, sg = self.source
                v += O.gaussian_pulse(t0 + n * self.dt, J0, tc, sg) * self.b
        return self.unflat(v)


# ----------------------------------------------------------------------------- adjoint
def _probe_attribution(R1: sp.csr_matrix, colors: np.ndarray, col) -> tuple:
    """For colour col: (outputs o, cells p) with p the one cell of that colour in R1(o)."""
    Rc = R1.tocoo()
    sel = colors[Rc.col] == col
    o, p = Rc.row[sel], Rc.col[sel]
    if np.unique(o).shape[0] != o.shape[0]:
        raise ValueError(f"material colour {col} occurs twice next to one cell: the colouring is not valid")
    return o, p


class LinearAdjoint:
    """Reverse mode of a run of LinearStep steps, by definition:

      lam^n = A^T lam^{n+1}  (the step's Jacobian, transposed), and
      dJ/dm_p += lam^{n+1} . dPhi(U^n)/dm_p  for m = 1/eps (and 1/mu).

    The output of cell o depends on m_p only for p = o or a face neighbour of o (the cell's own
    update factor, and the face-average material of the equilibrium time derivative on its
    faces), and at most quadratically, so a central difference of the step in m_p is exact.
    Cells that never neighbour one output are perturbed together (a distance-2 colouring): for
    colour c, B_c U = Phi(U; m + h e_c) - Phi(U; m - h e_c) with both steps probed as
    LinearStep maps, and each output's share lam_o . (B_c U)_o is credited to the one cell of
    colour c next to o, divided by 2 h_p."""

    def __init__(self, fwd: LinearStep, materials=("eps",)):
        self.fwd = fwd
        mesh = fwd.mesh
        nc = mesh.ncells
        A1 = _adjacency(mesh)
        colors = greedy_colors(A1)            # conflict: (A1 A1)[p, q] != 0
        self.terms = {}
        for which in materials:
            base = fwd.epsinv if which == "eps" else fwd.muinv
            base = np.ones(nc) if base is None else np.asarray(base, dtype=np.float64)
            h = 0.5 * np.maximum(1.0, np.abs(base))
            terms = []
            for col in np.unique(colors):
                mask = colors == col
                up, dn = base.copy(), base.copy()
                up[mask] += h[mask]
                dn[mask] -= h[mask]
                steps = []
                for m in (up, dn):
                    kw = dict(epsinv=m, muinv=fwd.muinv) if which == "eps" else dict(epsinv=fwd.epsinv, muinv=m)
                    steps.append(LinearStep(mesh, fwd.dt, fwd.tau, fwd.c, source=fwd.source, comps=fwd.comps,
                                            colors=fwd.colors, gradient=fwd.gradient, **kw))
                B = (steps[0].A - steps[1].A).tocsr()
                bs = None if fwd.source is None else steps[0].b - steps[1].b
                o, p = _probe_attribution(A1, colors, col)
                S = sp.csr_matrix((1.0 / (2.0 * h[p]), (p, o)), shape=(nc, nc))
                terms.append((B, bs, S))
            self.terms[which] = terms

    def gradients(self, states, lam_end, t0=0.0):
        """states: [U^0 .. U^N] (each (ncells, 6)); lam_end = dJ/dU^N (ncells, 6).  Returns
        (dJ/dU^0 as (ncells, 6), {material: dJ/dm per cell})."""
        fwd = self.fwd
        nk, nc = len(fwd.comps), fwd.mesh.ncells
        lam = fwd.flat(lam_end)
        g = {k: np.zeros(nc) for k in self.terms}
        AT = fwd.A.T.tocsr()
        for n in reversed(range(len(states) - 1)):
            u = fwd.flat(states[n])
            amp = 0.0
            if fwd.source is not None:
                _, _, J0, tc, sg = fwd.source
                amp = O.gaussian_pulse(t0 + n * fwd.dt, J0, tc, sg)
            for which, terms in self.terms.items():
                for B, bs, S in terms:
                    d = B @ u
                    if bs is not None:
                        d = d + amp * bs
                    share = (lam * d).reshape(nk, nc).sum(axis=0)
                    g[which] += S @ share
            lam = AT @ lam
        return fwd.unflat(lam), g

    def run(self, U0, nsteps, t0=0.0):
        """Forward states [U^0 .. U^N] of the affine map."""
        fwd = self.fwd
        states = [np.asarray(U0, dtype=np.float64)]
        v = fwd.flat(U0)
        for n in range(nsteps):
            v = fwd.A @ v
            if fwd.b is not None:
                _, _, J0, tc, sg = fwd.source
                v += O.gaussian_pulse(t0 + n * fwd.dt, J0, tc, sg) * fwd.b
            states.append(fwd.unflat(v))
        return states
