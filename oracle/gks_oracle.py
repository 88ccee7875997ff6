"""FP64 CPU oracle of the GKS step for Maxwell's equations -- Python side.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the HIP library: it builds its own
mesh geometry, computes its own time-integrated coefficients and calls its own literal C
implementation of the step (``gks_oracle.c``).

Contents
  * ``coefficients(dt, tau)``: C1..C5 of the time-integrated flux (Sec. 3.1, numerical flux
    coefficients), evaluated in 80-digit decimal arithmetic from the printed closed forms, so
    that they are exact to double rounding for every tau (including tau -> 0 and tau -> inf).
  * mesh builders: Cartesian 2D/3D grids (periodic, non-reflecting or PEC sides), windows of a
    Cartesian grid (for sampled checks of large problems) and triangle meshes.
  * ``step`` / ``run``: the explicit update (Sec. 3.1), literal per-face flux in the face frame.
  * ``energy``: W = 1/2 sum |Omega_i| (eps_i |E_i|^2 + mu_i |H_i|^2 (+ phi^2 + psi^2)).

States are arrays of shape (ncells, 6) holding (Ex, Ey, Ez, Hx, Hy, Hz); 2D TM problems use
columns 2, 3, 4 (Ez, Hx, Hy).  The perfectly hyperbolic Maxwell (PHM) system of Sec. 2.1 adds
the divergence-cleaning potentials phi and psi: its states have shape (ncells, 8), columns 6
and 7, and its couplings chi and gamma are keyword arguments of ``step`` and ``run``.  The C
code always carries eight components; six-component states are the chi = gamma = 0 case with
zero potentials, padded on the way in and cut on the way out.
"""
from __future__ import annotations

import ctypes
import decimal
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gks_oracle.c")
LIB = os.path.join(HERE, "liboracle_gks.so")

BC_PERIODIC, BC_NONREFLECT, BC_PEC = 0, 1, 2
TM = (2, 3, 4)  # Ez, Hx, Hy columns of the six-component state
TM_PHM = (2, 3, 4, 7)  # Ez, Hx, Hy, psi columns of the eight-component state
NC = 8  # components the C code carries per cell


def _widen(U: np.ndarray, nc: int) -> tuple:
    """(ncells, 6 or 8) -> contiguous (ncells, 8) and the width given."""
    U = np.asarray(U, dtype=np.float64)
    w = U.shape[-1] if U.ndim == 2 else U.size // nc
    if w not in (6, 8):
        raise ValueError(f"states have 6 or 8 components per cell, not {w}")
    U = U.reshape(nc, w)
    if w == 8:
        return np.ascontiguousarray(U), 8
    V = np.zeros((nc, NC))
    V[:, :6] = U
    return V, 6


# ----------------------------------------------------------------------------- build / load
def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP over cells and faces)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("ncells", ctypes.c_int64), ("nfaces", ctypes.c_int64),
                ("vol", ctypes.c_void_p), ("face_L", ctypes.c_void_p), ("face_R", ctypes.c_void_p),
                ("normal", ctypes.c_void_p), ("area", ctypes.c_void_p), ("dL", ctypes.c_void_p),
                ("dR", ctypes.c_void_p), ("cf_ptr", ctypes.c_void_p), ("cf_idx", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("dt", ctypes.c_double), ("C", ctypes.c_double * 5),
                ("gradient", ctypes.c_int32), ("limiter", ctypes.c_int32), ("chi", ctypes.c_double),
                ("gamma", ctypes.c_double)]

GRAD_GREEN_GAUSS, GRAD_LSQ = 0, 1
LIMITER_NONE, LIMITER_MINMOD = 0, 1


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _lib.orc_step.restype = ctypes.c_int
        _lib.orc_step.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Params)] + [ctypes.c_void_p] * 5
        _lib.orc_face_flux.restype = None
        _lib.orc_face_flux.argtypes = [ctypes.c_int, ctypes.POINTER(_Params)] + [ctypes.c_void_p] * 4 + \
            [ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        _lib.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_lattice.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
        _lib.orc_rotation.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_gradients.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_gradients_lsq.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_gradients_limited.restype = ctypes.c_int
        _lib.orc_gradients_limited.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_void_p, ctypes.c_void_p]
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# ----------------------------------------------------------------------------- coefficients
def coefficients(dt: float, tau: float) -> tuple:
    """C1..C5 of the time-integrated interface flux (Sec. 3.1).

    The printed closed forms, with e = exp(-dt/tau):
        C1 = dt - tau (1 - e)
        C2 = tau (-dt + 2 tau (1 - e) - dt e)
        C3 = dt^2/2 - tau dt - tau^2 e + tau^2
        C4 = tau (1 - e)
        C5 = -tau dt e + tau^2 (1 - e)
    evaluated with 80 significant digits so that the cancellation at large tau costs nothing.
    tau = 0 and tau = inf are the limits (dt, 0, dt^2/2, 0, 0) and (0, 0, 0, dt, dt^2/2).
    """
    if tau == 0.0:
        return (dt, 0.0, 0.5 * dt * dt, 0.0, 0.0)
    if math.isinf(tau):
        return (0.0, 0.0, 0.0, dt, 0.5 * dt * dt)
    with decimal.localcontext() as ctx:
        ctx.prec = 80
        D = decimal.Decimal
        t, T = D(dt), D(tau)
        e = (-(t / T)).exp()
        C1 = t - T * (1 - e)
        C2 = T * (-t + 2 * T * (1 - e) - t * e)
        C3 = t * t / 2 - T * t - T * T * e + T * T
        C4 = T * (1 - e)
        C5 = -T * t * e + T * T * (1 - e)
        return tuple(float(x) for x in (C1, C2, C3, C4, C5))


# ----------------------------------------------------------------------------- meshes
@dataclass
class Mesh:
    """Face-based finite-volume mesh (Sec. 3.1)."""
    dim: int
    vol: np.ndarray
    face_L: np.ndarray
    face_R: np.ndarray
    normal: np.ndarray
    area: np.ndarray
    dL: np.ndarray
    dR: np.ndarray
    centroid: np.ndarray
    cf_ptr: np.ndarray = None
    cf_idx: np.ndarray = None

    def __post_init__(self):
        self.vol = np.ascontiguousarray(self.vol, dtype=np.float64)
        self.face_L = np.ascontiguousarray(self.face_L, dtype=np.int64)
        self.face_R = np.ascontiguousarray(self.face_R, dtype=np.int64)
        self.normal = np.ascontiguousarray(self.normal, dtype=np.float64).reshape(-1, 3)
        self.area = np.ascontiguousarray(self.area, dtype=np.float64)
        self.dL = np.ascontiguousarray(self.dL, dtype=np.float64).reshape(-1, 3)
        self.dR = np.ascontiguousarray(self.dR, dtype=np.float64).reshape(-1, 3)
        nc = self.vol.shape[0]
        # cell -> faces (CSR), faces of a cell in increasing face order
        owners = np.concatenate([self.face_L, self.face_R[self.face_R >= 0]])
        fidx = np.concatenate([np.arange(self.nfaces), np.nonzero(self.face_R >= 0)[0]])
        order = np.lexsort((fidx, owners))
        self.cf_idx = np.ascontiguousarray(fidx[order], dtype=np.int64)
        counts = np.bincount(owners, minlength=nc)
        self.cf_ptr = np.zeros(nc + 1, dtype=np.int64)
        np.cumsum(counts, out=self.cf_ptr[1:])

    @property
    def ncells(self) -> int:
        return int(self.vol.shape[0])

    @property
    def nfaces(self) -> int:
        return int(self.face_L.shape[0])

    def _struct(self) -> _Mesh:
        return _Mesh(self.dim, self.ncells, self.nfaces, _ptr(self.vol), _ptr(self.face_L),
                     _ptr(self.face_R), _ptr(self.normal), _ptr(self.area), _ptr(self.dL),
                     _ptr(self.dR), _ptr(self.cf_ptr), _ptr(self.cf_idx))


def cart2d(nx: int, ny: int, lo=(0.0, 0.0), hi=(1.0, 1.0), bc=(0, 0, 0, 0)) -> Mesh:
    """Uniform Cartesian grid; cell (ix, iy) has index ix + nx*iy.  bc = (x-, x+, y-, y+);
    a periodic direction needs both of its sides periodic."""
    return cart3d(nx, ny, 1, (lo[0], lo[1], 0.0), (hi[0], hi[1], 1.0), tuple(bc) + (None, None), dim=2)


def cart3d(nx: int, ny: int, nz: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(0,) * 6,
           dim: int = 3) -> Mesh:
    """Uniform Cartesian grid; cell (ix, iy, iz) has index ix + nx*(iy + ny*iz).
    bc = (x-, x+, y-, y+, z-, z+); for dim=2 the z sides are absent."""
    n = (nx, ny, nz)
    h = tuple((hi[d] - lo[d]) / n[d] for d in range(3))
    ncell = nx * ny * nz
    idx = np.arange(ncell).reshape(nz, ny, nx)
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    centroid = np.stack([lo[0] + (cx + 0.5) * h[0], lo[1] + (cy + 0.5) * h[1],
                         lo[2] + (cz + 0.5) * h[2]], axis=-1).reshape(-1, 3)
    vol = np.full(ncell, h[0] * h[1] * h[2])
    FL, FR, NRM, AR, DL, DR = [], [], [], [], [], []
    ndirs = 2 if dim == 2 else 3
    for d in range(ndirs):
        area = h[0] * h[1] * h[2] / h[d]
        e = np.zeros(3)
        e[d] = 1.0
        lo_bc, hi_bc = bc[2 * d], bc[2 * d + 1]
        periodic = lo_bc == BC_PERIODIC and hi_bc == BC_PERIODIC
        a = np.moveaxis(idx, 2 - d, 0)            # axis d first
        # interior faces between slices k and k+1
        L = a[:-1].reshape(-1)
        R = a[1:].reshape(-1)
        if periodic:
            L = np.concatenate([L, a[-1].reshape(-1)])
            R = np.concatenate([R, a[0].reshape(-1)])
        m = L.shape[0]
        FL.append(L); FR.append(R)
        NRM.append(np.tile(e, (m, 1))); AR.append(np.full(m, area))
        DL.append(np.tile(0.5 * h[d] * e, (m, 1))); DR.append(np.tile(-0.5 * h[d] * e, (m, 1)))
        if not periodic:
            for side, bcv, sl in ((-1, lo_bc, a[0]), (+1, hi_bc, a[-1])):
                if bcv == BC_PERIODIC:
                    raise ValueError("a periodic direction needs both sides periodic")
                L = sl.reshape(-1)
                m = L.shape[0]
                FL.append(L); FR.append(np.full(m, -(1 + bcv)))
                NRM.append(np.tile(side * e, (m, 1))); AR.append(np.full(m, area))
                DL.append(np.tile(0.5 * h[d] * side * e, (m, 1))); DR.append(np.zeros((m, 3)))
    mesh = Mesh(dim, vol, np.concatenate(FL), np.concatenate(FR), np.concatenate(NRM),
                np.concatenate(AR), np.concatenate(DL), np.concatenate(DR), centroid)
    mesh.shape = (nx, ny, nz)
    mesh.h = h
    return mesh


def cart_window(n, lo, hi, bc, w0, w1, dim) -> Mesh:
    """The sub-grid of cells w0 <= (ix, iy[, iz]) < w1 of a Cartesian grid with sides ``bc``.
    Sides of the window that are sides of the domain keep their boundary condition; cut sides
    get a non-reflecting boundary (values near a cut side are wrong and are not compared).
    A periodic direction whose window spans the full grid stays periodic."""
    h = [(hi[d] - lo[d]) / n[d] for d in range(3)]
    wlo = [lo[d] + w0[d] * h[d] for d in range(3)]
    whi = [lo[d] + w1[d] * h[d] for d in range(3)]
    wbc = []
    for d in range(dim):
        full = w0[d] == 0 and w1[d] == n[d]
        per = bc[2 * d] == BC_PERIODIC
        if per and full:
            wbc += [BC_PERIODIC, BC_PERIODIC]
            continue
        wbc.append(bc[2 * d] if (w0[d] == 0 and not per) else BC_NONREFLECT)
        wbc.append(bc[2 * d + 1] if (w1[d] == n[d] and not per) else BC_NONREFLECT)
    m = [w1[d] - w0[d] for d in range(3)]
    if dim == 2:
        return cart2d(m[0], m[1], wlo[:2], whi[:2], wbc)
    return cart3d(m[0], m[1], m[2], wlo, whi, wbc)


def tri_mesh(verts: np.ndarray, tris: np.ndarray, face_cells: np.ndarray, face_verts: np.ndarray) -> Mesh:
    """Triangle mesh: geometry computed here from the vertices.
    face_cells[s] = (owner, neighbour or -(1+bc)); the normal points owner -> neighbour."""
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int64)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    vol = 0.5 * np.abs(area2)
    cen2 = (a + b + c) / 3.0
    fc = np.asarray(face_cells, dtype=np.int64)
    fv = np.asarray(face_verts, dtype=np.int64)
    p, q = v[fv[:, 0]], v[fv[:, 1]]
    mid = 0.5 * (p + q)
    length = np.hypot(q[:, 0] - p[:, 0], q[:, 1] - p[:, 1])
    nrm = np.stack([(q[:, 1] - p[:, 1]) / length, -(q[:, 0] - p[:, 0]) / length], axis=1)
    L = fc[:, 0]
    # orient the normal away from the owner's centroid
    flip = np.einsum("ij,ij->i", nrm, mid - cen2[L]) < 0
    nrm[flip] *= -1.0
    R = fc[:, 1]
    dL = np.zeros((fc.shape[0], 3)); dR = np.zeros((fc.shape[0], 3))
    dL[:, :2] = mid - cen2[L]
    inner = R >= 0
    dR[inner, :2] = mid[inner] - cen2[R[inner]]
    n3 = np.zeros((fc.shape[0], 3)); n3[:, :2] = nrm
    cen = np.zeros((t.shape[0], 3)); cen[:, :2] = cen2
    return Mesh(2, vol, L, R, n3, length, dL, dR, cen)


def tet_mesh(verts: np.ndarray, tets: np.ndarray, face_cells: np.ndarray, face_verts: np.ndarray) -> Mesh:
    """Tetrahedral mesh: geometry computed here from the vertices (cell volumes and centroids,
    face areas, unit normals and centroids).  face_cells[s] = (owner, neighbour or -(1+bc));
    the normal points owner -> neighbour."""
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tets, dtype=np.int64)
    a, b, c, d = (v[t[:, k]] for k in range(4))
    vol = np.abs(np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a)) / 6.0
    cen = (a + b + c + d) / 4.0
    fc = np.asarray(face_cells, dtype=np.int64)
    fv = np.asarray(face_verts, dtype=np.int64)
    p, q, r = v[fv[:, 0]], v[fv[:, 1]], v[fv[:, 2]]
    cr = np.cross(q - p, r - p)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    mid = (p + q + r) / 3.0
    L, R = fc[:, 0], fc[:, 1]
    flip = np.einsum("ij,ij->i", nrm, mid - cen[L]) < 0
    nrm[flip] *= -1.0
    dL = mid - cen[L]
    dR = np.zeros_like(dL)
    inner = R >= 0
    dR[inner] = mid[inner] - cen[R[inner]]
    return Mesh(3, vol, L, R, nrm, area, dL, dR, cen)


# ----------------------------------------------------------------------------- the step
def step(mesh: Mesh, U: np.ndarray, dt: float, tau: float, c: float = 1.0, epsinv=None,
         muinv=None, J=None, C=None, gradient: int = GRAD_GREEN_GAUSS, limiter: int = LIMITER_NONE,
         chi: float = 0.0, gamma: float = 0.0) -> np.ndarray:
    """One explicit GKS step (Sec. 3.1).  U: (ncells, 6), or (ncells, 8) for the PHM system with
    couplings chi and gamma (Sec. 2.1).  J: (ncells, 3) current density or None.
    gradient: GRAD_GREEN_GAUSS (the paper's) or GRAD_LSQ (least squares over the face neighbours).
    limiter: LIMITER_MINMOD replaces the gradients by minmod-limited slopes (Cartesian meshes).
    Returns a state of the width given."""
    nc = mesh.ncells
    U, width = _widen(U, nc)
    if width == 6 and (chi != 0.0 or gamma != 0.0):
        raise ValueError("chi or gamma nonzero: pass the eight-component PHM state")
    out = np.empty_like(U)
    ei = np.ones(nc) if epsinv is None else np.ascontiguousarray(epsinv, dtype=np.float64)
    mi = np.ones(nc) if muinv is None else np.ascontiguousarray(muinv, dtype=np.float64)
    Jp = None
    if J is not None:
        Jp = np.ascontiguousarray(J, dtype=np.float64).reshape(nc, 3)
    prm = _Params(c, dt, (ctypes.c_double * 5)(*(C if C is not None else coefficients(dt, tau))), int(gradient),
                  int(limiter), float(chi), float(gamma))
    ms = mesh._struct()
    rc = lib().orc_step(ctypes.byref(ms), ctypes.byref(prm), _ptr(U), _ptr(out), _ptr(ei), _ptr(mi),
                        _ptr(Jp) if Jp is not None else None)
    if rc == -2:
        raise ValueError("the limiter needs a Cartesian mesh")
    if rc != 0:
        raise MemoryError("oracle step could not allocate its work arrays")
    return out if width == 8 else np.ascontiguousarray(out[:, :6])


def gaussian_pulse(t: float, J0: float, t0: float, sigma_t: float) -> float:
    """Amplitude J0 exp(-((t - t0)/sigma_t)^2) of the point source."""
    return J0 * math.exp(-((t - t0) / sigma_t) ** 2)


def run(mesh: Mesh, U: np.ndarray, nsteps: int, dt: float, tau: float, c: float = 1.0,
        epsinv=None, muinv=None, source=None, t0: float = 0.0, energy_every: int = 0,
        eps=None, mu=None, gradient: int = GRAD_GREEN_GAUSS, limiter: int = LIMITER_NONE,
        chi: float = 0.0, gamma: float = 0.0):
    """nsteps explicit steps from time t0; t^n = t0 + n dt.
    source: None or (cells, weights, J0, tc, sigma_t): J_z = weight * J0 exp(-((t^n-tc)/sigma_t)^2).
    Returns the final state (and the energy history when energy_every > 0)."""
    C = coefficients(dt, tau)
    hist = []
    for n in range(nsteps):
        tn = t0 + n * dt
        J = None
        if source is not None:
            cells, w, J0, tc, sg = source
            J = np.zeros((mesh.ncells, 3))
            J[np.asarray(cells), 2] = np.asarray(w) * gaussian_pulse(tn, J0, tc, sg)
        U = step(mesh, U, dt, tau, c, epsinv, muinv, J, C, gradient, limiter, chi, gamma)
        if energy_every and (n + 1) % energy_every == 0:
            hist.append(energy(mesh, U, eps, mu))
    return (U, hist) if energy_every else U


def energy(mesh: Mesh, U: np.ndarray, eps=None, mu=None) -> float:
    """W = 1/2 sum_i |Omega_i| (eps_i |E_i|^2 + mu_i |H_i|^2), plus 1/2 sum_i |Omega_i| (phi_i^2 +
    psi_i^2) for PHM states (the quadratic form the PHM system conserves in vacuum, c = 1)."""
    U, width = _widen(U, mesh.ncells)
    e = np.ones(mesh.ncells) if eps is None else np.asarray(eps)
    m = np.ones(mesh.ncells) if mu is None else np.asarray(mu)
    return float(0.5 * np.sum(mesh.vol * (e * np.sum(U[:, :3] ** 2, axis=1) + m * np.sum(U[:, 3:6] ** 2, axis=1)
                                          + np.sum(U[:, 6:] ** 2, axis=1))))


def gradients(mesh: Mesh, U: np.ndarray, gradient: int = GRAD_GREEN_GAUSS, limiter: int = LIMITER_NONE) -> np.ndarray:
    """Cell gradients (Green-Gauss, least squares, or minmod-limited slopes), shape
    (ncells, 3, width) for a state of width 6 or 8."""
    U, width = _widen(U, mesh.ncells)
    g = np.empty((mesh.ncells, 3, NC))
    ms = mesh._struct()
    if limiter:
        if lib().orc_gradients_limited(ctypes.byref(ms), _ptr(U), _ptr(g)) != 0:
            raise ValueError("the limiter needs a Cartesian mesh")
    else:
        fn = lib().orc_gradients_lsq if gradient == GRAD_LSQ else lib().orc_gradients
        fn(ctypes.byref(ms), _ptr(U), _ptr(g))
    return g if width == 8 else np.ascontiguousarray(g[:, :, :6])


# ----------------------------------------------------------------------------- unit-level access
def _pad(x, shape):
    a = np.zeros(shape)
    x = np.asarray(x, dtype=np.float64)
    a[..., :x.shape[-1]] = x
    return a


def face_flux(dim, dt, tau, Ul, Ur, dUl, dUr, minvE=1.0, minvH=1.0, c=1.0, C=None, chi=0.0, gamma=0.0) -> np.ndarray:
    """Local-frame interface flux (normal along local x) for the unit tests; states of width 6 or 8
    (slopes (3, width)), the flux returned with the same width."""
    width = np.asarray(Ul).shape[-1]
    prm = _Params(c, dt, (ctypes.c_double * 5)(*(C if C is not None else coefficients(dt, tau))), 0, 0,
                  float(chi), float(gamma))
    a = [_pad(Ul, NC), _pad(Ur, NC), _pad(dUl, (3, NC)), _pad(dUr, (3, NC))]
    F = np.empty(NC)
    lib().orc_face_flux(dim, ctypes.byref(prm), *[_ptr(x) for x in a], minvE, minvH, _ptr(F))
    return F[:width].copy()


def equilibrium(dim, V, c=1.0, chi=0.0, gamma=0.0) -> np.ndarray:
    """g_k(V), shape (4, width) for V of width 6 or 8."""
    width = np.asarray(V).shape[-1]
    g = np.empty((4, NC))
    V = _pad(V, NC)
    lib().orc_equilibrium(dim, c, float(chi), float(gamma), _ptr(V), _ptr(g))
    return g[:, :width].copy()


def lattice(dim, c=1.0) -> np.ndarray:
    u = np.empty((4, 3))
    lib().orc_lattice(dim, c, _ptr(u))
    return u


def rotation(n) -> np.ndarray:
    T = np.empty((3, 3))
    n = np.ascontiguousarray(n, dtype=np.float64)
    lib().orc_rotation(_ptr(n), _ptr(T))
    return T


# ----------------------------------------------------------------------------- layout helpers
def from_soa(fields: np.ndarray, model: str) -> np.ndarray:
    """SoA (nfields, ncells) -> oracle state; model 'tm2d' (Ez,Hx,Hy) or 'em3d' give (ncells, 6),
    'tm2d_phm' (Ez,Hx,Hy,psi) or 'em3d_phm' (all eight) give (ncells, 8)."""
    f = np.asarray(fields, dtype=np.float64)
    if model == "tm2d":
        U = np.zeros((f.shape[1], 6))
        U[:, list(TM)] = f.T
        return U
    if model == "tm2d_phm":
        U = np.zeros((f.shape[1], 8))
        U[:, list(TM_PHM)] = f.T
        return U
    return np.ascontiguousarray(f.T)


def to_soa(U: np.ndarray, model: str) -> np.ndarray:
    U = np.asarray(U)
    if model == "tm2d":
        return np.ascontiguousarray(U[:, list(TM)].T)
    if model == "tm2d_phm":
        return np.ascontiguousarray(U[:, list(TM_PHM)].T)
    return np.ascontiguousarray(U.T)
