"""ctypes binding of libgks (include/gks.h): argument marshalling only.

Every step of the GKS path runs in the HIP kernels of libgks.so; this module checks tensor
shapes, dtypes and devices, passes raw device pointers and the current HIP stream, and turns
error codes into exceptions.  PyTorch provides device memory and streams.  There is no CPU
fallback: if the library is missing the import of ``lib()`` fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libgks.so")

GKS_CART2D, GKS_CART3D, GKS_TRI2D, GKS_TET3D = 0, 1, 2, 3
GKS_TM2D, GKS_EM3D, GKS_TM2D_PHM, GKS_EM3D_PHM = 0, 1, 2, 3
BC = {"periodic": 0, "nonreflecting": 1, "pec": 2}
PRECISION = {"fp64": 0, "fp32": 1}
STATUS = {0: "GKS_OK", -1: "GKS_EINVAL", -2: "GKS_ENOMEM", -3: "GKS_EDEVICE", -4: "GKS_EUNSTABLE",
          -5: "GKS_ENONFINITE", -6: "GKS_ESTATE"}

# entry points declared in include/gks.h
EXPORTS = ("gks_init_mesh", "gks_destroy", "gks_last_error", "gks_get_dt", "gks_flux_coefficients",
           "gks_set_material", "gks_set_point_source", "gks_step", "gks_run", "gks_adjoint_step",
           "gks_energy", "gks_probe_energy", "gks_probe_energy_grad", "gks_adjoint_step_noalloc")


class GKSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("model", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("batch", ctypes.c_int64), ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int32 * 6), ("ncells", ctypes.c_int64),
                ("nfaces", ctypes.c_int64), ("nverts", ctypes.c_int64), ("vert_xy", ctypes.c_void_p),
                ("cell_verts", ctypes.c_void_p), ("face_cells", ctypes.c_void_p), ("face_verts", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("cfl", ctypes.c_double), ("dt", ctypes.c_double),
                ("tau_over_dt", ctypes.c_double), ("energy_every", ctypes.c_int32),
                ("unstable_growth", ctypes.c_double), ("gradient", ctypes.c_int32), ("limiter", ctypes.c_int32),
                ("chi", ctypes.c_double), ("gamma", ctypes.c_double)]


GRADIENT = {"green_gauss": 0, "lsq": 1}
LIMITER = {"none": 0, "minmod": 1}


_lib = None


def lib():
    """Loads libgks.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the process's HIP runtime first)
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is not built; run `python -m paper_2412_16845_amd.build`")
    L = ctypes.CDLL(LIBPATH)
    vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    sig = {
        "gks_init_mesh": [ctypes.POINTER(MeshDesc), ctypes.POINTER(Params), vp, ctypes.POINTER(vp)],
        "gks_destroy": [vp],
        "gks_get_dt": [vp, ctypes.POINTER(dbl)],
        "gks_flux_coefficients": [dbl, dbl, ctypes.POINTER(dbl)],
        "gks_set_material": [vp, vp, vp],
        "gks_set_point_source": [vp, i64, vp, vp, dbl, dbl, dbl],
        "gks_step": [vp, vp, vp, dbl],
        "gks_run": [vp, vp, i64, dbl, vp],
        "gks_adjoint_step": [vp, vp, vp, vp, vp, vp, dbl],
        "gks_adjoint_step_noalloc": [vp, vp, vp, vp, vp, vp, dbl],
        "gks_energy": [vp, vp, vp],
        "gks_probe_energy": [vp, vp, vp, vp],
        "gks_probe_energy_grad": [vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.gks_last_error.argtypes = [vp]
    L.gks_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def flux_coefficients(dt: float, tau: float):
    """C1..C5 of the time-integrated interface flux as the library computes them."""
    out = (ctypes.c_double * 5)()
    st = lib().gks_flux_coefficients(dt, tau, out)
    if st != 0:
        raise GKSError(st, "invalid dt or tau")
    return tuple(out)


def _ptr(t) -> int:
    return t.data_ptr()


class Solver:
    """A libgks context on one GPU.

    kind 'cart2d' (TM fields Ez, Hx, Hy on an nx x ny grid) or 'cart3d' (six fields on
    nx x ny x nz) or 'tri2d' (TM fields on a triangle mesh: pass ``tri=(verts, tris,
    face_cells, face_verts)``) or 'tet3d' (six fields on a tetrahedral mesh: pass
    ``tet=(verts (nv, 3), tets (nc, 4), face_cells (nf, 2), face_verts (nf, 3))``; each face is
    evaluated from its owner face_cells[s, 0]).  Field tensors have shape (batch, nfields, *grid) with
    grid = (ny, nx) / (nz, ny, nx) / (ncells,), contiguous, on the solver's device, dtype
    float64 ('fp64') or float32 ('fp32').  gradient: 'green_gauss' (the paper's) or 'lsq'
    (least squares; differs only on triangle meshes).  limiter: 'none' or 'minmod' (limited
    slopes for discontinuous data, Cartesian grids; the adjoint refuses a limited solver).
    phm: None, or (chi, gamma) for the perfectly hyperbolic Maxwell system: the fields become
    (Ez, Hx, Hy, psi) in 2D (Cartesian or triangles) and (Ex, Ey, Ez, Hx, Hy, Hz, phi, psi) in
    3D, with divergence errors of E and H carried off at chi c and gamma c.
    cfl: c dt / h (h the smallest cell width, or the smallest inradius on unstructured meshes),
    used when dt is 0.  The library refuses values above the step's stability limit: 0.5 on 2D
    grids and unstructured meshes, 1/3 on 3D grids, and with the PHM couplings nonzero 0.42 on
    2D grids and 0.3 on 3D grids.
    """

    def __init__(self, kind: str = "cart2d", n: Sequence[int] = (64, 64), lo=None, hi=None,
                 bc: Sequence[str] = ("periodic",) * 4, precision: str = "fp64", batch: int = 1,
                 c: float = 1.0, cfl: float = 0.5, dt: float = 0.0, tau_over_dt: float = 0.01,
                 energy_every: int = 0, unstable_growth: float = 0.0, device=None, tri=None, tet=None,
                 gradient: str = "green_gauss", limiter: str = "none", phm=None):
        import torch
        L = lib()
        self.torch = torch
        self._init = dict(kind=kind, n=n, lo=lo, hi=hi, bc=bc, precision=precision, batch=batch, c=c, cfl=cfl, dt=dt,
                          tau_over_dt=tau_over_dt, energy_every=energy_every, unstable_growth=unstable_growth,
                          device=device, tri=tri, tet=tet, gradient=gradient, limiter=limiter, phm=phm)
        self._source = None
        self._twin = None
        self.kind = kind
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.batch = int(batch)
        d = MeshDesc()
        d.precision = PRECISION[precision]
        d.batch = self.batch
        self._keep = []
        if kind in ("cart2d", "cart3d"):
            nd = 2 if kind == "cart2d" else 3
            d.kind = GKS_CART2D if nd == 2 else GKS_CART3D
            d.model = GKS_TM2D if nd == 2 else GKS_EM3D
            if phm is not None:
                d.model = GKS_TM2D_PHM if nd == 2 else GKS_EM3D_PHM
            n = list(n) + [1] * (3 - len(n))
            lo = list(lo) if lo is not None else [0.0] * nd
            hi = list(hi) if hi is not None else [1.0] * nd
            for i in range(3):
                d.n[i] = int(n[i])
                d.lo[i] = float(lo[i]) if i < nd else 0.0
                d.hi[i] = float(hi[i]) if i < nd else 1.0
            bcs = list(bc) + ["periodic"] * (6 - len(bc))
            for i in range(6):
                d.bc[i] = BC[bcs[i]] if isinstance(bcs[i], str) else int(bcs[i])
            self.nfields = (4 if phm is not None else 3) if nd == 2 else (8 if phm is not None else 6)
            self.grid = (int(n[1]), int(n[0])) if nd == 2 else (int(n[2]), int(n[1]), int(n[0]))
            self.n = tuple(int(v) for v in n[:nd])
        elif kind == "tri2d":
            verts, tris, face_cells, face_verts = tri
            verts = np.ascontiguousarray(verts, dtype=np.float64)
            tris = np.ascontiguousarray(tris, dtype=np.int32)
            face_cells = np.ascontiguousarray(face_cells, dtype=np.int32)
            face_verts = np.ascontiguousarray(face_verts, dtype=np.int32)
            self._keep += [verts, tris, face_cells, face_verts]
            d.kind, d.model = GKS_TRI2D, GKS_TM2D
            d.nverts, d.ncells, d.nfaces = verts.shape[0], tris.shape[0], face_cells.shape[0]
            d.vert_xy = verts.ctypes.data
            d.cell_verts = tris.ctypes.data
            d.face_cells = face_cells.ctypes.data
            d.face_verts = face_verts.ctypes.data
            self.nfields = 3
            self.grid = (int(tris.shape[0]),)
            if phm is not None:
                d.model = GKS_TM2D_PHM
                self.nfields = 4
        elif kind == "tet3d":
            verts, tets, face_cells, face_verts = tet
            verts = np.ascontiguousarray(verts, dtype=np.float64)
            tets = np.ascontiguousarray(tets, dtype=np.int32)
            face_cells = np.ascontiguousarray(face_cells, dtype=np.int32)
            face_verts = np.ascontiguousarray(face_verts, dtype=np.int32)
            if verts.ndim != 2 or verts.shape[1] != 3 or tets.shape[1:] != (4,) or face_verts.shape[1:] != (3,):
                raise ValueError("tet3d needs verts (nv, 3), tets (nc, 4) and face_verts (nf, 3)")
            self._keep += [verts, tets, face_cells, face_verts]
            d.kind, d.model = GKS_TET3D, GKS_EM3D
            d.nverts, d.ncells, d.nfaces = verts.shape[0], tets.shape[0], face_cells.shape[0]
            d.vert_xy = verts.ctypes.data
            d.cell_verts = tets.ctypes.data
            d.face_cells = face_cells.ctypes.data
            d.face_verts = face_verts.ctypes.data
            self.nfields = 6
            self.grid = (int(tets.shape[0]),)
        else:
            raise ValueError(f"unknown mesh kind {kind!r}")
        grad = GRADIENT[gradient] if isinstance(gradient, str) else int(gradient)
        lim = LIMITER[limiter] if isinstance(limiter, str) else int(limiter)
        chi, gamma = (0.0, 0.0) if phm is None else (float(phm[0]), float(phm[1]))
        self.phm = None if phm is None else (chi, gamma)
        p = Params(c, cfl, dt, tau_over_dt, energy_every, unstable_growth, grad, lim, chi, gamma)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            st = L.gks_init_mesh(ctypes.byref(d), ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h))
        if st != 0:
            raise GKSError(st, L.gks_last_error(None).decode())
        self._h = h
        self.energy_every = energy_every
        self._material = (None, None)
        dtv = ctypes.c_double()
        L.gks_get_dt(self._h, ctypes.byref(dtv))
        self.dt = dtv.value

    # ------------------------------------------------------------------ helpers
    def _check(self, st: int):
        if st != 0:
            raise GKSError(st, lib().gks_last_error(self._h).decode())

    @property
    def shape(self):
        return (self.batch, self.nfields) + self.grid

    def _state(self, t, name, dtype=None):
        dtype = dtype or self.dtype
        if t.dtype != dtype or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor on {self.device}")
        if tuple(t.shape) != self.shape:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {self.shape}")
        return t

    def _cellmap(self, t, name, dtype=None):
        dtype = dtype or self.dtype
        if t is None:
            return None
        if t.dtype != dtype or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor on {self.device}")
        if tuple(t.shape) != (self.batch,) + self.grid:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {(self.batch,) + self.grid}")
        return t

    def zeros(self):
        return self.torch.zeros(self.shape, dtype=self.dtype, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            lib().gks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ entry points
    def set_material(self, epsinv=None, muinv=None):
        """Per-cell 1/eps, 1/mu maps of shape (batch, *grid); None = vacuum.  Kept alive here."""
        e = self._cellmap(epsinv, "epsinv")
        m = self._cellmap(muinv, "muinv")
        self._material = (e, m)
        self._check(lib().gks_set_material(self._h, _ptr(e) if e is not None else None,
                                           _ptr(m) if m is not None else None))

    def set_point_source(self, cells, weights, J0: float, t0: float, sigma_t: float):
        c = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1)
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
        if c.shape != w.shape:
            raise ValueError("cells and weights differ in length")
        self._check(lib().gks_set_point_source(self._h, c.shape[0], c.ctypes.data if c.size else None,
                                               w.ctypes.data if w.size else None, J0, t0, sigma_t))
        self._source = (c, w, J0, t0, sigma_t)
        if self._twin is not None:
            self._twin.set_point_source(*self._source)

    def twin(self):
        """A second solver of the same mesh, parameters, materials and source, bound to a stream of
        its own (made once and kept): its launches run concurrently with this solver's.  The
        caller orders the two streams (events) where one reads what the other writes."""
        if self._twin is None:
            side = self.torch.cuda.Stream(self.device)
            with self.torch.cuda.device(self.device), self.torch.cuda.stream(side):
                t = Solver(**self._init)
            if self._source is not None:
                t.set_point_source(*self._source)
            self._twin = t
        self._twin.set_material(*self._material)
        return self._twin

    def step(self, U, out=None, t: float = 0.0):
        self._state(U, "U")
        if out is None:
            out = self.torch.empty_like(U)
        self._state(out, "out")
        self._check(lib().gks_step(self._h, _ptr(U), _ptr(out), float(t)))
        return out

    def run(self, U, nsteps: int, t0: float = 0.0, energy: bool = False):
        """nsteps steps in place; returns the energy history (nsteps // energy_every, batch) when asked."""
        self._state(U, "U")
        rec = None
        if energy and self.energy_every > 0:
            rec = np.zeros((nsteps // self.energy_every, self.batch), dtype=np.float64)
        self._check(lib().gks_run(self._h, _ptr(U), int(nsteps), float(t0),
                                  rec.ctypes.data if rec is not None and rec.size else None))
        return rec

    def adjoint_step(self, U_n, lam_np1, lam_n=None, g_epsinv=None, g_muinv=None, t: float = 0.0):
        self._state(U_n, "U_n")
        self._state(lam_np1, "lam_np1")
        if lam_n is None:
            lam_n = self.torch.empty_like(lam_np1)
        self._state(lam_n, "lam_n")
        ge = self._cellmap(g_epsinv, "g_epsinv", self.torch.float64)
        gm = self._cellmap(g_muinv, "g_muinv", self.torch.float64)
        self._check(lib().gks_adjoint_step(self._h, _ptr(U_n), _ptr(lam_np1), _ptr(lam_n),
                                           _ptr(ge) if ge is not None else None,
                                           _ptr(gm) if gm is not None else None, float(t)))
        return lam_n

    def adjoint_step_noalloc(self, U_n, lam_np1, lam_n, g_epsinv=None, g_muinv=None, t: float = 0.0):
        """adjoint_step through gks_adjoint_step_noalloc (the library's static scratch, no device
        allocation in the call): every output buffer is passed in."""
        self._state(U_n, "U_n")
        self._state(lam_np1, "lam_np1")
        self._state(lam_n, "lam_n")
        ge = self._cellmap(g_epsinv, "g_epsinv", self.torch.float64)
        gm = self._cellmap(g_muinv, "g_muinv", self.torch.float64)
        self._check(lib().gks_adjoint_step_noalloc(self._h, _ptr(U_n), _ptr(lam_np1), _ptr(lam_n),
                                                   _ptr(ge) if ge is not None else None,
                                                   _ptr(gm) if gm is not None else None, float(t)))
        return lam_n

    def energy(self, U) -> np.ndarray:
        self._state(U, "U")
        out = np.zeros(self.batch)
        self._check(lib().gks_energy(self._h, _ptr(U), out.ctypes.data))
        return out

    def probe_energy(self, U, box) -> np.ndarray:
        self._state(U, "U")
        b = np.ascontiguousarray(list(box) + [0, 1] * ((6 - len(box)) // 2), dtype=np.int64)
        out = np.zeros(self.batch)
        self._check(lib().gks_probe_energy(self._h, _ptr(U), b.ctypes.data, out.ctypes.data))
        return out

    def probe_energy_grad(self, U, box, lam=None):
        self._state(U, "U")
        if lam is None:
            lam = self.torch.empty_like(U)
        self._state(lam, "lam")
        b = np.ascontiguousarray(list(box) + [0, 1] * ((6 - len(box)) // 2), dtype=np.int64)
        self._check(lib().gks_probe_energy_grad(self._h, _ptr(U), b.ctypes.data, _ptr(lam)))
        return lam
