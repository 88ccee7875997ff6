"""Seeded synthetic inputs for the GKS workloads (shared by the tests, the benchmark and the
oracle checks).  Pure NumPy; none of the scheme's arithmetic lives here.

All arrays are float64, structure-of-arrays: fields (batch, nfields, *grid) with grid =
(ny, nx) or (nz, ny, nx), material maps (batch, *grid).  Random draws use
numpy.random.default_rng(seed).

Workloads (names used across the repository):
  tm_gaussian_periodic  2D TM, periodic unit square, vacuum, periodic Gaussian Ez pulse
  tm_dielectric_nr      2D TM, non-reflecting sides, circular dielectric inclusions, Gaussian
                        point current source (and optionally an initial Gaussian pulse)
  em_blocks_pec         3D six-component, random dielectric blocks, PEC z walls, non-reflecting
                        x/y sides, Ez pulse uniform in z
  tm_batch_probe        2D TM batch of dielectric maps with a probe box (differentiable workload)
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PERIODIC, NONREFLECT, PEC = "periodic", "nonreflecting", "pec"


@dataclass
class Workload:
    name: str
    kind: str                       # 'cart2d' | 'cart3d' | 'tri2d'
    n: tuple                        # cells per axis (x, y[, z]) or (ncells,)
    lo: tuple
    hi: tuple
    bc: tuple                       # per side, x-, x+, y-, y+[, z-, z+]
    U0: np.ndarray                  # (batch, nfields, *grid)
    epsinv: Optional[np.ndarray]    # (batch, *grid) or None
    muinv: Optional[np.ndarray]
    cfl: float
    tau_over_dt: float
    nsteps: int
    source: Optional[dict] = None   # cells, weights, J0, t0, sigma_t
    probe: Optional[tuple] = None   # (i0, i1, j0, j1) cell box
    extra: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return int(self.U0.shape[0])

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n))


def centres_2d(nx, ny, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    """Cell-centre coordinates, arrays of shape (ny, nx)."""
    x = lo[0] + (np.arange(nx) + 0.5) * (hi[0] - lo[0]) / nx
    y = lo[1] + (np.arange(ny) + 0.5) * (hi[1] - lo[1]) / ny
    return np.meshgrid(x, y, indexing="xy")


def centres_3d(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Cell-centre coordinates, arrays of shape (nz, ny, nx)."""
    ax = [lo[d] + (np.arange(m) + 0.5) * (hi[d] - lo[d]) / m for d, m in enumerate((nx, ny, nz))]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return x, y, z


def gaussian(x, y, xc, yc, w, periodic=False):
    """exp(-|x - x_c|^2 / (2 w^2)); with periodic=True summed over the 3 x 3 unit-square images."""
    if not periodic:
        return np.exp(-((x - xc) ** 2 + (y - yc) ** 2) / (2 * w * w))
    out = np.zeros_like(x)
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            out += np.exp(-((x - xc - sx) ** 2 + (y - yc - sy) ** 2) / (2 * w * w))
    return out


def circles_eps(x, y, rng, count, r_range, eps_range):
    """Background eps = 1 with `count` discs painted in order at the cell centres."""
    eps = np.ones_like(x)
    cx = rng.uniform(0.05, 0.95, count)
    cy = rng.uniform(0.05, 0.95, count)
    r = rng.uniform(r_range[0], r_range[1], count)
    ev = rng.uniform(eps_range[0], eps_range[1], count)
    for i in range(count):
        eps[(x - cx[i]) ** 2 + (y - cy[i]) ** 2 <= r[i] ** 2] = ev[i]
    return eps


def boxes_eps(ax, ay, az, rng, count, side_range, eps_range):
    """Background eps = 1 with `count` axis-aligned boxes inside the unit cube, painted in order
    on the cells whose centre lies in the box.  ax, ay, az: 1D cell-centre coordinates; returns
    an array of shape (len(az), len(ay), len(ax))."""
    eps = np.ones((len(az), len(ay), len(ax)))
    for _ in range(count):
        s = rng.uniform(side_range[0], side_range[1], 3)
        a = rng.uniform(0.0, 1.0 - s)
        e = rng.uniform(eps_range[0], eps_range[1])
        ix = np.nonzero((ax >= a[0]) & (ax < a[0] + s[0]))[0]
        iy = np.nonzero((ay >= a[1]) & (ay < a[1] + s[1]))[0]
        iz = np.nonzero((az >= a[2]) & (az < a[2] + s[2]))[0]
        eps[np.ix_(iz, iy, ix)] = e
    return eps


def cell_containing(nx, ny, p, lo=(0.0, 0.0), hi=(1.0, 1.0)) -> int:
    ix = min(int((p[0] - lo[0]) / (hi[0] - lo[0]) * nx), nx - 1)
    iy = min(int((p[1] - lo[1]) / (hi[1] - lo[1]) * ny), ny - 1)
    return iy * nx + ix


# ----------------------------------------------------------------------------- workloads
def tm_gaussian_periodic(n=64, seed=0, nsteps=200, cfl=0.5, tau_over_dt=0.01, w=0.05) -> Workload:
    rng = np.random.default_rng(seed)
    xc, yc = rng.uniform(0.25, 0.75, 2)
    x, y = centres_2d(n, n)
    U = np.zeros((1, 3, n, n))
    U[0, 0] = gaussian(x, y, xc, yc, w, periodic=True)
    return Workload("tm_gaussian_periodic", "cart2d", (n, n), (0.0, 0.0), (1.0, 1.0), (PERIODIC,) * 4, U,
                    None, None, cfl, tau_over_dt, nsteps, extra={"centre": (xc, yc), "w": w})


def tm_dielectric_nr(nx=4096, ny=None, seed=0, nsteps=1000, cfl=0.5, tau_over_dt=0.01, ncircles=64,
                     pulse: Optional[float] = None, bc=(NONREFLECT,) * 4) -> Workload:
    """Non-reflecting box with circular inclusions (radii in [0.01, 0.04], eps in [1, 4]) and a
    Gaussian point source J_z = exp(-((t - 0.02)/0.005)^2) in the cell holding (0.5, 0.5).
    pulse: optional amplitude of an initial Ez Gaussian (w = 0.05 at (0.35, 0.6))."""
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    x, y = centres_2d(nx, ny)
    eps = circles_eps(x, y, rng, ncircles, (0.01, 0.04), (1.0, 4.0))
    U = np.zeros((1, 3, ny, nx))
    if pulse:
        U[0, 0] = pulse * gaussian(x, y, 0.35, 0.6, 0.05)
    src = {"cells": [cell_containing(nx, ny, (0.5, 0.5))], "weights": [1.0], "J0": 1.0, "t0": 0.02,
           "sigma_t": 0.005}
    return Workload("tm_dielectric_nr", "cart2d", (nx, ny), (0.0, 0.0), (1.0, 1.0), tuple(bc), U,
                    (1.0 / eps)[None], None, cfl, tau_over_dt, nsteps, source=src)


def tm_phm_dielectric_nr(nx=4096, ny=None, seed=0, nsteps=1000, cfl=0.4, tau_over_dt=0.01, ncircles=64,
                         chi=0.0, gamma=1.0, hbump=0.5, pulse: Optional[float] = 1.0, bc=(NONREFLECT,) * 4) -> Workload:
    """The dielectric workload of tm_dielectric_nr carried by the PHM fields (Ez, Hx, Hy, psi):
    the same inclusions, point source and initial Ez pulse, plus a divergence error to clean,
    an Hx Gaussian bump of amplitude hbump (w = 0.05 at (0.65, 0.35)), and psi = 0.  The PHM
    couplings (chi, gamma) travel in extra["phm"].  CFL 0.4: with the psi coupling the 2D step
    is stable up to 0.42 only (at 0.5 and gamma = 1 a Fourier mode gains 11% per step)."""
    base = tm_dielectric_nr(nx, ny, seed, nsteps, cfl, tau_over_dt, ncircles, pulse, bc)
    ny = base.n[1]
    x, y = centres_2d(nx, ny)
    U = np.zeros((1, 4, ny, nx))
    U[:, :3] = base.U0
    U[0, 1] += hbump * gaussian(x, y, 0.65, 0.35, 0.05)
    return Workload("tm_phm_dielectric_nr", "cart2d", base.n, base.lo, base.hi, base.bc, U, base.epsinv, None, cfl,
                    tau_over_dt, nsteps, source=base.source, extra={"phm": (float(chi), float(gamma))})


def em_blocks_pec(n=384, seed=0, nsteps=500, cfl=1.0 / 3.0, tau_over_dt=0.01, nboxes=32, w=0.05) -> Workload:
    """384^3 style 3D workload: dielectric blocks (sides in [0.05, 0.25], eps in [1, 6]), PEC on
    z = 0, 1, non-reflecting x, y sides; Ez = Gaussian in (x, y), uniform in z; H = 0."""
    nx = ny = nz = n if np.isscalar(n) else None
    if not np.isscalar(n):
        nx, ny, nz = n
    rng = np.random.default_rng(seed)
    ax, ay, az = ((np.arange(m) + 0.5) / m for m in (nx, ny, nz))
    eps = boxes_eps(ax, ay, az, rng, nboxes, (0.05, 0.25), (1.0, 6.0))
    xc, yc = rng.uniform(0.3, 0.7, 2)
    x, y = np.meshgrid(ax, ay, indexing="xy")
    U = np.zeros((1, 6, nz, ny, nx))
    U[0, 2] = np.exp(-((x - xc) ** 2 + (y - yc) ** 2) / (2 * w * w))[None]
    bc = (NONREFLECT, NONREFLECT, NONREFLECT, NONREFLECT, PEC, PEC)
    return Workload("em_blocks_pec", "cart3d", (nx, ny, nz), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), bc, U,
                    (1.0 / eps)[None], None, cfl, tau_over_dt, nsteps)


def em_phm_blocks_pec(n=384, seed=0, nsteps=500, cfl=0.3, tau_over_dt=0.01, nboxes=32, w=0.05, chi=1.0,
                      gamma=1.0, bump=0.5, bc=None) -> Workload:
    """The 3D workload of em_blocks_pec carried by the PHM fields (Ex, Ey, Ez, Hx, Hy, Hz, phi,
    psi), plus divergence errors to clean: an Ex and an Hy Gaussian bump of amplitude `bump`
    (w = 0.05 at (0.3, 0.6, 0.5) and (0.65, 0.35, 0.4)); phi = psi = 0.  The couplings travel in
    extra["phm"].  CFL 0.3: with the potentials coupled the 3D step is stable up to 0.30 only
    (at 1/3 and chi = gamma = 1 a Fourier mode gains 2.6% per step)."""
    base = em_blocks_pec(n, seed, nsteps, cfl, tau_over_dt, nboxes, w)
    nx, ny, nz = base.n
    x, y, z = np.meshgrid(*((np.arange(m) + 0.5) / m for m in (nx, ny, nz)), indexing="ij")
    g = lambda c: np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * 0.05 ** 2)).transpose(2, 1, 0)
    U = np.zeros((1, 8, nz, ny, nx))
    U[:, :6] = base.U0
    U[0, 0] += bump * g((0.3, 0.6, 0.5))
    U[0, 4] += bump * g((0.65, 0.35, 0.4))
    return Workload("em_phm_blocks_pec", "cart3d", base.n, base.lo, base.hi, base.bc if bc is None else tuple(bc), U,
                    base.epsinv, None, cfl, tau_over_dt, nsteps, extra={"phm": (float(chi), float(gamma))})


def tm_batch_probe(n=1024, batch=8, seed=0, nsteps=800, cfl=0.5, tau_over_dt=0.01, ncircles=16,
                   w=0.05) -> Workload:
    """Batch of dielectric maps (16 discs, radii [0.03, 0.1], eps [1, 4]); Ez Gaussian at
    (0.3, 0.5); probe box [0.55, 0.65] x [0.45, 0.55]; non-reflecting sides."""
    rng = np.random.default_rng(seed)
    x, y = centres_2d(n, n)
    eps = np.stack([circles_eps(x, y, rng, ncircles, (0.03, 0.1), (1.0, 4.0)) for _ in range(batch)])
    U = np.zeros((batch, 3, n, n))
    U[:, 0] = gaussian(x, y, 0.3, 0.5, w)[None]
    box = (int(0.55 * n), int(0.65 * n), int(0.45 * n), int(0.55 * n))
    return Workload("tm_batch_probe", "cart2d", (n, n), (0.0, 0.0), (1.0, 1.0), (NONREFLECT,) * 4, U,
                    1.0 / eps, None, cfl, tau_over_dt, nsteps, probe=box)


def random_smooth_tm(nx, ny, seed, modes=4, batch=1):
    """Sum of a few random Fourier modes per field (for symmetry and parity tests)."""
    rng = np.random.default_rng(seed)
    x, y = centres_2d(nx, ny)
    U = np.zeros((batch, 3, ny, nx))
    for b in range(batch):
        for f in range(3):
            for _ in range(modes):
                kx, ky = rng.integers(-3, 4, size=2)
                U[b, f] += rng.normal() * np.cos(2 * np.pi * (kx * x + ky * y) + rng.uniform(0, 2 * np.pi))
    return U


# ----------------------------------------------------------------------------- triangle meshes
def _hilbert_index(x, y, order=16):
    """Index along a Hilbert curve of points in [0, 1)^2 (order bits per axis), vectorised."""
    n = 1 << order
    xi = np.clip((x * n).astype(np.int64), 0, n - 1)
    yi = np.clip((y * n).astype(np.int64), 0, n - 1)
    d = np.zeros_like(xi)
    s = n >> 1
    while s > 0:
        rx = ((xi & s) > 0).astype(np.int64)
        ry = ((yi & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        # rotate the quadrant
        flip = ry == 0
        swap_x = flip & (rx == 1)
        xi = np.where(swap_x, s - 1 - xi, xi)
        yi = np.where(swap_x, s - 1 - yi, yi)
        xi, yi = np.where(flip, yi, xi), np.where(flip, xi, yi)
        s >>= 1
    return d


def _ellipse_points(centre, axes, h):
    """Points on the ellipse at arc-length spacing close to h (counter-clockwise)."""
    t = np.linspace(0.0, 2 * np.pi, 20001)
    x = centre[0] + axes[0] * np.cos(t)
    y = centre[1] + axes[1] * np.sin(t)
    s = np.concatenate([[0.0], np.cumsum(np.hypot(np.diff(x), np.diff(y)))])
    m = max(8, int(round(s[-1] / h)))
    tt = np.interp(np.arange(m) * s[-1] / m, s, t)
    return np.stack([centre[0] + axes[0] * np.cos(tt), centre[1] + axes[1] * np.sin(tt)], axis=1)


def tri_ellipse_mesh(h, seed=0, centre=(0.5, 0.5), axes=(0.2, 0.1), cache=True):
    """Cached form of _tri_ellipse_mesh (see there): large meshes take tens of seconds to
    triangulate, so they are kept in the temporary directory (or GKS_MESH_CACHE), keyed by the
    arguments and by this module's source."""
    import hashlib
    import os
    import tempfile
    if not cache:
        return _tri_ellipse_mesh(h, seed, centre, axes)
    with open(__file__, "rb") as f:
        tag = hashlib.sha256(f.read() + repr((h, seed, centre, axes)).encode()).hexdigest()[:20]
    d = os.environ.get("GKS_MESH_CACHE") or tempfile.gettempdir()
    path = os.path.join(d, f"gks_tri_{tag}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return z["verts"], z["tris"], z["face_cells"], z["face_verts"]
    out = _tri_ellipse_mesh(h, seed, centre, axes)
    try:
        tmp = path + f".{os.getpid()}.npz"
        np.savez(tmp, verts=out[0], tris=out[1], face_cells=out[2], face_verts=out[3])
        os.replace(tmp, path)
    except OSError:
        pass
    return out


def _tri_ellipse_mesh(h, seed=0, centre=(0.5, 0.5), axes=(0.2, 0.1)):
    """Triangle mesh of the unit square minus an elliptical hole.

    Jittered lattice (spacing h, jitter U[-h/4, h/4]^2) without the points closer than h/2 to
    the square's sides or to the ellipse (or inside it), plus boundary points at spacing h on
    the square and the ellipse; Delaunay triangulation; triangles whose centroid lies inside the
    ellipse dropped; cells in Hilbert order of their centroids.  Edges on the square are
    non-reflecting, edges on the ellipse PEC.
    Returns (verts (nv, 2), tris (nc, 3), face_cells (nf, 2), face_verts (nf, 2)) with
    face_cells[s] = (owner, neighbour or -(1 + bc))."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    n = int(round(1.0 / h))
    hh = 1.0 / n
    g = (np.arange(n) + 0.5) * hh
    X, Y = np.meshgrid(g, g, indexing="xy")
    P = np.stack([X.ravel(), Y.ravel()], axis=1) + rng.uniform(-0.25 * hh, 0.25 * hh, (n * n, 2))
    # exclusion bands
    keep = (P[:, 0] > 0.5 * hh) & (P[:, 0] < 1 - 0.5 * hh) & (P[:, 1] > 0.5 * hh) & (P[:, 1] < 1 - 0.5 * hh)
    E = _ellipse_points(centre, axes, hh)
    # distance to the ellipse, approximated by the distance to its dense polygon
    from scipy.spatial import cKDTree
    dense = _ellipse_points(centre, axes, hh / 16)
    dist, _ = cKDTree(dense).query(P, distance_upper_bound=0.5 * hh, workers=-1)
    inside = ((P[:, 0] - centre[0]) / axes[0]) ** 2 + ((P[:, 1] - centre[1]) / axes[1]) ** 2 < 1.0
    keep &= (dist > 0.5 * hh) & ~inside
    P = P[keep]
    side = np.arange(n + 1) * hh
    B = np.concatenate([np.stack([side, np.zeros_like(side)], 1), np.stack([side, np.ones_like(side)], 1),
                        np.stack([np.zeros_like(side[1:-1]), side[1:-1]], 1),
                        np.stack([np.ones_like(side[1:-1]), side[1:-1]], 1)])
    verts = np.concatenate([B, E, P])
    ne0 = B.shape[0]
    tri = Delaunay(verts).simplices.astype(np.int64)
    cen = verts[tri].mean(axis=1)
    inside = ((cen[:, 0] - centre[0]) / axes[0]) ** 2 + ((cen[:, 1] - centre[1]) / axes[1]) ** 2 < 1.0
    tri = tri[~inside]
    # counter-clockwise orientation
    a, b, c = verts[tri[:, 0]], verts[tri[:, 1]], verts[tri[:, 2]]
    cw = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]) < 0
    tri[cw] = tri[cw][:, [0, 2, 1]]
    # Hilbert order of the cells
    cen = verts[tri].mean(axis=1)
    tri = tri[np.argsort(_hilbert_index(cen[:, 0], cen[:, 1]), kind="stable")]
    # unique edges and their cells
    nc = tri.shape[0]
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    cell = np.tile(np.arange(nc), 3)
    e.sort(axis=1)
    key = e[:, 0] * verts.shape[0] + e[:, 1]
    order = np.argsort(key, kind="stable")
    key, cell, e = key[order], cell[order], e[order]
    first = np.concatenate([[True], key[1:] != key[:-1]])
    starts = np.nonzero(first)[0]
    counts = np.diff(np.concatenate([starts, [key.shape[0]]]))
    assert counts.max() <= 2, "an edge is shared by more than two triangles"
    face_verts = e[starts]
    owner = cell[starts]
    nb = np.where(counts == 2, cell[np.minimum(starts + 1, key.shape[0] - 1)], -1)
    # boundary edges: on the ellipse (both ends ellipse points) PEC, otherwise non-reflecting
    on_e = (face_verts >= ne0) & (face_verts < ne0 + E.shape[0])
    bnd = nb < 0
    pec = bnd & on_e.all(axis=1)
    nb = np.where(pec, -(1 + 2), np.where(bnd, -(1 + 1), nb))
    # every ellipse polygon edge is a mesh edge (the hole is resolved exactly by the mesh)
    m = E.shape[0]
    ring = np.stack([ne0 + np.arange(m), ne0 + (np.arange(m) + 1) % m], 1)
    ring.sort(axis=1)
    have = set((face_verts[pec, 0] * verts.shape[0] + face_verts[pec, 1]).tolist())
    assert all(int(r0) * verts.shape[0] + int(r1) in have for r0, r1 in ring), "ellipse edge missing from the mesh"
    face_cells = np.stack([owner, nb], axis=1)
    return verts, tri, face_cells, face_verts


def _morton3(q):
    """Morton (Z-order) key of integer coordinates q (n, 3), 10 bits each."""
    key = np.zeros(q.shape[0], dtype=np.int64)
    for bit in range(10):
        for d in range(3):
            key |= ((q[:, d] >> bit) & 1).astype(np.int64) << (3 * bit + d)
    return key


def tet_box_mesh(n, seed=0, jitter=0.15, sphere=None, bc=(NONREFLECT,) * 6):
    """Tetrahedral mesh of the unit cube: n^3 cubes (n = (nx, ny, nz) or one int), each split
    into the six tetrahedra around its main diagonal (a conforming subdivision), vertices
    jittered by U[-jitter h, jitter h] (boundary vertices only along their side, edges and
    corners not at all).  sphere = (centre, radius): tetrahedra with centroid inside are removed
    and the faces left open become PEC walls.  bc: the box sides x-, x+, y-, y+, z-, z+
    (non-reflecting or PEC).  Cells in Morton order of their centroids.
    Returns verts (nv, 3), tets (nc, 4), face_cells (nf, 2) = (owner, neighbour or -(1 + bc)) with
    the owner the lower cell index, face_verts (nf, 3)."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    rng = np.random.default_rng(seed)
    gi, gj, gk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    vid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k
    g = np.stack([gi.ravel(), gj.ravel(), gk.ravel()], axis=1)
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    verts = g * h
    top = np.array([nx, ny, nz])
    free = (g > 0) & (g < top)                     # a coordinate may move only off its side planes
    verts = verts + free * rng.uniform(-jitter, jitter, verts.shape) * h
    ci, cj, ck = (a.ravel() for a in np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"))
    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        p0 = np.stack([ci, cj, ck], axis=1)
        path = [p0]
        cur = p0.copy()
        for d in perm:
            cur = cur.copy()
            cur[:, d] += 1
            path.append(cur)
        tets.append(np.stack([vid(q[:, 0], q[:, 1], q[:, 2]) for q in path], axis=1))
    tets = np.concatenate(tets)
    cen = verts[tets].mean(axis=1)
    if sphere is not None:
        (cx, cy, cz), rad = sphere
        keep = (cen[:, 0] - cx) ** 2 + (cen[:, 1] - cy) ** 2 + (cen[:, 2] - cz) ** 2 >= rad * rad
        tets, cen = tets[keep], cen[keep]
    order = np.argsort(_morton3(np.minimum((cen * 1024).astype(np.int64), 1023)), kind="stable")
    tets, cen = tets[order], cen[order]
    nc = tets.shape[0]
    # faces: the four vertex triples of every tetrahedron, matched by their sorted vertex ids
    tri = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    owner = np.tile(np.arange(nc), 4)
    st = np.sort(tri, axis=1).astype(np.int64)
    assert verts.shape[0] < (1 << 21)
    key = (st[:, 0] << 42) | (st[:, 1] << 21) | st[:, 2]
    uniq, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    nf = uniq.shape[0]
    order_f = np.argsort(inv, kind="stable")
    first = np.zeros(nf, dtype=np.int64)
    np.cumsum(cnt[:-1], out=first[1:])
    cA = owner[order_f[first]]
    cB = np.where(cnt == 2, owner[order_f[np.minimum(first + 1, len(order_f) - 1)]], -1)
    fv = tri[order_f[first]]
    L = np.where(cB >= 0, np.minimum(cA, cB), cA)
    Rn = np.where(cB >= 0, np.maximum(cA, cB), -1)
    # boundary faces: a box side if all three vertices lie on it, otherwise the sphere (PEC)
    bnd = Rn < 0
    P = verts[fv[bnd]]
    num = {NONREFLECT: 1, PEC: 2}                   # boundary codes of the face list
    code = np.full(int(bnd.sum()), -(1 + num[PEC]))
    for d in range(3):
        for side, val in ((0, 0.0), (1, 1.0)):
            on = np.all(np.abs(P[:, :, d] - val) < 1e-12, axis=1)
            code[on] = -(1 + num[bc[2 * d + side]])
    Rn[bnd] = code
    face_cells = np.stack([L, Rn], axis=1)
    fo = np.lexsort((Rn < 0, L))                   # faces ordered by owner
    return verts, tets.astype(np.int32), face_cells[fo].astype(np.int32), fv[fo].astype(np.int32)


def tet_sphere_mesh(n, seed=0, radius=0.15, cache=True):
    """tet_box_mesh with a PEC sphere of the given radius at the centre and non-reflecting box
    sides, cached like tri_ellipse_mesh (large meshes take tens of seconds)."""
    import hashlib
    import os
    import tempfile
    args = (n, seed, radius)
    make = lambda: tet_box_mesh(n, seed=seed, sphere=((0.5, 0.5, 0.5), radius))
    if not cache:
        return make()
    with open(__file__, "rb") as f:
        tag = hashlib.sha256(f.read() + repr(args).encode()).hexdigest()[:20]
    d = os.environ.get("GKS_MESH_CACHE") or tempfile.gettempdir()
    path = os.path.join(d, f"gks_tet_{tag}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return z["verts"], z["tets"], z["face_cells"], z["face_verts"]
    out = make()
    try:
        tmp = path + f".{os.getpid()}.npz"
        np.savez(tmp, verts=out[0], tets=out[1], face_cells=out[2], face_verts=out[3])
        os.replace(tmp, path)
    except OSError:
        pass
    return out


def tet_sphere_workload(n=64, seed=0, nsteps=200, cfl=0.5, tau_over_dt=0.01, w=0.05, radius=0.15) -> Workload:
    """Tetrahedral workload (the unstructured 3D meshes of Sec. 5.5, with a sphere standing in
    for the paper's aircraft, whose geometry is not available): the unit cube as n^3 jittered
    cubes of six tetrahedra, a PEC sphere of the given radius at the centre, non-reflecting box
    sides; Ez = Gaussian (w) in (x, y) centred at (0.3, 0.5), uniform in z (a pulse that runs
    into the sphere), H = 0.  The time step is cfl x the smallest inradius (set by the caller's
    solver)."""
    verts, tets, face_cells, face_verts = tet_sphere_mesh(n, seed, radius)
    cen = verts[tets].mean(axis=1)
    U = np.zeros((1, 6, tets.shape[0]))
    U[0, 2] = np.exp(-((cen[:, 0] - 0.3) ** 2 + (cen[:, 1] - 0.5) ** 2) / (2 * w * w))
    return Workload("tet_sphere", "tet3d", (tets.shape[0],), (0.0,) * 3, (1.0,) * 3, (NONREFLECT,) * 6, U, None, None,
                    cfl, tau_over_dt, nsteps,
                    extra={"verts": verts, "tets": tets, "face_cells": face_cells, "face_verts": face_verts})


def tri_ellipse_workload(h=6.8e-4, seed=0, nsteps=2000, cfl=0.5, tau_over_dt=0.01, w=0.05, eps_discs=0,
                         batch=1) -> Workload:
    """2D TM on the square with an elliptical PEC hole (non-reflecting outer square): Ez
    Gaussian (w = 0.05) centred at a seeded point at least 0.15 from the ellipse, H = 0.
    eps_discs > 0 adds that many dielectric discs (radii [0.02, 0.06], eps [1, 4])."""
    verts, tri, fc, fv = tri_ellipse_mesh(h, seed)
    rng = np.random.default_rng(seed + 1)
    cen = verts[tri].mean(axis=1)
    while True:
        xc, yc = rng.uniform(0.15, 0.85, 2)
        if ((xc - 0.5) / 0.35) ** 2 + ((yc - 0.5) / 0.25) ** 2 > 1.0:
            break
    U = np.zeros((batch, 3, tri.shape[0]))
    U[:, 0] = gaussian(cen[:, 0], cen[:, 1], xc, yc, w)[None]
    epsinv = None
    if eps_discs:
        eps = circles_eps(cen[:, 0], cen[:, 1], rng, eps_discs, (0.02, 0.06), (1.0, 4.0))
        epsinv = np.repeat((1.0 / eps)[None], batch, axis=0)
    return Workload("tri_ellipse", "tri2d", (tri.shape[0],), (0.0, 0.0), (1.0, 1.0), (NONREFLECT, PEC), U, epsinv,
                    None, cfl, tau_over_dt, nsteps,
                    extra={"verts": verts, "tris": tri, "face_cells": fc, "face_verts": fv, "centre": (xc, yc)})
