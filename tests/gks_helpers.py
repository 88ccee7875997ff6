"""Test helpers: run the FP64 oracle on the same seeded workloads as the GPU path, and compare.

Only the input generators (paper_2412_16845_amd.inputs) are shared between the two sides.
"""
from __future__ import annotations

import numpy as np

from oracle import gks_oracle as O
from paper_2412_16845_amd import inputs as I

BCODE = {I.PERIODIC: O.BC_PERIODIC, I.NONREFLECT: O.BC_NONREFLECT, I.PEC: O.BC_PEC}


def model_of(wl):
    if wl.kind in ("cart2d", "tri2d"):
        return "tm2d_phm" if wl.U0.shape[1] == 4 else "tm2d"
    return "em3d_phm" if wl.U0.shape[1] == 8 else "em3d"


def phm_of(wl):
    """(chi, gamma) of a PHM workload, (0, 0) otherwise."""
    return wl.extra.get("phm", (0.0, 0.0))


def oracle_mesh(wl):
    bc = [BCODE[b] for b in wl.bc]
    if wl.kind == "cart2d":
        return O.cart2d(wl.n[0], wl.n[1], wl.lo, wl.hi, bc)
    if wl.kind == "cart3d":
        return O.cart3d(wl.n[0], wl.n[1], wl.n[2], wl.lo, wl.hi, bc)
    raise ValueError(wl.kind)


def oracle_source(wl):
    if wl.source is None:
        return None
    s = wl.source
    return (np.asarray(s["cells"]), np.asarray(s["weights"], dtype=np.float64), s["J0"], s["t0"], s["sigma_t"])


def oracle_run(wl, nsteps, dt, b=0, U0=None, t0=0.0, mesh=None, limiter=0):
    """FP64 oracle run of batch item b; returns the SoA state (nfields, *grid)."""
    mesh = mesh or oracle_mesh(wl)
    model = model_of(wl)
    U0 = wl.U0 if U0 is None else U0
    nf = U0.shape[1]
    U = O.from_soa(np.asarray(U0[b], dtype=np.float64).reshape(nf, -1), model)
    ei = None if wl.epsinv is None else np.asarray(wl.epsinv[b], dtype=np.float64).reshape(-1)
    mi = None if wl.muinv is None else np.asarray(wl.muinv[b], dtype=np.float64).reshape(-1)
    chi, gamma = phm_of(wl)
    out = O.run(mesh, U, nsteps, dt, wl.tau_over_dt * dt, epsinv=ei, muinv=mi, source=oracle_source(wl), t0=t0,
                limiter=limiter, chi=chi, gamma=gamma)
    return O.to_soa(out, model).reshape(U0.shape[1:])


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def window_check_2d(wl, U_start, U_end, nsteps, dt, t0, centres, half=None, b=0):
    """Sampled check of a large 2D run: for each centre (ix, iy) the oracle advances a window of
    the start state by nsteps and returns (gpu, oracle) values on the window's trusted core
    (cells farther than 2*nsteps + 2 from a cut side)."""
    nx, ny = wl.n[0], wl.n[1]
    margin = 2 * nsteps + 2
    half = half or margin + 8
    bc = [BCODE[v] for v in wl.bc]
    gpu_vals, orc_vals = [], []
    for (cx, cy) in centres:
        x0, x1 = max(cx - half, 0), min(cx + half, nx)
        y0, y1 = max(cy - half, 0), min(cy + half, ny)
        mesh = O.cart_window((nx, ny, 1), (wl.lo[0], wl.lo[1], 0.0), (wl.hi[0], wl.hi[1], 1.0), bc,
                             (x0, y0, 0), (x1, y1, 1), 2)
        sub = np.asarray(U_start[b][:, y0:y1, x0:x1], dtype=np.float64)
        nf, model = sub.shape[0], model_of(wl)
        U = O.from_soa(sub.reshape(nf, -1), model)
        ei = None if wl.epsinv is None else np.ascontiguousarray(wl.epsinv[b][y0:y1, x0:x1]).reshape(-1)
        mi = None if wl.muinv is None else np.ascontiguousarray(wl.muinv[b][y0:y1, x0:x1]).reshape(-1)
        src = None
        if wl.source is not None:
            cells, wts = [], []
            for c, w in zip(wl.source["cells"], wl.source["weights"]):
                ix, iy = c % nx, c // nx
                if x0 <= ix < x1 and y0 <= iy < y1:
                    cells.append((iy - y0) * (x1 - x0) + (ix - x0))
                    wts.append(w)
            if cells:
                src = (np.array(cells), np.array(wts), wl.source["J0"], wl.source["t0"], wl.source["sigma_t"])
        chi, gamma = phm_of(wl)
        out = O.run(mesh, U, nsteps, dt, wl.tau_over_dt * dt, epsinv=ei, muinv=mi, source=src, t0=t0, chi=chi,
                    gamma=gamma)
        ref = O.to_soa(out, model).reshape(nf, y1 - y0, x1 - x0)
        # trusted core: away from cut sides (domain sides are exact)
        lx = 0 if x0 == 0 else margin
        hx = (x1 - x0) if x1 == nx else (x1 - x0) - margin
        ly = 0 if y0 == 0 else margin
        hy = (y1 - y0) if y1 == ny else (y1 - y0) - margin
        assert hx > lx and hy > ly, "window too small for the step count"
        orc_vals.append(ref[:, ly:hy, lx:hx].ravel())
        gpu_vals.append(np.asarray(U_end[b][:, y0 + ly:y0 + hy, x0 + lx:x0 + hx], dtype=np.float64).ravel())
    return np.concatenate(gpu_vals), np.concatenate(orc_vals)


def window_check_3d(wl, U_start, U_end, nsteps, dt, t0, centres, half=None, b=0):
    """The 3D form of window_check_2d: centres (ix, iy, iz); returns (gpu, oracle) values on
    the trusted cores of the windows."""
    n = wl.n
    margin = 2 * nsteps + 2
    half = half or margin + 4
    bc = [BCODE[v] for v in wl.bc]
    gpu_vals, orc_vals = [], []
    for c in centres:
        lo = [max(c[d] - half, 0) for d in range(3)]
        hi = [min(c[d] + half, n[d]) for d in range(3)]
        mesh = O.cart_window(tuple(n), tuple(wl.lo), tuple(wl.hi), bc, tuple(lo), tuple(hi), 3)
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        sub = np.asarray(U_start[b][(slice(None),) + sl], dtype=np.float64)
        nf, model = sub.shape[0], model_of(wl)
        U = O.from_soa(sub.reshape(nf, -1), model)
        ei = None if wl.epsinv is None else np.ascontiguousarray(wl.epsinv[b][sl], dtype=np.float64).reshape(-1)
        mi = None if wl.muinv is None else np.ascontiguousarray(wl.muinv[b][sl], dtype=np.float64).reshape(-1)
        chi, gamma = phm_of(wl)
        out = O.run(mesh, U, nsteps, dt, wl.tau_over_dt * dt, epsinv=ei, muinv=mi, t0=t0, chi=chi, gamma=gamma)
        m = [hi[d] - lo[d] for d in range(3)]
        ref = O.to_soa(out, model).reshape(nf, m[2], m[1], m[0])
        core = []
        for d in range(3):
            a = 0 if lo[d] == 0 else margin
            z = m[d] if hi[d] == n[d] else m[d] - margin
            assert z > a, "window too small for the step count"
            core.append((a, z))
        cs = (slice(None), slice(*core[2]), slice(*core[1]), slice(*core[0]))
        gs = (slice(None),) + tuple(slice(lo[d] + core[d][0], lo[d] + core[d][1]) for d in (2, 1, 0))
        orc_vals.append(ref[cs].ravel())
        gpu_vals.append(np.asarray(U_end[b][gs], dtype=np.float64).ravel())
    return np.concatenate(gpu_vals), np.concatenate(orc_vals)
