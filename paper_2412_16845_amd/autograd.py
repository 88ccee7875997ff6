"""Differentiable 2D GKS runs for PyTorch (reverse mode through the library's adjoint step).

``run(solver, U0, nsteps, epsinv=None, muinv=None, t0=0.0, checkpoint_every=50)`` returns the
state after ``nsteps`` steps and is differentiable with respect to U0, 1/eps and 1/mu:

  forward   gks_run in segments of ``checkpoint_every`` steps; the state at the start of every
            segment is kept (one state per segment instead of one per step);
  backward  segment by segment, the last first: the segment's states are recomputed from its
            checkpoint with gks_step, then gks_adjoint_step walks back through them, carrying
            the co-state lambda and accumulating the 1/eps, 1/mu gradients in double precision.

``probe_energy(solver, U, box)`` is the probe-box field energy sum |Omega| Ez^2 per batch item
(gks_probe_energy, with gks_probe_energy_grad as its derivative): the loss of the inverse
design workload.

Memory: checkpoints hold ceil(nsteps / K) states and the backward pass K more (K =
checkpoint_every), plus two co-states and the library's adjoint scratch (the ghost positions
around the grid only: about 4 (nx + ny) positions per batch item).
"""
from __future__ import annotations

import torch

from .gks import Solver

__all__ = ["run", "probe_energy", "GKSFunction", "GKSRun", "ProbeEnergy"]


class GKSRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, epsinv, muinv, solver: Solver, nsteps: int, t0: float, K: int):
        if K < 1:
            raise ValueError("checkpoint_every must be >= 1")
        solver.set_material(epsinv, muinv)
        U = U0.detach().clone()
        ckpts = []
        segs = []
        for k in range(0, nsteps, K):
            m = min(K, nsteps - k)
            ckpts.append(U.clone())
            segs.append((k, m))
            solver.run(U, m, t0 + k * solver.dt)
        ctx.solver = solver
        ctx.t0 = t0
        ctx.segs = segs
        ctx.ckpts = ckpts
        ctx.save_for_backward(epsinv if epsinv is not None else torch.empty(0),
                              muinv if muinv is not None else torch.empty(0))
        ctx.has = (epsinv is not None, muinv is not None)
        return U

    @staticmethod
    def backward(ctx, gU):
        s: Solver = ctx.solver
        e_saved, m_saved = ctx.saved_tensors
        epsinv = e_saved if ctx.has[0] else None
        muinv = m_saved if ctx.has[1] else None
        s.set_material(epsinv, muinv)
        want_e = ctx.needs_input_grad[1]
        want_m = ctx.needs_input_grad[2]
        cell_shape = (s.batch,) + s.grid
        ge = torch.zeros(cell_shape, dtype=torch.float64, device=s.device) if want_e else None
        gm = torch.zeros(cell_shape, dtype=torch.float64, device=s.device) if want_m else None
        lam = gU.to(s.dtype).contiguous().clone()
        nxt = torch.empty_like(lam)
        for (k, m), ck in zip(reversed(ctx.segs), reversed(ctx.ckpts)):
            states = [ck]
            for j in range(m - 1):
                states.append(s.step(states[-1], t=ctx.t0 + (k + j) * s.dt))
            for j in reversed(range(m)):
                s.adjoint_step(states[j], lam, nxt, ge, gm, t=ctx.t0 + (k + j) * s.dt)
                lam, nxt = nxt, lam
            del states
        ctx.ckpts = None
        g_e = ge.to(epsinv.dtype) if (want_e and epsinv is not None) else (ge if want_e else None)
        g_m = gm.to(muinv.dtype) if (want_m and muinv is not None) else (gm if want_m else None)
        return lam, g_e, g_m, None, None, None, None


class ProbeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, solver: Solver, box):
        ctx.solver = solver
        ctx.box = tuple(int(v) for v in box)
        ctx.save_for_backward(U)
        vals = solver.probe_energy(U.detach(), ctx.box)
        return torch.tensor(vals, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, g):
        (U,) = ctx.saved_tensors
        lam = ctx.solver.probe_energy_grad(U.detach(), ctx.box)
        # chain rule with the upstream derivative of each batch item's energy
        lam = lam * g.to(lam.dtype).view((-1,) + (1,) * (lam.dim() - 1))
        return lam, None, None


def run(solver: Solver, U0, nsteps: int, epsinv=None, muinv=None, t0: float = 0.0, checkpoint_every: int = 50):
    """State after nsteps steps from U0 (differentiable in U0, epsinv, muinv)."""
    return GKSRun.apply(U0, epsinv, muinv, solver, int(nsteps), float(t0), int(checkpoint_every))


def probe_energy(solver: Solver, U, box):
    """(batch,) float64 probe-box energies sum |Omega| Ez^2 (differentiable in U)."""
    return ProbeEnergy.apply(U, solver, box)


class GKSFunction:
    """The differentiable run in one call, for callers that think of it as one function:

        GKSFunction.apply(solver, epsinv, muinv, U0, nsteps, t0=0.0, checkpoint_every=50, probe=None)

    returns the state after ``nsteps`` steps (``run``), or, with ``probe`` a box, the (batch,)
    probe-box energies of that state (``probe_energy``); differentiable in epsinv, muinv and U0.
    """

    @staticmethod
    def apply(solver: Solver, epsinv, muinv, U0, nsteps: int, t0: float = 0.0, checkpoint_every: int = 50,
              probe=None):
        UN = run(solver, U0, nsteps, epsinv, muinv, t0, checkpoint_every)
        return UN if probe is None else probe_energy(solver, UN, probe)
