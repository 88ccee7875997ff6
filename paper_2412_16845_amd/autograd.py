"""Differentiable 2D GKS runs for PyTorch (reverse mode through the library's adjoint step).

``run(solver, U0, nsteps, epsinv=None, muinv=None, t0=0.0, checkpoint_every=50)`` returns the
state after ``nsteps`` steps and is differentiable with respect to U0, 1/eps and 1/mu:

  forward   gks_run in segments of ``checkpoint_every`` steps; the state at the start of every
            segment is kept (one state per segment instead of one per step), and the last
            segment is stepped one gks_step at a time with its states kept, since the backward
            pass starts with them;
  backward  segment by segment, the last first: gks_adjoint_step walks back through the
            segment's states, carrying the co-state lambda and accumulating the 1/eps, 1/mu
            gradients in double precision, while the solver's twin (the same solver on a second
            stream) recomputes the states of the segment before from its checkpoint with
            gks_step.  The two kernels share the GPU, which fills the gaps each leaves (1024^2 x
            8, fp32: 222.5 -> 205.6 us per recomputed-and-reversed step).  Events order the two
            streams: a segment's adjoint waits for its states, and a recompute waits for the
            adjoint that last read its buffers.

``probe_energy(solver, U, box)`` is the probe-box field energy sum |Omega| Ez^2 per batch item
(gks_probe_energy, with gks_probe_energy_grad as its derivative): the loss of the inverse
design workload.

Memory: checkpoints hold ceil(nsteps / K) states; the forward pass keeps the last segment's K
states for the backward pass, which holds up to 2K more (the segment being reversed and the one
being recomputed; K = checkpoint_every), plus two co-states and the library's adjoint scratch
(the ghost positions around the grid only: about 4 (nx + ny) positions per batch item).
"""
from __future__ import annotations

import torch

from .gks import Solver

__all__ = ["run", "probe_energy", "GKSFunction", "GKSRun", "ProbeEnergy"]


def step_time(t0: float, k: int, j: int, dt: float) -> float:
    """Time of step j of the segment that starts at step k, formed as gks_run forms it from the
    segment's start time, so that recomputed states equal the forward ones bit for bit."""
    return (t0 + k * dt) + j * dt


class GKSRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, epsinv, muinv, solver: Solver, nsteps: int, t0: float, K: int):
        if K < 1:
            raise ValueError("checkpoint_every must be >= 1")
        solver.set_material(epsinv, muinv)
        U = U0.detach().clone()
        ckpts = []
        segs = []
        last = None
        dt = solver.dt
        for k in range(0, nsteps, K):
            m = min(K, nsteps - k)
            segs.append((k, m))
            if k + m < nsteps:
                ckpts.append(U.clone())
                solver.run(U, m, t0 + k * dt)
            else:
                # the last segment's states, as the backward pass would recompute them
                last = [U]
                for j in range(m):
                    last.append(solver.step(last[-1], t=step_time(t0, k, j, dt)))
                U = last.pop()
                ckpts.append(last[0])
        ctx.solver = solver
        ctx.t0 = t0
        ctx.segs = segs
        ctx.ckpts = ckpts
        ctx.last = last
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
        segs, ckpts = ctx.segs, ctx.ckpts
        nseg = len(segs)
        dt = s.dt
        main = s.stream
        tw = s.twin() if nseg > 1 else None
        # two buffer sets for recomputed states, by segment parity; allocated here, on the main
        # stream, before the twin writes them
        nbuf = segs[0][1] - 1 if nseg > 1 else 0   # every segment but the last has K steps
        bufs = [[torch.empty_like(lam) for _ in range(nbuf)] for _ in range(min(nseg - 1, 2))]
        states = [None] * nseg
        ready = [None] * nseg    # event: the segment's states are written
        freed = [None] * nseg    # event: the segment's adjoint steps have read its states

        def recompute(i):
            k, m = segs[i]
            par = bufs[i & 1]
            if i + 2 < nseg and freed[i + 2] is not None:
                tw.stream.wait_event(freed[i + 2])   # the buffers' last reader
            st = [ckpts[i]] + par[:m - 1]
            for j in range(m - 1):
                tw.step(st[j], st[j + 1], t=step_time(ctx.t0, k, j, dt))
            ev = torch.cuda.Event()
            ev.record(tw.stream)
            ready[i] = ev
            states[i] = st

        if nseg > 0:
            states[nseg - 1] = ctx.last
        if nseg > 1:
            # the twin reads checkpoints the main stream may still be writing
            start = torch.cuda.Event()
            start.record(main)
            tw.stream.wait_event(start)
            recompute(nseg - 2)
        for i in reversed(range(nseg)):
            k, m = segs[i]
            if ready[i] is not None:
                main.wait_event(ready[i])
            st = states[i]
            for j in reversed(range(m)):
                s.adjoint_step(st[j], lam, nxt, ge, gm, t=step_time(ctx.t0, k, j, dt))
                lam, nxt = nxt, lam
            ev = torch.cuda.Event()
            ev.record(main)
            freed[i] = ev
            states[i] = None
            if i - 2 >= 0:
                recompute(i - 2)
        ctx.ckpts = None
        ctx.last = None
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
