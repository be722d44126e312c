"""Differentiable receiver traces: a torch.autograd.Function over the C ABI.

traces = receiver_traces(solver, u0, ut0, amps, nsteps) runs the wave solver
forward from (u0, ut0) with its point source scaled per half step by amps,
and returns u at the receivers after each full step, [nsteps, n_rec]. Its
backward pass runs the library's adjoint sweep (transposed half steps,
hermite_adjoint_*), giving the gradients with respect to u0, ut0 and amps.

The problem is linear with state-independent operators, so the backward pass
needs no forward state: the adjoint sweep starts from zero at the final time
and takes the residuals at the receivers, which is all that the misfit's
gradient depends on. No checkpoints are stored or recomputed.

All tensors are CUDA float64; the solver runs on its own stream and both
passes synchronise with torch's stream around the library calls.
"""
from __future__ import annotations

import torch


class ReceiverTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, ut0, amps, solver, nsteps: int):
        torch.cuda.synchronize()
        solver.set_initial(u0.contiguous(), ut0.contiguous())
        if amps is not None:
            solver.set_source_series(amps.detach().contiguous())
        traces = torch.empty((nsteps, solver.nrec), dtype=torch.float64, device=u0.device)
        solver.step_record(nsteps, traces)
        solver.sync()
        ctx.solver, ctx.nsteps, ctx.has_amps = solver, nsteps, amps is not None
        ctx.shape = u0.shape
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        s = ctx.solver
        torch.cuda.synchronize()
        res = grad_traces.detach().contiguous()
        gu = torch.empty(ctx.shape, dtype=torch.float64, device=res.device)
        gut = torch.empty_like(gu)
        ga = torch.empty(2 * ctx.nsteps, dtype=torch.float64, device=res.device) if ctx.has_amps else None
        s.adjoint_init()
        s.adjoint_step(ctx.nsteps, res, ga)
        s.adjoint_gather(gu, gut)
        s.sync()
        return gu, gut, ga, None, None


def receiver_traces(solver, u0, ut0, amps, nsteps: int):
    """u at the solver's receivers after each of nsteps full steps from
    (u0, ut0), the source of half step h scaled by amps[h] (amps may be None
    when the solver has no source)."""
    return ReceiverTraces.apply(u0, ut0, amps, solver, nsteps)
