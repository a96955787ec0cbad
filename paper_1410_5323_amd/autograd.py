"""Differentiable propagation through the library's forward and adjoint kernels.

``propagate(u0, grid, x0, energy, charge, spacing, params)`` propagates the
particles from a fresh start in one field (section 3.2 grid, Lorentz-force
equation of section 2.1 in path length, Cash-Karp steps of section 3.1) and
returns the arrival direction, arrival time and energy.  Its backward pass
gives the gradients with respect to the initial direction, the initial
position, the energy (through the rigidity E/Z, which sets the deflection;
the output energy equals the input one) and the grid values.

The derivative is that of the replayed map: the accepted step sizes of the
forward run are held fixed and the sphere crossing of the last step is
differentiated through its defining equation.  Chaotic trajectories can
amplify a cotangent beyond the FP64 range: such particles keep their
non-finite gradients, and the grid gradient is taken over the other
particles (a second adjoint pass with the overflowed particles' cotangents
zeroed).  The grid gradient is returned in the grid's dtype: for an FP32 grid
the finite but huge gradients of long chaotic trajectories (1e38 and more)
become infinite there.  The forward records a
checkpoint every ``every_k`` accepted steps into a pool of records (run a
second time only if the pool was too small).  The backward pass replays each
segment from its checkpoint on the GPU and sweeps it in reverse.
"""
from __future__ import annotations

import torch

from . import crp

__all__ = ["propagate", "PropagateFunction"]


def _initial_state(u0, x0, energy, charge):
    n = u0.shape[0]
    dev = u0.device
    z = lambda dt: torch.zeros(n, dtype=dt, device=dev)  # noqa: E731
    return {"x": x0[:, 0].contiguous(), "y": x0[:, 1].contiguous(), "z": x0[:, 2].contiguous(),
            "ux": u0[:, 0].contiguous(), "uy": u0[:, 1].contiguous(), "uz": u0[:, 2].contiguous(),
            "energy": energy.contiguous(), "charge": charge.contiguous(), "mass": None,
            "length": z(torch.float64), "h_next": z(torch.float64), "time": z(torch.float64),
            "status": z(torch.int32), "param_index": None, "n_accepted": z(torch.int64),
            "n_rejected": z(torch.int64)}


class PropagateFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, grid, x0, energy, charge, spacing, origin, params, layout, every_k, tape_capacity,
                modulation):
        if u0.dtype != torch.float64 or x0.dtype != torch.float64 or energy.dtype != torch.float64:
            raise TypeError("u0, x0 and energy must be float64")
        if grid.dtype not in (torch.float64, torch.float32):
            raise TypeError("the grid must be float64 or float32")
        dt = "f64" if grid.dtype == torch.float64 else "f32"
        field = crp.make_field(grid.detach(), spacing, origin=origin, dtype=dt, layout=layout, modulation=modulation)
        u0d, x0d, charge = u0.detach(), x0.detach(), charge.to(torch.int32)
        init = _initial_state(u0d, x0d, energy.detach(), charge)
        n = u0.shape[0]
        tape = crp.Tape(n, every_k=every_k, capacity=tape_capacity, device=u0.device)
        st = crp.clone_particles(init)
        crp.crp_propagate([field], [params], st, tape=tape)
        if tape.overflowed():  # run again with exactly the records the run asked for
            tape = crp.Tape(n, every_k=every_k, capacity=tape.records_needed(), device=u0.device)
            st = crp.clone_particles(init)
            crp.crp_propagate([field], [params], st, tape=tape)
        ctx.field, ctx.params, ctx.init, ctx.tape = field, params, init, tape
        ctx.grid_shape, ctx.grid_dtype = tuple(grid.shape), grid.dtype
        direction = torch.stack([st["ux"], st["uy"], st["uz"]], dim=1)
        status = st["status"]
        ctx.mark_non_differentiable(status)
        return direction, st["time"], st["energy"].clone(), status

    @staticmethod
    def backward(ctx, g_dir, g_time, g_energy, g_status):
        n = ctx.init["energy"].numel()
        dev = ctx.init["energy"].device
        gd = (g_dir if g_dir is not None else torch.zeros(n, 3, dtype=torch.float64, device=dev))
        gd = gd.to(torch.float64).contiguous()
        gt = g_time.to(torch.float64).contiguous() if g_time is not None else None
        ge = g_energy.to(torch.float64).contiguous() if g_energy is not None else None
        grad_u0 = torch.empty(n, 3, dtype=torch.float64, device=dev)
        grad_x0 = torch.empty(n, 3, dtype=torch.float64, device=dev)
        grad_e = torch.empty(n, dtype=torch.float64, device=dev)
        grad_field = torch.zeros(ctx.grid_shape, dtype=torch.float64, device=dev)
        crp.crp_propagate_adjoint(ctx.field, ctx.params, ctx.init, ctx.tape, gd, gt, grad_u0, grad_field,
                                  grad_x0=grad_x0, gbar_energy=ge, grad_energy=grad_e)
        over = (ctx.tape.flags() & crp.CRP_TAPE_GRAD_OVERFLOW) != 0
        if ctx.needs_input_grad[1] and bool(over.any()):
            # chaotic particles whose cotangent left the FP64 range: the grid
            # gradient is taken over the other particles only (their own
            # gradients stay as computed, not finite)
            keep = (~over).to(torch.float64)
            grad_field.zero_()
            crp.crp_propagate_adjoint(ctx.field, ctx.params, ctx.init, ctx.tape, gd * keep[:, None],
                                      None if gt is None else gt * keep, torch.empty_like(grad_u0), grad_field,
                                      grad_x0=torch.empty_like(grad_x0),
                                      gbar_energy=None if ge is None else ge * keep,
                                      grad_energy=torch.empty_like(grad_e))
        ctx.overflowed = over
        gu = grad_u0 if ctx.needs_input_grad[0] else None
        gg = grad_field.to(ctx.grid_dtype) if ctx.needs_input_grad[1] else None
        gx = grad_x0 if ctx.needs_input_grad[2] else None
        gE = grad_e if ctx.needs_input_grad[3] else None
        return gu, gg, gx, gE, None, None, None, None, None, None, None, None


def propagate(u0, grid, x0, energy, charge, spacing: float, params, layout: str = "linear", every_k: int = 64,
              origin=(0.0, 0.0, 0.0), tape_capacity: int | None = None, modulation=None):
    """Differentiable propagation of n particles from a fresh start.

    u0, x0: (n, 3) float64 device tensors (direction need not be normalised;
    position in Mpc); grid: (n0, n1, n2, 3) float64/float32 device tensor of
    field values in nG with node spacing ``spacing`` Mpc, node (0, 0, 0) at
    ``origin``; energy: (n,) float64
    eV; charge: (n,) integer charge numbers; params: a crp_params.
    Returns (direction (n, 3), time (n,) s, energy (n,) eV, status (n,)).
    tape_capacity: checkpoint records to allocate (default 64 per particle);
    a run that needs more is repeated once with the exact number.
    modulation: a crp.Modulation multiplying the grid (section 3.2, modulated
    grids); the gradient is taken with respect to the vector grid only.  A
    reflective box or backtracking is set in params.  In a reflective box the
    derivative is that of the replayed map (steps and mirrors held fixed): it
    equals the forward run's in a field-free box and for particles that never
    reflect, not for particles that reflect in a field.
    """
    return PropagateFunction.apply(u0, grid, x0, energy, charge, float(spacing), tuple(float(o) for o in origin),
                                   params, layout, int(every_k), tape_capacity, modulation)
