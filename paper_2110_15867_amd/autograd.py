"""Gradients of a density-field loss through many Strang steps.

``VlasovRun.apply(f0, B, problem)`` advances f0 for ``problem.nsteps`` steps
of Eq. (5) with the acceleration field g(t) = sum_m B_m basis_m(t) and
returns the density rho(x) of the final state (vlasov_moments).  Its
backward runs the hand-written adjoints of the library -- vlasov_moments_adj
and vlasov_step_adj -- with segment checkpointing: the forward keeps f at
every K-th step, the backward recomputes each segment forward from its
checkpoint and walks it back step by step.  The field gradients lam_g(t) are
chained to the amplitudes by the (linear) field basis.

All sweep arithmetic runs in libvlasov; torch only holds the tensors and forms
g from B (the field parameterisation is input preparation, not a sweep).
"""
from __future__ import annotations

import dataclasses

import torch

from . import vlasov as V


@dataclasses.dataclass
class RunProblem:
    grid: object            # vlasov_grid
    basis: list             # basis[n]: FP32 tensor [modes, 3, nx, ny, nz] at t = n dt
    dt: float
    nsteps: int
    checkpoint_every: int = 2
    vbc: int = V.VBC_OUTFLOW
    a2inv: float = 1.0


def field_at(B: torch.Tensor, basis_n: torch.Tensor) -> torch.Tensor:
    """g = sum_m B_m basis_m, FP32 [3, nx, ny, nz]."""
    return torch.tensordot(B.to(basis_n.dtype), basis_n, dims=([0], [0])).contiguous()


def _step(p: RunProblem, f, g_n, g_np1, work):
    out = torch.empty_like(f)
    V.vlasov_step(p.grid, V.F32, p.vbc, f, None, out, None, g_n, g_np1, p.dt, p.a2inv, work,
                  work.numel(), None)
    return out


def run_forward(p: RunProblem, f0, B, keep_every=None):
    """Returns the final f and the checkpoints {step: f}."""
    fields = [field_at(B, b) for b in p.basis]
    work = torch.empty(V.vlasov_step_workspace_bytes(p.grid, V.F32), dtype=torch.uint8,
                       device=f0.device)
    ckpt = {}
    f = f0
    for n in range(p.nsteps):
        if keep_every and n % keep_every == 0:
            ckpt[n] = f
        f = _step(p, f, fields[n], fields[n + 1], work)
    return f, ckpt, fields


class VlasovRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, B, problem: RunProblem):
        f0 = f0.contiguous()
        f, ckpt, fields = run_forward(problem, f0, B, keep_every=problem.checkpoint_every)
        st = V.State(problem.grid, V.F32, f)
        rho, um, _ = V.moments(st)
        ctx.problem = problem
        ctx.ckpt = ckpt
        ctx.fields = fields
        ctx.save_for_backward(rho, um, B)
        return rho

    @staticmethod
    def backward(ctx, lam_rho):
        p: RunProblem = ctx.problem
        rho, um, B = ctx.saved_tensors
        grid = p.grid
        dev = rho.device
        shape = V.grid_shape(grid)
        lam_f = torch.zeros(shape, dtype=torch.float32, device=dev)
        V.vlasov_moments_adj(grid, rho, um, lam_rho.to(torch.float64).contiguous(), None, lam_f)
        lam_B = torch.zeros(B.shape, dtype=torch.float64, device=dev)
        work = torch.empty(V.vlasov_step_workspace_bytes(grid, V.F32), dtype=torch.uint8,
                           device=dev)
        awork_n = V.vlasov_step_adj_workspace_bytes(grid)
        awork = torch.empty(awork_n, dtype=torch.uint8, device=dev)
        K = p.checkpoint_every
        starts = sorted(ctx.ckpt)
        for s0 in reversed(starts):
            s1 = min(s0 + K, p.nsteps)
            # recompute the inputs of the segment's steps
            states = [ctx.ckpt[s0]]
            for n in range(s0, s1 - 1):
                states.append(_step(p, states[-1], ctx.fields[n], ctx.fields[n + 1], work))
            for n in range(s1 - 1, s0 - 1, -1):
                f_n = states[n - s0]
                lam_in = torch.empty_like(lam_f)
                lgn = torch.zeros((3,) + tuple(grid.n), dtype=torch.float32, device=dev)
                lgnp1 = torch.zeros_like(lgn)
                V.vlasov_step_adj(grid, p.vbc, f_n, ctx.fields[n], ctx.fields[n + 1], p.dt,
                                  p.a2inv, lam_f, lam_in, lgn, lgnp1, awork, awork_n)
                lam_f = lam_in
                lam_B += torch.tensordot(p.basis[n].double(), lgn.double(),
                                         dims=([1, 2, 3, 4], [0, 1, 2, 3]))
                lam_B += torch.tensordot(p.basis[n + 1].double(), lgnp1.double(),
                                         dims=([1, 2, 3, 4], [0, 1, 2, 3]))
        return lam_f, lam_B.to(B.dtype), None


def step_tangent(grid, f, g_n, g_np1, dt, v, gd_n=None, gd_np1=None, a2inv=1.0,
                 vbc=V.VBC_OUTFLOW):
    """Tangent of one Strang step: the nine tangent sweeps along the forward stages."""
    h = 0.5 * dt
    dta = dt * a2inv
    seq = [("ux", g_n, gd_n, h), ("uy", g_n, gd_n, h), ("uz", g_n, gd_n, h),
           ("z", None, None, dta), ("y", None, None, dta), ("x", None, None, dta),
           ("ux", g_np1, gd_np1, h), ("uy", g_np1, gd_np1, h), ("uz", g_np1, gd_np1, h)]
    x, t = f, v
    for ax, g, gd, d in seq:
        nt = torch.empty_like(t)
        nx = torch.empty_like(x)
        if ax in ("x", "y", "z"):
            getattr(V, f"vlasov_advect_{ax}_tan")(grid, x, t, nt, d)
            getattr(V, f"vlasov_advect_{ax}")(grid, V.F32, x, None, nx, None, d)
        else:
            getattr(V, f"vlasov_advect_{ax}_tan")(grid, vbc, x, g, gd, d, t, nt)
            getattr(V, f"vlasov_advect_{ax}")(grid, V.F32, vbc, x, None, nx, None, g, d, None)
        x, t = nx, nt
    return x, t
