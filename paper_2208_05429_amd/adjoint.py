"""Gradients of a loss of the final velocity field with respect to a per-cell
body force, through the library's discrete adjoint (argument marshalling only).

Forward: T time steps from f0 under the Guo force F, keeping the state every
`checkpoint` steps; each kept state is written by the out-of-place pass that
ends its interval, so keeping it costs no copy.  Backward: lambda_T = dL/df_T
from dL/du (lbm_macro_adjoint, which also adds the direct dL/dF), then for
each checkpoint interval in reverse: recompute the states the reverse steps start from (lbm_step_into,
out of place, so no state is ever copied), and run the adjoint backwards
(lbm_step_adjoint), accumulating dL/dF.  With spec["merged"] the reverse
steps go two at a time (the adjoint of the merged pass, f_{t+1} recomputed on
chip), so only every other state is needed.
"""
from __future__ import annotations

import torch

from . import capi
from .lattice import Lattice, real_dtype


def _ptr(t):
    return None if t is None else t.data_ptr()


class ForceAdjoint(torch.autograd.Function):
    """u_T = ForceAdjoint.apply(F, f0, spec); spec = dict(shape, tau, storage,
    faces, wall_u, steps, checkpoint[, merged, scheme, variant])."""

    @staticmethod
    def forward(ctx, F, f0, spec):
        shape, storage = tuple(spec["shape"]), spec["storage"]
        steps, k = int(spec["steps"]), int(spec["checkpoint"])
        lat = Lattice(shape, spec["tau"], storage, spec.get("scheme", "swap2"), spec["faces"],
                      spec.get("wall_u", (0.0, 0.0, 0.0)), force=F.detach(),
                      f=torch.empty(f0.shape, dtype=f0.dtype, device=f0.device), velocities=f0.shape[0],
                      variant=int(spec.get("variant", 0)))
        ckpts = [f0.detach().clone(memory_format=torch.contiguous_format)]
        t = 0
        while t < steps:
            n = min(k, steps - t)
            t += n
            dst = torch.empty_like(lat.f) if t < steps else None  # None: the final state, in lat.f
            forward_interval(lat, ckpts[-1], dst, n)
            if dst is not None:
                ckpts.append(dst)
        # with sums the call waits and reports a hazard wait that gave up in
        # any in-place pass of the forward (the gradient would be wrong)
        _, u, _, _ = lat.macroscopic(sums=True, want=("u",))
        ctx.lat, ctx.ckpts, ctx.spec = lat, ckpts, spec
        ctx.save_for_backward(F)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        lat, ckpts, spec = ctx.lat, ctx.ckpts, ctx.spec
        steps, k = int(spec["steps"]), int(spec["checkpoint"])
        merged = bool(spec.get("merged", False))
        shape = lat.shape
        rdt = real_dtype(lat.storage)
        dev = lat.device
        lam = torch.empty((lat.Q,) + shape, dtype=rdt, device=dev)
        lam2 = torch.empty_like(lam)
        gF = torch.zeros((3,) + shape, dtype=rdt, device=dev)
        gu = grad_u.to(device=dev, dtype=rdt).contiguous()
        capi.lbm_set_stream(lat.ctx, torch.cuda.current_stream().cuda_stream)
        capi.lbm_macro_adjoint(lat.ctx, _ptr(lat.f), _ptr(gu), _ptr(lam), _ptr(gF))
        pool = []  # state buffers reused across intervals
        for seg in range(len(ckpts) - 1, -1, -1):
            n = min(k, steps - seg * k)
            calls = reverse_schedule(n, merged)
            need = sorted({t0 for t0, _ in calls})
            states = {0: ckpts[seg]}
            prev = 0
            for j, t0 in enumerate(t for t in need if t > 0):
                while len(pool) <= j:
                    pool.append(torch.empty_like(lat.f))
                lat.step_into(states[prev], pool[j], t0 - prev)
                states[t0] = pool[j]
                prev = t0
            for t0, kk in calls:
                capi.lbm_step_adjoint(lat.ctx, _ptr(states[t0]), _ptr(lam), _ptr(lam2), _ptr(gF), kk)
                lam, lam2 = lam2, lam
        F, = ctx.saved_tensors
        return gF.to(F.dtype), None, None


def forward_interval(lat, src, dst, n):
    """n >= 1 steps from the state src into dst, or into lat.f (the lattice's
    own buffer) when dst is None.  src is left as it is and no state is copied:
    the first pass reads src, the last one writes dst, and the passes between
    run in place in lat.f (an out-of-place pass moves the same bytes as an
    in-place one)."""
    if dst is None:
        lat.step_into(src, lat.f, min(n, 2))
        if n > 2:
            lat.step(n - 2)
    elif n <= 2:
        lat.step_into(src, dst, n)
    else:
        last = 2 if n >= 4 else 1
        lat.step_into(src, lat.f, 2)
        if n - 2 - last:
            lat.step(n - 2 - last)
        lat.step_into(lat.f, dst, last)


def reverse_schedule(n, merged):
    """Reverse steps of an interval of n steps, latest first, as (start, k):
    the adjoint of steps start .. start+k-1 of the interval."""
    calls, t = [], n
    while t > 0:
        kk = 2 if merged and t >= 2 else 1
        calls.append((t - kk, kk))
        t -= kk
    return calls


def force_gradient(F, f0, spec, u_target):
    """(L, dL/dF) for L = sum (u_T - u*)^2, through ForceAdjoint."""
    Fp = F.detach().clone().requires_grad_(True)
    u = ForceAdjoint.apply(Fp, f0, spec)
    L = ((u - u_target) ** 2).sum()
    L.backward()
    return float(L.detach()), Fp.grad
