"""torch.autograd front end of the library (argument marshalling only).

AlchNonbonded.apply(context, pos, lam, sigma, epsilon, charge) returns
(E_total [K], forces [N,3], dU/dlambda [K], terms [K,10]).  Only E_total is
differentiable: its backward gives dL/dpos, dL/dlambda and per-type
dL/dsigma, dL/depsilon, dL/dcharge from the library's backward pass (the
saved forward state and one extra pass over the list for the parameters).
dL/depsilon is NaN for types with epsilon = 0 (the combination rule
sqrt(eps_i eps_j) has no derivative there); the library also reports the
derivative with respect to sqrt(epsilon), which is finite.

The forward reads the device flags (one synchronization): a list that
outgrew its capacity is re-planned and a fused list build that timed out is
redone per phase (both evaluated again); a fixed-point overflow or
non-finite positions raise, since the results would be wrong.

The parameter tensors must hold the values the context was created with;
gradients flow to them but changing them requires a new context.
"""
import numpy as np
import torch

from . import alchnb


class AlchNonbonded(torch.autograd.Function):
    @staticmethod
    def forward(ctx, context, pos, lam, sigma, epsilon, charge):
        for name, t, ref in (("sigma", sigma, context._sig), ("epsilon", epsilon, context._eps),
                             ("charge", charge, context._chg)):
            if not np.array_equal(t.detach().cpu().numpy().astype(np.float64), ref):
                raise ValueError("%s differs from the context's parameters; create a new context" % name)
        p = pos.detach().contiguous()
        lm = lam.detach().contiguous()
        out = context.compute_checked(p, lm, flags=alchnb.AUTO_REBUILD)
        bad = out["flags"] & (alchnb.FLAG_FIXED_OVERFLOW | alchnb.FLAG_NONFINITE | alchnb.FLAG_CAPACITY |
                              alchnb.FLAG_BARRIER_TIMEOUT)
        if bad:
            raise alchnb.AlchNBError("AlchNonbonded.forward (device flags %d)" % out["flags"], 4 if bad & 16 else 1)
        ctx.context = context
        ctx.generation = context.generation
        ctx.save_for_backward(p, lm)
        ctx.mark_non_differentiable(out["forces"], out["dudl"], out["terms"])
        return out["terms"][:, 8].clone(), out["forces"], out["dudl"], out["terms"]

    @staticmethod
    def backward(ctx, g_energy, g_forces, g_dudl, g_terms):
        for g in (g_forces, g_dudl, g_terms):
            if g is not None and bool(torch.any(g != 0)):
                raise RuntimeError("only E_total is differentiable (no gradients through forces, dU/dlambda or terms)")
        context = ctx.context
        pos, lam = ctx.saved_tensors
        if context.generation != ctx.generation:
            context.compute(pos, lam, flags=alchnb.AUTO_REBUILD)  # restore the forward state
        ge = g_energy.detach().to(torch.float64).contiguous()
        need = ctx.needs_input_grad
        d_pos = torch.zeros_like(pos) if need[1] else None
        d_lam = torch.zeros_like(lam) if need[2] else None
        T = context.n_types
        z = lambda: torch.zeros(T, dtype=torch.float64, device=pos.device)
        d_sig = z() if need[3] else None
        d_eps = z() if need[4] else None
        d_q = z() if need[5] else None
        context.backward(pos, lam, ge, d_pos=d_pos, d_lambda=d_lam, d_sigma=d_sig, d_charge=d_q, d_eps=d_eps)
        return (None, d_pos, d_lam, d_sig if need[3] else None, d_eps if need[4] else None,
                d_q if need[5] else None)


class DihedralCV(torch.autograd.Function):
    """xi [C] of atom quadruples idx [C,4] (int32, device); backward scatters dxi."""

    @staticmethod
    def forward(ctx, context, pos, idx):
        r = context.dihedrals(pos.detach().contiguous(), idx)
        ctx.save_for_backward(idx.to(torch.int64), r["dxi"])
        ctx.n = pos.shape[0]
        return r["xi"]

    @staticmethod
    def backward(ctx, g_xi):
        idx, dxi = ctx.saved_tensors
        d_pos = torch.zeros((ctx.n, 3), dtype=torch.float64, device=dxi.device)
        d_pos.index_add_(0, idx.reshape(-1), (g_xi.reshape(-1, 1, 1) * dxi).reshape(-1, 3))
        return None, d_pos, None


def dafed_energy(xi, s, kappa):
    """U = sum kappa/2 wrap(xi - s)^2 with the difference wrapped into (-pi, pi] (eq. 15)."""
    d = torch.remainder(xi - s + np.pi, 2 * np.pi) - np.pi
    d = torch.where(d == -np.pi, torch.full_like(d, np.pi), d)
    return 0.5 * torch.sum(kappa * d * d)
