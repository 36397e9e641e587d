"""torch.autograd.Function over the library's forward and adjoint.

The regenerated-photon loss (energy of one mode of the regenerated set over
the last columns after N steps) as a function of the seeded Fourier
coefficients of the first pulse's envelope and of the coupling g.  The state
is carried in scaled units (phi/g, E1/g^2), so the physical loss is
g^4 times the scaled one; the initial state is linear in the coefficients, so
dL/dc_q = g^4 Re<lambda^0, du^0/dc_q> with lambda^0 from qds_backward.
Argument marshalling only: the forward, the adjoint, the loss and the
projections run in libqds.
"""
from dataclasses import replace
from typing import Optional

import torch

from . import inputs as I
from . import qds


class EnvelopeLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeffs: torch.Tensor, g: torch.Tensor, wl: I.Workload, n_steps: int, ckpt_every: int,
                dtype: str = "f64", loss_mode: int = 1, x_begin: Optional[int] = None):
        if wl.s_phi != 1.0 or wl.s_j != 1.0:
            # L = g^4 L_hat and dL/dg = 4 g^3 L_hat hold in scaled units only
            raise ValueError("EnvelopeLoss needs the scaled units s_phi = s_j = 1 (the coupling enters as g^4)")
        c = tuple(float(v) for v in coeffs.detach().cpu().tolist())
        p0 = replace(wl.pulses[0], coeffs=c)
        wl2 = wl.with_(pulses=(p0,) + tuple(wl.pulses[1:]))
        s = qds.Solver(wl2, dtype=dtype)
        s.load_pulses()
        s.step(n_steps)
        torch.cuda.synchronize()
        L_hat = s.loss(1, loss_mode, x_begin)
        ctx.save_for_backward(coeffs, g)
        ctx.wl, ctx.n, ctx.ck, ctx.dtype, ctx.mode, ctx.x0 = wl2, n_steps, ckpt_every, dtype, loss_mode, x_begin
        ctx.L_hat = L_hat
        gv = float(g)
        return torch.tensor(gv ** 4 * L_hat, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        coeffs, g = ctx.saved_tensors
        gv = float(g)
        s = qds.Solver(ctx.wl, dtype=ctx.dtype)
        s.load_pulses()
        L_hat, lam, _ = s.backward(ctx.n, ctx.ck, 1, ctx.mode, ctx.x0)
        grads = torch.zeros_like(coeffs, dtype=torch.float64)
        for q in range(coeffs.numel()):
            b = qds.Solver(ctx.wl, dtype=ctx.dtype)
            b.load_pulses(basis=(0, q))
            grads[q] = s.dot(lam, b.bufs[b.state.cur])
            b.close()
        go = float(grad_out)
        dc = go * gv ** 4 * grads
        dg = torch.tensor(go * 4.0 * gv ** 3 * L_hat, dtype=torch.float64)
        return dc.to(coeffs.dtype), dg.to(g.dtype), None, None, None, None, None, None
