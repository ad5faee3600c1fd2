"""torch.autograd.Function for the Shannon throughput of eq. (loss) / Sec. IV.

forward(P) runs isrsgn_snr_grad (SNR, throughput and the adjoint gradient in one pass of the
library) when P requires grad, else isrsgn_snr; backward scales the saved gradient by the
incoming gradient of each plan's throughput.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from . import workloads as W


class ThroughputFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, engine: B.Engine, plan: W.Plan, nf, snr_trx_lin: float, plan_index):
        if P.requires_grad:
            snr, thr, g = engine.snr_grad(plan, P.detach(), nf, snr_trx_lin)
            ctx.save_for_backward(g, plan_index)
        else:
            snr, thr = engine.snr(plan, P.detach(), nf, snr_trx_lin)
        ctx.mark_non_differentiable(snr)
        return thr, snr

    @staticmethod
    def backward(ctx, gthr, gsnr):
        g, plan_index = ctx.saved_tensors
        return g * gthr[plan_index], None, None, None, None, None


class Throughput(torch.nn.Module):
    """Differentiable throughput (bit/s per plan) of a fixed channel plan and fibre."""

    def __init__(self, engine: B.Engine, plan: W.Plan, snr_trx_lin: float = 0.0):
        super().__init__()
        self.engine, self.plan, self.snr_trx = engine, plan, float(snr_trx_lin)
        self.nf = torch.tensor(plan.nf_lin, dtype=torch.float64, device="cuda")
        idx = np.repeat(np.arange(plan.n_batch), np.diff(plan.offsets))
        self.plan_index = torch.tensor(idx, dtype=torch.long, device="cuda")

    def forward(self, P):
        thr, snr = ThroughputFn.apply(P, self.engine, self.plan, self.nf, self.snr_trx, self.plan_index)
        return thr, snr


def optimise_launch_power(engine: B.Engine, plan: W.Plan, p_dbm0, steps: int = 50, lr_db: float = 0.05,
                          lo_dbm: float = -5.0, hi_dbm: float = 5.0, snr_trx_lin: float = 0.0, progress=None):
    """Projected gradient ascent (Adam) of the total throughput over per-channel launch powers in
    dBm, bounded to [lo_dbm, hi_dbm] as in Sec. IV.  Channels starting at -inf dBm (P = 0) are
    empty (guard) channels and stay empty.  Returns (p_dbm, history of throughput).
    progress(step, throughput) is called after each step when given."""
    model = Throughput(engine, plan, snr_trx_lin)
    p0 = np.asarray(p_dbm0, dtype=np.float64)
    occupied = np.isfinite(p0)
    occ = torch.tensor(occupied, device="cuda")
    x = torch.tensor(np.where(occupied, p0, lo_dbm), device="cuda", requires_grad=True)
    opt = torch.optim.Adam([x], lr=lr_db)
    hist = []
    for _ in range(steps):
        opt.zero_grad()
        P = torch.where(occ, 1e-3 * torch.pow(10.0, x / 10.0), torch.zeros_like(x))
        thr, _ = model(P)
        total = thr.sum()
        (-total).backward()
        opt.step()
        with torch.no_grad():
            x.clamp_(lo_dbm, hi_dbm)
        hist.append(total.item())
        if progress:
            progress(len(hist), hist[-1])
    return np.where(occupied, x.detach().cpu().numpy(), -np.inf), hist
