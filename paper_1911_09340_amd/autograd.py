"""torch.autograd wrapper of the seed RSS: forward through the scan kernels, backward
through the hand-written adjoint (RK4 recomputed in the backward pass)."""
from __future__ import annotations

import torch

from . import comet


class SeedRSS(torch.autograd.Function):
    """rss[s] = Eq. 1 RSS of seed s (seeds [6, S], float64, on the GPU).

    forward: comet_extrapolate_seeds + comet_dca_rss.
    backward: comet_rss_adjoint, which recomputes each track and sweeps back through
    the RK4 steps from every active wire's chord; d rss / d seed is exact for the
    piece of the (piecewise smooth) RSS the seed lies in.
    """

    @staticmethod
    def forward(ctx, seeds, wire_ends, wire_offsets, drift, cfg):
        seeds_c = seeds.detach().contiguous()
        S = seeds_c.shape[1]
        track = torch.empty(3, cfg.n_steps + 1, S, dtype=torch.float64, device=seeds.device)
        comet.extrapolate_seeds(seeds_c, cfg, track)
        rss = torch.empty(S, dtype=torch.float64, device=seeds.device)
        comet.dca_rss(track, wire_ends, wire_offsets, drift, cfg, rss,
                      comet.dca_workspace(S, cfg.n_steps + 1, int(wire_ends.shape[0]),
                                          seeds.device))
        ctx.save_for_backward(seeds_c, wire_ends, wire_offsets, drift)
        ctx.cfg = cfg
        return rss

    @staticmethod
    def backward(ctx, grad_rss):
        seeds, wire_ends, wire_offsets, drift = ctx.saved_tensors
        S = seeds.shape[1]
        grad = torch.empty(S, 6, dtype=torch.float64, device=seeds.device)
        comet.rss_adjoint(seeds, ctx.cfg, wire_ends, wire_offsets, drift, grad=grad)
        return (grad * grad_rss[:, None]).t().contiguous(), None, None, None, None


def seed_rss(seeds: torch.Tensor, event, cfg: comet.Config) -> torch.Tensor:
    """Differentiable RSS of seeds [6, S] against a scan.DeviceEvent."""
    return SeedRSS.apply(seeds, event.wire_ends, event.wire_offsets, event.drift, cfg)
