"""Differentiable coupled run: torch.autograd.Function over the library's
forward step and its hand-written adjoint, with sqrt(K) checkpointing.

    phiK, cK = gplbm_run(phi0, c0, lam, D_l, cfg, K, precision="fp64")

phi0, c0: float64 CUDA tensors of the grid's shape; lam, D_l: float64 scalar
tensors; cfg: the parameter mapping (its lam and D_l are replaced).  Any
torch objective J(phiK, cK) can then be differentiated: backward returns
dJ/dphi0, dJ/dc0, dJ/dlambda and dJ/dD_l, all computed by the GPU kernels of
libgplbm.so (this module only schedules them).  precision "fp32" runs the
forward (and its re-computation) in FP32 storage and arithmetic; the reverse
sweep stays FP64, taken at the FP32 states.  "fp16dev" / "bf16dev" (every
lattice combination, both h schemes, both free-energy forms) run the forward
in a deviation storage format and the FP64 reverse sweep at its decoded
states.

Checkpointing: forward keeps the state every s = ceil(sqrt(K)) steps;
backward rebuilds each segment from its checkpoint (gplbm_step_chain, no
copies) and runs the reverse steps over it (gplbm_adjoint_segment), one call
each per segment, so memory holds about 2 sqrt(K) states.
"""
from __future__ import annotations

import math

import torch

from . import binding as B


def _aligned(t: torch.Tensor) -> int:
    return (t.data_ptr() + 255) // 256 * 256


class _Run(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, c0, lam, D_l, cfg, K, seg, precision, schedule):
        cfg = dict(cfg, lam=float(lam), D_l=float(D_l))
        sim = B.Simulation(cfg, precision, schedule)
        dev = sim.device
        phi0d = phi0.detach().to(dev, torch.float64).contiguous()
        c0d = c0.detach().to(dev, torch.float64).contiguous()
        sim.init(phi0d, c0d)
        K = int(K)
        s = int(seg) if seg else max(1, math.ceil(math.sqrt(K)))
        ckpts = []
        n = 0
        while n < K:
            ckpts.append(sim.checkpoint())
            m = min(s, K - n)
            sim.step(m)
            n += m
        phiK, cK, _ = sim.fields_device()
        ctx.sim, ctx.ckpts, ctx.K, ctx.s = sim, ckpts, K, s
        ctx.inputs = (phi0d, c0d)
        ctx.shape = phi0.shape
        return phiK.reshape(phi0.shape), cK.reshape(phi0.shape)

    @staticmethod
    def backward(ctx, phi_bar, c_bar):
        sim, K, s = ctx.sim, ctx.K, ctx.s
        dev = sim.device
        nb = B.gplbm_adjoint_bytes(sim.params)
        work = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        pb = None if phi_bar is None else phi_bar.detach().to(dev, torch.float64).contiguous()
        cb = None if c_bar is None else c_bar.detach().to(dev, torch.float64).contiguous()
        B.gplbm_adjoint_begin(sim.ctx, _aligned(work), nb, pb.data_ptr() if pb is not None else 0,
                              cb.data_ptr() if cb is not None else 0)
        ck_bytes = B.gplbm_checkpoint_bytes(sim.params)
        # the s + 1 states of a segment, one after the other at a 256-byte stride
        stride = (ck_bytes + 255) // 256 * 256
        seg_buf = torch.empty((s + 1) * stride + 256, dtype=torch.uint8, device=dev)
        base = _aligned(seg_buf)
        off = base - seg_buf.data_ptr()
        state0 = seg_buf[off:off + ck_bytes]
        for (ck, n0) in reversed(ctx.ckpts):
            n1 = min(n0 + s, K)
            state0.copy_(ck)
            B.gplbm_step_chain(sim.ctx, base, stride, n1 - n0)
            B.gplbm_adjoint_segment(sim.ctx, base, stride, n1 - n0)
        phi0d, c0d = ctx.inputs
        g_phi0 = torch.empty_like(phi0d)
        g_c0 = torch.empty_like(c0d)
        dlam, ddl = B.gplbm_adjoint_finish(sim.ctx, phi0d.data_ptr(), c0d.data_ptr(),
                                           g_phi0.data_ptr(), g_c0.data_ptr())
        del seg_buf, work
        return (g_phi0.reshape(ctx.shape), g_c0.reshape(ctx.shape),
                torch.tensor(dlam, dtype=torch.float64), torch.tensor(ddl, dtype=torch.float64),
                None, None, None, None, None)


def gplbm_run(phi0, c0, lam, D_l, cfg, K, seg=None, precision="fp64", schedule="auto"):
    """(phi^K, c^K) after K steps; differentiable in phi0, c0, lam and D_l.
    precision: "fp64", "fp32", "fp16dev" or "bf16dev" (forward storage).
    schedule: "auto", "split" or "fused" for the forward steps and their
    re-computation (the schedules give the same bits, so the gradients do
    not depend on it)."""
    if precision not in ("fp64", "fp32", "fp16dev", "bf16dev"):
        raise ValueError(f"unknown precision {precision!r}")
    return _Run.apply(phi0, c0, lam, D_l, cfg, K, seg, precision, schedule)


def objectives(phi0, phiK, W):
    """J1 = final solid fraction mean(1 - phi^K); J2 = mean recession
    distance of the solid: (sum phi^K - sum phi0) / sum (4/W) phi^K (1 - phi^K)
    (volume dissolved over interface area)."""
    J1 = (1.0 - phiK).mean()
    area = ((4.0 / W) * phiK * (1.0 - phiK)).sum()
    J2 = (phiK.sum() - phi0.sum()) / area
    return J1, J2
