"""torch.autograd.Function over libppcg: (lambda, rho) = EigDensity.apply(V, cfg).

forward : the k lowest eigenpairs of H(V) = -1/2 Lap_h + diag(V) by ppcg_solve,
          and the density rho = sum_i |x_i|^2 by ppcg_density (real or complex
          Hermitian operators: cfg.kpt).
backward: dL/dV from the incoming gradients (g_lambda, g_rho) by ppcg_grad
          (Hellmann-Feynman for the eigenvalues, projected Sternheimer
          systems for the density).  Every step runs in libppcg.
"""
from __future__ import annotations

import dataclasses

import torch

from . import binding


@dataclasses.dataclass
class EigConfig:
    N: int
    k: int
    sbsize: int
    X0: torch.Tensor            # (n, K) start block, CUDA float64
    tol: float = 1e-10
    rr_period: int = 5
    h: float = 0.5
    order: int = 2
    kpt: tuple = (0.0, 0.0, 0.0)   # Bloch vector (nonzero: complex Hermitian operator)
    precision: str = "fp64"
    sternheimer_tol: float = 1e-10
    handle: binding.Handle | None = None


class EigDensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, cfg: EigConfig):
        h = cfg.handle or binding.Handle(cfg.precision)
        lam, X, info = h.solve(V.detach().contiguous(), cfg.N, cfg.k, cfg.sbsize, cfg.tol, cfg.rr_period,
                               cfg.X0, h=cfg.h, order=cfg.order, kpt=cfg.kpt)
        rho = h.density()
        ctx.handle = h
        ctx.cfg = cfg
        ctx.info = info
        return lam, rho

    @staticmethod
    def backward(ctx, g_lam, g_rho):
        h = ctx.handle
        if g_lam is None:
            g_lam = torch.zeros(ctx.cfg.k, dtype=torch.float64, device="cuda")
        dV, _ = h.grad(g_lam.contiguous(), None if g_rho is None else g_rho.contiguous(),
                       tol=ctx.cfg.sternheimer_tol)
        return dV, None
