"""torch.autograd integration of the NEP kernels.

`NEPFunction.apply(params, engine)` returns per-structure energies [S],
forces [3N] (SoA) and virials [S*6] computed by nep_energy_force_virial; its
backward calls nep_vjp with the incoming cotangents, so any loss written in
torch on (E, F, W) gets dL/dparams from the library's adjoint kernels (the
chain of Eqs. 13-16 with arbitrary cotangents).  Positions are not
differentiable inputs here.
"""
from __future__ import annotations

import torch

from . import nep


class NEPEngine:
    """Device state for one batch: model, batch arrays, neighbor lists and
    workspace.  `build_neighbors()` must run before energies or gradients."""

    def __init__(self, model: nep.Model, batch, device="cuda"):
        self.model = model
        self.batch = batch if isinstance(batch, nep.DeviceBatch) else nep.DeviceBatch(batch, device)
        self.S, self.N = self.batch.n_struct, self.batch.n_atom
        self.nbrs = nep.Neighbors(model, self.N, device)
        self.ws = nep.workspace(model, self.S, self.N, device)
        self.flags = torch.zeros(1, dtype=torch.int32, device=device)
        self.P = nep.param_count(model)
        self.sizes = torch.as_tensor(
            (self.batch.atom_offset[1:] - self.batch.atom_offset[:-1]).to(torch.float32), device=device)

    def build_neighbors(self, check=True):
        self.flags.zero_()
        nep.build_neighbors(self.model, self.batch, self.nbrs, self.ws, self.flags)
        if check:
            nep.check_flags(self.flags, "nep_build_neighbors")

    def energy_force_virial(self, params):
        e = torch.empty(self.S, device=params.device)
        f = torch.empty(3 * self.N, device=params.device)
        w = torch.empty(6 * self.S, device=params.device)
        nep.energy_force_virial(self.model, self.batch, self.nbrs, params, self.ws, None, e, f, w)
        return e, f, w

    def vjp(self, params, e_bar, f_bar, v_bar):
        g = torch.empty(self.P, device=params.device)
        nep.vjp(self.model, self.batch, self.nbrs, params, e_bar.contiguous(), f_bar.contiguous(),
                v_bar.contiguous(), g, self.ws)
        return g


class NEPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, engine):
        ctx.engine = engine
        ctx.save_for_backward(params)
        return engine.energy_force_virial(params.detach().contiguous())

    @staticmethod
    def backward(ctx, e_bar, f_bar, v_bar):
        (params,) = ctx.saved_tensors
        eng = ctx.engine
        z = lambda t, n: torch.zeros(n, device=params.device) if t is None else t.to(torch.float32)
        g = eng.vjp(params.detach().contiguous(), z(e_bar, eng.S), z(f_bar, 3 * eng.N), z(v_bar, 6 * eng.S))
        return g, None


def nep_loss(engine: NEPEngine, params, labels: nep.Labels, lam=(1.0, 1.0, 0.1)):
    """L = le*Le + lf*Lf + lv*Lv of Eqs. 9-12 written in torch on the outputs
    of NEPFunction; returns (L, Le, Lf, Lv)."""
    e, f, w = NEPFunction.apply(params, engine)
    n = engine.sizes
    S, N = engine.S, engine.N
    le = (((e - labels.energy) / n) ** 2).sum() / S
    lf = ((f - labels.force) ** 2).sum() / (3 * N)
    lv = ((((w - labels.virial).view(S, 6)) / n[:, None]) ** 2).sum() / (6 * S)
    L = lam[0] * le + lam[1] * lf + lam[2] * lv
    return L, le, lf, lv
