"""Helpers shared by the GPU parity tests: build a case (inputs, oracle
reference), run the library through its C ABI, compare with the A20 norm-wise
tolerance max|a - ref| / max|ref|."""
from __future__ import annotations

import numpy as np

from paper_2507_00528_amd import synth

TOL_E = 1e-5   # energy per atom
TOL_F = 1e-4   # forces, virials, parameter gradients


_STRUCTURES = {}


def structures(name):
    """synth.config_structures(name), generated once per test session (the
    c4 set takes most of a minute)."""
    if name not in _STRUCTURES:
        _STRUCTURES[name] = synth.config_structures(name)
    return _STRUCTURES[name]


def rel(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.abs(ref).max()
    return float(np.abs(a - ref).max() / den) if den > 0 else float(np.abs(a).max())


def param_blocks(sz):
    """name -> slice of the flat parameter vector."""
    T, H = sz.n_types, sz.hidden
    D = sz.n_desc
    out = {}
    o = T * T * sz.n_rad * sz.k_rad
    out["c_rad"] = slice(0, o)
    out["c_ang"] = slice(o, o + T * T * sz.n_ang * sz.k_ang)
    o += T * T * sz.n_ang * sz.k_ang
    blk = H * D + 2 * H + 1
    idx = {k: [] for k in ("W0", "b0", "w1", "b1")}
    for I in range(T):
        b = o + I * blk
        idx["W0"] += list(range(b, b + H * D))
        idx["b0"] += list(range(b + H * D, b + H * D + H))
        idx["w1"] += list(range(b + H * D + H, b + H * D + 2 * H))
        idx["b1"] += [b + blk - 1]
    out.update({k: np.array(v) for k, v in idx.items()})
    return out


class Case:
    """Structures + student/teacher parameters + oracle labels."""

    def __init__(self, sizes, structures, seed_student=11, seed_teacher=22, seed_noise=33, lam=(1.0, 1.0, 0.1),
                 with_oracle=True):
        from oracle import NEPOracle
        self.sizes = sizes
        self.structures = structures
        self.batch = synth.Batch(structures)
        self.lam = lam
        self.theta = synth.draw_params(sizes.n_params, seed_student)
        self.teacher = synth.draw_params(sizes.n_params, seed_teacher)
        self.oracle = NEPOracle(sizes)
        self.nbrs = [self.oracle.neighbors(st) for st in structures]
        tp = self.oracle.predict(self.teacher, structures, self.nbrs)
        de, df = synth.label_noise(self.batch, seed_noise)
        N = self.batch.n_atom
        offs = self.batch.atom_offset
        F = np.concatenate(tp["F"], 0) if N else np.zeros((0, 3))
        F = F + df.reshape(3, N).T if N else F
        self.labels = dict(energy=(tp["E"] + de).astype(np.float32).astype(np.float64),
                           force=F.astype(np.float32).astype(np.float64),
                           virial=tp["W"].astype(np.float32).astype(np.float64))
        self.labels_force_list = [self.labels["force"][offs[k]:offs[k + 1]] for k in range(len(structures))]
        if with_oracle:
            self.pred = self.oracle.predict(self.theta, structures, self.nbrs)
            self.loss, self.grad = self.oracle.loss_and_grad(
                self.theta, structures, dict(energy=self.labels["energy"], force=self.labels_force_list,
                                             virial=self.labels["virial"]), lam, nbr_cache=self.nbrs)


def oracle_lists(case, which):
    """Per-atom canonical neighbor entries (j_global << 5 | code) from the oracle."""
    out = []
    for k, st in enumerate(case.structures):
        p = case.nbrs[k][0 if which == "rad" else 1]
        base = int(case.batch.atom_offset[k])
        lists = [[] for _ in range(st.n)]
        for i, j, c in p:
            lists[i].append(((base + int(j)) << 5) | int(c))
        out.extend(lists)
    return out


class DeviceRun:
    """Device-side state for one case."""

    def __init__(self, case, cap_rad=64, cap_ang=32):
        import torch
        from paper_2507_00528_amd import nep
        self.nep = nep
        self.case = case
        self.model = nep.Model.of(case.sizes, cap_rad, cap_ang)
        self.batch = nep.DeviceBatch(case.batch)
        self.nbrs = nep.Neighbors(self.model, case.batch.n_atom)
        self.ws = nep.workspace(self.model, case.batch.n_struct, case.batch.n_atom)
        self.flags = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.params = torch.tensor(case.theta, device="cuda")
        b = case.batch
        self.labels = nep.Labels(torch.tensor(case.labels["energy"], dtype=torch.float32, device="cuda"),
                                 torch.tensor(np.ascontiguousarray(case.labels["force"].T).reshape(-1),
                                              dtype=torch.float32, device="cuda"),
                                 torch.tensor(case.labels["virial"].reshape(-1), dtype=torch.float32, device="cuda"))
        self.N, self.S = b.n_atom, b.n_struct

    def neighbors(self):
        self.nep.build_neighbors(self.model, self.batch, self.nbrs, self.ws, self.flags)

    def lists(self, which):
        import torch
        torch.cuda.synchronize()
        cap = self.model.cap_rad if which == "rad" else self.model.cap_ang
        idx = (self.nbrs.idx_rad if which == "rad" else self.nbrs.idx_ang).cpu().numpy().view(np.uint32)
        cnt = (self.nbrs.cnt_rad if which == "rad" else self.nbrs.cnt_ang).cpu().numpy()
        idx = idx.reshape(max(self.N, 1), cap)
        return [list(idx[i, :min(cnt[i], cap)]) for i in range(self.N)], cnt

    def efw(self):
        import torch
        e_atom = torch.zeros(self.N, device="cuda")
        e_s = torch.zeros(self.S, device="cuda")
        F = torch.zeros(3 * self.N, device="cuda")
        W = torch.zeros(6 * self.S, device="cuda")
        self.nep.energy_force_virial(self.model, self.batch, self.nbrs, self.params, self.ws, e_atom, e_s, F, W)
        torch.cuda.synchronize()
        return (e_atom.cpu().numpy(), e_s.cpu().numpy(), F.cpu().numpy().reshape(3, -1).T,
                W.cpu().numpy().reshape(-1, 6))

    def loss_grad(self):
        import torch
        loss = torch.zeros(4, device="cuda")
        grad = torch.zeros(self.params.numel(), device="cuda")
        e_s = torch.zeros(self.S, device="cuda")
        F = torch.zeros(3 * self.N, device="cuda")
        W = torch.zeros(6 * self.S, device="cuda")
        self.nep.loss_grad(self.model, self.batch, self.nbrs, self.params, self.labels, self.case.lam, loss, grad,
                           self.ws, self.flags, e_s, F, W)
        torch.cuda.synchronize()
        return loss.cpu().numpy(), grad.cpu().numpy(), e_s.cpu().numpy(), F.cpu().numpy().reshape(3, -1).T, \
            W.cpu().numpy().reshape(-1, 6)
