"""Mini-batch training driver for the NEP loss-and-gradient path.

One optimisation step is one mini-batch: neighbor lists, energies, forces
and virials, the weighted loss of Eqs. 9-12 normalised over the mini-batch,
its analytic gradient, and an Adam update whose learning rate follows the
warm-up plus cosine schedule of Eq. 17 (Sec. II D), with
N_warmup = warm-up epochs x batches per epoch and
N_total = epochs x batches per epoch.

Two ways to form mini-batches:

* fixed (default): the structures are split once, by a seeded permutation,
  into batches of `batch_size`; each batch keeps its own device arrays and a
  captured train-step graph, and every epoch replays the graphs in a fresh
  seeded order.  All graphs share the parameters, the Adam moments and the
  device step counter, so the Eq. 17 learning rate advances by one per
  replay.
* reshuffle: every epoch draws a new permutation and new batches; each step
  gathers its structures and runs the eager library calls, with the Eq. 17
  learning rate computed on the host.

The host-side bookkeeping (`epoch_batches`, `schedule_steps`) needs no GPU;
the `Trainer` drives the library on one.

    python -m paper_2507_00528_amd.train --config c1 --epochs 20 --batch-size 1
    python -m paper_2507_00528_amd.train --config c1 --sweep-batch 1,4,16,64 --epochs 10
    python -m paper_2507_00528_amd.train --config c1 --sweep-epochs 5,10,20 --batch-size 8

print one JSON line per epoch (or per sweep point) on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------- host logic
def epoch_batches(n_struct: int, batch_size: int, rng: np.random.Generator) -> list:
    """Split structure indices 0..n_struct-1 into consecutive batches of a
    random permutation; the last batch holds the remainder."""
    if n_struct <= 0 or batch_size <= 0:
        raise ValueError("need at least one structure and a positive batch size")
    perm = rng.permutation(n_struct)
    return [perm[k:k + batch_size] for k in range(0, n_struct, batch_size)]


def schedule_steps(epochs: int, warmup_epochs: float, batches_per_epoch: int) -> tuple:
    """(N_warmup, N_total) of Eq. 17 in optimisation steps."""
    return int(round(warmup_epochs * batches_per_epoch)), int(epochs * batches_per_epoch)


@dataclass
class LabelSet:
    """Training targets per structure: total energy, forces [n, 3] and total
    virial (xx, yy, zz, xy, yz, zx)."""
    energy: np.ndarray                       # [S]
    force: list                              # S arrays [n_s, 3]
    virial: np.ndarray                       # [S, 6]

    def subset(self, idx) -> "LabelSet":
        return LabelSet(self.energy[idx], [self.force[k] for k in idx], self.virial[idx])


# ---------------------------------------------------------------- device side
@dataclass
class _BatchState:
    idx: np.ndarray
    n_atom: int
    batch: object = None
    nbrs: object = None
    ws: object = None
    labels: object = None
    flags: object = None
    loss: object = None
    grad: object = None
    graph: object = None
    keep: list = field(default_factory=list)


def _device_labels(labels: LabelSet, device):
    import torch
    from . import nep
    f = np.concatenate(labels.force, 0) if labels.force else np.zeros((0, 3), np.float32)
    return nep.Labels(torch.tensor(np.asarray(labels.energy, np.float32), device=device),
                      torch.tensor(np.ascontiguousarray(f.T, dtype=np.float32).reshape(-1), device=device),
                      torch.tensor(np.asarray(labels.virial, np.float32).reshape(-1), device=device))


class Trainer:
    """Adam training of one NEP on a fixed set of structures (see module
    docstring).  `params` is the initial parameter vector (numpy, P floats)."""

    def __init__(self, sizes, structures, labels: LabelSet, params, batch_size=1, epochs=100, warmup_epochs=1.0,
                 lr_start=1e-3, lr_stop=1e-5, lam=(1.0, 1.0, 0.1), seed=0, reshuffle=False, cap_rad=64,
                 cap_ang=32, device="cuda"):
        import torch
        from . import nep, synth
        self.nep, self.synth, self.torch = nep, synth, torch
        self.structures, self.labels = list(structures), labels
        self.model = nep.Model.of(sizes, cap_rad, cap_ang)
        self.P = nep.param_count(self.model)
        if len(params) != self.P:
            raise ValueError(f"expected {self.P} parameters, got {len(params)}")
        self.device = device
        self.batch_size, self.epochs, self.lam = int(batch_size), int(epochs), tuple(lam)
        self.lr_start, self.lr_stop = float(lr_start), float(lr_stop)
        self.reshuffle = bool(reshuffle)
        self.rng = np.random.default_rng(seed)
        self.params = torch.tensor(np.asarray(params, np.float32), device=device)
        self.m = torch.zeros(self.P, device=device)
        self.v = torch.zeros(self.P, device=device)
        self.step = torch.ones(1, dtype=torch.int32, device=device)   # 1-based step of the next update
        self.stream = torch.cuda.Stream()
        nb = math.ceil(len(self.structures) / self.batch_size)
        self.batches_per_epoch = nb
        self.n_warmup, self.n_total = schedule_steps(self.epochs, warmup_epochs, nb)
        self.fixed = None if self.reshuffle else [self._prepare(idx, graph=True)
                                                  for idx in epoch_batches(len(self.structures), self.batch_size,
                                                                           self.rng)]
        # device arrays are filled on the default stream; the steps run on self.stream
        torch.cuda.synchronize()
        self.history = []

    # one mini-batch's device arrays (and, for fixed batches, its graph)
    def _prepare(self, idx, graph):
        nep, torch = self.nep, self.torch
        sts = [self.structures[k] for k in idx]
        b = self.synth.Batch(sts)
        st = _BatchState(idx=np.asarray(idx), n_atom=b.n_atom)
        st.batch = nep.DeviceBatch(b, self.device)
        st.nbrs = nep.Neighbors(self.model, b.n_atom, self.device)
        st.ws = nep.workspace(self.model, b.n_struct, b.n_atom, self.device)
        st.labels = _device_labels(self.labels.subset(st.idx), self.device)
        st.flags = torch.zeros(1, dtype=torch.int32, device=self.device)
        st.loss = torch.zeros(4, device=self.device)
        st.grad = torch.zeros(self.P, device=self.device)
        if graph:
            st.graph = nep.TrainStepGraph(self.model, st.batch, st.nbrs, st.labels, self.lam, self.params, self.m,
                                          self.v, st.grad, st.loss, self.step, st.ws, st.flags,
                                          lr_start=self.lr_start, lr_stop=self.lr_stop, n_warmup=self.n_warmup,
                                          n_total=self.n_total, stream=self.stream)
        return st

    def _eager_step(self, st):
        nep = self.nep
        s = int(self.step_host)
        lr = nep.lr_schedule(s - 1, self.lr_start, self.lr_stop, self.n_warmup, self.n_total)
        with self.torch.cuda.stream(self.stream):
            st.flags.zero_()
            nep.build_neighbors(self.model, st.batch, st.nbrs, st.ws, st.flags, stream=self.stream)
            nep.loss_grad(self.model, st.batch, st.nbrs, self.params, st.labels, self.lam, st.loss, st.grad, st.ws,
                          st.flags, stream=self.stream)
            # an overflowing list or a non-finite loss must not reach the optimizer state
            nep.check_flags(st.flags, "training step")
            nep.adam_step(self.params, self.m, self.v, st.grad, lr, s, stream=self.stream)
        self.step_host += 1

    def train_epoch(self) -> dict:
        """One pass over every structure; returns the atom-weighted mean of the
        mini-batch losses (each taken before its own update) and timing."""
        torch = self.torch
        t0 = time.perf_counter()
        if self.reshuffle:
            self.step_host = int(self.step.item())
            order = [self._prepare(idx, graph=False)
                     for idx in epoch_batches(len(self.structures), self.batch_size, self.rng)]
            torch.cuda.synchronize()   # batch arrays come from the default stream
            for st in order:
                self._eager_step(st)
            self.step.fill_(self.step_host)
        else:
            order = [self.fixed[k] for k in self.rng.permutation(len(self.fixed))]
            for st in order:
                st.graph.launch(self.stream)
        self.stream.synchronize()
        secs = time.perf_counter() - t0
        w = np.array([st.n_atom for st in order], np.float64)
        ls = torch.stack([st.loss for st in order]).cpu().numpy().astype(np.float64)
        for st in order:
            self.nep.check_flags(st.flags, "training step")
        rec = {"epoch": len(self.history) + 1, "loss": float((w[:, None] * ls).sum(0)[0] / w.sum()),
               "loss_e": float((w * ls[:, 1]).sum() / w.sum()), "loss_f": float((w * ls[:, 2]).sum() / w.sum()),
               "loss_v": float((w * ls[:, 3]).sum() / w.sum()), "seconds": secs,
               "steps": int(self.step.item()) - 1,
               "lr": self.nep.lr_schedule(int(self.step.item()) - 2, self.lr_start, self.lr_stop, self.n_warmup,
                                          self.n_total)}
        self.history.append(rec)
        return rec

    def evaluate(self, structures=None, labels: LabelSet | None = None) -> dict:
        """RMSE of energy per atom (eV/atom), force components (eV/A) and
        virial per atom (eV/atom) at the current parameters."""
        nep, torch = self.nep, self.torch
        sts = self.structures if structures is None else list(structures)
        lab = self.labels if labels is None else labels
        b = self.synth.Batch(sts)
        db = nep.DeviceBatch(b, self.device)
        nb = nep.Neighbors(self.model, b.n_atom, self.device)
        ws = nep.workspace(self.model, b.n_struct, b.n_atom, self.device)
        fl = torch.zeros(1, dtype=torch.int32, device=self.device)
        nep.build_neighbors(self.model, db, nb, ws, fl)
        e = torch.zeros(b.n_struct, device=self.device)
        f = torch.zeros(3 * b.n_atom, device=self.device)
        wv = torch.zeros(6 * b.n_struct, device=self.device)
        nep.energy_force_virial(self.model, db, nb, self.params, ws, None, e, f, wv)
        torch.cuda.synchronize()
        nep.check_flags(fl, "evaluation neighbors")
        n = np.diff(b.atom_offset).astype(np.float64)
        de = (e.cpu().numpy().astype(np.float64) - np.asarray(lab.energy, np.float64)) / n
        df = f.cpu().numpy().reshape(3, -1).T.astype(np.float64) - np.concatenate(lab.force, 0)
        dw = (wv.cpu().numpy().reshape(-1, 6).astype(np.float64) - np.asarray(lab.virial, np.float64)) / n[:, None]
        return {"rmse_e": float(np.sqrt(np.mean(de ** 2))), "rmse_f": float(np.sqrt(np.mean(df ** 2))),
                "rmse_v": float(np.sqrt(np.mean(dw ** 2)))}

    def close(self):
        for st in self.fixed or []:
            if st.graph is not None:
                st.graph.close()


# ---------------------------------------------------------------- synthetic data
def teacher_labels(sizes, structures, seed_teacher, seed_noise, device="cuda") -> LabelSet:
    """Labels of a teacher NEP (parameters drawn from seed_teacher) computed by
    the library, plus seeded noise (1 meV/atom on energies, 10 meV/A on force
    components)."""
    import torch
    from . import nep, synth
    model = nep.Model.of(sizes)
    b = synth.Batch(structures)
    db = nep.DeviceBatch(b, device)
    nb = nep.Neighbors(model, b.n_atom, device)
    ws = nep.workspace(model, b.n_struct, b.n_atom, device)
    fl = torch.zeros(1, dtype=torch.int32, device=device)
    theta = torch.tensor(synth.draw_params(sizes.n_params, seed_teacher), device=device)
    nep.build_neighbors(model, db, nb, ws, fl)
    e = torch.zeros(b.n_struct, device=device)
    f = torch.zeros(3 * b.n_atom, device=device)
    w = torch.zeros(6 * b.n_struct, device=device)
    nep.energy_force_virial(model, db, nb, theta, ws, None, e, f, w)
    torch.cuda.synchronize()
    nep.check_flags(fl, "teacher neighbors")
    de, df = synth.label_noise(b, seed_noise)
    e = e.cpu().numpy() + de
    f = (f.cpu().numpy() + df).reshape(3, -1).T
    off = b.atom_offset
    return LabelSet(e.astype(np.float32), [f[off[k]:off[k + 1]].astype(np.float32) for k in range(b.n_struct)],
                    w.cpu().numpy().reshape(-1, 6).astype(np.float32))


def _run(args, sizes, structures, labels, batch_size, epochs, log_epochs=True):
    from . import synth
    tr = Trainer(sizes, structures, labels, synth.draw_params(sizes.n_params, synth.SEEDS["student"]),
                 batch_size=batch_size, epochs=epochs, warmup_epochs=args.warmup_epochs, lr_start=args.lr_start,
                 lr_stop=args.lr_stop, seed=args.seed, reshuffle=args.reshuffle)
    t0 = time.perf_counter()
    for _ in range(epochs):
        rec = tr.train_epoch()
        if log_epochs:
            print(json.dumps({**rec, "batch_size": batch_size}), flush=True)
    wall = time.perf_counter() - t0
    ev = tr.evaluate()
    tr.close()
    return {"batch_size": batch_size, "epochs": epochs, "final_loss": tr.history[-1]["loss"],
            "train_seconds": wall, **ev}


def main(argv=None):
    from . import synth
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", default="c1", help="synthetic workload (c0..c4)")
    ap.add_argument("--sizes", default=None, choices=["small", "large", "tiny", "l8"],
                    help="model sizes in place of the workload's own (l8: 3-body degrees up to 8)")
    ap.add_argument("--structures", type=int, default=None, help="use only the first n structures")
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch-size", type=int, default=1)
    ap.add_argument("--warmup-epochs", type=float, default=1.0)
    ap.add_argument("--lr-start", type=float, default=1e-3)
    ap.add_argument("--lr-stop", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--reshuffle", action="store_true")
    ap.add_argument("--sweep-batch", default=None, help="comma-separated batch sizes")
    ap.add_argument("--sweep-epochs", default=None, help="comma-separated epoch counts")
    args = ap.parse_args(argv)
    sizes = (synth.CONFIG_SIZES[args.config] if args.sizes is None else
             {"small": synth.SIZES_SMALL, "large": synth.SIZES_LARGE, "tiny": synth.SIZES_TINY,
              "l8": synth.SIZES_L8}[args.sizes])
    structures = synth.config_structures(args.config, n_struct=args.structures)
    labels = teacher_labels(sizes, structures, synth.SEEDS["teacher"], synth.SEEDS["noise"])
    print(f"[train] {args.config}: {len(structures)} structures, {sum(s.n for s in structures)} atoms",
          file=sys.stderr, flush=True)
    if args.sweep_batch:
        for bs in [int(x) for x in args.sweep_batch.split(",")]:
            print(json.dumps(_run(args, sizes, structures, labels, bs, args.epochs, log_epochs=False)), flush=True)
    elif args.sweep_epochs:
        for ep in [int(x) for x in args.sweep_epochs.split(",")]:
            print(json.dumps(_run(args, sizes, structures, labels, args.batch_size, ep, log_epochs=False)),
                  flush=True)
    else:
        print(json.dumps(_run(args, sizes, structures, labels, args.batch_size, args.epochs)), flush=True)


if __name__ == "__main__":
    main()
