"""Central differences of the FP64 oracle loss on the 64-structure
adjoint-check workload (48-320 atoms per structure, 3-body NEP, teacher labels
plus noise), written by the oracle only.

    python tests/golden/make_fd_c1.py

For 50 seeded parameters k: (L(theta + h e_k) - L(theta - h e_k)) / 2h at
h = 1e-5 and at 2h, on all 64 structures, plus the oracle's own gradient at
those entries.  The difference of the two step sizes estimates the truncation
error of each difference (it falls as h^2), which the GPU test uses as part of
its per-parameter floor.  Output: fd_c1.npz next to this script.
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from gpu_util import Case  # noqa: E402  (inputs and oracle references only)
from paper_2507_00528_amd import synth  # noqa: E402

H = 1e-5
_CASE = {}


def _case():
    if not _CASE:
        sts = synth.config_structures("c1")
        _CASE["case"] = Case(synth.SIZES_SMALL, sts, with_oracle=False)
    return _CASE["case"]


def _init():
    import torch
    torch.set_num_threads(1)
    _case()


def _loss(args):
    k, step = args
    c = _case()
    th = c.theta.astype(np.float64).copy()
    th[k] += step
    lab = dict(energy=c.labels["energy"], force=c.labels_force_list, virial=c.labels["virial"])
    L, _ = c.oracle.loss_and_grad(th, c.structures, lab, c.lam, need_grad=False, nbr_cache=c.nbrs)
    return float(L[0])


def main():
    t0 = time.time()
    c = _case()
    P = c.sizes.n_params
    idx = np.random.default_rng(synth.SEEDS["fd"]).choice(P, 50, replace=False)
    jobs = [(int(k), s * h) for k in idx for h in (H, 2 * H) for s in (1, -1)]
    # spawned workers, one torch thread each (a forked torch thread pool can deadlock)
    with mp.get_context("spawn").Pool(min(8, len(os.sched_getaffinity(0))), initializer=_init) as pool:
        vals = np.array(pool.map(_loss, jobs)).reshape(len(idx), 2, 2)
    fd_h = (vals[:, 0, 0] - vals[:, 0, 1]) / (2 * H)
    fd_2h = (vals[:, 1, 0] - vals[:, 1, 1]) / (4 * H)
    lab = dict(energy=c.labels["energy"], force=c.labels_force_list, virial=c.labels["virial"])
    loss, grad = c.oracle.loss_and_grad(c.theta, c.structures, lab, c.lam, nbr_cache=c.nbrs)
    out = os.path.join(HERE, "fd_c1.npz")
    np.savez_compressed(out, idx=idx, h=H, fd=fd_h, fd_2h=fd_2h, oracle_grad=grad[idx], loss=loss,
                        n_struct=c.batch.n_struct, n_atom=c.batch.n_atom)
    err = np.abs(fd_h - grad[idx])
    print(f"wrote {out}: {c.batch.n_struct} structures, {c.batch.n_atom} atoms; "
          f"max |fd - oracle grad| {err.max():.3e} (max |grad| {np.abs(grad).max():.3e}); "
          f"{time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
