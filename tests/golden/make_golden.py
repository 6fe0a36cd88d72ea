"""Expected values for the full-size GPU parity tests, written by the FP64
oracle only.

    python tests/golden/make_golden.py c2 c3 c4

For each workload: seeded structures (synth.config_structures), student
parameters, seeded random labels (synth.random_labels), and from the oracle:
the loss and its gradient, per-structure energies and virials, energies and
forces of 256 sampled atoms, energies and forces of every atom of sampled
whole structures (the largest structure and up to 31 (c2) or 63 (c4) more;
the single c3 cell whole), per-atom neighbor counts and a SHA-256 digest of
the canonical neighbor lists (i, j, code as int64, global atom indices).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import NEPOracle  # noqa: E402
from paper_2507_00528_amd import synth  # noqa: E402

LAM = (1.0, 1.0, 0.1)


def canonical_digest(lists):
    arr = np.concatenate(lists, 0).astype(np.int64) if lists else np.zeros((0, 3), np.int64)
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


def make(name):
    t0 = time.time()
    sts = synth.config_structures(name)
    batch = synth.Batch(sts)
    sz = synth.CONFIG_SIZES[name]
    o = NEPOracle(sz)
    theta = synth.draw_params(sz.n_params, synth.SEEDS["student"])
    e_t, f_t, w_t = synth.random_labels(batch, synth.SEEDS["labels"])
    N, S = batch.n_atom, batch.n_struct
    offs = batch.atom_offset
    nbrs, glob_r, glob_a = [], [], []
    cnt_r = np.zeros(N, np.int32)
    cnt_a = np.zeros(N, np.int32)
    for k, st in enumerate(sts):
        pr, pa = o.neighbors(st)
        nbrs.append((pr, pa))
        base = int(offs[k])
        for p, cnt, glob in ((pr, cnt_r, glob_r), (pa, cnt_a, glob_a)):
            g = p.copy()
            g[:, :2] += base
            glob.append(g)
            np.add.at(cnt, g[:, 0], 1)
    print(f"[{name}] neighbors done {time.time() - t0:.0f}s", flush=True)
    ftl = f_t.reshape(3, N).T.astype(np.float64)
    lab = dict(energy=e_t.astype(np.float64), force=[ftl[offs[k]:offs[k + 1]] for k in range(S)],
               virial=w_t.reshape(S, 6).astype(np.float64))
    pred = o.predict(theta, sts, nbrs)
    loss, grad = o.loss_and_grad(theta, sts, lab, LAM, nbr_cache=nbrs)
    print(f"[{name}] loss and gradient done {time.time() - t0:.0f}s", flush=True)
    F = np.concatenate(pred["F"], 0)
    Ei = np.concatenate(pred["Ei"], 0)
    sample = np.sort(np.random.default_rng(99).choice(N, min(256, N), replace=False))
    # whole structures: the largest, then a seeded draw of the rest
    nst = {"c2": 32, "c4": 64}.get(name, S)
    sizes = np.diff(offs)
    big = int(np.argmax(sizes))
    rest = np.setdiff1d(np.arange(S), [big])
    pick = np.random.default_rng(98).choice(rest, min(nst, S) - 1, replace=False) if S > 1 else rest
    struct_sample = np.sort(np.concatenate([[big], pick]).astype(np.int64))
    atoms = np.concatenate([np.arange(offs[k], offs[k + 1]) for k in struct_sample])
    out = os.path.join(HERE, f"full_{name}.npz")
    np.savez_compressed(out, loss=loss, grad=grad, e_struct=pred["E"], virial=pred["W"], sample=sample,
                        force_sample=F[sample], eatom_sample=Ei[sample], cnt_rad=cnt_r, cnt_ang=cnt_a,
                        struct_sample=struct_sample, struct_natoms=sizes[struct_sample].astype(np.int64),
                        force_struct=F[atoms].astype(np.float32), eatom_struct=Ei[atoms])
    meta = {"workload": name, "n_struct": S, "n_atom": N, "lambda": LAM, "seeds": synth.SEEDS,
            "sha256_rad": canonical_digest(glob_r), "sha256_ang": canonical_digest(glob_a),
            "oracle_seconds": round(time.time() - t0, 1)}
    json.dump(meta, open(os.path.join(HERE, f"full_{name}.json"), "w"), indent=1)
    print(f"[{name}] wrote {out} ({os.path.getsize(out)} bytes)", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["c2", "c3", "c4"]:
        make(name)
