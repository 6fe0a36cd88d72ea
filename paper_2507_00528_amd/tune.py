"""Autotuner of the captured train step's launch choices (nep_tuning).

For one model and batch it times replays of the captured step (HIP events on
the replay stream; median of `reps` replays after warm-up) and searches the
choices one at a time: starting from the library's defaults, each choice is
swept with the others held, and a value is kept only when it is faster by
more than `min_gain`; passes repeat until one changes nothing.  The choices
are cached per size class (model sizes and capacities, cell shape, atom count
rounded to a power of two, largest structure below or at least 1024 atoms)
in tuning.json next to this file; graph creation (nep.TrainStepGraph) reads
that cache.

    python -m paper_2507_00528_amd.tune --workload c2 c3 c4 [--reps 30] [--out FILE]

None of the choices changes a result beyond the order of floating-point
sums; tests/test_gpu_tuning.py runs the parity checks on tuned choices.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")

# values tried per choice (the library default first)
SPACE = {
    "persistent": [0, 1],
    "adjoint_waves": [3, 2],
    "forward_waves": [3, 2],
    "outer_blocks_w": [192, 96, 128, 256, 384],
    "outer_blocks_c": [64, 32, 128],
    "reduce_chunks": [128, 64, 256],
    "gather_lanes": [16, 8],
    "cell_min_atoms": [1024, 512, 2048],
    "reverse_branch": [1, 2],
}
DEFAULTS = {k: v[0] for k, v in SPACE.items()}

_cache = None


def size_class(model, batch) -> str:
    """Key of the batch's size class for this model."""
    n = max(int(batch.n_atom), 1)
    big = batch.max_atoms == 0 or batch.max_atoms >= 1024
    tri = getattr(batch, "tilt", None) is not None
    return (f"T{model.n_types}-R{model.n_rad}x{model.k_rad}-A{model.n_ang}x{model.k_ang}"
            f"-l{model.l3}.{model.l4}.{model.l5}-H{model.hidden}-cap{model.cap_rad}.{model.cap_ang}"
            f"-{'tri' if tri else 'orth'}-N2^{round(math.log2(n))}-{'large' if big else 'small'}")


def load_cache(path=CACHE) -> dict:
    global _cache
    if path == CACHE and _cache is not None:
        return _cache
    d = json.load(open(path)) if os.path.exists(path) else {}
    if path == CACHE:
        _cache = d
    return d


def lookup(model, batch, path=CACHE):
    """The cached choices for this model and batch, or None."""
    e = load_cache(path).get(size_class(model, batch))
    return dict(e["tuning"]) if e else None


def search(measure, space=None, min_gain=0.01, max_passes=3, log=None):
    """Coordinate search.  measure(choices) -> ms (None: the choices are not
    available for this batch).  Returns (best choices, best ms, default ms,
    every measurement as (choices, ms))."""
    space = space or SPACE
    best = {k: v[0] for k, v in space.items()}
    seen = {}

    def run(c):
        key = tuple(sorted(c.items()))
        if key not in seen:
            seen[key] = measure(dict(c))
            if log:
                log(f"  {c} -> {seen[key]}")
        return seen[key]

    base = run(best)
    best_ms = base
    for _ in range(max_passes):
        changed = False
        for k, vals in space.items():
            for v in vals:
                if v == best[k]:
                    continue
                cand = dict(best, **{k: v})
                ms = run(cand)
                if ms is not None and ms < best_ms * (1.0 - min_gain):
                    best, best_ms, changed = cand, ms, True
        if not changed:
            break
    return best, best_ms, base, [(dict(k), v) for k, v in seen.items()]


def nondefault(choices: dict, space=None) -> dict:
    """Only the choices that differ from the defaults (the first value of each
    choice in `space`), the form the cache keeps."""
    d = {k: v[0] for k, v in (space or SPACE).items()}
    return {k: v for k, v in choices.items() if d.get(k, DEFAULTS.get(k)) != v}


def time_graph(nep, model, dev, labels, lam, theta, N, S, choices, reps, stream, warmup=3):
    """Median ms of `reps` replays of the captured step with these choices
    (learning rate 0: the parameters stay put), or None when the library
    refuses the choices for this batch."""
    import numpy as np
    import torch
    P = theta.numel()
    params = theta.clone()
    m, v, grad = (torch.zeros(P, device="cuda") for _ in range(3))
    loss = torch.zeros(4, device="cuda")
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    nb = nep.Neighbors(model, N)
    ws = nep.workspace(model, S, N)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    try:
        g = nep.TrainStepGraph(model, dev, nb, labels, lam, params, m, v, grad, loss, step, ws, flags,
                               lr_start=0.0, lr_stop=0.0, stream=stream, tuning=choices)
    except nep.NEPError:
        return None
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            g.launch(stream)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        evs[0].record(stream)
        for k in range(reps):
            g.launch(stream)
            evs[k + 1].record(stream)
    stream.synchronize()
    nep.check_flags(flags, f"tuning {choices}")
    g.close()
    return float(np.median([evs[k].elapsed_time(evs[k + 1]) for k in range(reps)]))


def tune_workload(name, reps, log):
    import torch
    from . import nep, synth
    sizes = synth.SIZES_L8 if name == "l8" else synth.CONFIG_SIZES[name]
    sts = synth.config_structures("c2" if name == "l8" else name)
    batch = synth.Batch(sts)
    model = nep.Model.of(sizes)
    dev = nep.DeviceBatch(batch)
    N, S = batch.n_atom, batch.n_struct
    theta = torch.tensor(synth.draw_params(sizes.n_params, synth.SEEDS["student"]), device="cuda")
    e_t, f_t, w_t = synth.random_labels(batch, synth.SEEDS["labels"])
    labels = nep.Labels(*(torch.tensor(x, device="cuda") for x in (e_t, f_t, w_t)))
    stream = torch.cuda.Stream()
    space = dict(SPACE)
    if dev.max_atoms < 512:          # no structure reaches any cell-list threshold tried
        space.pop("cell_min_atoms")
    if sizes.l3 > 4:                 # the library's adjoint default with degrees l > 4
        space["adjoint_waves"] = [2, 3]
    log(f"[tune] {name}: {S} structures, {N} atoms, class {size_class(model, dev)}")
    t0 = time.time()
    best, best_ms, base_ms, table = search(
        lambda c: time_graph(nep, model, dev, labels, (1.0, 1.0, 0.1), theta, N, S, c, reps, stream), space,
        log=log)
    log(f"[tune] {name}: default {base_ms:.4f} ms -> tuned {best_ms:.4f} ms {nondefault(best, space)} "
        f"({len(table)} settings, {time.time() - t0:.0f} s)")
    return size_class(model, dev), {"tuning": nondefault(best, space), "ms": best_ms, "default_ms": base_ms,
                                    "workload": name, "atoms": N, "structures": S,
                                    "measurements": [{"choices": nondefault(c, space), "ms": ms} for c, ms in table]}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", nargs="+", default=["c2", "c3", "c4"])
    ap.add_argument("--reps", type=int, default=30)
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, flush=True)

    out = load_cache(args.out) if os.path.exists(args.out) else {}
    for w in args.workload:
        key, entry = tune_workload(w, args.reps, log)
        out[key] = entry
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
