"""Parity of the captured train step on launch choices other than the
defaults (nep_tuning), through the C ABI: against the FP64 oracle on small
batches, and, for the autotuner's cached choices of the full workloads,
against the oracle's golden loss and gradient."""
import json
import os

import numpy as np
import pytest

from paper_2507_00528_amd import synth, tune

from gpu_util import TOL_F, Case, DeviceRun, param_blocks, rel, structures

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

CHOICES = [
    {"outer_blocks_w": 96, "outer_blocks_c": 32, "reduce_chunks": 64, "gather_lanes": 8, "forward_waves": 2,
     "adjoint_waves": 2, "reverse_branch": 2},
    {"outer_blocks_w": 384, "outer_blocks_c": 128, "reduce_chunks": 256, "cell_min_atoms": 512, "reverse_branch": 2},
    {"persistent": 1, "outer_blocks_w": 128, "reduce_chunks": 64},
]


def _step(r, choices):
    import torch
    nep = r.nep
    P = r.params.numel()
    grad = torch.zeros(P, device="cuda")
    loss = torch.zeros(4, device="cuda")
    params = r.params.clone()
    m, v = torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda")
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    nb = nep.Neighbors(r.model, r.N)
    ws = nep.workspace(r.model, r.S, r.N)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    g = nep.TrainStepGraph(r.model, r.batch, nb, r.labels, r.case.lam, params, m, v, grad, loss, step, ws, flags,
                           tuning=choices)
    g.launch()
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    g.close()
    return loss.cpu().numpy(), grad.cpu().numpy()


@pytest.mark.parametrize("k", range(len(CHOICES)))
def test_tuned_choices_match_oracle(k):
    """A batch with one 600-atom structure (cell-list search from 512 atoms)
    among small ones."""
    rng = np.random.default_rng(17)
    sts = synth.config_structures("c2", n_struct=6) + [synth.random_structure(rng, 600, 0.031, 2.7, "amorphous")]
    case = _case_cache(sts)
    r = DeviceRun(case)
    print(f"[tuning {CHOICES[k]}] S={r.S} N={r.N}", flush=True)
    loss, grad = _step(r, CHOICES[k])
    np.testing.assert_allclose(loss, case.loss, rtol=1e-4)
    for blk, sl in param_blocks(case.sizes).items():
        assert rel(grad[sl], case.grad[sl]) < TOL_F, blk


_CASE = {}


def _case_cache(sts):
    if "c" not in _CASE:
        _CASE["c"] = Case(synth.SIZES_LARGE, sts)
    return _CASE["c"]


@pytest.mark.parametrize("name", ["c2", "c3", "c4"])
def test_cached_choices_full_size_against_golden(name):
    import torch
    from paper_2507_00528_amd import nep
    batch = synth.Batch(structures(name))
    sz = synth.CONFIG_SIZES[name]
    model = nep.Model.of(sz)
    dev = nep.DeviceBatch(batch)
    choices = tune.lookup(model, dev)
    if not choices:
        pytest.skip(f"no cached choices for {tune.size_class(model, dev)}")
    gd = np.load(os.path.join(HERE, "golden", f"full_{name}.npz"))
    meta = json.load(open(os.path.join(HERE, "golden", f"full_{name}.json")))
    N, S = batch.n_atom, batch.n_struct
    print(f"[cached tuning {name}] {choices} S={S} N={N}", flush=True)
    theta = torch.tensor(synth.draw_params(sz.n_params, synth.SEEDS["student"]), device="cuda")
    e_t, f_t, w_t = synth.random_labels(batch, synth.SEEDS["labels"])
    labels = nep.Labels(*(torch.tensor(x, device="cuda") for x in (e_t, f_t, w_t)))
    P = sz.n_params
    grad, loss = torch.zeros(P, device="cuda"), torch.zeros(4, device="cuda")
    m, v = torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda")
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    nb = nep.Neighbors(model, N)
    ws = nep.workspace(model, S, N)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    g = nep.TrainStepGraph(model, dev, nb, labels, meta["lambda"], theta.clone(), m, v, grad, loss, step, ws, flags)
    assert g.tuning == choices
    g.launch()
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    np.testing.assert_allclose(loss.cpu().numpy(), gd["loss"], rtol=1e-4)
    gg = grad.cpu().numpy()
    for blk, sl in param_blocks(sz).items():
        assert rel(gg[sl], gd["grad"][sl]) < TOL_F, blk
    g.close()


def test_reverse_branch_replays_equal_single_stream():
    """The captured step with the reverse index on its own branch (a second
    stream joined before the force gather) gives, replay after replay with
    eager work in between, bit for bit the loss, gradient and Adam update of
    the single-stream step: the branch only moves the launch."""
    import torch
    from paper_2507_00528_amd import nep
    rng = np.random.default_rng(17)
    sts = synth.config_structures("c2", n_struct=6) + [synth.random_structure(rng, 600, 0.031, 2.7, "amorphous")]
    case = _case_cache(sts)
    r = DeviceRun(case)
    P = r.params.numel()
    print(f"[reverse branch] S={r.S} N={r.N}", flush=True)

    def make(choice):
        st = dict(params=r.params.clone(), m=torch.zeros(P, device="cuda"), v=torch.zeros(P, device="cuda"),
                  grad=torch.zeros(P, device="cuda"), loss=torch.zeros(4, device="cuda"),
                  step=torch.ones(1, dtype=torch.int32, device="cuda"),
                  flags=torch.zeros(1, dtype=torch.int32, device="cuda"))
        st["g"] = nep.TrainStepGraph(r.model, r.batch, nep.Neighbors(r.model, r.N), r.labels, case.lam,
                                     st["params"], st["m"], st["v"], st["grad"], st["loss"], st["step"],
                                     nep.workspace(r.model, r.S, r.N), st["flags"], lr_start=1e-3, lr_stop=1e-3,
                                     tuning={"reverse_branch": choice})
        return st

    one, two = make(1), make(2)
    for _ in range(3):
        one["g"].launch()
        two["g"].launch()
        torch.cuda.synchronize()
        # eager work between replays
        nep.build_neighbors(r.model, r.batch, r.nbrs, r.ws, r.flags)
        torch.cuda.synchronize()
        for k in ("loss", "grad", "params", "m", "v"):
            assert torch.equal(one[k], two[k]), k
        assert int(one["flags"].item()) == 0 and int(two["flags"].item()) == 0
    assert int(two["step"].item()) == 4
    one["g"].close()
    two["g"].close()
