"""The persistent train step (NEP_GRAPH_PERSISTENT: species order, forward,
force gather, per-structure sums and loss, adjoint, gradient reductions and
Adam in one launch with a software grid barrier) against the FP64 oracle and
against the graph of separate launches, through the C ABI.

Bars as in the other parity tests: loss rtol 1e-4, every gradient block 1e-4
norm-wise; parameters after several replays (Adam on both paths) 1e-5
relative to their size."""
import json
import os

import numpy as np
import pytest

from paper_2507_00528_amd import synth

from gpu_util import TOL_F, Case, DeviceRun, param_blocks, rel, structures

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _graph(nep, model, dev, labels, lam, theta, N, S, persistent, lr=1e-3):
    import torch
    P = theta.numel()
    st = dict(params=theta.clone(), m=torch.zeros(P, device="cuda"), v=torch.zeros(P, device="cuda"),
              grad=torch.zeros(P, device="cuda"), loss=torch.zeros(4, device="cuda"),
              step=torch.ones(1, dtype=torch.int32, device="cuda"),
              nb=nep.Neighbors(model, N), ws=nep.workspace(model, S, N),
              flags=torch.zeros(1, dtype=torch.int32, device="cuda"))
    st["graph"] = nep.TrainStepGraph(model, dev, st["nb"], labels, lam, st["params"], st["m"], st["v"], st["grad"],
                                     st["loss"], st["step"], st["ws"], st["flags"], lr_start=lr, lr_stop=lr,
                                     persistent=persistent)
    return st


def _replay(st):
    import torch
    st["graph"].launch()
    torch.cuda.synchronize()
    assert int(st["flags"].item()) == 0
    return st["loss"].cpu().numpy().copy(), st["grad"].cpu().numpy().copy(), st["params"].cpu().numpy().copy()


@pytest.mark.parametrize("name", ["c0", "c2_head", "mono"])
def test_persistent_step_matches_oracle_and_separate_launches(name):
    rng = np.random.default_rng(5)
    if name == "c0":
        case = Case(synth.SIZES_SMALL, synth.config_structures("c0"))
    elif name == "c2_head":
        case = Case(synth.SIZES_LARGE, synth.config_structures("c2", n_struct=12))
    else:
        small = [synth.random_structure(rng, n, 0.031, 2.4, "liquid") for n in (10, 13, 40)]
        case = Case(synth.SIZES_MONO, [synth.Structure(s.pos, s.box, np.zeros(s.n, np.int32)) for s in small])
    r = DeviceRun(case)
    print(f"[persistent {name}] S={r.S} N={r.N}", flush=True)
    pers = _graph(r.nep, r.model, r.batch, r.labels, case.lam, r.params, r.N, r.S, True)
    sep = _graph(r.nep, r.model, r.batch, r.labels, case.lam, r.params, r.N, r.S, False)
    for k in range(3):
        lp, gp, pp = _replay(pers)
        ls, gs, ps = _replay(sep)
        if k == 0:
            np.testing.assert_allclose(lp, case.loss, rtol=1e-4)
            for blk, sl in param_blocks(case.sizes).items():
                assert rel(gp[sl], case.grad[sl]) < TOL_F, (blk, "oracle")
        np.testing.assert_allclose(lp, ls, rtol=1e-5)
        for blk, sl in param_blocks(case.sizes).items():
            assert rel(gp[sl], gs[sl]) < TOL_F, (blk, k)
        np.testing.assert_allclose(pp, ps, rtol=0, atol=1e-5 * np.abs(ps).max())
    pers["graph"].close()
    sep["graph"].close()


@pytest.mark.parametrize("name", ["c2", "c3", "c4"])
def test_persistent_step_full_size_against_golden(name):
    """The full workloads (c3 through the cell-list search and chunked
    per-structure sums) against the oracle's golden loss and gradient."""
    import torch
    from paper_2507_00528_amd import nep
    gd = np.load(os.path.join(HERE, "golden", f"full_{name}.npz"))
    meta = json.load(open(os.path.join(HERE, "golden", f"full_{name}.json")))
    batch = synth.Batch(structures(name))
    N, S = batch.n_atom, batch.n_struct
    print(f"[persistent full {name}] S={S} N={N}", flush=True)
    sz = synth.CONFIG_SIZES[name]
    model = nep.Model.of(sz)
    dev = nep.DeviceBatch(batch)
    theta = torch.tensor(synth.draw_params(sz.n_params, synth.SEEDS["student"]), device="cuda")
    e_t, f_t, w_t = synth.random_labels(batch, synth.SEEDS["labels"])
    labels = nep.Labels(*(torch.tensor(x, device="cuda") for x in (e_t, f_t, w_t)))
    st = _graph(nep, model, dev, labels, meta["lambda"], theta, N, S, True)
    loss, grad, _ = _replay(st)
    np.testing.assert_allclose(loss, gd["loss"], rtol=1e-4)
    for blk, sl in param_blocks(sz).items():
        assert rel(grad[sl], gd["grad"][sl]) < TOL_F, blk
    # a second replay (new step, new parameters) still runs to completion
    _replay(st)
    st["graph"].close()


def test_persistent_step_rejects_what_it_does_not_cover():
    """Triclinic batches and models with degrees l > 4 are refused on the
    host (the separate launches cover them)."""
    import torch
    from paper_2507_00528_amd import nep
    rng = np.random.default_rng(9)
    tri = [synth.triclinic_structure(rng, 40, 0.031, 2.5)]
    for sizes, sts in ((synth.SIZES_LARGE, tri), (synth.SIZES_L8, synth.config_structures("c0"))):
        case = Case(sizes, sts, with_oracle=False)
        r = DeviceRun(case)
        with pytest.raises(nep.NEPError) as e:
            _graph(nep, r.model, r.batch, r.labels, case.lam, r.params, r.N, r.S, True)
        assert e.value.code == -1
    torch.cuda.synchronize()
