"""Training driver on the GPU: captured mini-batch steps with the Eq. 17
learning rate equal the eager library calls, and training on synthetic
teacher labels lowers the loss and the RMSE (fixed and reshuffled batches)."""
import numpy as np
import pytest

from paper_2507_00528_amd import synth

pytestmark = pytest.mark.gpu


def data(n=16):
    from paper_2507_00528_amd.train import teacher_labels
    sts = synth.config_structures("c1", n_struct=n)
    lab = teacher_labels(synth.SIZES_SMALL, sts, synth.SEEDS["teacher"], synth.SEEDS["noise"])
    return sts, lab


def test_graph_epochs_equal_eager_steps_with_eq17_rate():
    import torch
    from paper_2507_00528_amd import nep
    from paper_2507_00528_amd.train import Trainer, _device_labels
    sts, lab = data(6)
    sz = synth.SIZES_SMALL
    theta = synth.draw_params(sz.n_params, synth.SEEDS["student"])
    print(f"[train graph] S={len(sts)}", flush=True)
    tr = Trainer(sz, sts, lab, theta, batch_size=len(sts), epochs=4, warmup_epochs=1, lr_start=2e-3, lr_stop=1e-4)
    for _ in range(3):
        tr.train_epoch()
    torch.cuda.synchronize()
    model = nep.Model.of(sz)
    b = synth.Batch(sts)
    db = nep.DeviceBatch(b)
    nb = nep.Neighbors(model, b.n_atom)
    ws = nep.workspace(model, b.n_struct, b.n_atom)
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    labels = _device_labels(lab, "cuda")
    p = torch.tensor(theta, device="cuda")
    m, v, g = (torch.zeros(sz.n_params, device="cuda") for _ in range(3))
    loss = torch.zeros(4, device="cuda")
    for s in range(1, 4):
        nep.build_neighbors(model, db, nb, ws, fl)
        nep.loss_grad(model, db, nb, p, labels, (1.0, 1.0, 0.1), loss, g, ws, fl)
        nep.adam_step(p, m, v, g, nep.lr_schedule(s - 1, 2e-3, 1e-4, 1, 4), s)
    torch.cuda.synchronize()
    np.testing.assert_allclose(tr.params.cpu().numpy(), p.cpu().numpy(), rtol=0, atol=1e-6)
    assert int(tr.step.item()) == 4
    tr.close()


@pytest.mark.parametrize("reshuffle", [False, True])
def test_training_lowers_loss_and_rmse(reshuffle):
    from paper_2507_00528_amd.train import Trainer
    sts, lab = data(16)
    sz = synth.SIZES_SMALL
    print(f"[train] reshuffle={reshuffle} S={len(sts)}", flush=True)
    tr = Trainer(sz, sts, lab, synth.draw_params(sz.n_params, synth.SEEDS["student"]), batch_size=1, epochs=6,
                 warmup_epochs=0.5, lr_start=3e-3, lr_stop=1e-4, reshuffle=reshuffle, seed=5)
    ev0 = tr.evaluate()
    hist = [tr.train_epoch() for _ in range(6)]
    ev1 = tr.evaluate()
    assert all(np.isfinite(h["loss"]) for h in hist)
    assert hist[-1]["loss"] < 0.5 * hist[0]["loss"], [h["loss"] for h in hist]
    assert ev1["rmse_f"] < ev0["rmse_f"] and ev1["rmse_e"] < ev0["rmse_e"], (ev0, ev1)
    assert hist[-1]["steps"] == 6 * 16
    tr.close()


def test_training_with_high_degrees_and_tilted_cells():
    """The training driver with 3-body degrees up to l = 8 on a mix of
    orthorhombic and triclinic cells lowers the loss and the force RMSE."""
    from paper_2507_00528_amd.train import Trainer, teacher_labels
    rng = np.random.default_rng(12)
    sts = synth.config_structures("c1", n_struct=6) + [synth.triclinic_structure(rng, n, 0.031, 2.3, 0.3)
                                                        for n in (60, 90, 120)]
    sz = synth.SIZES_L8
    lab = teacher_labels(sz, sts, synth.SEEDS["teacher"], synth.SEEDS["noise"])
    print(f"[train l8] S={len(sts)}", flush=True)
    tr = Trainer(sz, sts, lab, synth.draw_params(sz.n_params, synth.SEEDS["student"]), batch_size=3, epochs=8,
                 warmup_epochs=0.5, lr_start=3e-3, lr_stop=1e-4, seed=3)
    ev0 = tr.evaluate()
    hist = [tr.train_epoch() for _ in range(8)]
    ev1 = tr.evaluate()
    assert all(np.isfinite(h["loss"]) for h in hist)
    assert hist[-1]["loss"] < 0.5 * hist[0]["loss"], [h["loss"] for h in hist]
    assert ev1["rmse_f"] < ev0["rmse_f"], (ev0, ev1)
    tr.close()
