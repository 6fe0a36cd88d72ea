"""A captured training step must not move the optimizer state when its replay
raised a flag: a neighbor-list overflow (lists cut at a small capacity on
purpose; every access stays inside the capacity) or a step counter below 1.
The gradient is still written; params, m and v stay bit-identical."""
import numpy as np
import pytest

from paper_2507_00528_amd import synth

from gpu_util import Case, DeviceRun

pytestmark = pytest.mark.gpu


def _graph_run(cap_rad, cap_ang, step0):
    import torch
    from paper_2507_00528_amd import nep
    c = Case(synth.SIZES_SMALL, synth.config_structures("c0")[:3], with_oracle=False)
    r = DeviceRun(c, cap_rad=cap_rad, cap_ang=cap_ang)
    P = r.params.numel()
    g = torch.Generator(device="cpu").manual_seed(5)
    m = (0.01 * torch.randn(P, generator=g)).cuda()
    v = (1e-3 * torch.rand(P, generator=g)).cuda()
    grad = torch.zeros(P, device="cuda")
    loss = torch.zeros(4, device="cuda")
    step = torch.full((1,), step0, dtype=torch.int32, device="cuda")
    before = (r.params.clone(), m.clone(), v.clone())
    graph = nep.TrainStepGraph(r.model, r.batch, r.nbrs, r.labels, c.lam, r.params, m, v, grad, loss, step, r.ws,
                               r.flags, lr_start=1e-2, lr_stop=1e-2)
    torch.cuda.synchronize()
    graph.launch()
    torch.cuda.synchronize()
    graph.close()
    return r, before, (r.params, m, v), grad, step


def torch_equal(a, b):
    import torch
    return torch.equal(a, b)


def test_overflowing_replay_keeps_params_and_moments():
    from paper_2507_00528_amd import nep
    print("[guard] overflow replay, cap 8/4", flush=True)
    r, before, after, grad, step = _graph_run(8, 4, 3)
    assert int(r.flags.item()) & nep.NEP_FLAG_NBR_OVERFLOW
    for a, b in zip(before, after):
        assert torch_equal(a, b)
    gh = grad.cpu().numpy()
    assert np.all(np.isfinite(gh)) and np.abs(gh).max() > 0
    assert int(step.item()) == 4


def test_step_counter_below_one_keeps_params_and_raises_flag():
    from paper_2507_00528_amd import nep
    print("[guard] step counter 0", flush=True)
    r, before, after, grad, step = _graph_run(64, 32, 0)
    assert int(r.flags.item()) == nep.NEP_FLAG_STEP
    for a, b in zip(before, after):
        assert torch_equal(a, b)
    with pytest.raises(nep.NEPError) as e:
        nep.check_flags(r.flags)
    assert e.value.code == -1


def test_clean_replay_updates_params():
    print("[guard] clean replay", flush=True)
    r, before, after, grad, step = _graph_run(64, 32, 1)
    assert int(r.flags.item()) == 0
    assert not torch_equal(before[0], after[0])
    assert not torch_equal(before[1], after[1])
