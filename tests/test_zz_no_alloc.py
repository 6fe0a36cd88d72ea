"""nep_loss_grad_noalloc (static device scratch, no allocation) against the
workspace path nep_build_neighbors + nep_loss_grad, through the C ABI: two
calls in a row on the same GPU, the second on a smaller batch, so the second
runs on scratch that still holds the first call's contents.  Lists bit-exact;
loss, energies, forces, virials and every gradient block within the parity
bars (and the first call also against the FP64 oracle)."""
import numpy as np
import pytest

from paper_2507_00528_amd import synth

from gpu_util import TOL_E, TOL_F, Case, DeviceRun, param_blocks, rel

pytestmark = pytest.mark.gpu


def _run_noalloc(r):
    import torch
    nep = r.nep
    nb = nep.Neighbors(r.model, r.N)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    loss = torch.zeros(4, device="cuda")
    grad = torch.zeros(r.params.numel(), device="cuda")
    e_s = torch.zeros(r.S, device="cuda")
    F = torch.zeros(3 * r.N, device="cuda")
    W = torch.zeros(6 * r.S, device="cuda")
    nep.loss_grad_noalloc(r.model, r.batch, nb, r.params, r.labels, r.case.lam, loss, grad, flags, e_s, F, W)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    return (nb, loss.cpu().numpy(), grad.cpu().numpy(), e_s.cpu().numpy(), F.cpu().numpy().reshape(3, -1).T,
            W.cpu().numpy().reshape(-1, 6))


def _compare(r, got, want, sizes):
    nb, loss, grad, e_s, F, W = got
    loss_w, grad_w, e_w, F_w, W_w = want
    for which in ("rad", "ang"):
        ref, cnt_ref = r.lists(which)
        idx = (nb.idx_rad if which == "rad" else nb.idx_ang).cpu().numpy().view(np.uint32)
        cnt = (nb.cnt_rad if which == "rad" else nb.cnt_ang).cpu().numpy()
        cap = r.model.cap_rad if which == "rad" else r.model.cap_ang
        idx = idx.reshape(max(r.N, 1), cap)
        assert np.array_equal(cnt[:r.N], cnt_ref[:r.N]), which
        for i in range(r.N):
            assert [int(v) for v in idx[i, :min(cnt[i], cap)]] == [int(v) for v in ref[i]], (which, i)
    np.testing.assert_allclose(loss, loss_w, rtol=1e-5, atol=1e-12)
    n_at = np.diff(r.case.batch.atom_offset)
    assert rel(e_s / np.maximum(n_at, 1), e_w / np.maximum(n_at, 1)) < TOL_E
    assert rel(F, F_w) < TOL_F
    assert rel(W, W_w) < TOL_F
    for name, sl in param_blocks(sizes).items():
        assert rel(grad[sl], grad_w[sl]) < TOL_F, name


def test_noalloc_matches_workspace_path_twice_second_smaller():
    rng = np.random.default_rng(71)
    first = synth.config_structures("c2", n_struct=24)      # about 3,000 atoms, 3/4/5-body model
    second = [synth.random_structure(rng, n, 0.031, 2.5, "amorphous") for n in (17, 40, 96)]
    for k, sts in enumerate((first, second)):
        case = Case(synth.SIZES_LARGE, sts, with_oracle=(k == 0))
        r = DeviceRun(case)
        print(f"[noalloc call {k + 1}] S={r.S} N={r.N}", flush=True)
        got = _run_noalloc(r)
        r.neighbors()
        want = r.loss_grad()
        _compare(r, got, want, case.sizes)
        if k == 0:
            loss, grad = got[1], got[2]
            np.testing.assert_allclose(loss, case.loss, rtol=1e-4)
            for name, sl in param_blocks(case.sizes).items():
                assert rel(grad[sl], case.grad[sl]) < TOL_F, name


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    import torch
    from paper_2507_00528_amd import nep
    sts = synth.config_structures("c1")
    big = synth.Batch(sts * 2)                               # about 24,000 atoms: beyond 64 MiB
    model = nep.Model.of(synth.SIZES_LARGE)
    assert nep.workspace_bytes(model, big.n_struct, big.n_atom) > nep.STATIC_SCRATCH_BYTES
    db = nep.DeviceBatch(big)
    nb = nep.Neighbors(model, big.n_atom)
    P = nep.param_count(model)
    z = lambda n: torch.zeros(n, device="cuda")
    labels = nep.Labels(z(big.n_struct), z(3 * big.n_atom), z(6 * big.n_struct))
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(nep.NEPError) as e:
        nep.loss_grad_noalloc(model, db, nb, z(P), labels, (1.0, 1.0, 0.1), z(4), z(P), flags)
    assert e.value.code == -9
    torch.cuda.synchronize()
    assert int(flags.item()) == 0                            # nothing was launched
