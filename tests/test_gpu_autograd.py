"""The adjoint kernels behind torch.autograd (NEPFunction) on 64 uneven
structures of 48-320 atoms (rocksalt-like, liquid, amorphous; 3-body NEP):
gradients against the FP64 oracle, against FP64 central differences on 50
random parameters over all 64 structures (each parameter against its own
difference), and 200 Adam steps."""
import numpy as np
import pytest

from paper_2507_00528_amd import synth

from gpu_util import TOL_F, Case, param_blocks, rel

pytestmark = pytest.mark.gpu

_STATE = {}


def state():
    if not _STATE:
        import torch
        from paper_2507_00528_amd import autograd as ag, nep
        sts = synth.config_structures("c1")
        case = Case(synth.SIZES_SMALL, sts)
        print(f"[c1] S={case.batch.n_struct} N={case.batch.n_atom}", flush=True)
        model = nep.Model.of(synth.SIZES_SMALL)
        eng = ag.NEPEngine(model, case.batch)
        eng.build_neighbors()
        labels = nep.Labels(torch.tensor(case.labels["energy"], dtype=torch.float32, device="cuda"),
                            torch.tensor(np.ascontiguousarray(case.labels["force"].T).reshape(-1),
                                         dtype=torch.float32, device="cuda"),
                            torch.tensor(case.labels["virial"].reshape(-1), dtype=torch.float32, device="cuda"))
        _STATE.update(case=case, eng=eng, labels=labels)
    return _STATE


def test_autograd_gradient_matches_oracle_and_loss_grad():
    import torch
    from paper_2507_00528_amd import autograd as ag, nep
    st = state()
    case, eng, labels = st["case"], st["eng"], st["labels"]
    params = torch.tensor(case.theta, device="cuda", requires_grad=True)
    L, le, lf, lv = ag.nep_loss(eng, params, labels, case.lam)
    L.backward()
    g = params.grad.detach().cpu().numpy()
    np.testing.assert_allclose([float(L), float(le), float(lf), float(lv)], case.loss, rtol=1e-4)
    for blk, sl in param_blocks(case.sizes).items():
        assert rel(g[sl], case.grad[sl]) < TOL_F, blk
    # the fused loss-and-gradient call gives the same gradient
    loss = torch.zeros(4, device="cuda")
    grad = torch.zeros(eng.P, device="cuda")
    nep.loss_grad(eng.model, eng.batch, eng.nbrs, params.detach(), labels, case.lam, loss, grad, eng.ws, eng.flags)
    assert rel(grad.cpu().numpy(), g) < 1e-5


def test_autograd_gradient_against_fp64_central_differences():
    """50 seeded parameters, central differences (h = 1e-5) of the FP64 oracle
    loss over all 64 structures, read from tests/golden/fd_c1.npz (written by
    tests/golden/make_fd_c1.py, which calls only the oracle).  Each parameter
    is compared with its own difference:
        |g_k - fd_k| <= 1e-4 |fd_k| + 3 t_k + 1e-5 max|fd|,
    t_k = |fd_k(h) - fd_k(2h)| / 3 the truncation estimate of the difference and
    1e-5 max|fd| the FP32 floor (sums over about 1.2e4 atoms carry about
    sqrt(1.2e4) 2^-24 ~ 7e-6 of the largest term), besides the block-wise
    norm test."""
    import os
    import torch
    from paper_2507_00528_amd import autograd as ag
    st = state()
    case, eng, labels = st["case"], st["eng"], st["labels"]
    gold = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_c1.npz"))
    assert int(gold["n_struct"]) == case.batch.n_struct == 64
    assert int(gold["n_atom"]) == case.batch.n_atom
    idx = gold["idx"]
    expect = np.random.default_rng(synth.SEEDS["fd"]).choice(case.sizes.n_params, 50, replace=False)
    assert np.array_equal(idx, expect)
    np.testing.assert_allclose(gold["loss"], case.loss, rtol=1e-12)
    p = torch.tensor(case.theta, device="cuda", requires_grad=True)
    L, *_ = ag.nep_loss(eng, p, labels, case.lam)
    L.backward()
    g = p.grad.detach().cpu().numpy()[idx].astype(np.float64)
    fd, fd2 = gold["fd"], gold["fd_2h"]
    trunc = np.abs(fd - fd2) / 3
    err = np.abs(g - fd)
    bound = 1e-4 * np.abs(fd) + 3 * trunc + 1e-5 * np.abs(fd).max()
    worst = int(np.argmax(err / bound))
    print(f"[c1 fd] max |g - fd| {err.max():.3e}, max |fd| {np.abs(fd).max():.3e}, "
          f"worst ratio {err[worst] / bound[worst]:.3f} at param {int(idx[worst])} "
          f"(g {g[worst]:.6e} fd {fd[worst]:.6e})", flush=True)
    assert np.all(err <= bound), [(int(idx[k]), g[k], fd[k]) for k in np.nonzero(err > bound)[0]]
    assert rel(g, fd) < TOL_F


def test_200_adam_steps_through_autograd():
    import torch
    from oracle import adam_step as oracle_adam
    from paper_2507_00528_amd import autograd as ag, nep
    st = state()
    case, eng, labels = st["case"], st["eng"], st["labels"]
    params = torch.tensor(case.theta, device="cuda", requires_grad=True)
    m = torch.zeros(eng.P, device="cuda")
    v = torch.zeros(eng.P, device="cuda")
    losses = []
    ref = (case.theta.astype(np.float64), np.zeros(eng.P), np.zeros(eng.P))
    for step in range(1, 201):
        params.grad = None
        L, *_ = ag.nep_loss(eng, params, labels, case.lam)
        L.backward()
        losses.append(float(L))
        if step == 1:
            # first update against the oracle's Adam on the oracle gradient
            ref = oracle_adam(*ref, case.grad, 1, 1e-3)
        nep.adam_step(params.data, m, v, params.grad, 1e-3, step)
        if step == 1:
            # well-conditioned entries (|g| well above Adam's eps) move like the oracle's step
            big = np.abs(case.grad) > 1e-4 * np.abs(case.grad).max()
            d_gpu = params.detach().cpu().numpy()[big] - case.theta[big]
            assert rel(d_gpu, (ref[0] - case.theta)[big]) < 1e-3
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])
