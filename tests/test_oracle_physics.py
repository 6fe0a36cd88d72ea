"""Pins of the oracle's neighbor sets, forces, virials, loss and gradient:
brute force by image replication, central finite differences, invariances,
special cases with closed forms, and library optimizers."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

from oracle import NEPOracle, adam_step, lr_schedule, neighbor_pairs, unpack, voigt
from oracle.nep_oracle import SHIFTS
from paper_2507_00528_amd import synth

from _helpers import cluster, small_structures

DT = torch.float64
SZT = synth.SIZES_TINY


# ---------------------------------------------------------------- neighbors
def replicate_neighbors(pos, box, rc):
    """Independent neighbor set: replicate the cell into its 27 images and
    take scipy distances (only used where no pair is within 1e-9 of r_c)."""
    x = pos.astype(np.float64)
    L = box.astype(np.float64)
    out = set()
    margin = False
    for c, s in enumerate(SHIFTS):
        d = cdist(x, x + s * L)
        if np.any(np.abs(d - rc) < 1e-9):
            margin = True
        ii, jj = np.nonzero(d < rc)
        for i, j in zip(ii, jj):
            if not (i == j and c == 13):
                out.add((int(i), int(j), c))
    return out, margin


@pytest.mark.parametrize("n,dmin,seed", [(9, 2.3, 0), (20, 2.5, 1), (64, 2.6, 2), (120, 2.5, 3)])
def test_neighbors_match_replicated_brute_force(n, dmin, seed):
    rng = np.random.default_rng(seed)
    st = synth.random_structure(rng, n, 0.031, dmin, "x")
    for rc in (6.0, 4.0):
        p = neighbor_pairs(st.pos, st.box, rc)
        ref, margin = replicate_neighbors(st.pos, st.box, rc)
        assert not margin
        assert set(map(tuple, p.tolist())) == ref
        # canonical order: (i, j, code) strictly increasing lexicographically
        key = (p[:, 0] * st.n + p[:, 1]) * 27 + p[:, 2]
        assert np.all(np.diff(key) > 0)
        # symmetric: (i, j, s) present iff (j, i, -s) present
        rev = set((j, i, 26 - c) for i, j, c in ref)
        assert rev == ref


def test_neighbors_small_cell_has_multiple_images():
    rng = np.random.default_rng(7)
    st = synth.random_structure(rng, 12, 0.031, 2.4, "x")   # L = 7.3 < 2 r_c
    p = neighbor_pairs(st.pos, st.box, 6.0)
    ij = p[:, 0] * 100 + p[:, 1]
    _, counts = np.unique(ij, return_counts=True)
    assert counts.max() > 1
    assert not np.any(p[:, 0] == p[:, 1])   # L >= r_c: no atom sees its own image


def test_neighbor_predicate_is_strict_and_float64():
    # a pair at exactly r_c is excluded; one ulp inside is included
    box = np.array([20.0, 20.0, 20.0], np.float32)
    pos = np.array([[1.0, 1.0, 1.0], [7.0, 1.0, 1.0], [1.0, 1.0, 1.0]], np.float32)
    pos[2, 0] = np.nextafter(np.float32(7.0), np.float32(0.0))
    pos[2, 1] = 5.0
    p = neighbor_pairs(pos[:2], box, 6.0)
    assert len(p) == 0
    pos2 = pos.copy()
    pos2[1, 0] = np.nextafter(np.float32(7.0), np.float32(0.0))
    p2 = neighbor_pairs(pos2[:2], box, 6.0)
    assert p2.tolist() == [[0, 1, 13], [1, 0, 13]]


# ----------------------------------------------------------------- forces
def fd_energy(o, theta, st, nbrs, x64, L64, strain=None):
    """Energy with float64 positions (bypassing float32 rounding) for finite
    differences; neighbor lists fixed."""
    p = unpack(o.sz, theta)
    pr, pa = nbrs
    x = torch.tensor(x64, dtype=DT)
    L = torch.tensor(L64, dtype=DT)
    eps = torch.zeros(3, 3, dtype=DT) if strain is None else torch.tensor(strain, dtype=DT)

    def vec(pairs):
        i, j, c = (torch.as_tensor(pairs[:, k]) for k in range(3))
        d = (x[j] - x[i]) + torch.as_tensor(SHIFTS)[c] * L
        return d + d @ eps.T

    G = o.descriptors(p, st.types, st.n, pr, vec(pr), pa, vec(pa))
    return float(o.atom_energies(p, st.types, G).sum())


@pytest.mark.parametrize("sizes", [synth.SIZES_TINY, synth.SIZES_LARGE])
def test_forces_and_virial_by_finite_differences(sizes):
    o = NEPOracle(sizes)
    st = small_structures(sizes=(11,))[0]
    th = torch.tensor(synth.draw_params(sizes.n_params, 8).astype(np.float64), dtype=DT)
    nbrs = o.neighbors(st)
    r = o.structure(th, st, nbrs)
    F = r["F"].numpy()
    W = r["W"].numpy()
    x0 = st.pos.astype(np.float64)
    L0 = st.box.astype(np.float64)
    h = 1e-5
    rng = np.random.default_rng(0)
    for i in rng.choice(st.n, 4, replace=False):
        for a in range(3):
            xp, xm = x0.copy(), x0.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(fd_energy(o, th, st, nbrs, xp, L0) - fd_energy(o, th, st, nbrs, xm, L0)) / (2 * h)
            assert fd == pytest.approx(F[i, a], abs=1e-7 * max(1, np.abs(F).max()))
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            fd = -(fd_energy(o, th, st, nbrs, x0, L0, e) - fd_energy(o, th, st, nbrs, x0, L0, -e)) / (2 * h)
            assert fd == pytest.approx(W[a, b], abs=1e-7 * max(1, np.abs(W).max()))
    # zero net force (Eq. 3) and symmetric virial
    np.testing.assert_allclose(F.sum(0), 0, atol=1e-11 * max(1, np.abs(F).max()))
    np.testing.assert_allclose(W, W.T, atol=1e-11 * max(1, np.abs(W).max()))


def test_forces_rotate_with_cluster_and_energy_invariant():
    sz = synth.SIZES_LARGE
    o = NEPOracle(sz)
    st = cluster(n=9)
    th = synth.draw_params(sz.n_params, 2)
    a = o.predict(th, [st])
    q, r = np.linalg.qr(np.random.default_rng(1).normal(size=(3, 3)))
    R = q * np.sign(np.diag(r))
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    c = st.box / 2
    p_rot = ((st.pos.astype(np.float64) - c) @ R.T + c).astype(np.float32)
    b = o.predict(th, [synth.Structure(p_rot, st.box, st.types)])
    assert b["E"][0] == pytest.approx(a["E"][0], rel=1e-6)
    np.testing.assert_allclose(b["F"][0], a["F"][0] @ R.T, atol=2e-5 * np.abs(a["F"][0]).max())


# ------------------------------------------------------------------ loss
def labels_from(o, th, sts, noise=0.0, seed=0):
    pr = o.predict(th, sts)
    rng = np.random.default_rng(seed)
    return dict(energy=pr["E"] + noise * rng.normal(size=len(sts)),
                force=[f + noise * rng.normal(size=f.shape) for f in pr["F"]],
                virial=pr["W"] + noise * rng.normal(size=pr["W"].shape))


def test_loss_zero_when_labels_are_own_predictions():
    o = NEPOracle(SZT)
    sts = small_structures()
    th = synth.draw_params(SZT.n_params, 1)
    L, g = o.loss_and_grad(th, sts, labels_from(o, th, sts))
    assert np.all(np.abs(L) < 1e-24)
    assert np.abs(g).max() < 1e-12


def test_loss_gradient_by_finite_differences():
    o = NEPOracle(SZT)
    sts = small_structures()
    th_s = synth.draw_params(SZT.n_params, 1)
    th_t = synth.draw_params(SZT.n_params, 2)
    lab = labels_from(o, th_t, sts, noise=0.05)
    lam = (1.0, 1.0, 0.1)
    L0, g = o.loss_and_grad(th_s, sts, lab, lam)
    nbrs = [o.neighbors(st) for st in sts]
    th64 = th_s.astype(np.float64)
    h = 1e-5
    idx = np.random.default_rng(44).choice(SZT.n_params, 50, replace=False)

    def loss_at(t):
        # loss_and_grad rounds theta to float32; evaluate on float64 directly
        theta = torch.tensor(t, dtype=DT)
        S = len(sts); N = sum(s.n for s in sts)
        tot = 0.0
        for k, st in enumerate(sts):
            r = o.structure(theta, st, nbrs[k])
            e = (float(r["E"]) - lab["energy"][k]) / st.n
            lf = float(((r["F"].numpy() - lab["force"][k]) ** 2).sum())
            w = (voigt(r["W"]).numpy() - lab["virial"][k]) / st.n
            tot += lam[0] * e * e / S + lam[1] * lf / (3 * N) + lam[2] * (w * w).sum() / (6 * S)
        return tot

    assert loss_at(th64) == pytest.approx(L0[0], rel=1e-12)
    for k in idx:
        tp, tm = th64.copy(), th64.copy()
        tp[k] += h
        tm[k] -= h
        fd = (loss_at(tp) - loss_at(tm)) / (2 * h)
        assert fd == pytest.approx(g[k], abs=1e-8 * max(1.0, np.abs(g).max()))


def test_energy_only_b1_gradient_closed_form():
    """With lambda_f = lambda_v = 0: dL/db1^(I) = sum_n eps_n N_n^(I),
    eps_n = 2 (E(n) - E_tar(n)) / (N_str N_n^2)."""
    o = NEPOracle(SZT)
    sts = small_structures()
    th = synth.draw_params(SZT.n_params, 1)
    pred = o.predict(th, sts)
    Et = pred["E"] + np.array([0.3, -0.2])
    lab = dict(energy=Et, force=pred["F"], virial=pred["W"])
    _, g = o.loss_and_grad(th, sts, lab, (1.0, 0.0, 0.0))
    S = len(sts)
    for I in range(SZT.n_types):
        exp = sum(2 * (pred["E"][k] - Et[k]) / (S * st.n ** 2) * np.sum(st.types == I) for k, st in enumerate(sts))
        base = SZT.n_types ** 2 * (SZT.n_rad * SZT.k_rad + SZT.n_ang * SZT.k_ang)
        blk = SZT.hidden * o.sz.n_desc + 2 * SZT.hidden + 1
        assert g[base + I * blk + blk - 1] == pytest.approx(exp, rel=1e-10)


def test_frozen_cotangent_surrogate_equals_loss_gradient():
    """dL/dtheta = d/dtheta [ sum_i eps_i E_i - D_t E ] with the cotangents
    frozen, where D_t E = sum_pairs (dE_i/dd_ij) . t_ij and
    t_ij = Fbar_j - Fbar_i + Gamma d_ij.  This is the identity the GPU adjoint
    is built on (the E, F and V terms of Eqs. 13-16 contracted)."""
    o = NEPOracle(SZT)
    sts = small_structures()
    th_s = synth.draw_params(SZT.n_params, 1)
    lab = labels_from(o, synth.draw_params(SZT.n_params, 2), sts, noise=0.05)
    lam = (1.0, 1.0, 0.1)
    _, g_ref = o.loss_and_grad(th_s, sts, lab, lam)
    theta = torch.tensor(th_s.astype(np.float64), dtype=DT, requires_grad=True)
    S = len(sts); N = sum(s.n for s in sts)
    pred = o.predict(th_s, sts)
    phi = 0
    for k, st in enumerate(sts):
        eps = 2 * lam[0] * (pred["E"][k] - lab["energy"][k]) / (S * st.n ** 2)
        Fbar = 2 * lam[1] * (pred["F"][k] - lab["force"][k]) / (3 * N)
        Wbar = 2 * lam[2] * (pred["W"][k] - lab["virial"][k]) / (6 * S * st.n ** 2)
        Gam = np.zeros((3, 3))
        for c, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0)]):
            Gam[a, b] = Wbar[c]
        pr, pa = o.neighbors(st)
        x = st.pos.astype(np.float64)
        L = st.box.astype(np.float64)
        h = torch.zeros((), dtype=DT, requires_grad=True)

        def vec(pairs):
            d = (x[pairs[:, 1]] - x[pairs[:, 0]]) + SHIFTS[pairs[:, 2]] * L
            t = Fbar[pairs[:, 1]] - Fbar[pairs[:, 0]] + d @ Gam.T
            return torch.tensor(d, dtype=DT) + h * torch.tensor(t, dtype=DT)

        p = unpack(o.sz, theta)
        G = o.descriptors(p, st.types, st.n, pr, vec(pr), pa, vec(pa))
        Ei = o.atom_energies(p, st.types, G)
        (DtE,) = torch.autograd.grad(Ei.sum(), h, create_graph=True)
        phi = phi + eps * Ei.sum() - DtE
    (g_phi,) = torch.autograd.grad(phi, theta)
    np.testing.assert_allclose(g_phi.numpy(), g_ref, atol=1e-12 * np.abs(g_ref).max())


# -------------------------------------------------------------- optimizer
def test_adam_matches_torch_optim():
    rng = np.random.default_rng(0)
    th = rng.normal(size=20)
    m = np.zeros(20)
    v = np.zeros(20)
    tt = torch.tensor(th, dtype=DT, requires_grad=True)
    opt = torch.optim.Adam([tt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=20)
        th, m, v = adam_step(th, m, v, g, step, 1e-3)
        tt.grad = torch.tensor(g, dtype=DT)
        opt.step()
        np.testing.assert_allclose(th, tt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_first_step_moves_by_lr_sign():
    g = np.array([3.0, -0.02, 1e-3])
    th, _, _ = adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 1e-3)
    np.testing.assert_allclose(th, -1e-3 * np.sign(g), rtol=1e-4)


def test_lr_schedule_eq17():
    a, b, nw, nt = 1e-3, 1e-5, 10, 110
    assert lr_schedule(0, a, b, nw, nt) == pytest.approx(b)
    assert lr_schedule(5, a, b, nw, nt) == pytest.approx(b + 0.5 * (a - b))
    assert lr_schedule(10, a, b, nw, nt) == pytest.approx(a)
    assert lr_schedule(60, a, b, nw, nt) == pytest.approx(b + (a - b) * 0.5)
    assert lr_schedule(110, a, b, nw, nt) == pytest.approx(b)
