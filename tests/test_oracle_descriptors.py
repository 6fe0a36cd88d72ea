"""Pins of the oracle's descriptors (Eqs. 5-8 and the 4-/5-body invariants)
against closed forms for one and two neighbors, and invariance checks."""
import math

import numpy as np
import pytest
import torch

from oracle import NEPOracle, harmonics as hm, unpack
from oracle.nep_oracle import four_body, five_body
from paper_2507_00528_amd import synth

from _helpers import cluster

DT = torch.float64


def g_closed(c_row, r, rc):
    """g_n(r) from the trig form of T_k and the cosine cutoff, independent of
    the oracle's recursion."""
    K = len(c_row)
    xi = 2 * (r / rc - 1) ** 2 - 1
    fk = 0.5 * (np.cos(np.arange(K) * np.arccos(xi)) + 1) * 0.5 * (1 + np.cos(np.pi * r / rc))
    return float(np.dot(c_row, fk))


def setup_pair_geometry(sz, d_list, types, seed=0):
    """Descriptors of atom 0 with neighbors at displacement vectors d_list."""
    o = NEPOracle(sz)
    th = torch.tensor(synth.draw_params(sz.n_params, seed).astype(np.float64), dtype=DT)
    p = unpack(o.sz, th)
    n = 1 + len(d_list)
    pairs = np.array([[0, j + 1, 13] for j in range(len(d_list))])
    d = torch.tensor(np.array(d_list, np.float64), dtype=DT)
    G = o.descriptors(p, np.array(types), n, pairs, d, pairs, d)
    return o, p, G[0].numpy()


SZ = synth.NEPSizes(n_types=2, n_rad=3, n_ang=3, k_rad=5, k_ang=4, l3=8, l4=2, l5=1, hidden=4)


def test_one_neighbor_closed_forms():
    r = 2.9
    u = np.array([0.3, -0.5, 0.81])
    u /= np.linalg.norm(u)
    o, p, G = setup_pair_geometry(SZ, [r * u], [0, 1])
    cR = p["c_rad"][0, 1].numpy()
    cA = p["c_ang"][0, 1].numpy()
    gR = [g_closed(cR[n], r, SZ.rc_rad) for n in range(SZ.n_rad)]
    gA = [g_closed(cA[n], r, SZ.rc_ang) for n in range(SZ.n_ang)]
    np.testing.assert_allclose(G[:SZ.n_rad], gR, rtol=1e-12)
    off = SZ.n_rad
    for l in range(1, SZ.l3 + 1):
        for n in range(SZ.n_ang):
            # q_nl = (2l+1)/(4 pi) g_n^2 for a single neighbor
            assert G[off] == pytest.approx((2 * l + 1) / (4 * math.pi) * gA[n] ** 2, rel=1e-11)
            off += 1
    for n in range(SZ.n_ang):
        assert G[off + n] == pytest.approx(2.0 / 9.0 * gA[n] ** 3, rel=1e-11)        # q4
        assert G[off + SZ.n_ang + n] == pytest.approx(gA[n] ** 4, rel=1e-11)         # q5


def test_two_neighbors_closed_forms():
    r1, r2 = 2.7, 3.4
    u1 = np.array([1.0, 0.2, -0.3]); u1 /= np.linalg.norm(u1)
    u2 = np.array([-0.4, 0.9, 0.5]); u2 /= np.linalg.norm(u2)
    cos = float(u1 @ u2)
    o, p, G = setup_pair_geometry(SZ, [r1 * u1, r2 * u2], [1, 0, 1], seed=3)
    cA1 = p["c_ang"][1, 0].numpy()   # center type 1, neighbor types 0 and 1
    cA2 = p["c_ang"][1, 1].numpy()
    off = SZ.n_rad
    g1 = [g_closed(cA1[n], r1, SZ.rc_ang) for n in range(SZ.n_ang)]
    g2 = [g_closed(cA2[n], r2, SZ.rc_ang) for n in range(SZ.n_ang)]
    for l in range(1, SZ.l3 + 1):
        for n in range(SZ.n_ang):
            exp = (2 * l + 1) / (4 * math.pi) * (g1[n] ** 2 + g2[n] ** 2 + 2 * g1[n] * g2[n] * hm.legendre_P(l, cos))
            assert G[off] == pytest.approx(exp, rel=1e-10, abs=1e-14)
            off += 1
    for n in range(SZ.n_ang):
        a, b = g1[n], g2[n]
        q4 = 2.0 / 9.0 * (a ** 3 + b ** 3) + a * b * (a + b) * (cos ** 2 - 1.0 / 3.0)
        q5 = (a * a + b * b + 2 * a * b * cos) ** 2
        assert G[off + n] == pytest.approx(q4, rel=1e-10, abs=1e-14)
        assert G[off + SZ.n_ang + n] == pytest.approx(q5, rel=1e-10, abs=1e-14)


def random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_four_and_five_body_rotation_invariant():
    rng = np.random.default_rng(9)
    S1 = torch.tensor(rng.normal(size=(4, 3)), dtype=DT)
    S2 = torch.tensor(rng.normal(size=(4, 5)), dtype=DT)
    # rotate the underlying tensors: M -> R M R^T, v -> R v
    R = torch.tensor(random_rotation(rng), dtype=DT)
    s0, s1, s2, s3, s4 = (S2[:, m] for m in range(5))
    M = torch.stack([torch.stack([-s0 / 6 + s3 / 2, s4 / 2, s1], -1),
                     torch.stack([s4 / 2, -s0 / 6 - s3 / 2, s2], -1),
                     torch.stack([s1, s2, s0 / 3], -1)], -2)
    Mr = R @ M @ R.T
    S2r = torch.stack([3 * Mr[:, 2, 2], Mr[:, 0, 2], Mr[:, 1, 2], Mr[:, 0, 0] - Mr[:, 1, 1], 2 * Mr[:, 0, 1]], -1)
    np.testing.assert_allclose(four_body(S2r).numpy(), four_body(S2).numpy(), rtol=1e-12)
    # l = 1 sums are (z, x, y) components
    v = S1[:, [1, 2, 0]] @ R.T
    S1r = v[:, [2, 0, 1]]
    np.testing.assert_allclose(five_body(S1r).numpy(), five_body(S1).numpy(), rtol=1e-12)


def test_descriptors_rotation_translation_permutation_invariant():
    sz = synth.SIZES_LARGE
    o = NEPOracle(sz)
    st = cluster(n=8)
    th = synth.draw_params(sz.n_params, 4)
    G0 = o.predict(th, [st])["G"][0]
    rng = np.random.default_rng(2)
    R = random_rotation(rng)
    c = st.box / 2
    p_rot = ((st.pos - c) @ R.T + c + np.array([0.3, -1.1, 0.7])).astype(np.float32)
    st_r = synth.Structure(p_rot, st.box, st.types)
    G1 = o.predict(th, [st_r])["G"][0]
    np.testing.assert_allclose(G1, G0, rtol=1e-5, atol=1e-9 * np.abs(G0).max())
    perm = rng.permutation(st.n)
    st_p = synth.Structure(st.pos[perm], st.box, st.types[perm])
    G2 = o.predict(th, [st_p])["G"][0]
    np.testing.assert_allclose(G2, G0[perm], rtol=1e-12, atol=1e-14)


def test_descriptor_dimension_and_order():
    sz = synth.SIZES_LARGE
    o = NEPOracle(sz)
    assert o.sz.n_desc == 37 and o.sz.n_params == 4430
    assert NEPOracle(synth.SIZES_SMALL).sz.n_desc == 25 and NEPOracle(synth.SIZES_SMALL).sz.n_params == 1982
