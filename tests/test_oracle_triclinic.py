"""Pins of the oracle on triclinic cells (edge vectors a = (lx,0,0),
b = (xy,ly,0), c = (xz,yz,lz)): neighbor sets against brute force over 125
images, the zero-tilt case against the orthorhombic search, sheared
representations of an orthorhombic lattice (same physics, different cell
vectors), and forces and virials by central finite differences."""
import itertools

import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

from oracle import NEPOracle, neighbor_pairs, unpack
from oracle.nep_oracle import _neighbor_pairs_triclinic
from paper_2507_00528_amd import synth

from _helpers import grid_structure, hmat, sheared, small_structures, widths

DT = torch.float64


def brute_force(st, rc, reach=2):
    """(i, j, code) for every image s in {-reach..reach}^3 within rc; asserts
    that no image beyond {-1,0,1}^3 is in range and that no distance lies
    within 1e-9 of rc."""
    x = st.pos.astype(np.float64)
    H = hmat(st.box, st.tilt)
    out = set()
    for s in itertools.product(range(-reach, reach + 1), repeat=3):
        d = cdist(x, x + H @ np.array(s, np.float64))
        assert not np.any(np.abs(d - rc) < 1e-9)
        ii, jj = np.nonzero(d < rc)
        for i, j in zip(ii, jj):
            if i == j and s == (0, 0, 0):
                continue
            assert max(abs(v) for v in s) <= 1, (i, j, s)
            out.add((int(i), int(j), 9 * (s[0] + 1) + 3 * (s[1] + 1) + (s[2] + 1)))
    return out


@pytest.mark.parametrize("n,tf,seed", [(40, 0.3, 0), (90, 0.45, 1), (150, 0.2, 2)])
def test_triclinic_neighbors_match_125_image_brute_force(n, tf, seed):
    st = synth.triclinic_structure(np.random.default_rng(seed), n, 0.031, 2.3, tf)
    for rc in (6.0, 4.0):
        assert widths(hmat(st.box, st.tilt)).min() >= rc
        p = neighbor_pairs(st.pos, st.box, rc, tilt32=st.tilt)
        assert set(map(tuple, p.tolist())) == brute_force(st, rc)
        key = (p[:, 0] * st.n + p[:, 1]) * 27 + p[:, 2]
        assert np.all(np.diff(key) > 0)
        assert set(map(tuple, p.tolist())) == set((j, i, 26 - c) for i, j, c in p.tolist())


def test_zero_tilt_search_equals_the_orthorhombic_search():
    sts = small_structures(sizes=(12, 60))   # the first cell is shorter than 2 rc
    for st in sts:
        for rc in (6.0, 3.7):
            a = neighbor_pairs(st.pos, st.box, rc)
            b = _neighbor_pairs_triclinic(st.pos, st.box, rc, None, np.zeros(3, np.float32))
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("L,tilt_of", [
    (20.0, lambda L: (L, 0.0, 0.0)),        # b' = b + a
    (20.0, lambda L: (0.0, L, L)),          # c' = c + a + b
    (20.0, lambda L: (-L, L, -L)),
    (13.0, lambda L: (L, 0.0, 0.0)),        # width L / sqrt(2): between rc and 2 rc
])
def test_sheared_cell_reproduces_the_orthorhombic_results(L, tilt_of):
    sz = synth.SIZES_TINY
    o = NEPOracle(sz)
    st = grid_structure(4, 24, L)
    tri = sheared(st, tilt_of(L))
    assert widths(hmat(tri.box, tri.tilt)).min() >= sz.rc_rad
    assert not np.array_equal(tri.pos, st.pos)
    th = synth.draw_params(sz.n_params, 9)
    a, b = o.predict(th, [st]), o.predict(th, [tri])
    # the same pairs, by (i, j, displacement)
    for rc in (sz.rc_rad, sz.rc_ang):
        pa = neighbor_pairs(st.pos, st.box, rc)
        pb = neighbor_pairs(tri.pos, tri.box, rc, tilt32=tri.tilt)
        assert len(pa) == len(pb)
    np.testing.assert_allclose(b["Ei"][0], a["Ei"][0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b["F"][0], a["F"][0], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(b["W"], a["W"], rtol=1e-10, atol=1e-12)


def test_triclinic_forces_and_virial_by_finite_differences():
    sz = synth.SIZES_TINY
    o = NEPOracle(sz)
    st = synth.triclinic_structure(np.random.default_rng(5), 30, 0.031, 2.2, 0.4)
    H = hmat(st.box, st.tilt)
    assert widths(H).min() >= sz.rc_rad
    th = torch.tensor(synth.draw_params(sz.n_params, 8).astype(np.float64), dtype=DT)
    nbrs = o.neighbors(st)
    r = o.structure(th, st, nbrs)
    F, W = r["F"].numpy(), r["W"].numpy()
    # shift vectors from the cell matrix, independently of the oracle's table
    S = np.array(list(itertools.product((-1, 0, 1), repeat=3)), np.float64)

    def energy(x64, Hm):
        pr, pa = nbrs
        x = torch.tensor(x64, dtype=DT)
        HS = torch.tensor(S @ Hm.T, dtype=DT)

        def vec(pairs):
            i, j, c = (torch.as_tensor(pairs[:, k]) for k in range(3))
            return (x[j] - x[i]) + HS[c]

        G = o.descriptors(unpack(sz, th), st.types, st.n, pr, vec(pr), pa, vec(pa))
        return float(o.atom_energies(unpack(sz, th), st.types, G).sum())

    x0 = st.pos.astype(np.float64)
    h = 1e-5
    for i in (0, 7, 19):
        for a in range(3):
            xp, xm = x0.copy(), x0.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(energy(xp, H) - energy(xm, H)) / (2 * h)
            assert fd == pytest.approx(F[i, a], abs=1e-7 * max(1, np.abs(F).max()))
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            Ep = energy(x0 @ (np.eye(3) + e).T, (np.eye(3) + e) @ H)
            Em = energy(x0 @ (np.eye(3) - e).T, (np.eye(3) - e) @ H)
            assert -(Ep - Em) / (2 * h) == pytest.approx(W[a, b], abs=1e-7 * max(1, np.abs(W).max()))
    np.testing.assert_allclose(F.sum(0), 0, atol=1e-11 * max(1, np.abs(F).max()))
    np.testing.assert_allclose(W, W.T, atol=1e-11 * max(1, np.abs(W).max()))
