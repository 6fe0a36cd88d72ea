"""Triclinic cells on the GPU against the FP64 oracle:
- a batch of tilted cells (wide ones through the single-image decision, a
  narrow one through the float64 test of all 27 images) and an orthorhombic
  cell: lists bit-exact; energies, forces, virials, loss and gradient within
  tolerance;
- sheared cells that hold an orthorhombic crystal: the same physics as the
  orthorhombic cell;
- the box and position flags of tilted cells;
- three velocity-Verlet steps in a tilted cell against the same integrator
  driven by oracle forces."""
import numpy as np
import pytest

from paper_2507_00528_amd import md, synth

from _helpers import grid_structure, hmat, sheared, widths
from gpu_util import TOL_E, TOL_F, Case, DeviceRun, oracle_lists, param_blocks, rel

pytestmark = pytest.mark.gpu
RC = synth.SIZES_LARGE.rc_rad
WIDE = 2 * (RC + 0.01)


def tri_structures():
    rng = np.random.default_rng(21)
    sts = [synth.triclinic_structure(rng, n, 0.031, 2.3, tf) for n, tf in ((150, 0.3), (96, 0.45), (200, 0.15))]
    sts.append(synth.triclinic_structure(rng, 30, 0.031, 2.2, 0.4))
    sts.append(synth.config_structures("c0")[0])
    return sts


def test_triclinic_batch_against_oracle():
    import torch
    sts = tri_structures()
    w = [widths(hmat(st.box, st.tilt if st.tilt is not None else np.zeros(3))).min() for st in sts]
    assert min(w[:3]) >= WIDE and RC <= w[3] < WIDE     # both decision paths are taken
    c = Case(synth.SIZES_LARGE, sts)
    r = DeviceRun(c)
    print(f"[triclinic] N={c.batch.n_atom} widths={np.round(w, 2).tolist()}", flush=True)
    r.neighbors()
    torch.cuda.synchronize()
    assert int(r.flags.item()) == 0
    for which in ("rad", "ang"):
        got, cnt = r.lists(which)
        ref = oracle_lists(c, which)
        assert cnt.tolist() == [len(x) for x in ref]
        assert all([int(v) for v in g] == x for g, x in zip(got, ref))
    e_atom, e_s, F, W = r.efw()
    sizes = np.diff(c.batch.atom_offset)
    assert rel(e_atom, np.concatenate(c.pred["Ei"])) < TOL_E
    assert rel(e_s / sizes, c.pred["E"] / sizes) < TOL_E
    assert rel(F, np.concatenate(c.pred["F"], 0)) < TOL_F
    assert rel(W, c.pred["W"]) < TOL_F
    loss, grad, *_ = r.loss_grad()
    np.testing.assert_allclose(loss, c.loss, rtol=1e-4)
    for blk, sl in param_blocks(c.sizes).items():
        assert rel(grad[sl], c.grad[sl]) < TOL_F, blk


@pytest.mark.parametrize("L,tilt", [(20.0, (20.0, 0.0, 0.0)), (20.0, (-20.0, 20.0, -20.0)), (13.0, (13.0, 0, 0))])
def test_sheared_cell_matches_the_orthorhombic_crystal(L, tilt):
    import torch
    st = grid_structure(4, 48, L)
    tri = sheared(st, tilt)
    c = Case(synth.SIZES_LARGE, [st])
    r = DeviceRun(GPUCase(c, [tri]))
    print(f"[sheared] L={L} tilt={tilt}", flush=True)
    r.neighbors()
    torch.cuda.synchronize()
    assert int(r.flags.item()) == 0
    e_atom, e_s, F, W = r.efw()
    assert rel(e_atom, c.pred["Ei"][0]) < TOL_E
    assert rel(F, c.pred["F"][0]) < TOL_F
    assert rel(W, c.pred["W"]) < TOL_F


class GPUCase:
    """A case whose GPU batch holds other structures (the same physics in
    another cell) than the oracle's."""

    def __init__(self, case, structures):
        self.__dict__.update(case.__dict__)
        self.batch = synth.Batch(structures)


def _flags(structures):
    import torch
    from paper_2507_00528_amd import nep
    b = synth.Batch(structures)
    model = nep.Model.of(synth.SIZES_SMALL)
    db = nep.DeviceBatch(b)
    nb = nep.Neighbors(model, b.n_atom)
    ws = nep.workspace(model, b.n_struct, b.n_atom)
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    nep.build_neighbors(model, db, nb, ws, fl)
    torch.cuda.synchronize()
    return int(fl.item()), nb.cnt_rad.cpu().numpy(), b


def test_triclinic_box_and_position_flags():
    from paper_2507_00528_amd import nep
    ok = synth.triclinic_structure(np.random.default_rng(2), 60, 0.031, 2.3, 0.2)
    # a tilted cell whose width across b (Ly = 5.5 A) is below rc = 6 A
    narrow_box = np.array([9.0, 5.5, 9.0], np.float32)
    narrow = synth.Structure(np.array([[1.0, 1.0, 1.0], [3.0, 2.0, 4.0]], np.float32), narrow_box,
                             np.zeros(2, np.int32), "narrow", np.array([2.0, 0.0, 0.0], np.float32))
    fl, cnt, b = _flags([ok, narrow])
    assert fl & nep.NEP_FLAG_BOX and nep.flags_status(fl) == -2
    assert (cnt[b.atom_offset[1]:] == 0).all() and (cnt[:b.atom_offset[1]] > 0).all()
    # an atom just outside the tilted cell (fractional coordinate -0.01 along a)
    H = hmat(ok.box, ok.tilt)
    pos = ok.pos.copy()
    f = np.linalg.solve(H, pos[5].astype(np.float64))
    f[0] = -0.01
    pos[5] = (H @ f).astype(np.float32)
    fl, _, _ = _flags([synth.Structure(pos, ok.box, ok.types, "out", ok.tilt)])
    assert fl & nep.NEP_FLAG_POSITION and nep.flags_status(fl) == -8
    fl, _, _ = _flags([ok])
    assert fl == 0


def test_triclinic_verlet_matches_oracle():
    import torch
    from oracle import NEPOracle
    from paper_2507_00528_amd import nep
    sz = synth.SIZES_TINY
    st = synth.triclinic_structure(np.random.default_rng(8), 120, 0.031, 2.3, 0.35)
    H = hmat(st.box, st.tilt)
    masses = [md.MASS["Sb"], md.MASS["Te"]]
    v0 = md.maxwell_velocities(st.types, masses, 900.0, seed=4)
    dt, n = 2.0, 3
    # translate the configuration (distances unchanged) so that the atoms with
    # the fastest fractional velocities along a and along c sit just inside
    # the faces they move towards: both cross in the first drift
    vf = np.linalg.solve(H, v0.reshape(3, -1).astype(np.float64)).T
    f = np.linalg.solve(H, st.pos.astype(np.float64).T).T
    shift = np.zeros(3)
    for ax in (0, 2):
        k = int(np.argmax(np.abs(vf[:, ax])))
        step = dt * vf[k, ax]
        shift[ax] = (1.0 - 0.3 * step if step > 0 else -0.3 * step) - f[k, ax]
    st = synth.Structure(synth.wrap_cell32((f + shift) @ H.T, st.box, st.tilt), st.box, st.types, "md", st.tilt)
    b = synth.Batch([st])
    model = nep.Model.of(sz)
    db = nep.DeviceBatch(b)
    nb = nep.Neighbors(model, b.n_atom)
    ws = nep.workspace(model, 1, b.n_atom)
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    theta = synth.draw_params(sz.n_params, synth.SEEDS["teacher"])
    p = torch.tensor(theta, device="cuda")
    mass = torch.tensor(masses, dtype=torch.float32, device="cuda")
    vel = torch.tensor(v0, device="cuda")
    force = torch.zeros(3 * b.n_atom, device="cuda")
    e_pot = torch.zeros(1, device="cuda")
    print(f"[triclinic md] N={b.n_atom}", flush=True)
    nep.build_neighbors(model, db, nb, ws, fl)
    nep.energy_force_virial(model, db, nb, p, ws, None, e_pot, force, None)
    nep.md_step(model, db, nb, p, mass, vel, force, dt, n, e_pot, ws, fl)
    torch.cuda.synchronize()
    assert int(fl.item()) == 0
    o = NEPOracle(sz)
    m = np.asarray(masses)[b.types][:, None]
    x = st.pos.astype(np.float64)
    v = v0.reshape(3, -1).T.astype(np.float64)
    F = o.predict(theta, [st])["F"][0]
    crossed = 0
    for _ in range(n):
        v += 0.5 * dt * md.ACCEL * F / m
        xn = x + dt * v
        fr = np.linalg.solve(H, xn.T).T
        crossed += int(((fr < 0) | (fr >= 1)).sum())
        cur = synth.Structure(synth.wrap_cell32(xn, st.box, st.tilt), st.box, st.types, "md", st.tilt)
        x = cur.pos.astype(np.float64)
        out = o.predict(theta, [cur])
        F = out["F"][0]
        v += 0.5 * dt * md.ACCEL * F / m
    assert crossed >= 2   # atoms were wrapped through tilted faces
    assert abs(float(e_pot[0]) - out["E"][0]) / st.n < TOL_E * max(1.0, abs(out["E"][0]) / st.n)
    xg = db.pos.cpu().numpy().reshape(3, -1).T.astype(np.float64)
    fg = np.linalg.solve(H, xg.T).T
    assert fg.min() >= -1e-5 and fg.max() < 1 + 1e-5
    # positions agree up to a lattice vector (an atom on a face may wrap on one side only)
    df = np.linalg.solve(H, (xg - x).T).T
    df -= np.round(df)
    assert np.abs(df @ H.T).max() < 1e-4
    assert rel(vel.cpu().numpy().reshape(3, -1).T, v) < 1e-4
