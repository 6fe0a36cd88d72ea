"""Inference helpers around nep_md_step: Maxwell-Boltzmann velocities,
NVE runs that record the energies, the energy-volume curve of a structure
under uniform scaling, and a host radial distribution function for
trajectory snapshots.  Units: eV, A, fs, amu, K."""
from __future__ import annotations

import numpy as np

KB = 8.617333262e-5          # eV / K
ACCEL = 9.648533212e-3       # (eV/A)/amu in A/fs^2
MASS = {"Sb": 121.760, "Te": 127.60}


def maxwell_velocities(types, masses, temperature, seed=0) -> np.ndarray:
    """SoA [3*n] velocities (A/fs) drawn at the given temperature, with the
    centre-of-mass drift removed."""
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, np.float64)[np.asarray(types)]
    sig = np.sqrt(KB * temperature * ACCEL / m)
    v = rng.normal(size=(len(m), 3)) * sig[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    return np.ascontiguousarray(v.T.reshape(-1)).astype(np.float32)


def run_nve(model, batch, nbrs, params, masses, vel, ws, flags, dt, n_chunks, chunk):
    """Velocity Verlet for n_chunks x chunk steps; returns per-chunk arrays of
    potential and kinetic energy per structure [n_chunks + 1, S]."""
    import torch
    from . import nep
    S, N = batch.n_struct, batch.n_atom
    force = torch.zeros(3 * N, device="cuda")
    e_pot = torch.zeros(S, device="cuda")
    e_kin = torch.zeros(S, device="cuda")
    nep.build_neighbors(model, batch, nbrs, ws, flags)
    nep.energy_force_virial(model, batch, nbrs, params, ws, None, e_pot, force, None)
    nep.md_step(model, batch, nbrs, params, masses, vel, force, dt, 0, e_pot, ws, flags)
    m = masses.cpu().numpy().astype(np.float64)[batch.type.cpu().numpy()]
    v = vel.cpu().numpy().reshape(3, -1).astype(np.float64)
    off = batch.atom_offset.cpu().numpy()
    ke0 = np.array([0.5 * (m[off[k]:off[k + 1]] * (v[:, off[k]:off[k + 1]] ** 2).sum(0)).sum() / ACCEL
                    for k in range(S)])
    pot, kin = [e_pot.cpu().numpy().astype(np.float64)], [ke0]
    for _ in range(n_chunks):
        nep.md_step(model, batch, nbrs, params, masses, vel, force, dt, chunk, e_pot, ws, flags, e_kin=e_kin)
        torch.cuda.synchronize()
        nep.check_flags(flags, "md")
        pot.append(e_pot.cpu().numpy().astype(np.float64))
        kin.append(e_kin.cpu().numpy().astype(np.float64))
    return np.array(pot), np.array(kin)


def scaled(structure, s):
    """The structure with positions and box scaled by s (uniform strain)."""
    from .synth import Structure, wrap32
    box = np.asarray(structure.box, np.float64) * s
    pos = wrap32(np.asarray(structure.pos, np.float64) * s, box)
    return Structure(pos, box.astype(np.float32), structure.types, structure.kind)


def rdf(pos, box, r_max, nbins=100):
    """g(r) of one periodic orthorhombic snapshot (minimum image; r_max must
    not exceed half the shortest edge).  Returns bin centres and g."""
    pos = np.asarray(pos, np.float64)
    box = np.asarray(box, np.float64)
    if r_max > 0.5 * box.min():
        raise ValueError("r_max exceeds half the shortest box edge")
    n = len(pos)
    d = pos[None, :, :] - pos[:, None, :]
    d -= box * np.round(d / box)
    r = np.sqrt((d ** 2).sum(-1))[np.triu_indices(n, 1)]
    h, edges = np.histogram(r, bins=nbins, range=(0.0, r_max))
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    rho = n / np.prod(box)
    g = 2.0 * h / (n * rho * shell)
    return 0.5 * (edges[1:] + edges[:-1]), g
