"""Seeded synthetic Sb-Te-shaped training batches.

The paper trains on a DFT dataset of crystalline (rocksalt-like metastable),
liquid and amorphous Sb-Te configurations (Sec. III.A).  That dataset is not
available, so the workloads here are synthetic stand-ins with the same shapes:
periodic orthorhombic cells at Sb-Te densities, species Sb:Te = 2:3, random
sequential addition (RSA) with a minimum pair distance for the disordered
phases, and perturbed rocksalt supercells for the crystalline phase.

This module draws random numbers and builds geometry.  It holds none of the
NEP arithmetic (no descriptors, no network, no loss): both the FP64 oracle and
the GPU path consume what it produces.  Everything is a pure function of the
seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SB, TE = 0, 1


# ----------------------------------------------------------------------------
# NEP sizes of the five synthetic workloads (index ranges are counts: n_rad =
# n_max_R + 1 radial channels, k_rad = basis_size + 1 Chebyshev terms).
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class NEPSizes:
    n_types: int = 2
    n_rad: int = 5
    n_ang: int = 5
    k_rad: int = 9
    k_ang: int = 9
    l3: int = 4      # 3-body angular degrees l = 1..l3
    l4: int = 0      # 0 or 2: 4-body term built from the l = 2 sums
    l5: int = 0      # 0 or 1: 5-body term built from the l = 1 sums
    hidden: int = 30
    rc_rad: float = 6.0
    rc_ang: float = 4.0

    @property
    def n_desc(self) -> int:
        return (self.n_rad + self.n_ang * self.l3
                + (self.n_ang if self.l4 else 0) + (self.n_ang if self.l5 else 0))

    @property
    def n_params(self) -> int:
        t2 = self.n_types * self.n_types
        nn = self.hidden * self.n_desc + 2 * self.hidden + 1
        return t2 * (self.n_rad * self.k_rad + self.n_ang * self.k_ang) + self.n_types * nn


SIZES_SMALL = NEPSizes()  # 3-body only, hidden 30
SIZES_LARGE = NEPSizes(n_rad=7, n_ang=5, k_rad=11, k_ang=11, l3=4, l4=2, l5=1, hidden=50)
SIZES_TINY = NEPSizes(n_rad=3, n_ang=2, k_rad=4, k_ang=3, l3=4, l4=2, l5=1, hidden=6)
SIZES_MONO = NEPSizes(n_types=1, n_rad=4, n_ang=3, k_rad=6, k_ang=5, l3=2, l4=2, l5=0, hidden=8)
SIZES_L8 = NEPSizes(n_rad=5, n_ang=4, k_rad=8, k_ang=8, l3=8, l4=2, l5=1, hidden=16)   # 3-body l up to 8


@dataclass
class Structure:
    pos: np.ndarray      # float32 [n, 3], wrapped into the cell
    box: np.ndarray      # float32 [3], cell lengths (lx, ly, lz)
    types: np.ndarray    # int32 [n]
    kind: str = ""
    # float32 [3] tilts (xy, xz, yz) of a triclinic cell with edge vectors
    # a = (lx, 0, 0), b = (xy, ly, 0), c = (xz, yz, lz); None: orthorhombic
    tilt: np.ndarray = None

    @property
    def n(self) -> int:
        return int(self.types.shape[0])


@dataclass
class Batch:
    """Concatenated structure-of-arrays layout consumed by the library."""
    structures: list
    pos_soa: np.ndarray = field(init=False)      # float32 [3*N]: x block, y block, z block
    types: np.ndarray = field(init=False)        # int32 [N]
    atom_offset: np.ndarray = field(init=False)  # int32 [S+1]
    box: np.ndarray = field(init=False)          # float32 [S*3]
    tilt: np.ndarray = field(init=False)         # float32 [S*3] (xy, xz, yz), zeros when orthorhombic

    def __post_init__(self):
        sizes = [s.n for s in self.structures]
        self.atom_offset = np.zeros(len(sizes) + 1, np.int32)
        self.atom_offset[1:] = np.cumsum(sizes)
        pos = np.concatenate([s.pos for s in self.structures], 0) if sizes else np.zeros((0, 3), np.float32)
        self.pos_soa = np.ascontiguousarray(pos.T.reshape(-1)).astype(np.float32)
        self.types = np.concatenate([s.types for s in self.structures]).astype(np.int32) if sizes else np.zeros(0, np.int32)
        self.box = np.concatenate([s.box for s in self.structures]).astype(np.float32) if sizes else np.zeros(0, np.float32)
        self.tilt = (np.concatenate([np.zeros(3, np.float32) if s.tilt is None else np.asarray(s.tilt, np.float32)
                                     for s in self.structures]).astype(np.float32) if sizes else np.zeros(0, np.float32))

    @property
    def triclinic(self) -> bool:
        return bool(np.any(self.tilt != 0))

    @property
    def n_struct(self) -> int:
        return len(self.structures)

    @property
    def n_atom(self) -> int:
        return int(self.atom_offset[-1])


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def wrap32(pos: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Wrap float64 positions into [0, L) and round to float32 so that every
    float32 coordinate is strictly below the float32 edge length."""
    box32 = box.astype(np.float32)
    p = np.mod(pos, box.astype(np.float64)).astype(np.float32)
    p = np.where(p >= box32, np.float32(0.0), p)
    p = np.where(p < 0, np.float32(0.0), p)
    return p.astype(np.float32)


def cell_matrix(box, tilt=None) -> np.ndarray:
    """Columns are the edge vectors a = (lx, 0, 0), b = (xy, ly, 0),
    c = (xz, yz, lz), in float64 from the float32 lengths and tilts."""
    lx, ly, lz = (float(np.float32(v)) for v in box)
    xy, xz, yz = (0.0, 0.0, 0.0) if tilt is None else (float(np.float32(v)) for v in tilt)
    return np.array([[lx, xy, xz], [0.0, ly, yz], [0.0, 0.0, lz]])


def wrap_cell32(pos: np.ndarray, box, tilt) -> np.ndarray:
    """Wrap float64 positions into a triclinic cell (fractional coordinates
    in [0, 1)) and round to float32."""
    H = cell_matrix(box, tilt)
    f = np.linalg.solve(H, np.asarray(pos, np.float64).T).T
    f -= np.floor(f)
    return (f @ H.T).astype(np.float32)


_IMAGES27 = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], np.float64)


def triclinic_structure(rng, n: int, density: float, dmin: float, tilt_frac: float = 0.3,
                        kind: str = "triclinic") -> Structure:
    """Random sequential packing (periodic minimum distance dmin) in a cell of
    volume n/density with edge lengths within 10% of the cube's and tilts
    xy, xz (yz) drawn uniformly in +-tilt_frac lx (ly)."""
    L = (n / density) ** (1.0 / 3.0)
    box = (L * rng.uniform(0.9, 1.1, 3)).astype(np.float32)
    tilt = np.array([rng.uniform(-tilt_frac, tilt_frac) * box[0], rng.uniform(-tilt_frac, tilt_frac) * box[0],
                     rng.uniform(-tilt_frac, tilt_frac) * box[1]], np.float32)
    H = cell_matrix(box, tilt)
    images = _IMAGES27 @ H.T
    pts = np.zeros((0, 3))
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > 200 * n:
            raise RuntimeError("packing failed: lower the density or dmin")
        x = H @ rng.uniform(0.0, 1.0, 3)
        if len(pts):
            d = (pts[:, None, :] + images[None]) - x
            if np.min(np.einsum("ijk,ijk->ij", d, d)) < dmin * dmin:
                continue
        pts = np.vstack([pts, x])
    return Structure(wrap_cell32(pts, box, tilt), box, assign_types(rng, n), kind, tilt)


def rsa_positions(rng: np.random.Generator, n: int, box: np.ndarray, dmin: float,
                  max_tries: int = 400_000_000) -> np.ndarray:
    """Random sequential addition in a periodic orthorhombic box: uniform
    candidates are accepted when no accepted atom lies closer than dmin
    (minimum-image distance).

    A cell grid with edge <= dmin/sqrt(3) holds at most one atom per cell, so a
    candidate only needs the cells within ceil(dmin/edge) of its own.  Once the
    acceptance rate falls (dense amorphous cells approach the RSA jamming
    fraction), candidates are drawn uniformly from the voxels not yet wholly
    inside some atom's exclusion sphere; every candidate still gets the exact
    distance test, so accepted points stay uniform on the available volume."""
    box = np.asarray(box, np.float64)
    if np.any(box < 2 * dmin):
        raise ValueError("box too small for RSA minimum-image check")
    nc = np.ceil(box / (dmin / math.sqrt(3.0))).astype(np.int64)
    edge = box / nc
    reach = int(np.ceil(dmin / edge.min()))
    r1 = np.arange(-reach, reach + 1)
    offs = np.stack(np.meshgrid(r1, r1, r1, indexing="ij"), -1).reshape(-1, 3)
    grid = -np.ones(tuple(nc), np.int64)
    pos = np.zeros((n, 3), np.float64)
    d2min = dmin * dmin
    state = {"placed": 0, "tries": 0}

    # voxel exclusion map, built lazily when acceptance drops
    nv = np.ceil(box / (dmin / 8.0)).astype(np.int64)
    hv = box / nv
    half_diag = 0.5 * float(np.sqrt((hv * hv).sum()))
    vr = int(np.ceil(dmin / hv.min()))
    rv = np.arange(-vr, vr + 1)
    voffs = np.stack(np.meshgrid(rv, rv, rv, indexing="ij"), -1).reshape(-1, 3)
    vdist = np.sqrt(((voffs * hv) ** 2).sum(1))
    voffs = voffs[vdist + 2.0 * half_diag <= dmin]
    excluded = None

    def exclude(p):
        iv = np.minimum((p / hv).astype(np.int64), nv - 1)
        cells = (iv[None, :] + voffs) % nv
        excluded[cells[:, 0], cells[:, 1], cells[:, 2]] = True

    def place(cand, ci):
        cells = (ci[:, None, :] + offs[None, :, :]) % nc
        ids = grid[cells[..., 0], cells[..., 1], cells[..., 2]]
        occ = ids >= 0
        nb = pos[np.where(occ, ids, 0)]
        dv = nb - cand[:, None, :]
        dv -= box * np.round(dv / box)
        bad = np.any(occ & (np.einsum("kox,kox->ko", dv, dv) < d2min), axis=1)
        ok = np.nonzero(~bad)[0]
        if len(ok) == 0:
            return 0
        sv = cand[ok]
        dd = sv[:, None, :] - sv[None, :, :]
        dd -= box * np.round(dd / box)
        clash = np.einsum("abx,abx->ab", dd, dd) < d2min
        keep = np.zeros(len(ok), bool)
        for a in range(len(ok)):
            if state["placed"] >= n:
                break
            if np.any(clash[a, :a] & keep[:a]):
                continue
            keep[a] = True
            k = state["placed"]
            pos[k] = sv[a]
            cc = ci[ok[a]]
            grid[cc[0], cc[1], cc[2]] = k
            if excluded is not None:
                exclude(sv[a])
            state["placed"] = k + 1
        return len(ok)

    p_acc = 1.0
    while state["placed"] < n:
        if excluded is None and p_acc < 0.05:
            excluded = np.zeros(tuple(nv), bool)
            for k in range(state["placed"]):
                exclude(pos[k])
            p_acc = 1.0
        k = int(min(16384, max(32, 24.0 / max(p_acc, 1e-6))))
        if excluded is None:
            cand = rng.uniform(0.0, 1.0, (k, 3)) * box
        else:
            free = np.flatnonzero(~excluded.reshape(-1))
            if len(free) == 0:
                raise RuntimeError(f"RSA jammed at {state['placed']}/{n} atoms")
            pick = free[rng.integers(0, len(free), k)]
            vi = np.stack(np.unravel_index(pick, tuple(nv)), -1)
            cand = (vi + rng.uniform(0.0, 1.0, (k, 3))) * hv
        state["tries"] += k
        if state["tries"] > max_tries:
            raise RuntimeError(f"RSA stalled at {state['placed']}/{n} atoms")
        ci = np.minimum((cand / edge).astype(np.int64), nc - 1)
        n_ok = place(cand, ci)
        p_acc = 0.7 * p_acc + 0.3 * (n_ok / k)
    return pos


ROCKSALT_SITES = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],   # fcc sublattice
    [0.5, 0.0, 0.0], [0.5, 0.5, 0.5], [0.0, 0.0, 0.5], [0.0, 0.5, 0.0],   # shifted by a/2
])


def rocksalt_reps(target: int, lo: int, hi: int):
    """Orthorhombic repeat counts (n1<=n2<=n3) of the 8-atom rocksalt cube with
    8*n1*n2*n3 in [lo, hi], closest to target, most cubic on ties."""
    best = None
    for n1 in range(1, 12):
        for n2 in range(n1, 12):
            for n3 in range(n2, 12):
                na = 8 * n1 * n2 * n3
                if na < lo or na > hi:
                    continue
                # within 15% of the target size, prefer near-cubic cells
                key = (abs(na - target) > 0.15 * target, n3 - n1, abs(na - target))
                if best is None or key < best[0]:
                    best = (key, (n1, n2, n3))
    if best is None:
        raise ValueError("no rocksalt supercell in range")
    return best[1]


def rocksalt_positions(rng, reps, density: float, sigma: float):
    a = (8.0 / density) ** (1.0 / 3.0)
    n1, n2, n3 = reps
    grid = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1).reshape(-1, 3)
    frac = (grid[:, None, :] + ROCKSALT_SITES[None]).reshape(-1, 3)
    pos = frac * a
    pos = pos + rng.normal(0.0, sigma, pos.shape)
    box = np.array([n1 * a, n2 * a, n3 * a])
    return pos, box


def assign_types(rng, n: int, frac_sb: float = 0.4) -> np.ndarray:
    n_sb = int(round(frac_sb * n))
    t = np.full(n, TE, np.int32)
    t[:n_sb] = SB
    return t[rng.permutation(n)].astype(np.int32)


def random_structure(rng, n: int, density: float, dmin: float, kind: str) -> Structure:
    L = (n / density) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    pos = rsa_positions(rng, n, box, dmin)
    return Structure(wrap32(pos, box), box.astype(np.float32), assign_types(rng, n), kind)


def lattice_structure(rng, target: int, lo: int, hi: int, density: float, sigma: float = 0.1) -> Structure:
    reps = rocksalt_reps(target, lo, hi)
    pos, box = rocksalt_positions(rng, reps, density, sigma)
    n = pos.shape[0]
    return Structure(wrap32(pos, box), box.astype(np.float32), assign_types(rng, n), "rocksalt")


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
KINDS3 = ("rocksalt", "liquid", "amorphous")
DMIN = {"liquid": 2.5, "amorphous": 2.7, "hot_liquid": 2.3}


def _mixed(rng, sizes, densities, kinds, lo, hi):
    out = []
    for n, rho, kind in zip(sizes, densities, kinds):
        if kind == "rocksalt":
            out.append(lattice_structure(rng, int(n), lo, hi, float(rho)))
        else:
            out.append(random_structure(rng, int(n), float(rho), DMIN[kind], kind))
    return out


def config_structures(name: str, seed: int = 1234, n_struct: int | None = None):
    """Structures of a named workload.  `n_struct` truncates the list (the
    random draws of the first structures do not depend on it)."""
    rng = np.random.default_rng(seed)
    if name == "c0":
        # 8 periodic cubic cells of 64 atoms, density 0.031, RSA dmin 2.6
        S = 8 if n_struct is None else n_struct
        return [random_structure(rng, 64, 0.031, 2.6, "amorphous") for _ in range(S)]
    if name == "c1":
        S = 64
        sizes = rng.integers(48, 321, S)
        kinds = [KINDS3[k % 3] for k in range(S)]
        dens = np.full(S, 0.031)
    elif name == "c2":
        S = 512
        sizes = np.rint(np.exp(rng.uniform(math.log(32), math.log(512), S))).astype(int)
        kinds = [KINDS3[k % 3] for k in range(S)]
        dens = rng.uniform(0.029, 0.033, S)
    elif name == "c3":
        S = 1
        sizes = np.array([27000])
        kinds = ["amorphous"]
        dens = np.array([0.031])
    elif name == "c4":
        S = 2000
        u = rng.uniform(0.0, 1.0, S)
        sizes = np.rint(1.0 / (1.0 / 32 - u * (1.0 / 32 - 1.0 / 1024))).astype(int)
        kinds = ["hot_liquid" if k % 10 == 9 else KINDS3[k % 3] for k in range(S)]
        dens = rng.uniform(0.029, 0.033, S)
    else:
        raise ValueError(name)
    lo, hi = {"c1": (48, 320), "c2": (32, 512), "c3": (27000, 27000), "c4": (32, 1024)}[name]
    if n_struct is not None:
        sizes, kinds, dens = sizes[:n_struct], kinds[:n_struct], dens[:n_struct]
    if name == "c3":
        # exactly 10,800 Sb and 16,200 Te
        L = (27000 / 0.031) ** (1.0 / 3.0)
        box = np.array([L, L, L])
        pos = rsa_positions(rng, 27000, box, 2.7)
        return [Structure(wrap32(pos, box), box.astype(np.float32), assign_types(rng, 27000), "amorphous")]
    return _mixed(rng, sizes, dens, kinds, lo, hi)


CONFIG_SIZES = {"c0": SIZES_SMALL, "c1": SIZES_SMALL, "c2": SIZES_LARGE,
                "c3": SIZES_LARGE, "c4": SIZES_LARGE}


def draw_params(n_params: int, seed: int, sigma: float = 0.1) -> np.ndarray:
    """Every parameter (descriptor coefficients, weights, biases) ~ N(0, sigma^2)."""
    return np.random.default_rng(seed).normal(0.0, sigma, n_params).astype(np.float32)


def label_noise(batch: Batch, seed: int, e_sigma: float = 1e-3, f_sigma: float = 1e-2):
    """Noise added to teacher labels: per-atom energy noise (so a structure's
    total moves by N_n * eta) and per-component force noise; virials carry none.
    Returns (dE [S] float64, dF [3*N] float64 SoA)."""
    rng = np.random.default_rng(seed)
    sizes = np.diff(batch.atom_offset).astype(np.float64)
    de = sizes * rng.normal(0.0, e_sigma, batch.n_struct)
    df = rng.normal(0.0, f_sigma, 3 * batch.n_atom)
    return de, df


def random_labels(batch: Batch, seed: int):
    """Seeded labels of Sb-Te-like magnitude without a teacher model: total
    energies -0.35 eV/atom with 0.05 eV/atom spread, force components N(0, 0.5)
    eV/A, virial components N_n * N(0, 0.05) eV.  Returns float32 arrays
    (energy [S], force SoA [3N], virial [S*6])."""
    rng = np.random.default_rng(seed)
    sizes = np.diff(batch.atom_offset).astype(np.float64)
    e = sizes * (-0.35 + rng.normal(0.0, 0.05, batch.n_struct))
    f = rng.normal(0.0, 0.5, 3 * batch.n_atom)
    w = (sizes[:, None] * rng.normal(0.0, 0.05, (batch.n_struct, 6))).reshape(-1)
    return e.astype(np.float32), f.astype(np.float32), w.astype(np.float32)


SEEDS = {"data": 1234, "student": 11, "teacher": 22, "noise": 33, "fd": 44, "labels": 55}
