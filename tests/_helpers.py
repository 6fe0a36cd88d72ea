"""Small shared fixtures for the oracle pin tests (inputs only)."""
import numpy as np

from paper_2507_00528_amd import synth


def small_structures(seed=5, sizes=(10, 14), density=0.031, dmin=2.4):
    rng = np.random.default_rng(seed)
    return [synth.random_structure(rng, n, density, dmin, "liquid") for n in sizes]


def cluster(seed=3, n=7, spread=2.0, box=40.0):
    """An isolated cluster in a large periodic box (no image is in range)."""
    rng = np.random.default_rng(seed)
    while True:
        p = rng.normal(0, spread, (n, 3))
        d = np.linalg.norm(p[:, None] - p[None], axis=-1) + np.eye(n) * 9
        if d.min() > 1.6:
            break
    p = p - p.mean(0) + box / 2
    return synth.Structure(p.astype(np.float32), np.full(3, box, np.float32),
                           (np.arange(n) % 2).astype(np.int32), "cluster")


# ---------------------------------------------------------------- triclinic cells
def hmat(box, tilt):
    lx, ly, lz = np.asarray(box, np.float32).astype(np.float64)
    xy, xz, yz = np.asarray(tilt, np.float32).astype(np.float64)
    return np.array([[lx, xy, xz], [0, ly, yz], [0, 0, lz]])


def widths(H):
    a, b, c = H.T
    V = abs(np.linalg.det(H))
    return np.array([V / np.linalg.norm(np.cross(b, c)), V / np.linalg.norm(np.cross(c, a)),
                     V / np.linalg.norm(np.cross(a, b))])


def grid_structure(seed, n, L):
    """An orthorhombic cell of edge L whose coordinates are multiples of 1/256,
    so that adding an edge vector is exact in float32."""
    rng = np.random.default_rng(seed)
    while True:
        p = np.round(rng.uniform(0, L, (n, 3)) * 256) / 256
        p = np.where(p >= L, 0.0, p)
        box = np.full(3, L)
        d = np.linalg.norm((p[:, None] - p[None] + L / 2) % L - L / 2, axis=-1) + np.eye(n) * 9
        if d.min() > 1.9:
            break
    return synth.Structure(p.astype(np.float32), box.astype(np.float32), (np.arange(n) % 2).astype(np.int32), "grid")


def sheared(st, tilt):
    """The same crystal in the cell with the given tilts, which are integer
    combinations of the orthorhombic edges: positions moved by whole edge
    vectors into the new cell (exact in float32)."""
    H = hmat(st.box, tilt)
    x = st.pos.astype(np.float64)
    f = np.linalg.solve(H, x.T).T
    k = np.floor(f)
    x2 = x - k @ H.T
    assert np.all(x2.astype(np.float32).astype(np.float64) == x2)
    return synth.Structure(x2.astype(np.float32), st.box, st.types, "sheared", np.asarray(tilt, np.float32))
