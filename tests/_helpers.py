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
