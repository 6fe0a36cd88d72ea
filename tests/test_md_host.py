"""Host helpers of the inference path: Maxwell-Boltzmann velocities and the
radial distribution function (an ideal gas has g(r) = 1)."""
import numpy as np

from paper_2507_00528_amd import md


def test_maxwell_velocities_temperature_and_zero_momentum():
    types = np.array([0, 1] * 2000)
    masses = [121.76, 127.6]
    v = md.maxwell_velocities(types, masses, 600.0, seed=4).reshape(3, -1).astype(np.float64)
    m = np.asarray(masses)[types]
    ke = 0.5 * (m * (v ** 2).sum(0)).sum() / md.ACCEL
    t = 2 * ke / (3 * len(types) * md.KB)
    assert abs(t - 600.0) / 600.0 < 0.05
    assert np.abs((m * v).sum(1)).max() < 1e-3


def test_rdf_of_uniform_points_is_one():
    rng = np.random.default_rng(1)
    box = np.array([30.0, 30.0, 30.0])
    pos = rng.uniform(0, 30.0, size=(3000, 3))
    r, g = md.rdf(pos, box, 12.0, nbins=24)
    assert np.abs(g[4:] - 1.0).max() < 0.1


def test_rdf_of_simple_cubic_lattice_has_its_shells():
    a = 3.0
    grid = np.arange(8) * a
    pos = np.stack(np.meshgrid(grid, grid, grid, indexing="ij"), -1).reshape(-1, 3)
    r, g = md.rdf(pos, np.array([24.0] * 3), 7.0, nbins=70)
    peaks = r[g > 1.0]
    assert np.all(np.abs(peaks[:, None] - np.array([3.0, 3.0 * 2 ** 0.5, 3.0 * 3 ** 0.5, 6.0, 3.0 * 5 ** 0.5])[None, :]).min(1) < 0.1)
    assert g[r < 2.9].max() == 0.0
