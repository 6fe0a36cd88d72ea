"""Host-side bookkeeping of the training driver: mini-batch partitions and
the step counts of the Eq. 17 schedule (Sec. II D)."""
import numpy as np
import pytest

from paper_2507_00528_amd.train import LabelSet, epoch_batches, schedule_steps


@pytest.mark.parametrize("n,bs", [(1, 1), (7, 1), (7, 3), (64, 8), (65, 8), (5, 10)])
def test_epoch_batches_cover_every_structure_once(n, bs):
    batches = epoch_batches(n, bs, np.random.default_rng(3))
    assert len(batches) == -(-n // bs)
    assert all(len(b) == bs for b in batches[:-1]) and 1 <= len(batches[-1]) <= bs
    assert sorted(np.concatenate(batches).tolist()) == list(range(n))


def test_epoch_batches_are_seeded():
    a = epoch_batches(50, 4, np.random.default_rng(11))
    b = epoch_batches(50, 4, np.random.default_rng(11))
    c = epoch_batches(50, 4, np.random.default_rng(12))
    assert all((x == y).all() for x, y in zip(a, b))
    assert any((x != y).any() for x, y in zip(a, c))


def test_epoch_batches_reject_empty():
    with pytest.raises(ValueError):
        epoch_batches(0, 1, np.random.default_rng(0))
    with pytest.raises(ValueError):
        epoch_batches(4, 0, np.random.default_rng(0))


def test_schedule_steps_follow_the_epoch_definitions():
    # N_warmup = warm-up epochs x batches per epoch, N_total = epochs x batches per epoch
    assert schedule_steps(100, 1, 512) == (512, 51200)
    assert schedule_steps(10, 0.5, 8) == (4, 80)
    assert schedule_steps(3, 0, 5) == (0, 15)


def test_label_subset_keeps_structure_order():
    lab = LabelSet(np.arange(4.0), [np.full((k + 1, 3), k) for k in range(4)], np.arange(24.0).reshape(4, 6))
    sub = lab.subset(np.array([2, 0]))
    assert sub.energy.tolist() == [2.0, 0.0]
    assert [f.shape[0] for f in sub.force] == [3, 1]
    assert sub.virial[0, 0] == 12.0
