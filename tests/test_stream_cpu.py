"""Host logic of the in-situ loop: the replay buffer (newest pair always in the
batch, the others drawn uniformly without replacement, FIFO capacity,
deterministic per seed)."""
from paper_2103_10975_amd.stream import ReplayBuffer


def test_replay_fifo_and_sampling():
    rb = ReplayBuffer(64, seed=4000)
    for t in range(100):
        rb.push(t, t - 1, t)
    assert len(rb) == 64 and rb.items[0][0] == 36 and rb.items[-1][0] == 99
    for _ in range(50):
        idx = rb.sample_indices(8)
        assert idx[0] == 63 and len(idx) == 8 and len(set(idx)) == 8
        assert all(0 <= i < 63 for i in idx[1:])


def test_replay_small_and_deterministic():
    a, b = ReplayBuffer(64, seed=1), ReplayBuffer(64, seed=1)
    for t in range(3):
        a.push(t, 0, 0)
        b.push(t, 0, 0)
    assert a.sample_indices(8) == b.sample_indices(8)
    assert sorted(a.sample_indices(8)) == [0, 1, 2]
    one = ReplayBuffer(4, seed=0)
    one.push("x", 0, 0)
    assert one.sample(8) == [("x", 0, 0)]


def test_replay_uniform_coverage():
    rb = ReplayBuffer(64, seed=7)
    for t in range(64):
        rb.push(t, 0, 0)
    counts = [0] * 63
    for _ in range(3000):
        for i in rb.sample_indices(8)[1:]:
            counts[i] += 1
    mean = sum(counts) / 63
    assert min(counts) > 0.7 * mean and max(counts) < 1.3 * mean
