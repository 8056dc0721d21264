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


# ---------------------------------------------------------------- Algorithm 1
import numpy as np

from paper_2103_10975_amd.stream import SelectiveCollector, cosine, moving_average


def test_moving_average_is_the_mean_of_the_last_p():
    ys = [5.0, 1.0, 2.0, 3.0, 10.0]
    assert moving_average(ys, 3) == (2.0 + 3.0 + 10.0) / 3
    assert moving_average(ys[:2], 4) == 3.0              # fewer than p values: all of them
    assert moving_average([7.0], 10) == 7.0


def test_collector_passes_only_below_both_averages():
    c = SelectiveCollector(p=4, f_r=100)
    x = np.ones(3)
    # E_k and TOS both falling: each new value is below the mean that includes it
    for e, t in [(1.0, 1.0), (0.5, 0.9), (0.4, 0.8)]:
        c.observe(e, t, ("pair", e), x * e)
    assert c.failures == 1                               # the first step equals its own mean
    # E_k below average but TOS above: under-performing
    assert not c.passes(0.1, 5.0)
    # both below
    assert c.passes(0.05, 0.1)


def test_collector_orthogonality_filter_and_retrain_trigger():
    c = SelectiveCollector(p=3, f_r=3, cos_max=0.9)
    e1, e2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    # three under-performing steps (rising E_k and TOS never pass)
    assert c.observe(1.0, 1.0, "a", e1) is False          # candidate (set was empty)
    assert c.observe(2.0, 2.0, "b", 3.0 * e1 + 0.1 * e2) is False   # |cos| > 0.9: rejected
    assert c.observe(3.0, 3.0, "c", e2) is True            # orthogonal: kept; f_r reached
    assert c.candidates == ["a", "c"] and c.retained == 2 and c.seen == 3
    assert c.drain() == ["a", "c"]
    assert c.candidates == [] and c.failures == 0
    # cosine is the absolute normalised inner product, 0 for a zero vector
    assert abs(cosine(e1, -2.0 * e1) - 1.0) < 1e-15 and cosine(e1, np.zeros(3)) == 0.0


def test_block_growth_on_stagnation():
    from paper_2103_10975_amd.stream import BlockGrowth
    g = BlockGrowth(window=4, min_gain=0.1, max_blocks=2)
    # falling fast: no growth
    for v in [100, 90, 80, 70, 50, 45, 40, 35]:
        assert not g.observe(v)
    # window mean 40 vs previous 42.5: less than 10 % better -> grow
    grown = [g.observe(v) for v in [41, 40, 40, 39]]
    assert grown == [False, False, False, True] and g.blocks == 1 and g.events == [(12, 1)]
    # the comparison restarts: the next window only sets the reference
    assert not any(g.observe(v) for v in [40, 40, 40, 40])
    for v in [40, 40, 40]:
        assert not g.observe(v)
    assert g.observe(40) and g.blocks == 2
    # at the cap nothing more grows
    for _ in range(3):
        assert not any(g.observe(40) for _ in range(4))
    assert g.blocks == 2


def test_fluid_levels():
    from paper_2103_10975_amd.stream import fluid_levels
    assert fluid_levels((512, 512)) == 6
    assert fluid_levels((256, 256)) == 6
    assert fluid_levels((64, 64)) == 4       # 64 -> 8 at the coarsest
    assert fluid_levels((96, 136)) == 4      # 136 = 8 * 17
    assert fluid_levels((50, 64)) == 2       # 50 = 2 * 25
    assert fluid_levels((7, 9)) == 1


def test_record_json_writes_nan_as_null():
    import json
    from paper_2103_10975_amd.stream import StepRecord, record_json
    rec = StepRecord(3, "learned", 17, 1, 1.3e-5, 2e-9, 9e-9, 4.7e-4, relres_iter5=float("nan"))
    rec.extra["train_steps"] = 1
    d = json.loads(record_json(rec))
    assert d["t"] == 3 and d["guess"] == "learned" and d["iters"] == 17
    assert d["relres_iter5"] is None and d["loss"] is None
    assert d["extra"] == {"train_steps": 1}
    assert list(d) == sorted(d)
