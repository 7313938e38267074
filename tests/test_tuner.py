"""Autotuner host logic (CPU): size buckets, which buckets are tuned, and the
saved table."""
import numpy as np

from paper_2012_12618_amd import binding, tuner


def test_size_buckets():
    assert tuner.size_bucket(0) == 0 and tuner.size_bucket(63) == 0
    assert tuner.size_bucket(64) == 1 and tuner.size_bucket(127) == 1
    assert tuner.size_bucket(128) == 2
    assert tuner.size_bucket(64 << 6) == binding.RV_TUNE_BUCKETS - 1
    assert tuner.size_bucket(10**7) == binding.RV_TUNE_BUCKETS - 1
    for b in range(1, binding.RV_TUNE_BUCKETS - 1):
        assert tuner.size_bucket(32 << b) == b and tuner.size_bucket((64 << b) - 1) == b


def test_buckets_in_use_skip_single_pass_sizes():
    offsets = np.cumsum([0, 8, 200, 256, 257, 3000, 9000]).astype(np.int32)
    # only clusters longer than the smallest tile (4 rows = 256 points) can be affected
    assert tuner.buckets_in_use(offsets) == [tuner.size_bucket(257), tuner.size_bucket(3000),
                                             tuner.size_bucket(9000)]


def test_table_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert tuner.load(path, "gfx950", 512) is None
    t = binding.RVTuning.from_dict({"rows_max": [1, 2, 3, 4, 5, 6, 7, 8], "blocks_per_cu": 3})
    tuner.save(path, "gfx950", 512, t)
    tuner.save(path, "gfx950", 1024, binding.RVTuning.from_dict({"rows_max": [16] * 8}))
    got = tuner.load(path, "gfx950", 512)
    assert got.to_dict() == t.to_dict()
    assert tuner.load(path, "gfx950", 1024).to_dict()["rows_max"] == [16] * 8
    assert tuner.load(path, "other", 512) is None
