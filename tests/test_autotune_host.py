"""Host logic of the autotuner, without a GPU: size buckets and the JSON cache (round trip,
atomic replace, unreadable files ignored)."""
import json

from paper_1404_3456_amd import autotune


def test_buckets_are_the_next_power_of_two():
    assert [autotune._bucket(x) for x in (0, 1, 2, 3, 4, 5, 1000, 1024, 1025)] == \
        [1, 1, 2, 4, 4, 8, 1024, 1024, 2048]


def test_cache_round_trip_and_bad_files(tmp_path):
    path = str(tmp_path / "sub" / "cache.json")
    assert autotune._load(path) == {}
    data = {"dev|n1024|sets1": {"digit_bits": 9, "block_threads": 1024, "items_per_thread": 16}}
    autotune._save(path, data)
    assert autotune._load(path) == data
    assert not (tmp_path / "sub" / "cache.json.tmp").exists()
    (tmp_path / "sub" / "cache.json").write_text("{not json")
    assert autotune._load(path) == {}
    json.loads(json.dumps(data))  # entries stay plain JSON


def test_candidates_are_accepted_tunings():
    from paper_1404_3456_amd import _abi
    for d, b, i in autotune.TILE_CANDIDATES:
        assert _abi.sa_build_ws_bytes(1000, _abi.Tuning(d, b, i, 0)) > 0, (d, b, i)
