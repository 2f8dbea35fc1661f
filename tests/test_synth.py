"""Seeded generators: deterministic, right shapes, valid alphabet (no GPU)."""
import numpy as np

from paper_1404_3456_amd import synth


def test_small_plain_shape_and_determinism():
    a = synth.small_plain()
    b = synth.small_plain()
    assert a.n == 80_400 and a.m == 400
    assert a.sha256() == b.sha256()
    assert np.all(a.lengths == 200)
    assert a.text[-1] == ord("$")
    assert set(np.unique(a.text).tolist()) <= set(b"ACGT$")
    # error-free: each read equals the genome window it was cut from (checked via read overlap)
    seps = np.flatnonzero(a.text == ord("$"))
    assert np.array_equal(seps, np.arange(1, 401) * 201 - 1)


def test_large_plain_sample_scaled():
    s = synth.large_plain(scale=0.01)
    assert s.m == 1000 and s.n == 1000 * 501
    assert np.all(np.diff(np.flatnonzero(s.text == ord("$"))) == 501)


def test_repeat_genome_small():
    rng = np.random.default_rng(0)
    g = synth.repeat_genome(rng, 200_000, n_copies=3, rep_len=5000, n_tandem=20)
    assert g.size == 200_000 and g.max() <= 3


def test_batched_and_serving_generators():
    sets = synth.batched_sets(n_sets=3, g_hi=50_000)
    assert len(sets) == 3
    for s in sets:
        assert s.text[-1] == ord("$")
        assert 100 <= s.lengths.min() and s.lengths.max() <= 1000
    arr, jobs = synth.serving_jobs(n_jobs=4, g_hi=20_000)
    assert arr.size == 4 and np.all(np.diff(arr) >= 0) and arr[0] == 0
    for j in jobs:
        assert j.lengths.min() >= 150 or j.genome_len < 150


def test_text_from_strings():
    t = synth.text_from_strings(["AC", "", "G"])
    assert t.tobytes() == b"AC$$G$"
