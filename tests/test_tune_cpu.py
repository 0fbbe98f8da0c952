"""Host logic of the autotuner (paper_2308_10960_amd/tune.py) with the
library calls replaced by stand-ins: which launch strings each candidate
and each (tile shape, column-tile variant) pair is timed with, that the
fastest is returned and left set, and the tune-cache file format.  No GPU
needed."""

import sys
import types

import pytest

from paper_2308_10960_amd import tune


class FakeMatrix:
    def __init__(self, shape=None):
        self.handle = object()
        self.shape = shape
        self.closed = False

    def close(self):
        self.closed = True


class Stand:
    """set_launch records the strings per matrix; the time of a call is
    cost(matrix, its last launch string)."""

    def __init__(self):
        self.calls = {}
        self.cost = lambda D, last: 1.0

    def set_launch(self, handle, text):
        self.calls.setdefault(id(handle), []).append(text)

    def time(self, D, step, reps):
        return self.cost(D, self.calls[id(D.handle)][-1])

    def launches(self, D):
        return self.calls[id(D.handle)]


@pytest.fixture
def stand(monkeypatch):
    s = Stand()
    monkeypatch.setattr(tune.hm, "hm_matrix_set_launch", s.set_launch)
    monkeypatch.setattr(tune, "_time", s.time)
    # tune() and tune_shape() synchronise through torch: a stand-in module
    monkeypatch.setitem(sys.modules, "torch", types.SimpleNamespace(
        cuda=types.SimpleNamespace(synchronize=lambda: None, empty_cache=lambda: None)))
    return s


def test_tune_picks_fastest_candidate_and_leaves_it_set(stand):
    D = FakeMatrix()
    fastest = tune.CANDIDATES[3]
    stand.cost = lambda D, last: 0.5 if last == fastest else 1.0 + tune.CANDIDATES.index(last)
    best, times = tune.tune(D, lambda: None, reps=2, warmup=1)
    assert best == fastest
    assert set(times) == set(tune.CANDIDATES) and times[fastest] == 0.5
    assert stand.launches(D)[-1] == fastest            # the matrix is left on the best


def test_tune_shape_times_every_variant_per_shape(stand):
    made = []

    def make(chunk, tile, mix):
        D = FakeMatrix((chunk, tile, mix))
        made.append(D)
        return D

    def cost(D, last):                                 # cheapest: 256 x 32, one format, a wave per tile
        c, t, mx = D.shape
        base = {512: 3.0, 256: 1.0, 128: 2.0, 64: 4.0}[c] + (0.0 if t == 32 else 0.5) + (mx - 1) * 0.25
        return base - (0.125 if last.endswith("colw=2") else 0.0)

    stand.cost = cost
    best, times = tune.tune_shape(make, lambda D: (lambda: None), "schedule=0 unroll=4",
                                  variants=tune.COLW_VARIANTS, reps=1, warmup=0)
    assert best == (256, 32, 1, "colw=2")
    assert len(times) == len(tune.SHAPE_CANDIDATES) * len(tune.COLW_VARIANTS)
    assert [D.shape for D in made] == list(tune.SHAPE_CANDIDATES)
    assert all(D.closed for D in made)                 # every shape's matrix is released
    for D in made:                                     # each variant after the launch line
        assert stand.launches(D) == ["schedule=0 unroll=4 " + v for v in tune.COLW_VARIANTS]


def test_tune_shape_without_variants_keeps_the_launch_line(stand):
    made = []

    def make(chunk, tile, mix):
        D = FakeMatrix((chunk, tile, mix))
        made.append(D)
        return D

    stand.cost = lambda D, last: float(D.shape[0])
    best, times = tune.tune_shape(make, lambda D: (lambda: None), "schedule=0 unroll=8 colb=1",
                                  candidates=[(512, 64, 1), (128, 64, 1)], reps=1, warmup=0)
    assert best == (128, 64, 1, "")
    assert all(stand.launches(D) == ["schedule=0 unroll=8 colb=1"] for D in made)


def test_write_cache_replaces_the_key_line(tmp_path):
    path = str(tmp_path / "cache.txt")
    tune.write_cache(path, "acc0-fmt1-n2^18-r3", "schedule=0 unroll=8")
    tune.write_cache(path, "acc0-fmt16-n2^18-r3", "schedule=0 unroll=4 colw=2")
    tune.write_cache(path, "acc0-fmt1-n2^18-r3", "schedule=1 unroll=4 colw=0")
    assert open(path).read().splitlines() == ["acc0-fmt16-n2^18-r3 schedule=0 unroll=4 colw=2",
                                              "acc0-fmt1-n2^18-r3 schedule=1 unroll=4 colw=0"]
