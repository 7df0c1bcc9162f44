"""Host logic of the tile-shape autotuner (no device work)."""
from paper_2204_13241_amd import tune


def test_candidate_spaces_hold_the_default_shapes():
    assert (32, 0, 64) in tune.FWD_CANDIDATES and (8, 4, 64) in tune.FWD_CANDIDATES
    assert (2, 5, 8192) in tune.GRAD_CANDIDATES and (32, 0, 128) in tune.GRAD_CANDIDATES


def test_current_shape_is_timed_first_and_the_rest_keep_their_order():
    cands = tune.GRAD_CANDIDATES
    order = tune._current_first(cands, (2, 5, 8192))
    assert order[0] == (2, 5, 8192)
    assert sorted(order) == sorted(cands) and len(order) == len(cands)
    rest = [c for c in cands if c != (2, 5, 8192)]
    assert order[1:] == rest
    # a shape outside the list leaves the list unchanged
    assert tune._current_first(cands, (3, 0, 1)) == list(cands)


def test_bucket_is_the_nearest_power_of_two():
    assert tune._bucket(0) == 0
    assert tune._bucket(65536) == 16
    assert tune._bucket(262144) == 18
    assert tune._bucket(90000) == 16 and tune._bucket(100000) == 17


def test_cache_roundtrip_and_unreadable_file(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert tune._load_cache(p) == {}
    tune._store_cache(p, {"k": {"forward": {"q_per_lane": 8}}})
    assert tune._load_cache(p) == {"k": {"forward": {"q_per_lane": 8}}}
    with open(p, "w") as fh:
        fh.write("{not json")
    assert tune._load_cache(p) == {}
    assert 0.0 < tune.TIE < 0.1


def test_pick_keeps_the_installed_shape_within_the_margin():
    cur = (8, 4, 64)
    t = {cur: 1.00, (8, 0, 32): 0.98, (4, 4, 64): 1.20}
    assert tune._pick(t, cur) == cur
    t[(8, 0, 32)] = 0.95
    assert tune._pick(t, cur) == (8, 0, 32)
    # a shape that is not a candidate: the fastest wins
    assert tune._pick({(1, 0, 16): 2.0, (2, 0, 16): 1.5}, cur) == (2, 0, 16)


def test_search_times_the_installed_shape_twice_and_keeps_the_better():
    calls = []
    seq = iter([1.10, 1.05, 1.20, 0.99])

    def timer(c):
        calls.append(c)
        return next(seq)
    cands = [(1, 0, 16), (8, 4, 64), (2, 0, 16)]
    times = tune._search(cands, (8, 4, 64), timer)
    assert calls == [(8, 4, 64), (1, 0, 16), (2, 0, 16), (8, 4, 64)]
    assert times[(8, 4, 64)] == 0.99 and times[(1, 0, 16)] == 1.05


def test_per_pair_search_leaves_out_the_factorized_shapes():
    f0, g0 = tune.candidates(tune.FWD_CANDIDATES, 0), tune.candidates(tune.GRAD_CANDIDATES, 0)
    assert f0 and g0 and all(c[0] in (1, 2, 4, 8) for c in f0 + g0)
    assert (32, 0, 64) in tune.candidates(tune.FWD_CANDIDATES, 1)
    assert len(tune.candidates(tune.GRAD_CANDIDATES, 1)) == len(tune.GRAD_CANDIDATES)
