"""Host logic of the launch-shape tuner: size classes, the cached lookups,
and the batch option chosen from timed results (no GPU)."""

from paper_1606_07801_amd import tune


def test_size_classes():
    assert tune.size_class((64, 64)) == "tiny"
    assert tune.size_class((4097,)) == "small"
    assert tune.size_class((256, 256)) == "medium"
    assert tune.size_class((4096, 4096)) == "large"
    assert tune.size_class((512, 512, 512)) == "large"


def test_cached_configs_are_valid():
    for d, prec, dims in [(1, 4, (1 << 22,)), (2, 4, (4096, 4096)), (2, 8, (4096, 4096)), (3, 4, (512,) * 3),
                          (2, 4, (32, 32))]:
        cfg = tune.best_config(d, prec, dims)
        assert cfg["kernel"] in ("auto", "plain", "rows", "flat", "resident", "two")
        if cfg["kernel"] == "two":
            assert d == 2
    b = tune.batch_config()
    assert set(b) == set(tune.BATCH_DEFAULT)
    assert b["depth"] in (1, 2) and b["tiling"] in (0, 1) and b["chunk"] >= 1


def test_pick_batch_prefers_whole_member_tiles_on_a_near_tie():
    res = [dict(depth=2, tiling=1, chunk=32, ms=0.4226), dict(depth=2, tiling=0, chunk=32, ms=0.4228),
           dict(depth=2, tiling=0, chunk=8, ms=0.4266), dict(depth=1, tiling=0, chunk=32, ms=0.6172)]
    assert tune.pick_batch(res) == res[1]
    # a clear win for row tiles stands
    res[0]["ms"] = 0.40
    assert tune.pick_batch(res) == res[0]
    # otherwise the fastest
    assert tune.pick_batch([dict(depth=1, tiling=0, chunk=8, ms=1.0), dict(depth=2, tiling=0, chunk=8, ms=0.5)])[
        "depth"] == 2


def test_configs_beyond_the_32_bit_plane_limit_take_the_defaults():
    # D2Q5 FP64 at 4096^2 is tuned to the two-step kernel; a box whose
    # Q N precision reaches 2^32 cannot use it
    small = tune.best_config(2, 8, (4096, 4096))
    big = tune.best_config(2, 8, (10243, 10483))      # 5 * 8 * 10243 * 10483 >= 2^32
    edge = tune.best_config(2, 8, (10243, 10482))     # just below
    if small["kernel"] in ("two", "flat"):
        assert big == tune.DEFAULTS[2] and edge == small
    assert big["kernel"] not in ("two", "flat")
