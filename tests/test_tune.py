"""Host logic of the switch-threshold autotuner (no device)."""
from paper_1208_2675_amd import tune


def test_switch_for_picks_the_bucket_then_the_nearest():
    table = {"iters": 1, "buckets": [
        {"lo": 20, "hi": 60, "symmetric": True, "switch_permille": 40},
        {"lo": 60, "hi": 100, "symmetric": True, "switch_permille": 10},
        {"lo": 20, "hi": 60, "symmetric": False, "switch_permille": 80},
    ]}
    assert tune.switch_for(table, 20, True) == 40
    assert tune.switch_for(table, 59, True) == 40
    assert tune.switch_for(table, 60, True) == 10
    assert tune.switch_for(table, 500, True) == 10      # nearest bucket
    assert tune.switch_for(table, 5, True) == 40
    assert tune.switch_for(table, 90, False) == 80      # the only asymmetric bucket
    assert tune.switch_for(None, 90, False) == 10       # no table: the library default


def test_representatives_have_the_bucket_shape():
    ch = tune._representative(100, 140, False, 1000)
    assert ch.n == 120 and not ch.symmetric and ch.iters == 1000
    assert (ch.A.diagonal() == 0).all()
    ch = tune._representative(20, 60, True, 10)
    assert ch.n == 40 and (ch.A == ch.A.T).all() and (ch.B == ch.B.T).all()


def test_dispatch_for_takes_the_nearest_measured_size():
    table = {"iters": 1, "entries": [
        {"n": 200, "symmetric": True, "flags": tune.FLAG_SINGLE_WG, "scan_window": 1024},
        {"n": 700, "symmetric": True, "flags": tune.FLAG_MULTI_WG, "scan_window": 4096},
        {"n": 300, "symmetric": False, "flags": tune.FLAG_MULTI_WG, "scan_window": 16384},
    ]}
    assert tune.dispatch_for(table, 200, True) == (tune.FLAG_SINGLE_WG, 1024)
    assert tune.dispatch_for(table, 449, True) == (tune.FLAG_SINGLE_WG, 1024)
    assert tune.dispatch_for(table, 451, True) == (tune.FLAG_MULTI_WG, 4096)
    assert tune.dispatch_for(table, 5000, True) == (tune.FLAG_MULTI_WG, 4096)
    assert tune.dispatch_for(table, 120, True) == (0, 0)       # one workgroup's LDS: the library decides
    assert tune.dispatch_for(table, 2000, False) == (tune.FLAG_MULTI_WG, 16384)
    assert tune.dispatch_for(None, 2000, False) == (0, 0)
