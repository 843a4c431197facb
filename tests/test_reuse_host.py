"""The host replay of the exact walker's loads (tests/host/reuse_host.hip):
its stack-distance LRU counts against a plain LRU cache run over the same
request sequence, and its bookkeeping invariants."""
import collections
import shutil

import numpy as np
import pytest

import inputs
from tests import reuse_replay as R


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    return R.build(str(tmp_path_factory.mktemp("reusehost")))


@pytest.fixture(scope="module")
def tiny():
    return inputs.load_workload("tiny", keep_dvr=False)


def lru_hits(lines, streams, cap):
    """Hits per stream of one LRU cache of `cap` lines, request by request."""
    cache = collections.OrderedDict()
    hits = np.zeros(4)
    for line, s in zip(lines.tolist(), streams.tolist()):
        if line in cache:
            hits[s] += 1
            cache.move_to_end(line)
        else:
            cache[line] = True
            if len(cache) > cap:
                cache.popitem(last=False)
    return hits


@pytest.mark.parametrize("theta", [25.0, -60.0])
def test_stack_distances_match_a_plain_lru(lib, tiny, theta):
    """One 8x8 frame is one tile: the replay's counts at every capacity equal
    those of an LRU cache simulated request by request."""
    cam = inputs.orbit_camera(theta)
    lines, streams = R.tile_trace(lib, tiny, cam, 8, 8, 0, 0)
    assert len(lines) > 200
    st = R.replay(lib, tiny, cam, 8, 8, 1, caps=(1, 4, 16, 64, 1 << 30))
    assert np.array_equal(st[:, 0], np.bincount(streams, minlength=4))
    firsts = {}
    for i, line in enumerate(lines.tolist()):
        firsts.setdefault(line, i)
    cold = np.bincount(streams[sorted(firsts.values())], minlength=4)
    assert np.array_equal(st[:, 1], cold)
    for c, cap in enumerate((1, 4, 16, 64, 1 << 30)):
        assert np.array_equal(st[:, 2 + c], lru_hits(lines, streams, cap)), cap


def test_bookkeeping(lib, tiny):
    """Hits never fall as the cache grows; unbounded, every request after a
    line's first hits."""
    st = R.replay(lib, tiny, inputs.orbit_camera(40.0), 64, 48, 1)
    assert st[:, 0].sum() > 0
    assert np.all(np.diff(st[:, 2:], axis=1) >= 0)
    assert np.array_equal(st[:, -1], st[:, 0] - st[:, 1])
    # every exact ray reads at least its first list's count
    assert st[0, 0] > 0 and st[2, 0] > 0
