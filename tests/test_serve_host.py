"""Host logic of the solve server's HBM admission (no GPU): entries of
problem shapes are created while the budget allows, idle shapes are evicted
least recently used first, busy or in-flight shapes never, and a shape that
cannot fit even alone is refused.  The device entry is replaced by a stand-in
with the same footprint fields."""

import pytest

from paper_2512_20269_amd import serve


class FakeEntry:
    def __init__(self, key, slots, tune, device, k, graphs):
        self.key = key
        self.bytes = SIZES[key][0]
        self.busy = {}
        self.inflight = False
        self.free = list(range(slots))


# (entry bytes, N) per shape
SIZES = {(2, 64, 3): (1000, 10), (3, 32, 3): (3000, 100), (3, 64, 4): (9000, 500)}


@pytest.fixture
def server(monkeypatch):
    monkeypatch.setattr(serve, "_Entry", FakeEntry)
    monkeypatch.setattr(serve.SolveServer, "entry_bytes",
                        classmethod(lambda cls, key, slots: SIZES.get(key, (None, None))))
    return serve.SolveServer(hbm_budget=10000, slots=4)


def test_entries_created_within_budget(server):
    e1 = server._entry_for((2, 64, 3), now=0.0)
    e2 = server._entry_for((3, 32, 3), now=1.0)
    assert e1 is not None and e2 is not None
    assert server.used == 4000 and server.peak == 4000
    # the same shape again: the existing entry, moved to most recently used
    assert server._entry_for((2, 64, 3), now=2.0) is e1
    assert list(server.entries) == [(3, 32, 3), (2, 64, 3)]


def test_idle_shapes_evicted_least_recently_used_first(server):
    server._entry_for((2, 64, 3), now=0.0)
    server._entry_for((3, 32, 3), now=1.0)
    server._entry_for((2, 64, 3), now=2.0)            # (3, 32, 3) is now the oldest
    e = server._entry_for((3, 64, 4), now=3.0)        # 9000 + 8*500 > 10000 even when empty
    assert e is None
    assert list(server.entries) == [(3, 32, 3), (2, 64, 3)]   # nothing evicted in vain
    assert not server.fits_alone(serve.Request(0, 0.0, 3, 64, 4, None))
    SIZES[(3, 48, 4)] = (5500, 100)
    try:
        e = server._entry_for((3, 48, 4), now=4.0)     # 5500 + 800: evict (3, 32, 3) only
        assert e is not None
        assert list(server.entries) == [(2, 64, 3), (3, 48, 4)]
        assert server.used == 1000 + 5500
    finally:
        del SIZES[(3, 48, 4)]


def test_busy_or_inflight_shapes_are_never_evicted(server):
    a = server._entry_for((2, 64, 3), now=0.0)
    b = server._entry_for((3, 32, 3), now=1.0)
    a.busy[0] = object()
    b.inflight = True
    SIZES[(3, 40, 4)] = (6500, 100)
    try:
        assert server._entry_for((3, 40, 4), now=2.0) is None   # nothing evictable
        assert set(server.entries) == {(2, 64, 3), (3, 32, 3)}
        assert server.used == 4000
        b.inflight = False
        assert server._entry_for((3, 40, 4), now=3.0) is not None   # b goes, a stays
        assert set(server.entries) == {(2, 64, 3), (3, 40, 4)}
    finally:
        del SIZES[(3, 40, 4)]


def test_unsupported_shape_refused(server):
    assert server._entry_for((3, 100, 3), now=0.0) is None
    assert not server.fits_alone(serve.Request(0, 0.0, 3, 100, 3, None))
