"""The batch decomposition of the batched path (static schedule of work
units over the persistent kernel's waves), checked on the host through
tsqbx_schedule_preview: no device is touched."""
import numpy as np
import pytest

from paper_1811_01110_amd import _lib as L
from paper_1811_01110_amd import api


def _covered(units, items):
    seen = [np.zeros(len(r), dtype=np.int64) for r, _, _ in items]
    for it, first, cnt in units:
        assert cnt > 0
        seen[it][first:first + cnt] += 1
    return seen


def _random_items(seed, n, max_t=300, max_len=400):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        t = int(rng.integers(0, max_t))
        out.append((rng.integers(0, max_len, t), int(rng.choice([0, 4, 8, 16, 24])),
                    int(rng.choice([1, 2, 3, 4, 7]))))
    return out


@pytest.mark.parametrize("G", [16, 32, 64])
@pytest.mark.parametrize("max_waves", [1, 7, 64, 5000])
def test_every_target_once_and_waves_contiguous(G, max_waves):
    items = _random_items(G * 1000 + max_waves, 12)
    units, wb = api.schedule_preview(items, group_lanes=G, max_waves=max_waves)
    assert all(np.all(s == 1) for s in _covered(units, items))
    assert wb[0] == 0 and wb[-1] == len(units) and np.all(np.diff(wb) >= 0)
    assert 1 <= len(wb) - 1 <= max_waves
    # within a wave, consecutive units of one item are merged into one run
    for w in range(len(wb) - 1):
        us = units[wb[w]:wb[w + 1]]
        for a, b in zip(us[:-1], us[1:]):
            assert not (a[0] == b[0] and a[1] + a[2] == b[1])
    # group-sized steps: unit boundaries fall on multiples of 64/G targets
    tpw = 64 // G
    for it, first, cnt in units:
        assert first % tpw == 0
        assert cnt % tpw == 0 or first + cnt == len(items[it][0])


def test_items_largest_first():
    """Items are laid out by estimated cost, largest first (ties in order)."""
    rl = lambda t, n: np.full(t, n, dtype=np.int64)
    items = [(rl(10, 50), 8, 1), (rl(200, 300), 16, 3), (rl(50, 100), 4, 1), (rl(200, 300), 16, 3)]
    units, _ = api.schedule_preview(items, group_lanes=64, max_waves=3)
    order = []
    for it, _, _ in units:
        if not order or order[-1] != it:
            order.append(int(it))
    assert order == [1, 3, 2, 0]


def test_equal_steps_are_dealt_evenly():
    """Uniform items: every wave gets the same number of targets, give or take
    one wave-step."""
    items = [(np.full(640, 200, dtype=np.int64), 16, 1) for _ in range(4)]
    units, wb = api.schedule_preview(items, group_lanes=16, max_waves=32)
    per_wave = [int(units[wb[w]:wb[w + 1], 2].sum()) for w in range(len(wb) - 1)]
    assert len(per_wave) == 32 and sum(per_wave) == 2560
    assert max(per_wave) - min(per_wave) <= 4


def test_edge_cases_and_errors():
    units, wb = api.schedule_preview([], group_lanes=16, max_waves=8)
    assert len(units) == 0 and list(wb) == [0]
    units, wb = api.schedule_preview([(np.zeros(0, dtype=np.int64), 8, 1)], 16, 8)
    assert len(units) == 0
    units, wb = api.schedule_preview([(np.zeros(5, dtype=np.int64), 8, 1)], 64, 8)
    assert int(units[:, 2].sum()) == 5  # empty lists still get a unit (their outputs are written)
    with pytest.raises(api.TsqbxError) as e:
        api.schedule_preview([(np.ones(3, dtype=np.int64), 33, 1)], 16, 8)
    assert e.value.code == L.E_RANGE
    with pytest.raises(api.TsqbxError) as e:
        api.schedule_preview([(np.ones(3, dtype=np.int64), 8, 0)], 16, 8)
    assert e.value.code == L.E_INVALID
    with pytest.raises(api.TsqbxError) as e:
        api.schedule_preview([(np.ones(3, dtype=np.int64), 8, 1)], 8, 8)
    assert e.value.code == L.E_INVALID
    with pytest.raises(api.TsqbxError) as e:
        api.schedule_preview([(-np.ones(3, dtype=np.int64), 8, 1)], 16, 8)
    assert e.value.code == L.E_RANGE
    lib = api._lib()
    assert lib.tsqbx_schedule_preview(1, None, None, None, None, 16, 8, None, 0, None, None,
                                      None) == L.E_INVALID
