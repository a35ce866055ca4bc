"""Launch-parameter table of qless_tsqr_r (host side; no GPU needed)."""
import json

import pytest

import paper_2603_20889_amd as q
from paper_2603_20889_amd import autotune


@pytest.fixture(autouse=True)
def reset_tuning():
    yield
    for n in range(1, 65):
        q.qless_tune_set(n, 0, 0, 0)


def test_defaults_and_round_trip():
    # default fan-in for n <= 16: one panel (64 lanes x rows_per_lane rows) of
    # stacked n-row triangles per tree wavefront; 4 for wider n
    d = q.qless_tune_get(8)
    assert d == {"waves_per_cu": 8, "fan_in": 64 * 4 // 8, "rows_per_lane": 4}
    assert q.qless_tune_get(16)["fan_in"] == 64 * 4 // 16
    assert q.qless_tune_get(32)["fan_in"] == 4
    q.qless_tune_set(8, 12, 32, 4)
    assert q.qless_tune_get(8) == {"waves_per_cu": 12, "fan_in": 32, "rows_per_lane": 4}


def test_invalid_and_unsupported_values():
    with pytest.raises(q.QlessError):
        q.qless_tune_set(0, 8, 16, 0)
    with pytest.raises(q.QlessError):
        q.qless_tune_set(8, 64, 16, 0)
    with pytest.raises(q.QlessError):
        q.qless_tune_set(8, 8, 1, 0)
    with pytest.raises(q.QlessError) as e:
        q.qless_tune_set(8, 8, 16, 3)          # no compiled 3-rows-per-lane variant for n = 8
    assert e.value.status == q.QLESS_ERR_UNSUPPORTED


def test_tuning_changes_the_plan():
    base = q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, 50_000_000, 8)
    q.qless_tune_set(8, 16, 0, 0)     # twice the stage-1 blocks -> more stacked triangles
    assert q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, 50_000_000, 8) > base


def test_variants_listed():
    assert autotune.rows_per_lane_variants(8) == [4, 8]
    assert autotune.rows_per_lane_variants(16) == [4, 2, 3]
    # n > 16: the 8 x 8 column-group variants, the matrix-core fold (one row
    # per lane) and the 4 x 16 column-group fold (the default for 48 and 64)
    assert autotune.rows_per_lane_variants(32) == [16, 1, 8, 24]
    assert autotune.rows_per_lane_variants(48) == [16, 1, 10]
    assert autotune.rows_per_lane_variants(64) == [12, 1, 4, 7]
    assert autotune.rows_per_lane_variants(24) == [21]


def test_matrix_core_instance_selection():
    """n in (16, 64] with rows_per_lane 1 selects the matrix-core fold; the
    widths that pad to 24, 40 or 56 columns have no such instance."""
    q.qless_tune_set(32, 8, 0, 1)
    assert q.qless_tune_get(32)["rows_per_lane"] == 1
    q.qless_tune_set(61, 8, 0, 1)
    assert q.qless_tune_get(61)["rows_per_lane"] == 1
    for n in (24, 40, 56):
        with pytest.raises(q.QlessError) as e:
            q.qless_tune_set(n, 8, 0, 1)
        assert e.value.status == q.QLESS_ERR_UNSUPPORTED


def test_apply_and_cache_file(tmp_path, monkeypatch):
    table = {"8": {"rows_per_lane": 4, "waves_per_cu": 12, "fan_in": 8, "ms": 1.0}}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"fakegpu|v": table}))
    monkeypatch.setattr(autotune, "_key", lambda device: "fakegpu|v")
    got = autotune.apply_cached(device="x", path=str(path))
    assert got == table
    assert q.qless_tune_get(8) == {"waves_per_cu": 12, "fan_in": 8, "rows_per_lane": 4}
    monkeypatch.setenv("QLESS_TUNE", "off")
    assert autotune.apply_cached(device="x", path=str(path)) is None


def _fake_timer(monkeypatch, true_ms, lucky=None):
    """Replace the GPU timing by a function of the configuration in effect:
    true_ms(config) for every call, except that the configuration `lucky`
    times 20 % fast on its first (screening) call only."""
    seen = set()

    def fake(X, steps, flush=None):
        n = X.shape[1]
        t = q.qless_tune_get(n)
        c = (t["rows_per_lane"], t["waves_per_cu"], t["fan_in"])
        ms = true_ms(c)
        if c == lucky and c not in seen:
            seen.add(c)
            return 0.8 * ms
        return ms

    monkeypatch.setattr(autotune, "_time_tsqr", fake)


def test_tuner_keeps_default_against_a_lucky_screen(monkeypatch):
    """A configuration that is fast only on its screening call does not
    survive the confirmation rounds."""
    d = q.qless_tune_get(8)
    lucky = (8, 16, 32)
    _fake_timer(monkeypatch, lambda c: 1.0, lucky=lucky)
    table = autotune.tune_tsqr([8], device="cpu", m=1024, log=lambda *a: None)
    got = table[8]
    assert (got["rows_per_lane"], got["waves_per_cu"], got["fan_in"]) == (d["rows_per_lane"], d["waves_per_cu"], 0)
    assert got["ms"] == got["default_ms"] == 1.0


def test_tuner_takes_a_confirmed_gain(monkeypatch):
    """A configuration at least min_gain faster on every round is chosen; one
    under the threshold is not."""
    better = (8, 12, 16)
    _fake_timer(monkeypatch, lambda c: 0.95 if c == better else 1.0)
    got = autotune.tune_tsqr([8], device="cpu", m=1024, log=lambda *a: None)[8]
    assert (got["rows_per_lane"], got["waves_per_cu"], got["fan_in"]) == better
    assert q.qless_tune_get(8) == {"rows_per_lane": 8, "waves_per_cu": 12, "fan_in": 16}
    _fake_timer(monkeypatch, lambda c: 0.99 if c == better else 1.0)
    got = autotune.tune_tsqr([8], device="cpu", m=1024, log=lambda *a: None)[8]
    assert (got["waves_per_cu"], got["fan_in"]) == (q.qless_tune_get(8)["waves_per_cu"], 0)


def _fake_batched(monkeypatch, cost, lucky=None):
    """BatchPlan stand-in whose run() advances a fake clock by cost(key) per
    call ((tile_bytes, waves_per_cu) -> seconds); `lucky` runs 20 % fast in
    its first plan only."""
    import torch
    clock = [0.0]
    plans = []

    class FakePlan:
        def __init__(self, Xs, tile_bytes=0, waves_per_cu=0):
            self.key = (tile_bytes, waves_per_cu)
            self.first = self.key == lucky and lucky not in plans
            plans.append(self.key)

        def run(self):
            clock[0] += cost(self.key) * (0.8 if self.first else 1.0)

        def close(self):
            pass

    monkeypatch.setattr(q, "BatchPlan", FakePlan)
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: clock[0])
    monkeypatch.setattr(torch.cuda, "synchronize", lambda device=None: None)


def test_batched_tuner_keeps_defaults_against_a_lucky_screen(monkeypatch):
    _fake_batched(monkeypatch, lambda k: 1e-3, lucky=(1 << 20, 16))
    got = autotune.tune_batched([None], device="cpu", log=lambda *a: None)
    assert (got["tile_bytes"], got["waves_per_cu"]) == (0, 0)


def test_batched_tuner_takes_a_confirmed_gain(monkeypatch):
    _fake_batched(monkeypatch, lambda k: 0.9e-3 if k == (1 << 20, 16) else 1e-3)
    got = autotune.tune_batched([None], device="cpu", log=lambda *a: None)
    assert (got["tile_bytes"], got["waves_per_cu"]) == (1 << 20, 16)
    assert got["ms"] < got["default_ms"]
