"""Host logic of the launch-shape autotuner: cache keys and the JSON cache."""

from paper_1603_06400_amd import autotune, inputs


class FakeGeo:
    def __init__(self, geom, lr=1, td=0):
        self.geom = geom
        self.table_dtype = td
        self._lr = lr
        self.shapes = []

    def info(self):
        return {"symmetric_lr": self._lr}

    def set_launch(self, *s):
        self.shapes.append(s)


def test_size_key_separates_shapes():
    a = FakeGeo(inputs.standard_geometry(16, 8, ndet=10))
    b = FakeGeo(inputs.standard_geometry(16, 16, ndet=10))
    c = FakeGeo(inputs.standard_geometry(16, 8, ndet=10), lr=0)
    d = FakeGeo(inputs.standard_geometry(16, 8, ndet=10), td=1)
    keys = {autotune.size_key(g) for g in (a, b, c, d)}
    assert len(keys) == 4
    assert autotune.size_key(a) == autotune.size_key(FakeGeo(inputs.standard_geometry(16, 8, ndet=10)))


def test_cache_round_trip_and_reuse(tmp_path, monkeypatch):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    calls = []

    def fake_tune(geo, reps=5):
        calls.append(geo)
        return {"fwd_splits": 4, "fwd_qw": 32, "adj_qw": 64, "adj_splits": 2, "forward_ms": 1.0, "adjoint_ms": 2.0}

    monkeypatch.setattr(autotune, "tune", fake_tune)
    cache = {}
    g1 = FakeGeo(inputs.standard_geometry(16, 8, ndet=10))
    g2 = FakeGeo(inputs.standard_geometry(16, 8, ndet=10))
    autotune.tuned(g1, cache)
    autotune.tuned(g2, cache)
    assert len(calls) == 1 and g2.shapes == [(4, 32, 64, 2)]
    autotune.save_cache(cache, path)
    assert autotune.load_cache(path) == cache
    (tmp_path / "bad.json").write_text("{not json")
    assert autotune.load_cache(str(tmp_path / "bad.json")) == {}
