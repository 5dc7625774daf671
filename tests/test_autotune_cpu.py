"""Host-side logic of the autotuner: cache round trip and signatures."""
import json

from paper_2506_06040_amd import autotune as T


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "c.json")
    assert T._load(p) == {}
    T._store(p, "k1", {"best": {"a": 1}, "table": []})
    T._store(p, "k2", {"best": {"a": 2}, "table": [{"cfg": {"a": 2}, "ms": 0.5}]})
    d = json.load(open(p))
    assert d["k1"]["best"] == {"a": 1} and d["k2"]["table"][0]["ms"] == 0.5


def test_signature_depends_on_content():
    a = T._sig([[1, 2], [3]])
    assert a == T._sig([[1, 2], [3]]) and a != T._sig([[3], [1, 2]])
    assert len(T.DECODE_CANDIDATES) == 6


def test_batch_candidates_are_valid_and_distinct():
    # the library accepts work items of 64..65536 pixels in multiples of 64
    keys = set()
    for c in T.BATCH_CANDIDATES:
        assert 64 <= c["item_pixels"] <= 65536 and c["item_pixels"] % 64 == 0
        keys.add(tuple(sorted(c.items())))
    assert len(keys) == len(T.BATCH_CANDIDATES)


def test_cache_path_env(monkeypatch, tmp_path):
    monkeypatch.setenv("NTC_AUTOTUNE_CACHE", str(tmp_path / "x.json"))
    assert T.default_cache_path() == str(tmp_path / "x.json")
