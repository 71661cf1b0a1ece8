"""Host-side logic of the tile autotuner: size classes and the stored table."""
import json

import gen
from paper_1309_5571_amd import autotune


def test_size_classes():
    assert autotune.size_class([gen.config(3)]) == "dmax<=48"
    assert autotune.size_class([gen.config(2)]) == "dmax<=200"
    assert autotune.size_class(gen.batched_heisenberg(4, seed=777)) in ("dmax<=200", "dmax>200")
    assert autotune.key_of([gen.config(3)], "bf16") == "bf16|dmax<=48"


def test_save_and_load_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "tiles.json"
    res = {"key": "f64|dmax<=48", "best": {"bounds": [64, 1 << 30], "tiles": [16, 32], "us": 20.0},
           "results": []}
    autotune.save(res, str(path))
    monkeypatch.setattr(autotune, "TABLE_PATH", str(path))
    assert autotune.load_table("f64|dmax<=48") == ((64, 1 << 30), (16, 32))
    assert autotune.load_table("f32|dmax<=48") is None
    tab = json.load(open(path))
    assert tab["arch"] == "gfx950"


def test_stored_table_is_valid():
    """Every stored entry uses tiles the library accepts (16 or 32, bounds ascending)."""
    import os

    if not os.path.exists(autotune.TABLE_PATH):
        return
    tab = json.load(open(autotune.TABLE_PATH))
    for key, ent in tab["entries"].items():
        assert set(ent["tiles"]) <= {16, 32}, key
        assert list(ent["bounds"]) == sorted(ent["bounds"]), key
