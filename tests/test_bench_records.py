"""Host checks of the benchmark's measurement records (no GPU).

* The HBM-traffic record holds, per kernel, the source it was taken from, a
  SHA-256 of that source, and one or more (tile shape, read, write) entries;
  the benchmark's lookup returns the entry whose shape equals the timed one,
  and nothing for a shape that was not measured or a source that changed.
* Every command quoted in the committed rocprofv3 summaries runs committed
  files only (the benchmark script at the repository root).
"""
import json
import os
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
RECORD = os.path.join(ROOT, "profiles", "traffic_road1242x375_b256.json")


def load_bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_record_is_well_formed():
    rec = json.load(open(RECORD))
    kernels = {k: v for k, v in rec.items() if isinstance(v, dict)}
    assert kernels, "no kernel records"
    for name, r in kernels.items():
        assert os.path.exists(os.path.join(ROOT, r["source"])), name
        assert re.fullmatch(r"[0-9a-f]{64}", r["sha256"]), name
        entries = r.get("variants", [r])
        shapes = [json.dumps(e.get("tuning", {}), sort_keys=True) for e in entries]
        assert len(set(shapes)) == len(shapes), f"{name}: a tile shape recorded twice"
        for e in entries:
            assert e["read_bytes"] > 0 and e["write_bytes"] > 0, name


def test_lookup_follows_shape_and_source(tmp_path, monkeypatch):
    bench = load_bench()
    rec = json.load(open(RECORD))
    # a copy of the record next to a copy of one source, so the hash can be changed
    src_dir = tmp_path / "src"
    src_dir.mkdir()
    (tmp_path / "profiles").mkdir()
    name = next(k for k, v in rec.items() if isinstance(v, dict) and "variants" in v)
    r = rec[name]
    text = open(os.path.join(ROOT, r["source"]), "rb").read()
    (src_dir / "k.hip").write_bytes(text)
    r = dict(r, source="src/k.hip")
    (tmp_path / "profiles" / os.path.basename(RECORD)).write_text(json.dumps({name: r}))
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    for e in r["variants"]:
        shape = dict(e["tuning"], unrelated_knob=7)
        assert bench.measured_traffic(name, 256, shape) == e["read_bytes"] + e["write_bytes"]
    key = next(iter(r["variants"][0]["tuning"]))
    assert bench.measured_traffic(name, 256, {key: -1}) is None  # a shape never measured
    assert bench.measured_traffic(name, 64, dict(r["variants"][0]["tuning"])) is None  # another batch
    (src_dir / "k.hip").write_bytes(text + b"\n// changed\n")
    assert bench.measured_traffic(name, 256, dict(r["variants"][0]["tuning"])) is None  # another source


@pytest.mark.parametrize("md", sorted(f for f in os.listdir(os.path.join(ROOT, "profiles")) if f.endswith(".md")))
def test_profile_commands_run_committed_files(md):
    text = open(os.path.join(ROOT, "profiles", md)).read()
    cmds = [ln.strip() for ln in text.splitlines() if ln.strip().startswith("rocprofv3 ")]
    assert cmds, f"{md}: no rocprofv3 command"
    for c in cmds:
        prog = c.split(" -- ", 1)[1].split()
        assert prog[0] in ("python3", "python"), c
        script = next(a for a in prog[1:] if not a.startswith("-"))
        assert script == "bench.py" and os.path.exists(os.path.join(ROOT, script)), c
        assert "_work" not in c, c
