"""Workload files (paper_2501_16122_amd/configs): each equals the workload
the code defines under its name, carries only known solve options, and
every point the paper leaves open is listed once in the readings file with
the fields that carry its value."""
import dataclasses
import glob
import json
import os

import pytest

from paper_2501_16122_amd import synth

FILES = sorted(f for f in glob.glob(os.path.join(synth.CONFIG_DIR, "*.json")) if not f.endswith("readings.json"))


def test_every_named_workload_has_a_file_equal_to_it():
    loaded = {}
    for f in FILES:
        w, solve = synth.load_config(f)
        loaded[w.name] = w
        assert w == synth.CONFIGS[w.name], f
        # FP32 storage is solved in the mixed form, FP64 in the plain one
        assert solve["mixed"] == (1 if w.precision == "f32" else 0), f
        assert solve["tol"] == 1e-10
    assert sorted(loaded) == sorted(synth.CONFIGS)


def test_files_load_by_name_and_round_trip(tmp_path):
    w, solve = synth.load_config("gls")
    assert w == synth.C2_GLS
    p = tmp_path / "w.json"
    p.write_text(json.dumps(synth.config_dict(w.replace(n_det=3), solve)))
    w2, solve2 = synth.load_config(str(p))
    assert w2 == w.replace(n_det=3) and solve2 == solve


def test_solve_options_are_the_library_options():
    b = pytest.importorskip("paper_2501_16122_amd.binding")
    try:
        b.load()
    except Exception as e:  # the library is built by build()
        pytest.skip(f"library not built: {e}")
    for f in FILES:
        _, solve = synth.load_config(f)
        o = b.solve_opts(**solve)
        for k, v in solve.items():
            assert getattr(o, k) == pytest.approx(v), (f, k)


@pytest.mark.parametrize("edit", ["drop", "add", "solve"])
def test_malformed_files_are_refused(tmp_path, edit):
    d = json.load(open(synth.config_path("gls")))
    if edit == "drop":
        del d["workload"]["lam"]
    elif edit == "add":
        d["workload"]["lags"] = 4096
    else:
        d["solve"]["tolerance"] = 1e-8
    p = tmp_path / "bad.json"
    p.write_text(json.dumps(d))
    with pytest.raises(ValueError):
        synth.load_config(str(p))
    with pytest.raises(FileNotFoundError):
        synth.load_config("no_such_workload")


def test_readings_file_lists_every_reading_once():
    d = json.load(open(os.path.join(synth.CONFIG_DIR, "readings.json")))
    ids = [r["id"] for r in d["readings"]]
    assert ids == list(range(1, len(ids) + 1)) and len(ids) >= 23
    names = {f.name for f in dataclasses.fields(synth.Workload)} | set(synth.SOLVE_KEYS)
    for r in d["readings"]:
        assert r["point"] and r["reading"]
        assert set(r["fields"]) <= names, r
    for f in FILES:
        assert json.load(open(f))["readings"] == "readings.json"
