"""The autotuner's choice cache through the C ABI (host memory only, no GPU):
entries round-trip, a cached class takes a new choice, malformed entries
are refused with nothing added, and a JSON file named by MM_TUNE_CACHE
carries the choices from one process to the next."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _b():
    from paper_2501_16122_amd import binding
    try:
        binding.load()
    except Exception as e:
        pytest.skip(f"library not built: {e}")
    return binding


# classes no real solve in this process produces (device 7)
E1 = {"device": 7, "log2_samples": 28, "dtype": 0, "arith": 0, "n_rhs": 1, "ncomp": 3, "lambda": 4096,
      "noise_kind": 1, "op_variant": 16}
E2 = dict(E1, arith=1, op_variant=8)


def test_entries_round_trip_and_replace():
    b = _b()
    b.tune_cache_put([E1, E2])
    got = b.tune_cache_get()
    assert E1 in got and E2 in got
    n = len(got)
    b.tune_cache_put([dict(E1, op_variant=5)])
    got = b.tune_cache_get()
    assert len(got) == n and dict(E1, op_variant=5) in got and E1 not in got
    b.tune_cache_put([E1])


@pytest.mark.parametrize("bad", [dict(op_variant=32), dict(op_variant=-1), dict(ncomp=4), dict(dtype=2),
                                 dict(arith=5), dict(noise_kind=3), dict(lambda_=0), dict(n_rhs=0),
                                 dict(device=-1), dict(log2_samples=63)])
def test_malformed_entries_are_refused(bad):
    b = _b()
    before = b.tune_cache_get()
    e = dict(E1, device=6)
    e.update({("lambda" if k == "lambda_" else k): v for k, v in bad.items()})
    with pytest.raises(b.MapMakerError) as ex:
        b.tune_cache_put([dict(E1, device=5), e])  # a good entry before it is not added either
    assert ex.value.code == b.MM_EINVAL
    assert b.tune_cache_get() == before


def test_query_arguments_are_checked():
    b = _b()
    lib = b.load()
    assert lib.mm_tune_cache_get(None, 0, None) == b.MM_EINVAL
    n = b._c.c_int32()
    assert lib.mm_tune_cache_get(None, 1, b._c.byref(n)) == b.MM_EINVAL
    assert lib.mm_tune_cache_get(None, -1, b._c.byref(n)) == b.MM_EINVAL
    assert lib.mm_tune_cache_put(None, 1) == b.MM_EINVAL
    assert lib.mm_tune_cache_put(None, 0) == b.MM_OK


def test_file_carries_choices_across_processes(tmp_path):
    _b()
    path = tmp_path / "tune.json"
    env = dict(os.environ, MM_TUNE_CACHE=str(path), PYTHONPATH=ROOT)
    put = ("from paper_2501_16122_amd import binding as b; b.load(); "
           f"b.tune_cache_put([{E1!r}, {E2!r}])")
    subprocess.run([sys.executable, "-c", put], env=env, check=True, timeout=120)
    d = json.loads(path.read_text())
    assert E1 in d["entries"] and E2 in d["entries"]
    get = ("import json; from paper_2501_16122_amd import binding as b; b.load(); "
           "print(json.dumps(b.tune_cache_get()))")
    r = subprocess.run([sys.executable, "-c", get], env=env, check=True, timeout=120, capture_output=True, text=True)
    got = json.loads(r.stdout.strip().splitlines()[-1])
    assert E1 in got and E2 in got


@pytest.mark.parametrize("content", ["{not json", '{"entries": [{"device": 0}]}',
                                     '{"entries": [{"device": 0, "log2_samples": 28, "dtype": 0, "arith": 0, '
                                     '"n_rhs": 1, "ncomp": 3, "lambda": 4096, "noise_kind": 1, "op_variant": 99}]}'])
def test_broken_file_is_skipped_with_a_warning(tmp_path, content):
    _b()
    path = tmp_path / "tune.json"
    path.write_text(content)
    env = dict(os.environ, MM_TUNE_CACHE=str(path), PYTHONPATH=ROOT)
    code = ("import warnings; warnings.simplefilter('always'); "
            "from paper_2501_16122_amd import binding as b; lib = b.load(); print('abi', lib.mm_abi_version())")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "abi 5" in r.stdout and "not loaded" in r.stderr
