"""Tuning of launch shapes, through the C ABI: the single-instance tile height
(tile_rows = -1) and the batched group share, kept in memory and in the JSON
file named by POT_TUNE_CACHE.

* A tuned solve picks one of the candidate heights, records it under its
  architecture, cost kind and shape bucket, passes the Definition 1 check of
  tests/gpu_common.py, and equals bit for bit the solve run with that height
  given explicitly.
* A batched solve records its tuned (share, workgroups per CU).
* A cache file that does not parse is ignored and replaced.
"""
import json

import numpy as np
import pytest

from paper_2601_17196_amd import instances as I
from tests.gpu_common import check_definition1, gpu_solve

pytestmark = pytest.mark.gpu


def _read(path):
    with open(path) as f:
        return json.load(f)


def test_tile_tuning_recorded_and_reproducible(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("POT_TUNE_CACHE", str(path))
    inst = I.uniform_pair(600, 500, 2, 4101, mass_r=1.0, mass_c=1.1, s_frac=0.8)
    print("tile tuning: 600 x 500 FP32", flush=True)
    out = gpu_solve(inst, "f32", "aspot", tile_rows=-1)
    assert out.status == 0
    cache = _read(path)
    keys = [k for k in cache if "/tile/kind0/n512/m512" in k]
    assert len(keys) == 1, cache
    br = cache[keys[0]]
    assert len(br) == 1 and br[0] in (64, 128, 256)
    check_definition1(inst, "f32", "aspot", out, lp_key=None)
    ref = gpu_solve(inst, "f32", "aspot", tile_rows=br[0])
    assert ref.result["iters"] == out.result["iters"]
    assert ref.result["cost"] == out.result["cost"]
    assert np.array_equal(ref.u.cpu().numpy(), out.u.cpu().numpy())
    assert np.array_equal(ref.v.cpu().numpy(), out.v.cpu().numpy())
    # a second tuned solve takes the recorded height (no new entry)
    out2 = gpu_solve(inst, "f32", "aspot", tile_rows=-1)
    assert out2.result["cost"] == out.result["cost"]
    assert _read(path) == cache


def test_batched_tuning_recorded(tmp_path, monkeypatch):
    from paper_2601_17196_amd import pot
    path = tmp_path / "tune.json"
    monkeypatch.setenv("POT_TUNE_CACHE", str(path))
    insts = [I.uniform_pair(n, m, 3, 4200 + k) for k, (n, m) in enumerate([(300, 280), (260, 310), (290, 300)])]
    probs = []
    for inst in insts:
        d = pot.to_device_instance(inst, "cuda:0", kind="f32")
        probs.append(dict(r=d["r"], c=d["c"], s=d["s"], C=d["C"], kind=d["kind"], ldc=d["ldc"], cmax=1.0))
    print("batched tuning: 3 instances", flush=True)
    st, res, _ = pot.solve_batched(probs, insts[0].eps, want_duals=False)
    assert st == 0
    cache = _read(path)
    total = sum(i.n * i.m for i in insts)
    largest = max(i.n * i.m for i in insts)
    keys = [k for k in cache if "/batched/" in k and k.endswith(f"/b3/e{total >> 16}/l{largest}")]
    assert len(keys) == 1, cache
    share, per_cu = cache[keys[0]]
    assert share >= 1 << 15 and per_cu >= 1


def test_unparsable_cache_ignored(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    monkeypatch.setenv("POT_TUNE_CACHE", str(path))
    inst = I.uniform_pair(300, 260, 2, 4301)
    print("tile tuning over an unparsable cache file", flush=True)
    out = gpu_solve(inst, "f32", "aspot", tile_rows=-1)
    assert out.status == 0
    cache = _read(path)
    assert any("/tile/kind0/n256/m256" in k for k in cache)
    check_definition1(inst, "f32", "aspot", out, lp_key=None)


def test_recorded_height_outside_candidates_ignored(tmp_path, monkeypatch):
    """A recorded tile height that is not one of the tuned candidates (the
    workspace is sized for the candidates) is not used: the solve tunes
    again and records a candidate in its place."""
    import torch
    path = tmp_path / "tune.json"
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/tile/kind0/n1024/m1024"     # (a bucket no other test tunes: results stay in memory)
    path.write_text(json.dumps({key: [16]}))
    monkeypatch.setenv("POT_TUNE_CACHE", str(path))
    inst = I.uniform_pair(1100, 1000, 2, 4401, mass_r=1.0, mass_c=1.1, s_frac=0.8)
    print("tile tuning over a recorded height outside the candidates", flush=True)
    out = gpu_solve(inst, "f32", "aspot", tile_rows=-1)
    assert out.status == 0
    cache = _read(path)
    assert cache[key][0] in (64, 128, 256), cache
    check_definition1(inst, "f32", "aspot", out, lp_key=None)
