"""The committed rocprofv3 summaries under profiles/ and the hash that ties
their counters to the kernel sources (CPU only).

* Every traffic summary holds the scaled FETCH_SIZE and WRITE_SIZE of its
  kernel, the copy-derived scale factors, the command that made it and the
  hash of the sources it describes.
* The hash covers each HIP source's compiler flags as well as its text, so a
  flag change retires the recorded counters like a source change does.
* Every kernel-duration summary names its command.
"""
import glob
import json
import os

import pytest

from paper_2601_17196_amd import build as hipbuild
from paper_2601_17196_amd import profile_summary as PS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def _traffic_files():
    return sorted(glob.glob(os.path.join(PROFILES, "*_traffic.json")))


def test_traffic_summaries_well_formed():
    files = _traffic_files()
    assert files
    for f in files:
        d = json.load(open(f))
        for key in ("kernel", "fetch_bytes", "write_bytes", "traffic_bytes", "scale_fetch", "scale_write",
                    "kernel_sources", "kernel_source_hash", "command"):
            assert key in d, (f, key)
        assert d["traffic_bytes"] == pytest.approx(d["fetch_bytes"] + d["write_bytes"])
        # a plain copy reads as half its bytes on FETCH_SIZE and all of them on WRITE_SIZE
        assert d["scale_fetch"] == pytest.approx(2.0, rel=1e-2)
        assert d["scale_write"] == pytest.approx(1.0, rel=1e-2)
        assert d["fetch_bytes"] > 0 and d["write_bytes"] >= 0
        assert "rocprofv3 --pmc FETCH_SIZE" in d["command"] and "rocprofv3 --pmc WRITE_SIZE" in d["command"]
        for src in d["kernel_sources"]:
            assert os.path.exists(os.path.join(ROOT, "paper_2601_17196_amd", src)), src
        assert len(d["kernel_source_hash"]) == 16


def test_kernel_stats_summaries_name_their_command():
    files = sorted(glob.glob(os.path.join(PROFILES, "*_kernel_stats.md")))
    assert files
    for f in files:
        text = open(f).read()
        assert "rocprofv3 --kernel-trace --stats" in text, f
        assert "| kernel | calls |" in text, f


def test_source_hash_covers_compiler_flags(monkeypatch):
    base = PS.kernel_source_hash(PS.BATCHED_SOURCES)
    assert base == PS.kernel_source_hash(PS.BATCHED_SOURCES)
    flags = dict(hipbuild.SOURCE_FLAGS)
    flags["pot_batched.hip"] = flags.get("pot_batched.hip", []) + ["-mllvm", "-some-other-option"]
    monkeypatch.setattr(hipbuild, "SOURCE_FLAGS", flags)
    assert PS.kernel_source_hash(PS.BATCHED_SOURCES) != base
    # the single-instance kernels' hash does not depend on the batched source's flags
    monkeypatch.undo()
    single = PS.kernel_source_hash()
    flags = dict(hipbuild.SOURCE_FLAGS)
    flags["pot_batched.hip"] = ["-O1"]
    monkeypatch.setattr(hipbuild, "SOURCE_FLAGS", flags)
    assert PS.kernel_source_hash() == single
