"""Host logic of bench.py that needs no GPU: the one-GPU guard, and the HBM
traffic figure it reads back from the committed counter summary, which is
keyed to the HIP sources it was taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _summary(tmp_path, digest):
    rec = {"source_sha256": digest, "fetch_factor": 2.0, "write_factor": 1.0,
           "kernels": {"colpass": {"fetch_kib": 100.0, "write_kib": 10.0, "dispatches": 3}}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "counters_w_fp64.md").write_text("# summary\n\ntraffic_json: " + json.dumps(rec) + "\n")


def test_stored_traffic_is_keyed_to_the_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: "abc")
    _summary(tmp_path, "abc")
    # FETCH_SIZE and WRITE_SIZE in KiB, each scaled by its copy calibration
    assert bench.stored_traffic("w", "fp64", "colpass") == pytest.approx(1024.0 * (100.0 * 2.0 + 10.0))
    assert bench.stored_traffic("w", "fp64", "rowpass") is None      # kernel not in the summary
    assert bench.stored_traffic("w", "fp32", "colpass") is None      # no summary for it
    monkeypatch.setattr(bench, "source_digest", lambda: "other")
    assert bench.stored_traffic("w", "fp64", "colpass") is None      # other kernel sources


def test_source_digest_covers_the_single_path_sources(tmp_path, monkeypatch):
    """The digest changes with any source of the single-instance path's
    kernels and launches, and not with the batched solver's own file."""
    csrc = tmp_path / "paper_2308_00637_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.PATH_SOURCES:
        (csrc / f).write_text(f)
    (csrc / "qpk_batch.hip").write_text("z")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.source_digest()
    (csrc / "qpk_batch.hip").write_text("z // other")
    assert bench.source_digest() == d0
    for f in bench.PATH_SOURCES:
        (csrc / f).write_text(f + " // comment")
        d1 = bench.source_digest()
        assert d1 != d0
        d0 = d1
    assert set(bench.PATH_SOURCES) == {"qpk_api.hip", "qpk_internal.h", "qpk_kernels.hip"}