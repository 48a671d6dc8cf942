"""Host logic of bench.py's rooflines: the counter figures it reads from the
committed rocprofv3 summaries are used only while the kernel sources hash as
they did when the counters were taken, and the batched roofline only for the
launch parameters and batch the counters were taken with.  Each test works on
a copy of a summary keyed to a copy of the sources, so it checks the logic
whether or not the committed summary is current."""
import os
import re
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

PARAMS = {"seg_log2": 20, "wg_size": 1024, "window": 16384, "wg_per_cu": 0,
          "bucket_log2": 0, "bucket_mib": 0}


def _tree(tmp_path, monkeypatch, profile, sources, key):
    """A copy of one summary and of the sources, the summary's hash line
    rewritten to the copied sources' hash."""
    for rel in (os.path.join("profiles", profile),) + tuple(sources):
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    prof = tmp_path / "profiles" / profile
    text = prof.read_text()
    assert re.search(r"\b%s: [0-9a-f]+" % key, text)
    prof.write_text(re.sub(r"\b%s: [0-9a-f]+" % key, "%s: %s" % (key, bench.kernel_sha(sources)),
                           text))
    return tmp_path


def test_batch_figures_follow_the_sources(tmp_path, monkeypatch):
    root = _tree(tmp_path, monkeypatch, "batched_4096.md", bench.BATCH_SOURCES,
                 "batch_kernel_source_sha256_16")
    fig = bench.batch_profile_figures()
    assert fig is not None and fig["params"] == [20, 1024, 16384, 24]
    ev = int(fig["batch_evens_per_launch"])
    r = bench.batch_roofline(PARAMS, ev, 170.0)
    assert r is not None and r["bound"] == "alu"
    assert r["frac"] == pytest.approx(64 * fig["launch_valu_instructions"] / 0.170
                                      / bench.VALU_PEAK_OPS)
    assert set(r["per_kernel"]) == {"bucket_fill_kernel", "sieve_probe_kernel"}
    # other launch parameters, another batch: no figures
    assert bench.batch_roofline(dict(PARAMS, window=4096), ev, 170.0) is None
    assert bench.batch_roofline(dict(PARAMS, bucket_log2=23), ev, 170.0) is None
    assert bench.batch_roofline(PARAMS, ev + 1, 170.0) is None
    # a changed kernel source: the counters no longer describe it
    src = root / bench.BATCH_SOURCES[-1]
    src.write_text(src.read_text() + "\n")
    assert bench.batch_profile_figures() is None
    assert bench.batch_roofline(PARAMS, ev, 170.0) is None


def test_wide_and_headline_figures_follow_the_sources(tmp_path, monkeypatch):
    root = _tree(tmp_path, monkeypatch, "wide_probe_2_64.md", bench.WIDE_SOURCES,
                 "wide_kernel_source_sha256_16")
    _tree(tmp_path, monkeypatch, "sieve_probe_1e12.md", bench.KERNEL_SOURCES,
          "kernel_source_sha256_16")
    w = bench.wide_profile_figures()
    assert w is not None and w["valu_instructions_per_even_2_26"] > 0
    traffic, issue, prices = bench.profile_figures()
    assert traffic and issue and prices
    for rel in (bench.WIDE_SOURCES[0], bench.KERNEL_SOURCES[0]):
        p = root / rel
        p.write_text(p.read_text() + "\n")
    assert bench.wide_profile_figures() is None
    assert bench.profile_figures() == (None, None, None)
