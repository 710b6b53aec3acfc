"""Consistency of the committed measurement record (CPU only): the bench line
in profiles/ keeps the bench.py output contract, its roofline figures follow
from one another, its traffic figure is the counter record's for the kernel
source it was taken on, and the kernel trace summary's average for the
collide-stream kernel agrees with the bench line's own events."""
import hashlib
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROF = os.path.join(ROOT, "profiles")
BENCH = os.path.join(PROF, "bench_c4_ensemble_256_fp16.json")
TRAFFIC = os.path.join(PROF, "collide_stream_traffic.json")
TRACE = os.path.join(PROF, "trace_collide_particle_c4_ensemble_256_fp16.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2403_05443_amd", "csrc", "k_stream.hip")
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


def _bench():
    return json.loads(open(BENCH).read().strip().splitlines()[-1])


def test_bench_line_contract():
    d = _bench()
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["higher_is_better"] is True and d["value"] > 0
    assert d["config"]["workload"] == "c4_ensemble_256"
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-3)
    # achieved = algorithmic bytes per launch over the measured launch duration
    assert r["achieved"] == pytest.approx(r["bytes_per_launch"] / (r["avg_launch_ms"] * 1e-3) / 1e9, rel=2e-3)
    # 19 populations per site in the stored format, read once and written once
    assert r["bytes_per_launch"] == 2 * 19 * STORAGE_BYTES[d["config"]["storage"]] * d["config"]["sites"]
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["sample"]


def test_traffic_matches_counter_record():
    """The line reports counter traffic only from a record of the kernel
    source it ran (the line carries that source's hash when it has one)."""
    d = _bench()
    r = d["roofline"]
    rec = json.load(open(TRAFFIC))
    ent = rec["entries"].get(f"{d['config']['workload']}/{d['config']['storage']}/v{r['variant']}")
    sha = r.get("source_sha256", rec["source_sha256"])
    if r["traffic"] is not None:
        assert rec["source_sha256"] == sha and ent is not None
        assert r["traffic"] == ent["traffic_bytes_per_launch"]
        # the counters' bytes are the record's, and never below the algorithmic bytes
        assert r["traffic"] >= 0.999 * r["bytes_per_launch"]
    else:
        # counters taken on another kernel source are not reported
        assert ent is None or rec["source_sha256"] != sha


def test_trace_agrees_with_bench_events():
    """The trace summary names the collide-stream kernel of the line's
    variant; its average over the traced launches agrees with the line's own
    HIP events within 3%."""
    d = _bench()
    r = d["roofline"]
    text = open(TRACE).read()
    m = re.search(r"Collide-stream kernel of variant (\d+): ((?:`[^`]+`(?:, )?)+)", text)
    assert m and int(m.group(1)) == r["variant"]
    names = re.findall(r"`([^`]+)`", m.group(2))
    avg = {}
    for line in text.splitlines():
        t = re.match(r"\| `([^`]+)` \| (\d+) \| ([0-9.]+) \|", line)
        if t:
            avg[t.group(1)] = float(t.group(3))
    us = [avg[n] for n in names]
    assert sum(us) / len(us) == pytest.approx(r["avg_launch_ms"] * 1e3, rel=0.03)
