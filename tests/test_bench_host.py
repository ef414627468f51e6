"""Host-side checks of bench.py's bookkeeping (no GPU): a counter-table row
is reported only for the workload, launch shape and kernel source it was
taken on, and a size subset of the batch never borrows the whole batch's row."""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _args(**kw):
    a = argparse.Namespace(workload="jet", storage="f16", exact_time=False, sides=None)
    for k, v in kw.items():
        setattr(a, k, v)
    return a


def test_workload_keys():
    assert bench.workload_key(_args()) == "jet"
    assert bench.workload_key(_args(workload="batch")) == "batch-f16"
    assert bench.workload_key(_args(workload="batch", storage="bf16")) == "batch-bf16"
    assert bench.workload_key(_args(exact_time=True)) == "jet-exact"
    assert bench.workload_key(_args(workload="batch", sides="1024")) == "batch-f16-sides1024"


def test_traffic_rows_match_source_and_shape():
    rows = []
    with open(bench.TRAFFIC_TABLE) as fh:
        for ln in fh:
            if ln.strip() and not ln.startswith("#"):
                rows.append(ln.split())
    assert rows, "the counter table holds no rows"
    kid = bench.kernel_source_id()
    for r in rows:
        if r[1] != kid:
            # taken on another kernel source: never reported
            continue
        tw, th, w, order, orient, bx, by, bz, sync, k = [int(x) for x in r[2].split(",")]
        tuning = {"tile": [tw, th], "waves_per_cu": w, "order": order, "orient": orient,
                  "brick": [bx, by, bz], "depth_sync": sync, "cells_per_batch": k}
        assert bench.tuning_key(tuning) == r[2]
        traffic, src = bench.measured_traffic(r[0], tuning)
        assert traffic == float(r[3]) + float(r[4]), src
        hit = bench.counter_row(r[0], tuning)[2]
        assert hit == (float(r[5]) if len(r) >= 6 else None)
        assert hit is None or 0.0 <= hit <= 1.0
        # another launch shape, or a size subset of the batch: no row
        taken = {tuple(x[2].split(",")) for x in rows if x[0] == r[0] and x[1] == r[1]}
        wo = next(c for c in range(4, 68, 4)
                  if tuple(bench.tuning_key(dict(tuning, waves_per_cu=c)).split(",")) not in taken)
        other = dict(tuning, waves_per_cu=wo)
        assert bench.measured_traffic(r[0], other)[0] is None
        assert bench.measured_traffic(r[0] + "-sides128", tuning)[0] is None


def test_tuning_strings_are_normalised():
    assert bench.normalise_tuning("64,1,8,3,0,1,8,1") == "64,1,8,3,0,1,8,1,0,4"
    assert bench.normalise_tuning("64,1,8,3,0,1,8,1,2") == "64,1,8,3,0,1,8,1,2,4"
    assert bench.normalise_tuning("64,1,8,3,0,1,8,1,2,8") == "64,1,8,3,0,1,8,1,2,8"
