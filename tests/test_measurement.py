"""Host logic of the measurement: the calibrated counter summary
(paper_2604_11959_amd.profile_traffic) and the bench line's comparison of the
general range's counter bytes with the cut-cell extras.  Synthetic counter
files, no GPU."""
import csv
import importlib.util
import json
import os

import numpy as np
import pytest

from paper_2604_11959_amd import profile_traffic as pt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KIB = 1024.0


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, val in rows:
            # two rows per dispatch (the counter is reported per XCD group);
            # the summary adds them
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val / 2})
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val / 2})


def _pmc_dir(tmp_path):
    gen = ["void ebs::(anonymous namespace)::k_gen_prims<float>(ebs::GenArgs<float>)",
           "void ebs::(anonymous namespace)::k_gen_fhat<float>(ebs::GenArgs<float>)",
           "void ebs::(anonymous namespace)::k_gen_cut<float>(ebs::GenArgs<float>)",
           "void ebs::(anonymous namespace)::k_gen_update<float>(ebs::GenArgs<float>)",
           "ebs::(anonymous namespace)::k_qhat(ebs::AArgs)",
           "ebs::(anonymous namespace)::k_grad(ebs::AArgs)",
           "void ebs::(anonymous namespace)::k_final<float>(ebs::FArgs<float>)"]
    fetch, write = [], []
    d = 1
    # set-up kernels before the step (not counted)
    fetch.append((d, "k_sum<float>", 999.0)); write.append((d, "k_sum<float>", 999.0)); d += 1
    for stage in range(3):
        fetch.append((d, "void ebs::k_bulk<float, 64, 16, true, false, false>(ebs::BulkArgs<float>)", 1000.0 + stage))
        write.append((d, "void ebs::k_bulk<float, 64, 16, true, false, false>(ebs::BulkArgs<float>)", 500.0))
        d += 1
        for q, name in enumerate(gen):
            fetch.append((d, name, 10.0 * (q + 1)))
            write.append((d, name, 1.0 * (q + 1)))
            d += 1
    # after the step: sums and copies (not counted)
    fetch.append((d, "k_sum<float>", 777.0)); write.append((d, "k_sum<float>", 777.0))
    _write(tmp_path / "fetch_counter_collection.csv", "FETCH_SIZE", fetch)
    _write(tmp_path / "write_counter_collection.csv", "WRITE_SIZE", write)
    # the 2^30-byte copy: FETCH_SIZE reads half width, WRITE_SIZE exact
    _write(tmp_path / "cfetch_counter_collection.csv", "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", 2.0 ** 19)])
    _write(tmp_path / "cwrite_counter_collection.csv", "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", 2.0 ** 20)])
    return tmp_path


def test_counter_summary_scales_and_general_range(tmp_path):
    s = pt.summarize(str(_pmc_dir(tmp_path)))
    assert s["fetch_scale"] == pytest.approx(2.0)
    assert s["write_scale"] == pytest.approx(1.0)
    assert s["launches"] == 3
    # mean over the three regular-region launches: 2 x 1001 KiB read + 500 KiB written
    assert s["traffic_bytes_per_launch"] == pytest.approx((2 * 1001.0 + 500.0) * KIB)
    per = s["general_range_bytes_per_stage"]
    assert sorted(per) == sorted(pt.GENERAL_PASSES)
    for q, name in enumerate(pt.GENERAL_PASSES):
        # per stage: calibrated read 2 x 10 (q + 1) KiB and write (q + 1) KiB
        assert per[name] == pytest.approx((2 * 10.0 * (q + 1) + (q + 1)) * KIB), name
    assert s["general_source_sha256"] == pt.source_sha256(pt.GENERAL_SOURCES)


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_general_range_leg_against_extras(tmp_path, monkeypatch):
    import paper_2604_11959_amd as ebs

    bench = _bench()
    stats = np.zeros((4, 8), dtype=np.int64)
    stats[:, 0] = [100, 90, 80, 30]  # cut CV-instances
    stats[:, 1] = [10, 9, 8, 3]      # small CVs
    stats[0, 6] = 1000               # general cells
    per = {name: 1.0e6 * (q + 1) for q, name in enumerate(pt.GENERAL_PASSES)}
    summ = {"workload": "w", "general_range_bytes_per_stage": per,
            "general_source_sha256": pt.source_sha256(pt.GENERAL_SOURCES)}
    path = tmp_path / "summary.json"
    path.write_text(json.dumps(summ))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(path))
    leg = bench.general_range_leg(stats, ebs.EBS_F32_BULK, "w")
    ex = leg["extras_bytes_per_stage"]
    assert ex["state"] == round(1000 * 8 / 3 * 5 * 4)
    assert ex["geometry_records"] == round(300 * bench.GEOM_RECORD_BYTES)
    assert ex["uhat"] == 1000 * 80
    total = 1000 * 8 / 3 * 5 * 4 + 300 * bench.GEOM_RECORD_BYTES + 1000 * 80
    cb = leg["counter_bytes_per_stage"]
    assert cb["update_passes"] == round(1e6 * (1 + 2 + 3 + 4))
    assert cb["redistribution"] == round(1e6 * (5 + 6 + 7))
    assert leg["update_passes_over_extras"] == round(1e7 / total, 2)
    assert leg["total_over_extras"] == round(2.8e7 / total, 2)
    assert leg["redistribution_bytes_per_small_cv"] == round(1.8e7 / 30, 1)
    # another workload, or other general-range sources: no counter bytes
    assert bench.general_range_leg(stats, ebs.EBS_F32_BULK, "other")["counter_bytes_per_stage"] is None
    summ["general_source_sha256"] = "0" * 64
    path.write_text(json.dumps(summ))
    assert bench.general_range_leg(stats, ebs.EBS_F32_BULK, "w")["counter_bytes_per_stage"] is None
    # FP64 state: 8-byte elements in the state term
    assert bench.general_range_leg(stats, ebs.EBS_F64, "w")["extras_bytes_per_stage"]["state"] == round(
        1000 * 8 / 3 * 5 * 8)
