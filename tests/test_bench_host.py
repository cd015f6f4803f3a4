"""Host logic of bench.py on the CPU: the refusal of more than one GPU, the counter summary built from
rocprofv3's CSV output (synthetic rows here, in the layout rocprofv3 writes), and the rule that the
counter figures of the JSON line (roofline.traffic, roofline.valu_issue) apply only to the sources they
were taken on."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402

ROLES = ["fft1_row", "xop"]
KERNELS = {"fft1_row": "void nufds::fft_fixed_kernel<float, 16, 64, 1024>(nufds::PassDesc)",
           "xop": "void nufds::row_chain_kernel<25600, 1, true>(nufds::PassDesc)"}
COPY = "__amd_rocclr_copyBuffer"


def _csv(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def _counter_rows(per_role, copy_value=None):
    """Two steps of the roles in launch order, after a plan build kernel and a 1 GiB copy; per_role maps
    counter name -> {role: value}."""
    rows, disp = [], 0

    def add(kernel, grid, values):
        nonlocal disp
        disp += 1
        for name, v in values.items():
            rows.append({"Dispatch_Id": disp, "Kernel_Name": kernel, "Grid_Size": grid, "Counter_Name": name,
                         "Counter_Value": v})

    if copy_value is not None:
        add(COPY, 1 << 27, copy_value)
    add("void nufds::map_table_kernel(double*)", 4096, {k: 1.0 for k in per_role})
    for _ in range(2):
        for role in ROLES:
            add(KERNELS[role], 1024, {name: vals[role] for name, vals in per_role.items()})
    return rows


def _profile_dir(tmp_path):
    d = tmp_path / "prof"
    fields = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    # FETCH_SIZE reads half a 1 GiB copy's bytes (factor 2), WRITE_SIZE all of them (factor 1)
    _csv(str(d / "fetch" / "run_counter_collection.csv"), fields,
         _counter_rows({"FETCH_SIZE": {"fft1_row": 1000.0, "xop": 3000.0}}, {"FETCH_SIZE": 524288.0}))
    _csv(str(d / "write" / "run_counter_collection.csv"), fields,
         _counter_rows({"WRITE_SIZE": {"fft1_row": 2000.0, "xop": 5000.0}}, {"WRITE_SIZE": 1048576.0}))
    _csv(str(d / "valu" / "run_counter_collection.csv"), fields,
         _counter_rows({"SQ_INSTS_VALU": {"fft1_row": 4.0e8, "xop": 1.4e9},
                        "SQ_WAVES": {"fft1_row": 262144.0, "xop": 409600.0}}))
    _csv(str(d / "trace" / "run_kernel_stats.csv"), ["Name", "Calls", "AverageNs"],
         [{"Name": KERNELS[r], "Calls": 2, "AverageNs": 1e6 * (1.0 if r == "fft1_row" else 3.5)} for r in ROLES])
    with open(d / "roles.json", "w") as f:
        json.dump({"roles": ROLES, "bytes": {"fft1_row": 4.0e9, "xop": 1.0e10},
                   "avg_ms": {"fft1_row": 1.0, "xop": 3.5}, "ms_per_step": 4.5}, f)
    return str(d)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_summary_and_its_source_rule(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_JSON", str(tmp_path / "counters.json"))
    monkeypatch.setattr(bench, "PROFILE_MD", str(tmp_path / "kernels.md"))
    rec = bench.summarize_profile(_profile_dir(tmp_path))
    assert rec["calibration"]["FETCH_SIZE"]["factor"] == 2.0
    assert rec["calibration"]["WRITE_SIZE"]["factor"] == 1.0
    xop = rec["roles"]["xop"]
    # KiB per dispatch, times the copy's factor, averaged over the two steps
    assert xop["fetch_bytes"] == 3000.0 * 1024 * 2.0
    assert xop["write_bytes"] == 5000.0 * 1024
    assert xop["valu_insts"] == 1.4e9 and xop["waves"] == 409600.0
    assert rec["roles"]["fft1_row"]["valu_insts"] == 4.0e8
    md = open(tmp_path / "kernels.md").read()
    # VALU issue of xop: 1.4e9 instructions in 3.5 ms against 614.4 G/s
    assert f"{1.4e9 / 3.5e-3 / bench.VALU_ISSUE_PEAK:.2f} |" in md
    assert "rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES" in md
    # the JSON line's counter figures while the sources match ...
    assert bench.measured_traffic("xop") == xop["fetch_bytes"] + xop["write_bytes"]
    assert bench.measured_valu("xop") == 1.4e9
    assert bench.measured_valu("no_such_role") is None
    # ... and none once they differ
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("xop") is None
    assert bench.measured_valu("xop") is None
