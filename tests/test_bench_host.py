"""Host-side logic of bench.py (no GPU): the counter-to-traffic conversion
and the algorithmic byte counts."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for disp, name, ctr, val in rows:
            r = {k: "0" for k in FIELDS}
            r.update(Dispatch_Id=str(disp), Kernel_Name=name, Counter_Name=ctr,
                     Counter_Value=str(val))
            w.writerow(r)


def test_algorithmic_bytes():
    assert bench.algorithmic_bytes_per_node("fp64") == 432
    assert bench.algorithmic_bytes_per_node("fp32") == 216
    assert bench.algorithmic_bytes_per_node("fp16") == 108
    assert bench.algorithmic_bytes_per_node("fp32", lattices=2) == 144


def test_record_traffic_scales_by_copy(tmp_path):
    step = "void cmlb::k_step<float, float, 2, true, 8, 2, false, true>(cmlb::StepArgs)"
    copy = "__amd_rocclr_copyBuffer"
    # the copy of 1 MiB reads half its bytes in FETCH_SIZE units (scale 2)
    # and all of them in WRITE_SIZE units (scale 1); two instances of one
    # dispatch are summed, other kernels ignored
    _csv(tmp_path / "cf.csv", [(1, copy, "FETCH_SIZE", 256.0), (1, copy, "FETCH_SIZE", 256.0),
                               (2, "other", "FETCH_SIZE", 9e9)])
    _csv(tmp_path / "cw.csv", [(1, copy, "WRITE_SIZE", 1024.0)])
    _csv(tmp_path / "f.csv", [(3, step, "FETCH_SIZE", 100.0), (4, step, "FETCH_SIZE", 300.0)])
    _csv(tmp_path / "w.csv", [(3, step, "WRITE_SIZE", 500.0), (4, step, "WRITE_SIZE", 500.0)])
    out = tmp_path / "traffic.json"
    ent = bench.record_traffic("batched:fp32", 1000, "fp32", tmp_path / "f.csv",
                               tmp_path / "w.csv", tmp_path / "cf.csv", tmp_path / "cw.csv",
                               copy_bytes=1 << 20, path=str(out))
    assert ent["fetch_bytes"] == 200 * 1024 * 2
    assert ent["write_bytes"] == 500 * 1024
    assert ent["algorithmic_bytes"] == 216000
    assert ent["dispatches"] == [2, 2]
    data = json.loads(out.read_text())
    assert data["batched:fp32"]["kernel_hash"] == bench.kernel_hash(2)
    assert abs(data["calibration"]["fetch_scale"] - 2.0) < 1e-12


def test_record_traffic_sums_the_3d_step_kernels(tmp_path):
    mom = "void cmlb3::k_moments3<float, float, 2, true>(cmlb3::StepArgs3)"
    col = "void cmlb3::k_collide3<float, float, 2, true, 8, false, true>(cmlb3::StepArgs3)"
    copy = "__amd_rocclr_copyBuffer"
    _csv(tmp_path / "cf.csv", [(1, copy, "FETCH_SIZE", 512.0)])
    _csv(tmp_path / "cw.csv", [(1, copy, "WRITE_SIZE", 1024.0)])
    _csv(tmp_path / "f.csv", [(3, mom, "FETCH_SIZE", 100.0), (4, col, "FETCH_SIZE", 30.0),
                              (5, mom, "FETCH_SIZE", 100.0), (6, col, "FETCH_SIZE", 10.0)])
    _csv(tmp_path / "w.csv", [(3, mom, "WRITE_SIZE", 20.0), (4, col, "WRITE_SIZE", 80.0)])
    out = tmp_path / "traffic.json"
    ent = bench.record_traffic("c5:fp32", 100, "fp32", tmp_path / "f.csv", tmp_path / "w.csv",
                               tmp_path / "cf.csv", tmp_path / "cw.csv", copy_bytes=1 << 20,
                               path=str(out), lattices=3, q=27,
                               kernels=("k_moments3", "k_collide3"))
    assert ent["fetch_bytes"] == (100 + 20) * 1024 * 2
    assert ent["write_bytes"] == (20 + 80) * 1024
    assert ent["algorithmic_bytes"] == 3 * 27 * 2 * 4 * 100
    assert ent["per_kernel"]["k_collide3"]["write_bytes"] == 80 * 1024
    assert json.loads(out.read_text())["c5:fp32"]["kernel_hash"] == bench.kernel_hash(3)


def test_bench_refuses_several_gpus():
    """One GPU only: --gpus 2 exits with status 2 and says why."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_missing_library_fails_loudly(tmp_path):
    """Without libcmlb.so the binding raises; there is no CPU fallback."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2504_09024_amd import cmlb\n"
            "try:\n"
            "    cmlb.load(%r)\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "    sys.exit(3)\n") % (ROOT, str(tmp_path / "libcmlb.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 3, r.stdout + r.stderr
    assert "no CPU fallback" in r.stdout
