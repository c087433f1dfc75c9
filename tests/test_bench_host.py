"""Host logic of bench.py's counter summary (no GPU): kernel-name matching
for the multigrid groups and the scaling of FETCH_SIZE / WRITE_SIZE by the
run's reference copy, on a synthetic rocprofv3 counter CSV."""
import csv
import importlib.util
import io
import json
import os
import contextlib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_names_match_their_level_kind():
    b = _bench()
    ns = "void aao::(anonymous namespace)::"
    assert b._kernel_matches(ns + "k_up2d_march<0, 2, float, float, float, 32>(float const*)", "k_up2d_march", True)
    assert not b._kernel_matches(ns + "k_up2d_march<2, 2, float, float, float, 32>(float const*)", "k_up2d_march", True)
    assert b._kernel_matches(ns + "k_up2d_march<2, 2, float, float, float, 32>(float const*)", "k_up2d_march", False)
    # the 3D marches have no level kind in their template: level 0 only
    assert b._kernel_matches(ns + "k_down3d_march<float, float, float>(float const*)", "k_down3d_march", True)
    assert not b._kernel_matches(ns + "k_down3d_march<float, float, float>(float const*)", "k_down3d_march", False)
    assert not b._kernel_matches(ns + "k_up3d_march<float, float, float>(float const*)", "k_down3d_march", True)


def _csv(path, counter, rows):
    """rows: (kernel name, grid size, workgroup size, value in KiB)."""
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Workgroup_Size", "Counter_Name", "Counter_Value"])
        for d, (name, grid, wg, v) in enumerate(rows):
            w.writerow([d, grid, name, wg, counter, v])


def test_traffic_summary_scales_by_the_last_copy(tmp_path):
    b = _bench()
    GiB = 1 << 30
    ns = "void aao::(anonymous namespace)::"
    down = ns + "k_down3d_march<float, float, float>(float const*)"
    apply3 = ns + "k_apply_A_3d<3, 2, float>(float const*)"
    # counters read half the copy's reads and all its writes; the earlier,
    # larger copy (a right-hand side) must not be taken as the reference
    fetch = [("__amd_rocclr_copyBuffer", 1, 1, 3 * GiB // 1024), (down, 200 * 1024, 1024, 1000.0),
             (down, 3200 * 1024, 1024, 16000.0), (apply3, 512, 512, 2000.0), (apply3, 512, 512, 2000.0),
             ("__amd_rocclr_copyBuffer", 1, 1, GiB // 2 // 1024)]
    write = [("__amd_rocclr_copyBuffer", 1, 1, 6 * GiB // 1024), (down, 200 * 1024, 1024, 500.0),
             (down, 3200 * 1024, 1024, 8000.0), (apply3, 512, 512, 1000.0), (apply3, 512, 512, 1000.0),
             ("__amd_rocclr_copyBuffer", 1, 1, GiB // 1024)]
    _csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    members = [{"label": "k_down3d_march@0", "blocks": 1, "weight": 21, "workgroups": 200,
                "bytes_per_launch": 2560000.0},
               {"label": "k_down3d_march@0", "blocks": 32, "weight": 12, "workgroups": 3200,
                "bytes_per_launch": 40960000.0}]
    roof = {"vcycle_kernels": {"dominant": "k_down3d_march<level 0>",
                               "by_kernel": {"k_down3d_march<level 0>": {"members": members},
                                             "k_smooth<coarse levels>": {"members": [
                                                 {"label": "k_smooth@1", "blocks": 1, "weight": 1,
                                                  "workgroups": None, "bytes_per_launch": 1.0}]}}},
            "apply_A": {"kernel": "k_apply_A_3d", "bytes_per_launch": 5120000.0},
            "copy_reference": {"bytes": GiB}}
    (tmp_path / "r.json").write_text("[bench] log line\n" + json.dumps(roof) + "\n")
    out = io.StringIO()
    with contextlib.redirect_stdout(out):
        b.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "r.json"))
    text = out.getvalue()
    assert "(scale 2.000)" in text and "(scale 1.000)" in text
    # 1 block: 1000 KiB x 2 + 500 KiB = 2,560,000 B measured, ratio 1
    assert "| k_down3d_march<level 0> | `k_down3d_march@0` | 1 | 200 | 21 | 1,000 | 500 | 2,560,000 | 2,560,000 | 1.000 |" in text
    assert "| k_down3d_march<level 0> | 16,523,636 | 16,523,636 | 1.000 |" in text   # weighted 21 : 12
    assert "not matched): k_smooth<coarse levels>" in text
    # apply_A: 2000 KiB x 2 + 1000 KiB
    assert "5,120,000 B measured, 5,120,000 B algorithmic (ratio 1.000)" in text
    assert "traffic k_down3d_march<level0> source=paper_2609_16863_amd/csrc/kern_mg.hip" in text
