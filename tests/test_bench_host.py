"""Host logic of bench.py that needs no GPU: kernel-name shortening, the
rocprofv3 summaries (traffic scaled by the copy calibration, merged per leg,
tied to the hash of the HIP sources), and the refusal of several GPUs."""
import csv
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_short_kernel_names():
    assert bench.short_kernel_name("void divas::(anonymous namespace)::k_fuse_all<0>(divas::FuseArgs)") == "k_fuse_all"
    assert bench.short_kernel_name("void divas::(anonymous namespace)::k_fuse_all<0>(divas::FuseArgs)",
                                   keep_template=True) == "k_fuse_all<0>"
    assert bench.short_kernel_name("divas::(anonymous namespace)::k_cull(divas::ChunkBox const*, long const*)") == \
        "k_cull"
    assert bench.short_kernel_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"
    name = "void divas::(anonymous namespace)::k_fuse_targets<8, false>(divas::TargetArgs const*)"
    assert bench.short_kernel_name(name, keep_template=True) == "k_fuse_targets<8, false>"
    nested = ("void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<long>, "
              "std::array<char*, 1ul> >(int, at::native::FillFunctor<long>, std::array<char*, 1ul>)")
    assert bench.short_kernel_name(nested) == "vectorized_elementwise_kernel"


def _pmc_csv(path, counter, rows):
    """A counter_collection.csv with one row per (dispatch, kernel, KiB)."""
    fields = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
              "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
              "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields, quoting=csv.QUOTE_NONNUMERIC)
        w.writeheader()
        for d, (kernel, kib) in enumerate(rows):
            r = {k: 0 for k in fields}
            r.update(Dispatch_Id=d + 1, Kernel_Name=kernel, Counter_Name=counter, Counter_Value=float(kib))
            w.writerow(r)


def test_traffic_summary_scales_by_the_copy_and_merges_legs(tmp_path):
    fuse = "void divas::(anonymous namespace)::k_fuse_all<0>(divas::FuseArgs)"
    copy = "__amd_rocclr_copyBuffer"
    # the 64 MiB copy: FETCH_SIZE reads half of it, WRITE_SIZE all of it
    _pmc_csv(tmp_path / "cf.csv", "FETCH_SIZE", [(copy, 32768.0)] * 3)
    _pmc_csv(tmp_path / "cw.csv", "WRITE_SIZE", [(copy, 65536.0)] * 3)
    # three dispatches: the median is taken
    _pmc_csv(tmp_path / "f.csv", "FETCH_SIZE", [(fuse, 100.0), (fuse, 1000.0), (fuse, 120.0)])
    _pmc_csv(tmp_path / "w.csv", "WRITE_SIZE", [(fuse, 10.0), (fuse, 30.0), (fuse, 20.0)])
    out = tmp_path / "t.json"
    args = [str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv")]
    bench.summarize(["traffic", str(out), "-"] + args)
    bench.summarize(["traffic", str(out), "R2"] + args)
    doc = json.loads(out.read_text())
    assert doc["source_hash"] == bench.kernel_source_hash()
    assert abs(doc["factors"]["FETCH_SIZE"] - 2.0) < 1e-9 and abs(doc["factors"]["WRITE_SIZE"] - 1.0) < 1e-9
    k = doc["kernels"]["k_fuse_all"]
    assert k["read_bytes"] == 120 * 1024 * 2 and k["write_bytes"] == 20 * 1024
    assert k["bytes"] == k["read_bytes"] + k["write_bytes"]
    assert doc["legs"]["R2"]["kernels"]["k_fuse_all"] == k


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
