"""Host logic of bench.py (no GPU): the HBM traffic summary scales each
counter by what it reads for the 256 MiB calibration copy, and the
roofline's traffic field finds each stage's kernel in the committed
summaries by name, and only while the library code is the code the
counters were taken from (comments aside)."""
import csv
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WORKLOADS = ["tc-iso-n32", "tc-heated-n64", "tc-adjoint-n64", "tc-turb-n128",
             "tc-conv-n256", "pipe-n64"]
FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Agent_Id": "Agent 1", "Queue_Id": 1,
                        "Process_Id": 1, "Thread_Id": 1, "Grid_Size": grid, "Kernel_Id": i,
                        "Kernel_Name": name, "Workgroup_Size": 256, "LDS_Block_Size": 0,
                        "Scratch_Size": 0, "VGPR_Count": 8, "Accum_VGPR_Count": 0,
                        "SGPR_Count": 16, "Counter_Name": counter, "Counter_Value": value,
                        "Start_Timestamp": 0, "End_Timestamp": 1})


def test_traffic_report_scales_by_the_calibration_copy(bench, tmp_path):
    """FETCH_SIZE reads half the bytes of the copy and WRITE_SIZE all of
    them: a kernel reading 1 MiB as counted and writing 2 MiB comes out at
    2 + 2 MiB.  A larger non-library copy in the same run (a state clone)
    must not be taken for the calibration kernel."""
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(at::TensorIteratorBase&)::{lambda()#1}::operator()() const::{lambda()#3}::operator()() const::{lambda(double)#1}, std::array<char*, 2ul> >(int, at::native::neg_kernel_cuda(at::TensorIteratorBase&)::{lambda()#1}::operator()() const::{lambda()#3}::operator()() const::{lambda(double)#1}, std::array<char*, 2ul>)"
    kib = 256 * 1024
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    _csv(f, "FETCH_SIZE", [(neg, 8388608, kib / 2), ("__amd_rocclr_copyBuffer", 131072, 8 * kib),
                           ("void nsc::(anonymous namespace)::k_demo<float>(int)", 4096, 1024.0),
                           ("void nsc::(anonymous namespace)::k_demo<float>(int)", 4096, 1024.0)])
    _csv(w, "WRITE_SIZE", [(neg, 8388608, kib), ("__amd_rocclr_copyBuffer", 131072, 16 * kib),
                           ("void nsc::(anonymous namespace)::k_demo<float>(int)", 4096, 2048.0),
                           ("void nsc::(anonymous namespace)::k_demo<float>(int)", 4096, 2048.0)])
    text = bench.traffic_report("demo", str(f), str(w))
    assert "neg_kernel_cuda" in text.splitlines()[1]
    rows = {ln.split()[2]: float(ln.split()[1]) for ln in text.splitlines()
            if ln.startswith("bytes_per_launch")}
    assert rows == {"nsc::k_demo<float>": pytest.approx(4 * 1024 * 1024, rel=1e-12)}
    assert "code_sha256 " + bench.source_digest() in text


@pytest.mark.parametrize("name", WORKLOADS)
def test_committed_traffic_names_one_kernel_per_stage(bench, name):
    """Every timed stage of every configured workload matches exactly one
    kernel of its committed counter summary, of the mixed-precision family
    the stage launches."""
    path = os.path.join(ROOT, "profiles", f"hbm-traffic_{name}.txt")
    if not os.path.exists(path):
        pytest.skip("no committed counter summary")
    for stage in ("zinv", "theta", "zfwd", "rhs", "div", "sweep_pt", "vel_rhs", "sweep_vel",
                  "influence", "finalize"):
        dev, _ = bench.committed_traffic(name, stage)
        assert dev is not None, stage
        assert dev.startswith(bench.STAGE_KERNELS[stage]), (stage, dev)
        if stage in ("zinv", "theta", "zfwd"):
            assert "<float," in dev


def test_committed_traffic_only_for_the_same_code(bench, monkeypatch):
    dev, b = bench.committed_traffic("tc-heated-n64", "theta")
    if b is None:
        pytest.skip("the committed summary belongs to other library code")
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 64)
    dev2, b2 = bench.committed_traffic("tc-heated-n64", "theta")
    assert dev2 == dev and b2 is None


def test_code_digest_ignores_comments_only(bench, tmp_path, monkeypatch):
    """The digest sees code, not comments or layout."""
    src = tmp_path / "paper_1908_00587_amd" / "csrc"
    src.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (src / "a.hip").write_text("int f(int x) {  // twice\n  return 2 * x; /* doubled */ }\n")
    d0 = bench.source_digest()
    (src / "a.hip").write_text("int f(int x) {  // two times x\n\n  return 2 * x;\n}\n")
    assert bench.source_digest() == d0
    (src / "a.hip").write_text("int f(int x) { return 3 * x; }\n")
    assert bench.source_digest() != d0
