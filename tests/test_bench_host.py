"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic work
behind roofline.achieved, the comment-blind kernel fingerprint that keeps the
stored counters valid, and the counter summary behind roofline.traffic."""
import csv
import json
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("n", [1, 2, 3, 7, 20, 25])
def test_work_counts_every_internal_node_once(n):
    """A 2^n-leaf tree has 2^n - 1 internal nodes, 2^(n-1) of them bottom
    nodes (children are leaves): one key's work is their weighted sum."""
    for prf in ("aes128", "chacha20"):
        vf, vb = bench.VALU_NODE[prf]
        lf, lb = bench.LOOKUPS_NODE[prf]
        bottom, full = 1 << (n - 1), (1 << (n - 1)) - 1
        assert full + bottom == (1 << n) - 1
        assert bench.algorithmic_work(n, 1, 64, prf=prf) == (full * vf + bottom * vb, full * lf + bottom * lb)
        # linear in the batch; the VALU product adds a multiply and an add per leaf and column
        v3, l3 = bench.algorithmic_work(n, 3, 64, prf=prf)
        assert (v3, l3) == (3 * (full * vf + bottom * vb), 3 * (full * lf + bottom * lb))
        vp, lp = bench.algorithmic_work(n, 3, 10, valu_product=True, prf=prf)
        assert vp - v3 == 3 * (1 << n) * 2 * 10 and lp == l3


def test_work_of_the_benchmark_launch():
    """1024 keys on 2^20 leaves, the figures the design notes quote."""
    assert bench.algorithmic_work(20, 1024, 64) == (686_120_343_552, 360_776_896_512)
    assert bench.algorithmic_work(20, 1024, 64, prf="chacha20")[0] == 1_021_127_478_272
    assert bench.algorithmic_work(20, 1024, 64, prf="chacha20")[1] == 0


def test_kernel_digest_ignores_comments_and_layout(tmp_path, monkeypatch):
    src = tmp_path / "k.h"
    src.write_text("// header\nint f(int x) { return x + 1; } /* block\n comment */\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    d0 = bench.kernel_digest()
    src.write_text("// another header\n\nint f(int x)\n{\n    return x + 1; // same code\n}\n")
    assert bench.kernel_digest() == d0
    src.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_digest() != d0


def test_traffic_is_reported_only_for_the_profiled_kernel(tmp_path, monkeypatch):
    """roofline.traffic is the stored counter figure of the same workload while
    the kernel sources hash to the digest stored with it, and null once they do
    not, or for a workload with no stored figure."""
    summary = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", {("aes128", 20, 1024, 64): summary})
    summary.write_text(json.dumps({"kernel_digest": bench.kernel_digest(), "bytes_per_launch": 123}))
    assert bench.measured_traffic("aes128") == 123
    assert bench.measured_traffic("aes128", 20, 1024, 64) == 123
    assert bench.measured_traffic("aes128", 20, 1024, 128) is None
    assert bench.measured_traffic("aes128", 22, 1024, 64) is None
    assert bench.measured_traffic("aes128", 20, 512, 64) is None
    assert bench.measured_traffic("chacha20") is None
    summary.write_text(json.dumps({"kernel_digest": "0" * 16, "bytes_per_launch": 123}))
    assert bench.measured_traffic("aes128") is None
    summary.write_text("not json")
    assert bench.measured_traffic("aes128") is None


def write_pmc(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(w.fieldnames, r)))


def test_pmc_summary_averages_dispatches_and_scales_by_the_copy(tmp_path):
    """Counters of one dispatch are summed over their rows (one per agent
    block), averaged over dispatches of the batched kernel, and scaled by
    what the same counter reads for the largest copy (the calibration copy of
    256 MiB)."""
    waves = "void (anonymous namespace)::k_pir_waves<AesPrf, 4, true>(WaveTasks, unsigned int)"
    copy = "__amd_rocclr_copyBuffer"
    fetch = tmp_path / "fetch.csv"
    write_pmc(fetch, [(1, waves, "FETCH_SIZE", 60.0), (1, waves, "FETCH_SIZE", 40.0),
                      (2, waves, "FETCH_SIZE", 300.0),
                      (3, copy, "FETCH_SIZE", 10.0), (4, copy, "FETCH_SIZE", 65536.0),
                      (4, copy, "FETCH_SIZE", 65536.0), (5, "k_fill_zero", "FETCH_SIZE", 9.0)])
    write = tmp_path / "write.csv"
    write_pmc(write, [(1, waves, "WRITE_SIZE", 1000.0), (2, waves, "WRITE_SIZE", 3000.0),
                      (4, copy, "WRITE_SIZE", 262144.0)])
    avg, scale, dispatches = bench.pmc_summary([str(fetch), str(write)], copy_mib=256)
    assert avg == {"FETCH_SIZE": 200.0, "WRITE_SIZE": 2000.0}
    assert scale == {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
    assert dispatches == 4  # two dispatches in each file
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--pmc-summary", str(fetch), str(write),
                        "--calibrate-copy", "256"], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    assert out["bytes_per_launch"] == 1024 * (200 * 2 + 2000 * 1)
    assert out["kernel_digest"] == bench.kernel_digest()


def test_pmc_summary_of_another_kernel(tmp_path):
    """--pmc-kernel selects the dispatches summarised: here the single-key
    kernel's, ignoring the batched kernel's in the same file."""
    fused = "void (anonymous namespace)::k_pir_fused<AesPrf, 1, 1, true, true>(FusedArgs)"
    waves = "void (anonymous namespace)::k_pir_waves<AesPrf, 4, true>(WaveTasks, unsigned int)"
    copy = "__amd_rocclr_copyBuffer"
    fetch = tmp_path / "fetch.csv"
    write_pmc(fetch, [(1, waves, "FETCH_SIZE", 900.0), (2, fused, "FETCH_SIZE", 50.0),
                      (3, fused, "FETCH_SIZE", 70.0), (4, copy, "FETCH_SIZE", 131072.0)])
    write = tmp_path / "write.csv"
    write_pmc(write, [(1, waves, "WRITE_SIZE", 900.0), (2, fused, "WRITE_SIZE", 4.0),
                      (4, copy, "WRITE_SIZE", 262144.0)])
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--pmc-summary", str(fetch), str(write),
                        "--pmc-kernel", "k_pir_fused", "--calibrate-copy", "256"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    assert out["kernel"].startswith("k_pir_fused")
    assert out["counters_avg"] == {"FETCH_SIZE": 60.0, "WRITE_SIZE": 4.0}
    assert out["bytes_per_launch"] == 1024 * (60 * 2 + 4 * 1)


def test_every_stored_counter_summary_names_its_workload():
    """Each committed summary that roofline.traffic reads exists, and its note
    names the table shape and PRF of the key it is stored under."""
    for (prf, log_rows, keys, dim), path in bench.TRAFFIC_SUMMARY.items():
        t = json.loads(path.read_text())
        assert t["prf"] == prf and t["bytes_per_launch"] > 0
        assert f"{keys} keys, 2^{log_rows} x {dim} table" in t["note"], path
        assert (f"--dim {dim} " in t["command"]) == (dim != 64), path


def test_roofline_binds_on_lds_lookups_for_aes_and_the_valu_for_chacha():
    """AES-128 is bound by LDS table lookups: frac = algorithmic lookups per
    launch / launch time / the unit-count LDS peak; ChaCha20 has no table and
    is bound by the VALU."""
    kern_s = 0.021
    r, lds, valu = bench.rooflines("aes128", 20, 1024, 64, kern_s, "k_pir_waves")
    lookups = 360_776_896_512
    assert r["bound"] == "lds" and r["unit"] == "T lookups/s" and r["kernel"] == "k_pir_waves"
    assert r["lookups_per_launch"] == lookups == lds["lookups_per_launch"]
    assert abs(r["frac"] - lookups / kern_s / bench.PEAK_LDS_LOOKUPS) < 1e-4
    assert abs(r["peak"] - 19.661) < 1e-3 and r["frac"] == lds["frac"]
    assert abs(valu["frac"] - 686_120_343_552 / kern_s / bench.PEAK_INT32_OPS) < 1e-4
    r, lds, valu = bench.rooflines("chacha20", 20, 1024, 64, kern_s, "k_pir_waves")
    assert lds is None and r["bound"] == "alu" and r["frac"] == valu["frac"]
    assert r["valu_ops_per_launch"] == 1_021_127_478_272


def test_host_cpus_reports_what_the_oracle_runs_on():
    h = bench.host_cpus()
    assert 1 <= h["usable_cores"] <= h["nproc"] <= (h["os_cpu_count"] or h["nproc"])
    if h["cgroup_cpu_quota"]:
        assert h["usable_cores"] <= h["cgroup_cpu_quota"]
    assert h["cpu_model"] is None or isinstance(h["cpu_model"], str)
