"""The measurement contract of bench.py, checked on the host (no GPU):
roofline entries, the bound each kernel is priced against, and the refusal
of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

ROOF_KEYS = {"kernel", "bound", "achieved", "peak", "unit", "frac", "traffic", "avg_launch_us"}


def _counters(nl=10, active=1000.0, ms_apply=0.4, ms_update=0.4):
    return {"cg_timed_launches": nl, "cg_timed_active": active * nl, "cg_timed_columns": active * nl,
            "ms_cg_apply": ms_apply, "ms_cg_update": ms_update}


def test_rooflines_price_each_kernel_against_its_bound():
    # 6561-realization layout: sum R_i = 2560, sum R_i^2 = 181248, M = 1280
    sz = {"M": 1280, "darcy_flops": 21.7e9}
    k = bench.kernel_rooflines(sz, 2560, 181248, _counters(), 6.4, "fp64", "no-such-workload")
    for name in ("cg_update", "cg_apply", "darcy_basis"):
        assert ROOF_KEYS <= set(k[name]), name
        assert 0 < k[name]["frac"] and k[name]["achieved"] / k[name]["peak"] == pytest.approx(k[name]["frac"])
    upd = k["cg_update"]
    assert upd["bound"] == "hbm" and upd["unit"] == "GB/s" and upd["peak"] == 8000.0
    # 8 (sum R_i + 6 M) bytes per realization-iteration, 1000 active, 40 us per launch
    assert upd["bytes_per_unit"] == 8 * (2560 + 6 * 1280)
    assert upd["achieved"] == pytest.approx(upd["bytes_per_unit"] * 1000 / 40e-6 / 1e9)
    # 11.8 flop/B is above the FP64 MFMA ridge (78.6 / 8 = 9.8): priced against MFMA
    app = k["cg_apply"]
    assert app["bound"] == "mfma" and app["unit"] == "TFLOP/s" and app["peak"] == 78.6
    assert app["achieved"] == pytest.approx(2 * 181248 * 1000 / 40e-6 / 1e12)
    assert k["darcy_basis"]["bound"] == "mfma" and k["darcy_basis"]["peak"] == 78.6
    # the uneven layout: 2 sum R_i^2 = 203,904 flops against 23,040 bytes (8.9 flop/B) is HBM-bound
    k3 = bench.kernel_rooflines({"M": 960, "darcy_flops": 313e9}, 1920, 101952, _counters(), 42.0, "mixed",
                                "no-such-workload")
    assert k3["cg_apply"]["bound"] == "hbm" and k3["cg_apply"]["unit"] == "GB/s"
    # no counter summary for an unknown workload: traffic is null, not guessed
    assert k3["cg_apply"]["traffic"] is None and k3["cg_update"]["traffic"] is None


def test_traffic_is_reported_only_for_the_profiled_kernel_source():
    """A counter summary carries the hash of the kernel source it was taken
    with; the bench reports traffic from it only while the hash matches."""
    for kernel, name in (("cg_update2", "cg_update2_kernel"), ("cg_apply_mfma", "cg_apply_mfma_kernel")):
        path = os.path.join(ROOT, "profiles", "traffic_%s_cfg2.txt" % kernel)
        assert os.path.exists(path), path
        recorded = [ln.split(":", 1)[1].strip() for ln in open(path) if ln.startswith("kernel_source_sha256_16:")]
        assert len(recorded) == 1
        t = bench.read_traffic(kernel, "cfg2")
        if recorded[0] == bench.kernel_source_hash(name):
            assert t is not None and t > 0
        else:
            assert t is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--no-cpu-baseline"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_whole_cg_figure_adds_both_kernels():
    """The whole-CG figure counts the product's and the update's algorithmic
    bytes, 8 (M + sum R_i) + 8 (sum R_i + 6 M) per realization-iteration, and
    the product's 2 sum R_i^2 flops, over the CG wall time."""
    w = bench.cg_whole(2560, 181248, 1280, 1.0e6, 100.0)
    assert w["bytes_per_unit"] == 8 * (1280 + 2560) + 8 * (2560 + 6 * 1280) == 112640
    assert w["gbps"] == pytest.approx(112640 * 1.0e6 / 0.1 / 1e9)
    assert w["frac_hbm"] == pytest.approx(w["gbps"] / 8000.0)
    assert w["tflops"] == pytest.approx(2 * 181248 * 1.0e6 / 0.1 / 1e12)
    assert w["frac_fp64_mfma"] == pytest.approx(w["tflops"] / 78.6)
