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
    # 6561-realization layout: sum R_i^2 = 181248, M = 1280
    sz = {"M": 1280, "darcy_flops": 21.7e9}
    ms = {"basis_darcy": 6.4}
    k = bench.kernel_rooflines(sz, 1280, 181248, _counters(), ms, "fp64", "no-such-workload")
    for name in ("cg_update", "cg_apply", "darcy_basis"):
        assert ROOF_KEYS <= set(k[name]), name
        assert 0 < k[name]["frac"] and k[name]["achieved"] / k[name]["peak"] == pytest.approx(k[name]["frac"])
    upd = k["cg_update"]
    assert upd["bound"] == "hbm" and upd["unit"] == "GB/s" and upd["peak"] == 8000.0
    # the update streams 6 M doubles per realization-iteration on average (A p,
    # p and r read, r and p written, lambda read and written every other
    # iteration); 1000 active, 40 us per launch
    assert upd["bytes_per_unit"] == 6 * 1280 * 8
    assert upd["achieved"] == pytest.approx(upd["bytes_per_unit"] * 1000 / 40e-6 / 1e9)
    # the product: 2 sum R_i^2 flops per realization-iteration on FP64 MFMA
    app = k["cg_apply"]
    assert app["bound"] == "mfma" and app["unit"] == "TFLOP/s" and app["peak"] == 78.6
    assert app["achieved"] == pytest.approx(2 * 181248 * 1000 / 40e-6 / 1e12)
    # the FP64 basis build against the FP64 MFMA peak, the mixed one against FP32 MFMA
    assert k["darcy_basis"]["bound"] == "mfma" and k["darcy_basis"]["peak"] == 78.6
    assert k["darcy_basis"]["achieved"] == pytest.approx(21.7e9 / 6.4e-3 / 1e12)
    km = bench.kernel_rooflines(sz, 1280, 181248, _counters(), ms, "mixed", "no-such-workload")
    assert km["darcy_basis"]["peak"] == 157.3
    # no counter summary for an unknown workload: traffic is null, not guessed
    assert km["cg_apply"]["traffic"] is None and km["cg_update"]["traffic"] is None


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


def test_whole_cg_figure_uses_the_scope_table_counts():
    """The whole-CG figure prices a realization-iteration at 5 M 8 bytes (the
    CG vectors streamed once) and 2 sum R_i^2 flops, over the CG wall time."""
    w = bench.cg_whole(1280, 181248, 1.0e6, 100.0)
    assert w["bytes_per_unit"] == 5 * 1280 * 8 == 51200
    assert w["flops_per_unit"] == 2 * 181248 == 362496
    assert w["gbps"] == pytest.approx(51200 * 1.0e6 / 0.1 / 1e9)
    assert w["frac_hbm"] == pytest.approx(w["gbps"] / 8000.0)
    assert w["tflops"] == pytest.approx(362496 * 1.0e6 / 0.1 / 1e12)
    assert w["frac_fp64_mfma"] == pytest.approx(w["tflops"] / 78.6)


def test_moment_errors_are_relative_to_the_largest_entry():
    import numpy as np
    ref = {f: (np.array([1.0, -2.0]), np.array([0.5, 0.25])) for f in bench.FIELD_NAMES}
    mom = {f: (np.array([1.0, -2.0 + 2e-9]), np.array([0.5 + 5e-10, 0.25])) for f in bench.FIELD_NAMES}
    e = bench.moment_errors(mom, ref)
    for f in bench.FIELD_NAMES:
        assert e[f]["mean"] == pytest.approx(1e-9)
        assert e[f]["var"] == pytest.approx(1e-9)
