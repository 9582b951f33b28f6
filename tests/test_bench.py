"""Host-side logic of bench.py: the roofline record of the dominant kernel,
its HBM traffic from the committed counter summary, and the one-GPU guard.
No GPU is used."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import bench  # noqa: E402


def _report(svd_ms, env_ms, svd_fl=None, env_fl=None, env_by=None):
    n_svd, n_env = len(bench.SVD_KERNELS), len(bench.ENV_KERNELS)
    rep = {"svd_kind_ms": [0.0] * n_svd, "svd_kind_flops": [0.0] * n_svd, "svd_kind_launches": [0] * n_svd,
           "env_kind_ms": [0.0] * n_env, "env_kind_flops": [0.0] * n_env, "env_kind_bytes": [0.0] * n_env,
           "env_kind_launches": [0] * n_env}
    for k, (ms, launches) in svd_ms.items():
        rep["svd_kind_ms"][k], rep["svd_kind_launches"][k] = ms, launches
        rep["svd_kind_flops"][k] = (svd_fl or {}).get(k, 1e9)
    for k, (ms, launches) in env_ms.items():
        rep["env_kind_ms"][k], rep["env_kind_launches"][k] = ms, launches
        rep["env_kind_flops"][k] = (env_fl or {}).get(k, 1e9)
        rep["env_kind_bytes"][k] = (env_by or {}).get(k, 1e9)
    return rep


def test_jacobi_instantiations_priced_together():
    # k_jacobi<8> (kind 1) and k_jacobi<20> (kind 4) each below the channel
    # mix, together above it
    rep = _report({1: (300.0, 1000), 4: (250.0, 300)}, {1: (400.0, 72)},
                  svd_fl={1: 3e11, 4: 2e11})
    r = bench.roofline(rep)
    assert r["kernel"] == bench.JACOBI_FAMILY
    assert r["launches"] == 1300
    assert r["avg_launch_us"] == pytest.approx(550.0 * 1e3 / 1300)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(5e11 / 0.55 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.PEAK_FP64_TFLOPS)


def test_environment_kernel_priced_against_hbm():
    # a low-intensity environment kernel dominates: bandwidth roofline
    rep = _report({1: (100.0, 500)}, {1: (400.0, 72)}, env_fl={1: 1e11}, env_by={1: 1e12})
    r = bench.roofline(rep)
    assert r["kernel"] == "k_mix" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1e12 / 0.4 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.PEAK_HBM_GBS)


def test_traffic_record_matches_the_sources():
    # the committed counter summary covers the Jacobi kernel as it is now
    t = bench.measured_traffic(bench.JACOBI_FAMILY)
    assert t is not None and t["bytes_per_launch"] > 0
    assert t["bytes_per_launch"] == pytest.approx(t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"])
    assert bench.measured_traffic("k_no_such_kernel") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(os.path.dirname(HERE), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stdout
