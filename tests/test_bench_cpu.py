"""The bench line's roofline object from a kernel profile (host logic, no
GPU): the dominant class by total time, its arithmetic intensity against the
ridge of its operand type, and the resource that bounds it."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _prof(**classes):
    return {k: dict(v, bytes=v.get("bytes", 1.0)) for k, v in classes.items()}


def test_dominant_fp32_gemm_above_the_ridge_is_mfma_bound():
    # 1.2 GFLOP on 57 MB of optimiser state: 21 FLOP/B, above fp32's 19.7
    kp = _prof(**{"adj.fp32.t32x32": dict(launches=10, ms=0.4, flops=1.2e10, alg_bytes=5.7e8),
                  "bound.fp32.t32x32": dict(launches=10, ms=0.3, flops=1.2e10, alg_bytes=1e8)})
    r = bench.roofline(kp, "fp32")
    assert r["kernel"] == "adj.fp32.t32x32" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(1.2e10 / 0.4e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)


def test_bf16_gemm_below_the_ridge_is_hbm_bound():
    kp = _prof(**{"adj.bf16.t16x64": dict(launches=5, ms=0.15, flops=6e9, alg_bytes=2.85e8)})
    r = bench.roofline(kp, "bf16")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(2.85e8 / 0.15e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)


def test_direct_conv_is_bound_by_the_vector_alus():
    kp = _prof(**{"convT_conc.fp32.direct": dict(launches=1, ms=0.3, flops=7.25e9, alg_bytes=0.0)})
    r = bench.roofline(kp, "fp32")
    assert r["bound"] == "alu" and r["peak"] == 78.6
    assert r["frac"] == pytest.approx(7.25e9 / 0.3e-3 / 1e12 / 78.6)
