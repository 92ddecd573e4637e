"""Host-side pricing of bench.py's roofline (no device): each launch class is
bound by the larger of its flops at the MFMA peak and its bytes at the HBM
peak, and named by the kernel symbol rocprofv3 reports for it."""
import bench


def launch(cls, tile, level, ms, flops, nbytes, peak):
    return {"cls": cls, "tile": tile, "level": level, "ms": ms, "flops": flops, "bytes": nbytes, "peak_tf": peak,
            "max_prod_flops": flops / 2}


def test_price_picks_the_binding_roof():
    # 1 TFLOP in 20 ms at 78.6 TF peak (12.7 ms) vs 1 GB at 8 TB/s (0.125 ms): MFMA bound
    r = bench.price([launch("gemm35", 64, 3, 20.0, 1e12, 1e9, 78.6)], 0.0)
    assert r["bound"] == "mfma" and abs(r["achieved"] - 50.0) < 1e-9 and abs(r["frac"] - 50.0 / 78.6) < 1e-12
    # 1 GFLOP and 4 GB in 1 ms: HBM bound at 4 TB/s = half the peak
    r = bench.price([launch("gemm4", 64, 3, 1.0, 1e9, 4e9, 78.6)], 0.0)
    assert r["bound"] == "hbm" and abs(r["achieved"] - 4000.0) < 1e-6 and abs(r["frac"] - 0.5) < 1e-12
    # the event overhead comes off every launch interval, at most half of it
    r = bench.price([launch("gemm4", 64, 3, 1.0, 1e9, 4e9, 78.6)], 0.2)
    assert abs(r["mean_launch_ms"] - 0.8) < 1e-12
    r = bench.price([launch("gemm4", 64, 3, 1.0, 1e9, 4e9, 78.6)], 0.9)
    assert abs(r["mean_launch_ms"] - 0.5) < 1e-12


def test_roofline_takes_the_largest_class_and_names_its_kernel():
    ph = {"event_overhead_ms": 0.0, "launches": [
        launch("tri", 0, -1, 0.5, 1e9, 1e9, 78.6),
        launch("gemm35g", 32, 20, 2.0, 1e11, 1e9, 78.6),
        launch("gemm35g", 32, 21, 2.0, 1e11, 1e9, 78.6),
        launch("gemm35", 64, 5, 3.0, 1e11, 1e9, 78.6),
        launch("gemm4", 64, 5, 1.0, 1e9, 1e9, 78.6),
    ]}
    r = bench.roofline(ph, "fp64")
    assert r["class"] == "gemm35g" and r["launches"] == 2
    assert r["kernel"] == "selinv::gemm_g35<0, 32, 32, double>"
    r = bench.roofline(ph, "mixed_bf16x3")
    assert r["kernel"] == "selinv::gemm_g35<2, 32, 32, float>"
    lp = bench.largest_product(ph, "mixed_bf16x3")
    assert lp["level"] in (20, 21, 5) and abs(lp["issued_frac_of_bf16_peak"] - 3 * lp["useful_tflops"] / 2500) < 1e-12
