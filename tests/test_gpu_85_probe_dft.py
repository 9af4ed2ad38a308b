"""The DFT row-pass probe behind bench.py --probe-dft: both forms of the pass (the library's FFT
stages on the VALU, the dense DFT as an FP32 MFMA GEMM) reproduce numpy's FFT of every row at
L = 51, N_t = 128 before their timings mean anything."""
import pytest

from gpu_common import dev


@pytest.mark.gpu
def test_dft_row_pass_probe_matches_numpy_fft():
    import bench
    from workloads import PREC
    print("[case] probe dft row pass L51 Nt128", flush=True)
    r = bench.dft_pass(PREC, dev())
    for name in ("fft_valu", "dft_mfma_fp32"):
        assert r[name]["max_err_rel"] < 1e-5, (name, r[name])
        assert r[name]["us"] > 0
    assert 0 < r["dft_mfma_fp32"]["mfma_frac_of_fp32_peak"] <= 1
    # the matrix cores' own rate, measured beside the pass, is the datasheet's to within its clock
    for prec in ("fp32", "fp64"):
        assert 0.3 < r["mfma_rate"][prec]["frac_of_datasheet"] < 1.1, r["mfma_rate"]
