"""Measured device ceilings (iga_measure_peaks): each probe must land between a floor that a
working unit exceeds easily and the published peak of the MI355X with some clock headroom
(dense FP64 matrix cores 78.6 TFLOP/s, FP32 157.3, BF16 2500; HBM 8 TB/s)."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_physical(gpu_ctx):
    from paper_1811_06797_amd import iga
    pk = iga.measure_peaks(gpu_ctx)
    print(pk, flush=True)
    assert 20.0 < pk["mfma_f64_4x4x4_tflops"] < 1.1 * 78.6
    assert 10.0 < pk["mfma_f64_16x16x4_tflops"] < 1.1 * 78.6
    assert 40.0 < pk["mfma_f32_16x16x4_tflops"] < 1.1 * 157.3
    assert 400.0 < pk["mfma_bf16_16x16x32_tflops"] < 1.1 * 2500.0
    assert 1000.0 < pk["hbm_copy_gbps"] < 8000.0 * 1.05
    assert 1000.0 < pk["hbm_read_gbps"] < 8000.0 * 1.05


def test_measure_peaks_rejects_null(gpu_ctx):
    from paper_1811_06797_amd import iga
    assert iga.lib.iga_measure_peaks(gpu_ctx, None) == iga.EINVAL
