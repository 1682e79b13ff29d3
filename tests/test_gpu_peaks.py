"""The ceiling probes of the roofline (libadg_peaks.so): the copy moves the data and both
rates fall inside what the MI355X datasheet allows (8 TB/s HBM, 78.6 TFLOP/s FP64 vector)."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_ceilings_are_plausible():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_01747_amd import peaks

    m = peaks.measure(copy_bytes=256 << 20, n_reps=5)
    print(f"[peaks] copy {m['copy_GBps']:.0f} GB/s, FP64 {m['fp64_vector_TFLOPs']:.1f} TFLOP/s", flush=True)
    assert 1000.0 < m["copy_GBps"] < 8000.0
    assert 10.0 < m["fp64_vector_TFLOPs"] < 80.0
