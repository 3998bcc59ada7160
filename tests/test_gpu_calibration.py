"""The FLOP-accounting calibration kernel (hjpd_calibrate_fma): its exact
flop and instruction counts, and a rate within physical bounds."""
import pytest

pytestmark = pytest.mark.gpu


def test_fma_calibration_counts_and_rate():
    import torch

    from paper_1803_01215_amd import hjpd as C
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    r = C.hjpd_calibrate_fma(C.HJPD_F32, 8, 2, 200)
    insts = cus * 2 * 4 * 200 * 32 * 8
    assert r["wave_instructions"] == insts and r["flops"] == insts * 128
    assert 0 < r["flops"] / (r["ms"] * 1e-3) < 2 * 157.3e12
    r64 = C.hjpd_calibrate_fma(C.HJPD_F64, 4, 1, 100)
    assert r64["ms"] > 0 and r64["flops"] == cus * 4 * 100 * 32 * 4 * 128
