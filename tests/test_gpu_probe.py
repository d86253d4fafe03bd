"""The float64 MFMA-rate probe (the hardware reference quoted beside the roofline): it runs,
reports a positive rate no higher than the published peak, and rejects bad arguments."""
import pytest

pytestmark = pytest.mark.gpu


def test_mfma_probe_rate_and_errors():
    from paper_2101_07249_amd import Wc4dError
    from paper_2101_07249_amd import wc4d as W4
    print("[case] mfma probe", flush=True)
    r = W4.probe_mfma_f64(2, 500, 2)
    print("[result] TFLOP/s", r, flush=True)
    assert 0.0 < r <= 78.6 * 1.02
    with pytest.raises(Wc4dError):
        W4.probe_mfma_f64(0, 500, 2)
    with pytest.raises(Wc4dError):
        W4.probe_mfma_f64(2, 500, 2, device=99)
