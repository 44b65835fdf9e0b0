"""mcpt_device_rates: the FP64 pipe rates the roofline report quotes beside the published peak.

The measured rates must lie below the published dense FP64 peak of the MI355X
(78.6 TFLOP/s, matrix and vector alike), the clock below its 2.4 GHz peak
engine clock, and the compute units must come in whole XCDs.
"""
import pytest

pytestmark = pytest.mark.gpu


def test_device_rates_are_physical():
    import paper_1409_2700_amd as mc

    r = mc.device_rates(0)
    print(r, flush=True)
    assert r["compute_units"] >= 8 and r["compute_units"] % 8 == 0   # whole XCDs (256 on the MI355X)
    assert 10.0 < r["mfma_f64_tflops"] <= 78.6 * 1.02
    assert 10.0 < r["valu_f64_tflops"] <= 78.6 * 1.02
    assert 1.0 < r["clock_ghz"] <= 2.4 * 1.02


def test_device_rates_rejects_bad_device():
    import paper_1409_2700_amd as mc

    with pytest.raises(mc.MCPTError):
        mc.device_rates(99)
