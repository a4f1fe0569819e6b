"""The peak probes of the C ABI run and return plausible values on the GPU: the STREAM
triad's bandwidth, the matrix cores' FP32 / FP64 throughput and the co-execution timings
(products alone, vector FMAs alone, both)."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_probes_return_plausible_values():
    from paper_1802_05246_amd import binding as B
    gbs = B.hw_probe_stream_triad(1 << 26)
    t32 = B.hw_probe_mfma(B.HW_FP32)
    t64 = B.hw_probe_mfma(B.HW_FP64)
    co = B.hw_probe_coexec()
    print(f"[probes] triad {gbs:.0f} GB/s, mfma fp32 {t32:.1f} / fp64 {t64:.1f} TFLOP/s, coexec ms {co}", flush=True)
    # within published peaks (8 TB/s, 157.3 / 78.6 TFLOP/s dense), and not absurdly low
    assert 500.0 < gbs < 8000.0
    assert 10.0 < t32 < 160.0 and 5.0 < t64 < 80.0
    assert all(x > 0.0 for x in co)
    # running both kinds of work takes at least as long as the longer of the two alone
    assert co[2] >= 0.95 * max(co[0], co[1])


def test_probe_rejects_bad_arguments():
    from paper_1802_05246_amd import binding as B
    with pytest.raises(B.HwError):
        B.hw_probe_stream_triad(7)
    with pytest.raises(B.HwError):
        B.hw_probe_mfma(B.HW_BF16)
