"""The matrix-core probe (hfx_mfma_peak) on the GPU: each MFMA kind the build uses reports a
throughput of the order of the part's data-sheet peak (between a fifth and two and a half times
it: the probe ran and counted its FLOPs per instruction right) and a positive shader clock; the
measured values are what bench.py reports beside the data-sheet peak."""
import pytest

from test_gpu_parity import log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["fp64", "fp32", "bf16"])
def test_probe_reports_a_plausible_peak(kind):
    from paper_2009_12505_amd import peak
    log(f"case matrix-core probe {kind}")
    tf, mhz = peak.mfma_peak(kind)
    ref = peak.DATASHEET_TFLOPS[kind]
    log(f"  {kind}: {tf:.1f} TFLOP/s measured ({tf / ref:.3f} of {ref}), shader clock {mhz:.0f} MHz")
    assert 0.2 * ref < tf < 2.5 * ref
    assert mhz > 0

