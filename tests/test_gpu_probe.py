"""The attainable-rate probe the benchmark's rooflines use: its arithmetic
is exact for m = c = 1 (each chain counts its fused multiply-adds)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_fp64_probe_counts_its_fmas():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_10987_amd import hydro
    print("case: FP64 FMA probe, 4 x 256 threads, 1000 iterations", flush=True)
    out = torch.full((4 * 256,), -1.0, dtype=torch.float64, device="cuda")
    hydro.fp64_probe(out, 4, 1000)
    torch.cuda.synchronize()
    t = np.arange(4 * 256, dtype=np.float64)
    assert np.array_equal(out.cpu().numpy(), 8 * t + 28 + 8 * 1000)
    with pytest.raises(hydro.HydroError):
        hydro.fp64_probe(out, 0, 10)
