"""The measured ceilings that the benchmark reports beside the published
peaks: register-only matrix-core rates and a streaming HBM read rate."""
import math

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2506_06661_amd as p
    return p


def test_probe_mfma(pkg):
    published = {pkg.DFJK_F64: 78.6, pkg.DFJK_F32: 157.3, pkg.DFJK_BF16: 2516.6}
    for dt, peak in published.items():
        r = pkg.dfjk_probe_mfma(dt)
        print(f"dtype {dt}: {r:.1f} TFLOP/s", flush=True)
        assert math.isfinite(r) and 0.05 * peak < r < 1.05 * peak


def test_probe_hbm_read(pkg):
    buf = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    r = pkg.dfjk_probe_hbm_read(buf)
    print(f"streaming read {r:.0f} GB/s", flush=True)
    assert math.isfinite(r) and 500.0 < r < 8000.0 * 1.05
    with pytest.raises(pkg.DFJKError):
        pkg.dfjk_probe_hbm_read(buf, 8)
