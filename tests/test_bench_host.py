"""Host-side parts of the benchmark that need no GPU: the refusal of more
than one GPU, the algorithmic flop count the roofline line divides by, the
validity gate behind ``invalid_pairs``, and the rule that an HBM-traffic
summary taken on other kernel sources is not reported."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and r.stdout == ""


def test_forward_flop_count():
    """L s complex N^3 products at 8 flops per complex MAC per pair, (8/3 + 8)
    N^3 per transformation and (8/3) N^3 for each pair's final solve; the
    N = 61 gradient workload's launch (128 pairs, 400 slices, 7 stages,
    19925 transformations in all) is the 6.99e11 flops the roofline uses."""
    N, L, s = 5, 3, 7
    assert bench._flops_forward(N, L, s, 0, 1) == pytest.approx(L * s * 8 * N**3 + 8 / 3 * N**3)
    assert bench._flops_forward(N, L, s, 4, 2) - bench._flops_forward(N, L, s, 0, 2) == pytest.approx(4 * 32 / 3 * N**3)
    assert bench._flops_forward(61, 400, 7, 19925, 128) == pytest.approx(6.99e11, rel=1e-3)


def test_validity_gate():
    import torch
    ok = torch.tensor([[0.2, 0.3, 0.0], [0.5, 0.5, 0.0]], dtype=torch.float64)
    st = torch.zeros(2, dtype=torch.int32)
    assert bench.invalid_pairs(ok, st, 0.1) == 0
    cases = [torch.tensor([[0.7, 0.4, 0.0]]),            # more flux out than in under absorption
             torch.tensor([[0.1, -1e-3, 0.0]]),          # a negative intensity
             torch.tensor([[0.1, float("nan"), 0.0]])]   # not finite
    for c in cases:
        assert bench.invalid_pairs(c.double(), torch.zeros(1, dtype=torch.int32), 0.1) == 1
    # without absorption the flux bound is not applied
    assert bench.invalid_pairs(cases[0].double(), torch.zeros(1, dtype=torch.int32), 0.0) == 0
    # a failure status counts whatever the curve
    assert bench.invalid_pairs(ok, torch.tensor([0, 3], dtype=torch.int32), 0.1) == 1


def test_traffic_summary_on_other_sources_is_not_used(tmp_path, monkeypatch):
    summary = tmp_path / "summary.md"
    monkeypatch.setattr(bench, "traffic_summary", lambda split: str(summary))
    summary.write_text(f"- HBM bytes per launch: 1.5e+10\n- source sha256: `{bench.kernel_source_hash()}`\n")
    assert bench.traffic_from_profile(True) == pytest.approx(1.5e10)
    summary.write_text("- HBM bytes per launch: 1.5e+10\n- source sha256: `" + "0" * 64 + "`\n")
    assert bench.traffic_from_profile(True) is None
    summary.unlink()
    assert bench.traffic_from_profile(True) is None
