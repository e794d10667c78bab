"""bench.py's byte model and its single-GPU contract (CPU only).

The roofline counts compulsory bytes per 5D output site: the input and output
spinor once and the links once per launch (8 SU(3) matrices per 4D site,
shared by the Ls slices); the figures below are those bytes written out per
precision (FP64 192 B, FP32 96 B, FP16S 48 B of values + 4 B of scale per
spinor; links 8 x 9 complex per 4D site)."""
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))
import bench  # noqa: E402


@pytest.mark.parametrize("prec,Ls,per_site", [
    (0, 16, 2 * 192 + 8 * 9 * 16 / 16),  # FP64: 456 B
    (0, 12, 2 * 192 + 8 * 9 * 16 / 12),  # FP64: 480 B
    (1, 12, 2 * 96 + 8 * 9 * 8 / 12),    # FP32: 240 B
    (2, 16, 2 * 52 + 8 * 9 * 4 / 16),    # FP16S: 122 B
])
def test_hop_bytes_per_site(prec, Ls, per_site):
    assert bench.hop_bytes(prec, Ls, 1000) == pytest.approx(per_site * 1000)


def test_fused_bytes_add_the_epilogue_fields():
    hop = bench.hop_bytes(2, 16, 1)
    # K1 reads and writes one spinor, K2 also reads p~, K4 also reads w and r and writes r
    assert bench.role_bytes(0, 2, 16, 1) == pytest.approx(hop)
    assert bench.role_bytes(1, 2, 16, 1) == pytest.approx(hop + 52)
    assert bench.role_bytes(3, 2, 16, 1) == pytest.approx(hop + 2 * 52)


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                         timeout=300, cwd=ROOT)
    assert out.returncode != 0
    assert "single GPU" in out.stderr + out.stdout
