"""Host-side logic of bench.py (no GPU): the algorithmic byte model the
roofline divides by, the kernel-source hash that keys the stored traffic
counters, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_reconstruction_bytes_model():
    # two scans reading I and J and writing J (6 B/px), 10 + 2c bytes per queue item
    assert bench.algorithmic_bytes("mr16k_conn8", "mr_propagate", 100, 7, 8) == 6 * 100 + 26 * 7
    assert bench.algorithmic_bytes("mr16k_conn4", "mr_propagate", 100, 7, 4) == 6 * 100 + 18 * 7
    assert bench.algorithmic_bytes("mr16k_conn8", "reset", 100, 7, 8) == 0.0


def test_edt_bytes_model():
    # initialisation 5 B/px; rounds 12 B/px plus 24 + 4c bytes per frontier item
    assert bench.algorithmic_bytes("edt4k_conn8", "edt_init", 100, 7, 8) == 500
    assert bench.algorithmic_bytes("edt4k_conn8", "edt_rounds", 100, 7, 8) == 12 * 100 + 56 * 7
    assert bench.algorithmic_bytes("edt4k_conn4", "edt_rounds", 100, 7, 4) == 12 * 100 + 40 * 7


def test_kernel_source_hash_is_stable_and_covers_the_kernels():
    h = bench.kernel_source_sha()
    assert h == bench.kernel_source_sha()
    assert len(h) == 16 and int(h, 16) >= 0
    names = sorted(os.listdir(bench.CSRC))
    assert "iwpp_mr.hip" in names and "iwpp_edt.hip" in names


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
