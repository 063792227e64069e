"""Host logic of bench.py: the algorithmic bytes behind the roofline, the
committed counter traffic being tied to the current kernel sources, and the
refusal of more than one GPU."""
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("dim,N,elt,state", [
    (3, 4, 4, 992),   # D3Q19, N = 4, float32: the impurities workload
    (2, 2, 4, 344),   # D2Q9, N = 2: the droplet
    (2, 3, 4, 424),   # D2Q9, N = 3: the compound droplet
    (2, 2, 8, 688),   # float64 parity mode
])
def test_state_bytes_per_cell_is_every_population_and_lagged_field_read_and_written_once(dim, N, elt, state):
    Q = 9 if dim == 2 else 19
    b = bench.algorithmic_bytes_per_cell(dim, N, elt)
    assert b["step"] == state == 2 * elt * ((N + 2) * Q + (N + dim + 3))


def test_pass_bytes_cover_the_state():
    """The two passes together move the state plus the moments pass's
    re-read of g and h and the moment planes: never less than the state."""
    for dim, N in ((2, 2), (2, 3), (3, 4)):
        b = bench.algorithmic_bytes_per_cell(dim, N, 4)
        Q = 9 if dim == 2 else 19
        assert b["moments"] == 4 * ((N + 1) * Q + 2 + (N + 1))
        assert b["collide"] + b["moments"] > b["step"]


def test_committed_traffic_matches_the_current_kernel_sources():
    with open(os.path.join(ROOT, "profiles", "traffic_impurities_fp32.json")) as f:
        rec = json.load(f)
    assert rec["kernel_hash"] == bench.kernel_hash()
    assert bench.measured_traffic("impurities", "fp32") == rec["bytes_per_launch"]
    # the traffic is within 10 % of the collide kernel's algorithmic bytes
    alg = bench.algorithmic_bytes_per_cell(3, 4, 4)["collide"] * 192 ** 3
    assert rec["algorithmic_bytes"] == alg
    assert 1.0 <= rec["bytes_per_launch"] / alg < 1.1


def test_more_than_one_gpu_is_refused_with_a_message():
    """bench.py times one GPU only: --gpus above 1 exits with status 2 and
    says why, before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_reverse_step_bytes_per_cell():
    """Compound 512^2, N = 3, float32: 736 B/cell for the collide reverse
    and 216 B/cell for the gather (their counters read 1.07x and 1.19x)."""
    b = bench.algorithmic_bytes_reverse(2, 3, 4)
    assert b["collide_reverse"] == 736 and b["gather"] == 216 and b["reverse_step"] == 952
