"""Host-side checks of bench.py's contract that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_algorithmic_counts_of_the_bench_workload():
    """The algorithmic flops of the translations (8 x 4 x Q^2 per pair) and the
    phase byte counts are the ones the roofline lines divide by."""
    sys.path.insert(0, ROOT)
    import bench
    info = {"n_rwg": 201720, "L": 5, "l0": 2, "n_box": [56, 272, 1160, 4544],
            "n_pairs": [2504, 12216, 54000, 205824], "near_entries": 134473164,
            "near_entries_half": 73234866, "near_transposed": 1349520}
    Q = [441, 196, 81, 49]
    alg = bench.algorithmic(info, Q, 8)
    assert abs(alg["translate"]["flops"] - 57.75e9) < 0.01e9
    assert alg["radiate"]["bytes"] == 201720 * 4 * 49 * 8 + 201720 * 8 + 4544 * 4 * 49 * 8
    # half storage: 73.2M stored near entries, 1.35M transposed outputs
    assert alg["near_recv"]["bytes"] == (73234866 + 2 * 1349520 + 201720 * 4 * 49 + 2 * 201720
                                         + 4544 * 4 * 49) * 8
    assert alg["near_recv"]["flops"] == 8 * 134473164 + 8 * 4 * 49 * 201720
    json.dumps(alg)
