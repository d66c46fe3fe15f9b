"""Host logic of bench.py: algorithmic bytes per kernel for each storage form (no GPU)."""
import bench


def _info(**kw):
    base = dict(n=1000, kind=0, storage=0, elem_bytes=16, elems_forward=100, elems_coupling=200,
                elems_backward=300, elems_near=400, rank_space=10, partial_coupling=0, partial_near=0,
                elems_coupling_in=0)
    base.update(kw)
    return base


def test_general_form():
    ab = bench.algorithmic_bytes(_info(), 1000)
    assert ab["k_forward_tiles"] == 16 * 100 + 16 * (1000 + 10)
    assert ab["k_coupling"] == 16 * 200 + 16 * 20
    assert ab["k_backward"] == 16 * 700 + 16 * (2000 + 10)
    assert ab["total"] == 16 * 1000 + 16 * (2000 + 40)


def test_symmetric_form_counts_the_partial_sums():
    ab = bench.algorithmic_bytes(_info(storage=4, partial_coupling=50, partial_near=30), 1000)
    assert ab["k_coupling_sym"] == 16 * 200 + 16 * (20 + 50)
    assert ab["k_backward_sym"] == 16 * 700 + 16 * (2000 + 10 + 30)
    assert "k_coupling" not in ab and "k_backward" not in ab
    assert ab["total"] == 16 * 1000 + 16 * (2000 + 40 + 100 + 60)


def test_factored_form_counts_both_factors():
    ab = bench.algorithmic_bytes(_info(storage=5, elems_coupling_in=80), 1000)
    assert ab["k_factor_in"] == 16 * 80 + 16 * 20
    assert ab["total"] == 16 * 1080 + 16 * (2000 + 60)
    # complex64 vectors for the low-precision forms
    ab = bench.algorithmic_bytes(_info(storage=6, elem_bytes=8, elems_coupling_in=80), 1000)
    assert ab["k_forward_tiles"] == 8 * 100 + 8 * 1010


def test_bench_cli_on_the_host():
    """The parts of bench.py that need no GPU: more than one GPU is refused with a message,
    and the direct-construction mode runs end to end on a small cloud."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU only" in r.stderr
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--mode", "direct", "--n", "3000"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["ranks_equal"] and line["sampled_rel_diff"] <= 1e-12
    assert line["peak_factor_bytes"] < line["total_factor_bytes"]
