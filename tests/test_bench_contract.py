"""The benchmark's contract on the CPU: it measures one GPU and refuses any
other count before touching a device, and its plain-check accounting
(work per kernel vector of the per-ridge AND + popcount check) gives the
hand count on the Fano configuration."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.join(HERE, "..")


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_plain_check_accounting_on_fano():
    # Fano: 28 candidate facets in one word, 21 ridges with 4 parents each:
    # W (Gray XOR) + 21 x (AND + popcount on one word + compare) + W + 1
    sys.path.insert(0, ROOT)
    import bench
    import wpm_inputs as W
    from paper_2301_00806_amd import engine as E
    p = E.prepare(3, 7, lam=W.fano().lam)
    assert len(p.facets) == 28
    assert bench.ops_alg_plain(p) == 1 + 21 * 3 + 1 + 1 == 66
