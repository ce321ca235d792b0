"""bench.py's command-line contract on the CPU: more than one GPU is refused with a message."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in msg and "one GPU" in msg["error"]


def test_eq28_helpers_reproduce_the_papers_example():
    """Eq. 28 (Sec. IV.C): with the worked example's short/long counts (275/190, 13 PAOs, 4 LNOs)
    the ratio is the printed 0.37; the printed formula with the buffer at exactly kappa N_S
    (N_F = 167, N_S = 298) gives 0.33 instead, which is why the sweep reports both forms."""
    sys.path.insert(0, ROOT)
    import bench
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "region_counts.json")))
    c = g["cases"][0]
    assert round(bench.eq28_ratio(c["n_short"], c["n_long"], c["m_pao"], c["m_lno"]), 2) == c["time_ratio"]
    n_s = c["n_cluster"] - c["n_fna"]
    assert round(bench.eq28_kappa(c["n_fna"], n_s, c["m_pao"], c["m_lno"], g["kappa"]), 2) == 0.33
    # no LNO savings when M_L = M_P
    assert abs(bench.eq28_ratio(275, 190, 13, 13) - 1.0) < 1e-15
