"""bench.py on the host: the one-GPU contract and the algorithmic byte
model behind roofline.achieved (no device needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a configuration it does not run


def test_algorithmic_bytes_model():
    import bench
    n = 1000
    # init + fix-up: 8(n+1) row_ptr + 8n parent/depth + 8n final pass
    base = 8 * (n + 1) + 8 * n + 8 * n
    assert bench.algorithmic_bytes([], n) == base
    td = {"direction": 1, "frontier": 10, "frontier_edges": 100, "claimed": 40,
          "scanned": 100, "unvisited": 0}
    # top-down: 20 per frontier vertex, 8 per frontier edge, 12 per claim
    assert bench.algorithmic_bytes([td], n) == base + 20 * 10 + 8 * 100 + 12 * 40
    bu = {"direction": 2, "frontier": 40, "frontier_edges": 400, "claimed": 300,
          "scanned": 900, "unvisited": 500}
    # switch to bottom-up: 4 per frontier vertex + n/8; then 16 per unvisited
    # vertex, 4 per scanned entry, three bitmaps, 8 per find
    want_bu = 4 * 40 + n // 8 + 16 * 500 + 4 * 900 + 3 * n // 8 + 8 * 300
    assert bench.algorithmic_bytes([td, bu], n) == base + 20 * 10 + 8 * 100 + 12 * 40 + want_bu
    # a second bottom-up level pays no conversion
    want_bu2 = 16 * 500 + 4 * 900 + 3 * n // 8 + 8 * 300
    assert bench.algorithmic_bytes([td, bu, bu], n) == (base + 20 * 10 + 8 * 100 + 12 * 40 + want_bu
                                                       + want_bu2)
    # back to top-down: the frontier bitmap becomes the queue (20 per
    # frontier vertex + n/8), then the top-down level itself
    td2 = {"direction": 1, "frontier": 30, "frontier_edges": 60, "claimed": 5,
           "scanned": 60, "unvisited": 0}
    want_td2 = 20 * 30 + n // 8 + 20 * 30 + 8 * 60 + 12 * 5
    assert bench.algorithmic_bytes([td, bu, td2], n) == (base + 20 * 10 + 8 * 100 + 12 * 40 + want_bu
                                                        + want_td2)


def test_batch_algorithmic_bytes_model():
    """The multi-source byte model, term by term (64 lanes: W = 1; 100
    lanes: W = 2)."""
    import bench
    n = 1000
    for lanes, W in ((64, 1), (100, 2)):
        base = 24 * W * n + 8 * lanes * n
        assert bench.batch_algorithmic_bytes([], n, lanes) == base
        td = {"direction": 1, "frontier": 10, "frontier_edges": 100, "claimed": 40,
              "scanned": 100, "unvisited": 0}
        want_td = 24 * W * n + 8 * W * 10 + 16 * 10 + 100 * (4 + 8 * W)
        assert bench.batch_algorithmic_bytes([td], n, lanes) == base + want_td
        bu = {"direction": 2, "frontier": 40, "frontier_edges": 400, "claimed": 300,
              "scanned": 900, "unvisited": 500}
        want_bu = 24 * W * n + 16 * 500 + 16 * W * 500 + 900 * (4 + 8 * W)
        assert bench.batch_algorithmic_bytes([td, bu], n, lanes) == base + want_td + want_bu
