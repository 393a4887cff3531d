"""The benchmark's command line (host only): more than one GPU is refused with
a message before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workload_choices_are_listed():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for w in ("dvs", "precision", "batch", "diff", "quality", "threshold", "bandwidth", "multicrossing"):
        assert w in r.stdout


def test_kappa_histogram_bins():
    """Decade bins of the per-frame condition record: [1, 10) is bin 0, values
    below 1 count there too, 1e12 and above share the last bin, non-finite
    values are counted apart."""
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench
    k = np.array([0.5, 1.0, 9.99, 10.0, 3e5, 1e12, 1e30, np.inf, np.nan])
    h, nonfinite = bench.kappa_histogram(k)
    assert h.size == bench.KAPPA_DECADES
    assert h[0] == 3 and h[1] == 1 and h[5] == 1 and h[-1] == 2
    assert h.sum() == 7 and nonfinite == 2


def test_cpu_model_is_named():
    sys.path.insert(0, ROOT)
    import bench
    m = bench.cpu_model()
    assert isinstance(m, str) and m


def test_edge_split_classes_partition_the_events():
    """Every event falls in exactly one of the three places, and the shares
    are those of the distances passed in."""
    sys.path.insert(0, ROOT)
    import torch

    import bench
    from paper_2303_02608_amd import synth
    spec = synth.config_spec(0)["spec"]
    g = torch.Generator().manual_seed(3)
    n = 5000
    ev = {"t": torch.randint(0, spec.T, (n,), generator=g, dtype=torch.int32),
          "x": torch.randint(0, spec.W, (n,), generator=g, dtype=torch.int32),
          "y": torch.randint(0, spec.H, (n,), generator=g, dtype=torch.int32)}
    d = torch.rand(n, generator=g, dtype=torch.float64) * 0.01
    out = bench.edge_split(spec, ev, d, 5, [5e-3, 2e-2])
    assert sum(v["events"] for v in out.values()) == n
    assert all(v["events"] > 0 for v in out.values())
    for v in out.values():
        assert v["share"][1] == 1.0 and 0.0 < v["share"][0] < 1.0
