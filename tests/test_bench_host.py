"""bench.py's host-side contract, without a GPU: one GPU only, the metric's
name for a system size, and the traffic figure taken from the committed
rocprofv3 summary only when it matches the tile being measured."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_metric_names_the_system_size():
    assert bench.metric_at(10425).startswith("pair interactions/s + steps/s at N=10,425:")
    assert "N=131,072" in bench.metric_at(131072)


def test_traffic_only_for_the_profiled_tile():
    tile = {"targets_per_lane": 4, "waves": 4, "chunks": 1, "variant": 5}
    t = bench.read_traffic("force_fp64_n10425", tile)
    assert t is not None and t > 32 * 10425        # at least the source reads
    assert bench.read_traffic("force_fp64_n10425", dict(tile, variant=1)) is None
    assert bench.read_traffic("no_such_profile", tile) is None


def test_roofline_counts_twenty_flops_per_ordered_pair():
    """frac = 20 N (N - 1) per launch / launch time / 78.6 TFLOP/s, for the
    each-pair-once kernel too (its own 27-flop arithmetic beside it); the
    counter fractions and the clock / issue / mix decomposition come from
    the committed summaries taken with the same tile, and multiply back to
    the fraction."""
    tile = {"targets_per_lane": 4, "waves": 4, "chunks": 1, "variant": 5}
    n, ms = 10425, 0.0485
    r = bench.roofline(n, tile, ms, 0.038)
    want = 20 * n * (n - 1) / (ms * 1e-3) / 1e12
    assert abs(r["achieved"] - round(want, 3)) < 1e-9 and abs(r["frac"] - round(want / 78.6, 4)) < 1e-9
    assert r["own_arithmetic"]["flops_per_launch"] == 27 * n * (n - 1) // 2
    assert 0.3 < r["counter_frac_fp64"] < 0.6 and r["counter_frac_fp32"] == 0.0
    prod = r["clock_frac"] * r["issue_efficiency"] * r["mix_efficiency"]
    assert abs(prod - r["frac"]) < 2e-3
    # another tile: no counter figures
    r1 = bench.roofline(n, dict(tile, variant=1), ms, 0.038)
    assert "counter_frac_fp64" not in r1 and r1["traffic"] is None


def test_oracle_is_used_by_the_cpu_baseline_leg_only():
    """The oracle is test infrastructure: in bench.py it is imported only by
    the CPU-baseline leg's functions (all skipped by --no-cpu-baseline), and
    the package never imports it."""
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = set()
    for fn in ast.walk(tree):
        if isinstance(fn, ast.FunctionDef):
            for node in ast.walk(fn):
                if isinstance(node, ast.Import) and any(a.name == "oracle" for a in node.names):
                    users.add(fn.name)
                if isinstance(node, ast.ImportFrom) and node.module == "oracle":
                    users.add(fn.name)
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))
           and ("oracle" in [a.name for a in n.names] or getattr(n, "module", None) == "oracle")]
    assert not top
    assert users == {"cpu_baseline", "oracle_accel_errors", "oracle_scan_rates"}
    calls = {n.func.id for n in ast.walk(tree) if isinstance(n, ast.Call)
             and isinstance(n.func, ast.Name) and n.func.id in users}
    assert calls == users
    src = open(os.path.join(ROOT, "bench.py")).read()
    for name in users:   # every call sits behind the --no-cpu-baseline switch
        for line in [l for l in src.splitlines() if f"{name}(" in l and "def " not in l]:
            idx = src.index(line)
            assert "if not args.no_cpu_baseline" in src[max(0, idx - 400):idx], name
    pkg = os.path.join(ROOT, "paper_2112_15079_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            assert "import oracle" not in open(os.path.join(pkg, f)).read(), f
