"""CPU checks of bench.py: every global name its functions read is defined (a renamed
or dropped constant fails here instead of at the end of a GPU run), and --gpus N > 1
exits with a message before touching a GPU."""
import ast
import builtins
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _module_names(tree):
    names = set(dir(builtins))
    for node in tree.body:
        if isinstance(node, (ast.FunctionDef, ast.ClassDef)):
            names.add(node.name)
        elif isinstance(node, ast.Assign):
            for t in node.targets:
                for n in ast.walk(t):
                    if isinstance(n, ast.Name):
                        names.add(n.id)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            for a in node.names:
                names.add((a.asname or a.name).split(".")[0])
    return names


def _local_names(fn):
    names = {a.arg for a in fn.args.args + fn.args.kwonlyargs}
    if fn.args.vararg:
        names.add(fn.args.vararg.arg)
    if fn.args.kwarg:
        names.add(fn.args.kwarg.arg)
    for n in ast.walk(fn):
        if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
            names.add(n.id)
        elif isinstance(n, (ast.FunctionDef, ast.Lambda)) and n is not fn:
            args = n.args
            names |= {a.arg for a in args.args + args.kwonlyargs}
            if isinstance(n, ast.FunctionDef):
                names.add(n.name)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for a in n.names:
                names.add((a.asname or a.name).split(".")[0])
        elif isinstance(n, ast.comprehension):
            for t in ast.walk(n.target):
                if isinstance(t, ast.Name):
                    names.add(t.id)
        elif isinstance(n, ast.ExceptHandler) and n.name:
            names.add(n.name)
    return names


def test_bench_functions_read_only_defined_names():
    src = open(os.path.join(ROOT, "bench.py")).read()
    tree = ast.parse(src)
    glob = _module_names(tree)
    missing = []
    for fn in [n for n in tree.body if isinstance(n, ast.FunctionDef)]:
        local = _local_names(fn)
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load) and n.id not in local and n.id not in glob:
                missing.append((fn.name, n.id))
    assert not missing, missing


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_cpu_baseline_runs_concurrent_oracle_processes():
    """The CPU baseline leg on the small sphere workload: two concurrent one-thread oracle
    processes, each with its measured step parts; the record states the process count as
    cores, the host's CPU count and model, and what was measured and extrapolated."""
    sys.path.insert(0, ROOT)
    import bench
    samples, wall = bench.cpu_samples("sphere32", 2, n_pcg=4)
    assert len(samples) == 2 and all(r["pcg_iters"] == 4 and r["t_fixed"] > 0 for r in samples)
    case = bench.workload("sphere32")
    rec = bench.cpu_baseline(case, samples, wall, 40.0)
    assert rec["cores"] == 2 and rec["kind"] == "oracle" and rec["host_cpus"] == os.cpu_count()
    assert rec["measured_pcg_iters"] == 4 and rec["extrapolated_pcg_iters"] == 36.0
    assert rec["value"] > rec["single_process_value"] > 0
