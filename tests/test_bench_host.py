"""bench.py on the host: it imports without a GPU, its flags parse, and every
mode its main() dispatches to is defined (a mode whose function went missing
would only fail on the GPU)."""
import ast
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_every_called_module_function_is_defined():
    src = open(os.path.join(ROOT, "bench.py")).read()
    tree = ast.parse(src)
    defined = {n.name for n in tree.body if isinstance(n, (ast.FunctionDef, ast.ClassDef))}
    defined |= {t.id for n in tree.body if isinstance(n, ast.Assign) for t in n.targets if isinstance(t, ast.Name)}
    called = {n.func.id for n in ast.walk(tree) if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    import builtins as _b
    builtins = set(dir(_b))
    local = set()
    for n in ast.walk(tree):  # names bound inside functions (nested defs, lambdas, imports)
        if isinstance(n, (ast.FunctionDef, ast.Lambda)):
            for a in ast.walk(n.args):
                if isinstance(a, ast.arg):
                    local.add(a.arg)
        if isinstance(n, ast.FunctionDef):
            local.add(n.name)
        if isinstance(n, (ast.Import, ast.ImportFrom)):
            local |= {(al.asname or al.name).split(".")[0] for al in n.names}
        if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Store):
            local.add(n.id)
    missing = sorted(c for c in called if c not in defined | builtins | local)
    assert not missing, missing


def test_modes_exist_and_flags_parse():
    b = _bench()
    for name in ("bench_sweep", "bench_batch", "extra_fasta", "extra_batch", "cpu_baseline", "stream_read_probe",
                 "counters_from_profiles", "scan_source_hash"):
        assert callable(getattr(b, name)), name
    src = open(os.path.join(ROOT, "bench.py")).read()
    for flag in ("--sweep", "--serve", "--config", "--steps", "--warmup", "--gpus", "--no-extras"):
        assert flag in src, flag


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "RANK": "0", "WORLD_SIZE": "1"})
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)


def test_counters_are_used_only_for_the_profiled_sources():
    """The committed counter runs carry the hash of the scan sources they were
    taken on: the bench takes traffic and VALU figures from them only for
    that hash (any other gives nothing, and the line reports null)."""
    import json
    b = _bench()
    for name in ("scan_genome", "scan_batch"):
        taken_on = json.load(open(os.path.join(ROOT, "profiles", "%s_counters.json" % name)))["scan_src_sha256"]
        d = b.counters_from_profiles(name, taken_on)
        assert d is not None and d["hbm_bytes_per_launch"] > 0 and d["valu_insts_per_launch"] > 0
        assert b.counters_from_profiles(name, "0" * 64) is None
    assert b.traffic_from_profiles("0" * 64) is None
    if b.counters_from_profiles("scan_genome", b.scan_source_hash()) is None:
        print("note: the scan sources changed since profiles/ was taken; the bench reports traffic as null")
