"""bench.py on the host: every function it calls is defined, the slot model
matches its documented counts, and more than one GPU is refused with a message
(no GPU call in any of these)."""
import ast
import builtins
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_called_functions_exist():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    defined = {n.name for n in ast.walk(tree) if isinstance(n, ast.FunctionDef)}
    imported = set()
    for n in ast.walk(tree):
        if isinstance(n, ast.Import):
            imported |= {a.asname or a.name.split(".")[0] for a in n.names}
        elif isinstance(n, ast.ImportFrom):
            imported |= {a.asname or a.name for a in n.names}
    assigned = {t.id for n in ast.walk(tree) if isinstance(n, ast.Assign)
                for t in n.targets if isinstance(t, ast.Name)}
    params = {a.arg for n in ast.walk(tree) if isinstance(n, ast.FunctionDef)
              for a in n.args.args + n.args.kwonlyargs}
    known = defined | imported | assigned | params | set(dir(builtins))
    called = {n.func.id for n in ast.walk(tree)
              if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    assert not called - known, sorted(called - known)


def test_slot_model():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.valu_slots_per_eval(10, 2, "fp64") == 373
    assert bench.valu_slots_per_eval(10, 2, "fp32") == 282
    assert bench.valu_slots_per_eval(16, 4, "fp32") == 815


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
