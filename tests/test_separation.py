"""The HIP path and the oracle share no code: no file of the library or of the
input generators imports the oracle, the oracle imports neither of them, and
bench.py reaches the oracle only inside its CPU-baseline leg (the pool and its
worker processes)."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    tree = ast.parse(open(path).read(), path)
    out = []
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out += [a.name.split(".")[0] for a in node.names]
        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
            out.append(node.module.split(".")[0])
    return out


def _py_files(folder):
    for dirpath, _, files in os.walk(os.path.join(ROOT, folder)):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(dirpath, f)


def test_library_and_generators_do_not_import_the_oracle():
    for folder in ("paper_1411_2141_amd", "synth"):
        for path in _py_files(folder):
            assert "oracle" not in _imports(path), path


def test_oracle_imports_neither_the_library_nor_the_generators():
    for path in _py_files("oracle"):
        imps = _imports(path)
        assert "paper_1411_2141_amd" not in imps and "synth" not in imps, path


def test_native_sources_do_not_reference_the_oracle():
    csrc = os.path.join(ROOT, "paper_1411_2141_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f), errors="replace").read()
        assert "oracle" not in text.lower(), f


def test_bench_uses_the_oracle_only_in_its_cpu_baseline():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    for fn in [n for n in tree.body if isinstance(n, ast.FunctionDef)]:
        uses = any(isinstance(n, ast.ImportFrom) and n.module and n.module.startswith("oracle")
                   for n in ast.walk(fn))
        assert not uses or fn.name in ("cpu_baseline", "cpu_baseline_worker"), fn.name
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    assert all("oracle" not in ast.dump(n) for n in top)
