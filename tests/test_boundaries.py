"""Static checks of the separation between the product path, the oracle and
the shared input generators:

  - nothing in the package (Python or HIP/C++ sources) refers to the oracle;
  - the oracle refers to nothing of the package and includes no HIP header;
  - the input generators (workloads/) import neither of the two;
  - outside tests/, only bench.py's CPU-baseline functions and
    __graft_entry__'s build() / smoke() import the oracle.
"""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2111_05960_amd")


def _files(d, exts):
    for dirpath, dirnames, files in os.walk(d):
        dirnames[:] = [x for x in dirnames if x != "__pycache__"]
        for f in files:
            if f.endswith(exts):
                yield os.path.join(dirpath, f)


def _imports(path):
    """(top-level module, enclosing function or None) of every import."""
    tree = ast.parse(open(path).read())
    out = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else func
            if isinstance(child, ast.Import):
                out.extend((a.name.split(".")[0], f) for a in child.names)
            elif isinstance(child, ast.ImportFrom) and child.module and child.level == 0:
                out.append((child.module.split(".")[0], f))
            visit(child, f)

    visit(tree, None)
    return out


def test_package_never_refers_to_the_oracle():
    for path in _files(PKG, (".py",)):
        mods = [m for m, _ in _imports(path)]
        assert "oracle" not in mods, path
    for path in _files(os.path.join(PKG, "csrc"), (".h", ".hip", ".cpp")):
        text = open(path).read()
        assert not re.search(r'#include\s*["<][^">]*oracle', text), path
        assert "orc_" not in text, path


def test_oracle_refers_to_nothing_of_the_package():
    for path in _files(os.path.join(ROOT, "oracle"), (".py",)):
        mods = [m for m, _ in _imports(path)]
        assert "paper_2111_05960_amd" not in mods, path
        assert "workloads" not in mods, path
    for path in _files(os.path.join(ROOT, "oracle"), (".c", ".h")):
        text = open(path).read()
        assert "hip" not in " ".join(re.findall(r"#include\s*[\"<]([^\">]*)", text)).lower(), path
        assert "gplbm" not in text, path


def test_input_generators_import_neither_side():
    for path in _files(os.path.join(ROOT, "workloads"), (".py",)):
        mods = [m for m, _ in _imports(path)]
        assert "oracle" not in mods and "paper_2111_05960_amd" not in mods, path


def test_oracle_imported_only_by_the_allowed_entry_points():
    allowed = {"bench.py": {"cpu_baseline", "cpu_single_thread"},
               "__graft_entry__.py": {"build", "smoke"}}
    for name, funcs in allowed.items():
        for mod, func in _imports(os.path.join(ROOT, name)):
            if mod == "oracle":
                assert func in funcs, (name, func)
    # a committed script that runs a string of code importing the oracle is
    # counted through the string: the CPU single-thread timing in bench.py
    src = open(os.path.join(ROOT, "bench.py")).read()
    for m in re.finditer(r"import oracle", src):
        line = src.count("\n", 0, m.start()) + 1
        owner = None
        for node in ast.walk(ast.parse(src)):
            if isinstance(node, ast.FunctionDef) and node.lineno <= line <= node.end_lineno:
                owner = node.name
        assert owner in allowed["bench.py"], (line, owner)
