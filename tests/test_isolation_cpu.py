"""Separation of the oracle and the product path (host checks).

The oracle is test infrastructure: it shares no code with the HIP path and
neither side imports the other; outside tests/ only bench.py's CPU baseline
and __graft_entry__.smoke() use it.  The product path has no CPU fallback:
without the built library the binding refuses to load."""
import ast
import os
import re
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2507_12349_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _files(top, exts):
    for d, dirs, names in os.walk(top):
        dirs[:] = [x for x in dirs if x not in ("__pycache__", "_build")]
        for f in names:
            if f.endswith(exts):
                yield os.path.join(d, f)


def _imports(path):
    tree = ast.parse(open(path).read(), path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name.split(".")[0]
        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
            yield node.module.split(".")[0]


def test_oracle_does_not_use_the_package():
    files = list(_files(ORACLE, (".py", ".c", ".h")))
    assert files
    for f in files:
        txt = open(f).read()
        if f.endswith(".py"):
            assert "paper_2507_12349_amd" not in set(_imports(f)), f
            assert "libcos.so" not in txt, f   # no loading of the built library either
        else:
            # system headers, and quoted includes only of the oracle's own files
            for q, inc in re.findall(r'#\s*include\s*([<"])([^>"]+)[>"]', txt):
                if q == '"':
                    assert os.path.exists(os.path.join(os.path.dirname(f), inc)), (f, inc)
                else:
                    assert not inc.startswith(("cos_", "libcos")), (f, inc)


def test_package_does_not_use_the_oracle():
    for f in _files(PKG, (".py",)):
        assert "oracle" not in set(_imports(f)), f
    for f in _files(os.path.join(PKG, "csrc"), (".hip", ".cpp", ".hpp", ".h")):
        txt = open(f).read()
        for inc in re.findall(r'#\s*include\s*[<"]([^>"]+)[>"]', txt):
            assert "oracle" not in inc, (f, inc)


def test_only_tests_bench_and_smoke_use_the_oracle():
    users = set()
    for f in _files(ROOT, (".py",)):
        rel = os.path.relpath(f, ROOT)
        if rel.startswith(("oracle" + os.sep, "tests" + os.sep, "_work" + os.sep)):
            continue
        if "oracle" in set(_imports(f)):
            users.add(rel)
    assert users <= {"bench.py", "__graft_entry__.py"}, users
    # inside __graft_entry__ only smoke() calls the oracle (build() compiles it)
    tree = ast.parse(open(os.path.join(ROOT, "__graft_entry__.py")).read())
    for fn in tree.body:
        if isinstance(fn, ast.FunctionDef) and fn.name not in ("smoke", "build"):
            assert "oracle" not in ast.unparse(fn), fn.name


def test_binding_refuses_to_load_without_the_library():
    """The binding's module code run with the library path pointing at a file
    that does not exist raises ImportError (no fallback)."""
    src = open(os.path.join(PKG, "_binding.py")).read()
    src = src.replace('LIB_PATH = os.path.join(_HERE, "libcos.so")',
                      'LIB_PATH = os.path.join(_HERE, "no-such-libcos.so")')
    assert "no-such-libcos.so" in src
    mod = types.ModuleType("binding_without_library")
    mod.__file__ = os.path.join(PKG, "_binding.py")
    with pytest.raises(ImportError, match="libcos.so is not built"):
        exec(compile(src, mod.__file__, "exec"), mod.__dict__)
