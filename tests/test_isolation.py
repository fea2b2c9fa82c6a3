"""The oracle and the product path share no code, and the product path never falls back.

- The package (Python binding and HIP sources), the C header and the input generators never
  import, include or load anything of the oracle.
- The oracle never imports the package or includes its headers; its C file includes only
  its own header and the C library.
- The input generators hold no reference to either side.
- The binding raises when the compiled library is missing instead of computing elsewhere.
"""
import ast
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2607_04127_amd")


def _files(top, exts):
    for d, _, names in os.walk(top):
        if "__pycache__" in d:
            continue
        for n in sorted(names):
            if n.endswith(exts):
                yield os.path.join(d, n)


def _py_imports(path):
    tree = ast.parse(open(path, encoding="utf-8").read(), filename=path)
    out = []
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out += [a.name for a in node.names]
        elif isinstance(node, ast.ImportFrom):
            out.append("." * node.level + (node.module or ""))
    return out


def _c_includes(path):
    return re.findall(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', open(path, encoding="utf-8").read(), re.M)


def test_package_never_references_the_oracle():
    for path in _files(PKG, (".py",)):
        for mod in _py_imports(path):
            assert "oracle" not in mod.split("."), (path, mod)
        text = open(path, encoding="utf-8").read()
        assert "liblgsr_ref" not in text and "lgsr_ref" not in text, path
    for path in list(_files(os.path.join(PKG, "csrc"), (".hip", ".h", ".cpp"))) + list(
            _files(os.path.join(ROOT, "include"), (".h",))):
        for inc in _c_includes(path):
            assert "lgsr_ref" not in inc and "oracle" not in inc, (path, inc)


def test_oracle_never_references_the_package():
    for path in _files(os.path.join(ROOT, "oracle"), (".py",)):
        for mod in _py_imports(path):
            top = mod.lstrip(".").split(".")[0]
            assert top not in ("paper_2607_04127_amd", "scenegen", "tests"), (path, mod)
    allowed = {"lgsr_ref.h", "math.h", "stdlib.h", "string.h", "stdint.h", "stddef.h", "stdio.h", "float.h",
               "omp.h"}
    for path in _files(os.path.join(ROOT, "oracle"), (".c", ".h")):
        for inc in _c_includes(path):
            assert inc in allowed, (path, inc)


def test_input_generators_reference_neither_side():
    for path in _files(os.path.join(ROOT, "scenegen"), (".py",)):
        for mod in _py_imports(path):
            top = mod.lstrip(".").split(".")[0]
            assert top not in ("oracle", "paper_2607_04127_amd"), (path, mod)


def test_binding_raises_without_the_library(monkeypatch, tmp_path):
    from paper_2607_04127_amd import lgsr
    monkeypatch.setattr(lgsr, "LIB_PATH", str(tmp_path / "missing" / "liblgsr.so"))
    monkeypatch.setattr(lgsr, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        lgsr.lib()
