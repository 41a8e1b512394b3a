"""The product path stands on the HIP library alone: it raises when the library
is missing (there is no CPU fallback), and neither the package nor the native
sources reach into the oracle."""
import ast
import os

import pytest

from paper_1209_5942_amd import tmqcd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1209_5942_amd")


def test_missing_library_raises(tmp_path, monkeypatch):
    monkeypatch.setattr(tmqcd, "LIB_PATH", str(tmp_path / "libtmqcd.so"))
    monkeypatch.setattr(tmqcd, "_lib", None)
    with pytest.raises(tmqcd.TmqcdLibraryMissing):
        tmqcd.lib()
    prob = tmqcd.Problem((4, 4, 4, 4), 0.15, 0.01, (1, 1, 1, -1))
    with pytest.raises(tmqcd.TmqcdLibraryMissing):
        tmqcd.gauge_bytes(prob)


def _python_sources():
    for dirpath, _, files in os.walk(PKG):
        if "__pycache__" in dirpath or "_build" in dirpath:
            continue
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(dirpath, f)


def test_package_never_imports_the_oracle():
    for path in _python_sources():
        with open(path) as fh:
            tree = ast.parse(fh.read(), path)
        for node in ast.walk(tree):
            names = []
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            for n in names:
                assert n.split(".")[0] != "oracle", f"{path} imports {n}"


def test_native_sources_include_nothing_from_the_oracle():
    csrc = os.path.join(PKG, "csrc")
    for f in os.listdir(csrc):
        with open(os.path.join(csrc, f)) as fh:
            for line in fh:
                if line.lstrip().startswith("#include"):
                    assert "oracle" not in line, f"{f}: {line.strip()}"


def test_oracle_reads_only_the_input_generator_from_the_package():
    """The oracle shares no arithmetic with the product: the only product module it may
    import is the seeded input generator (no tables, constants or helpers)."""
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if not f.endswith(".py"):
            continue
        path = os.path.join(odir, f)
        with open(path) as fh:
            tree = ast.parse(fh.read(), path)
        for node in ast.walk(tree):
            names = []
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            for n in names:
                if n.split(".")[0] == "paper_1209_5942_amd":
                    assert n == "paper_1209_5942_amd.synth", f"{path} imports {n}"
