"""The oracle and the HIP path share no code: neither imports the other,
and only the seeded input generators (scenegen) serve both."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    tree = ast.parse(open(path).read())
    mods = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            mods.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
            mods.add(node.module.split(".")[0])
    return mods


def _py_files(d):
    for base, _, files in os.walk(os.path.join(ROOT, d)):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(base, f)


def test_oracle_imports_no_product_code():
    for f in _py_files("oracle"):
        assert "paper_2404_09531_amd" not in _imports(f), f


def test_product_imports_neither_oracle_nor_generators():
    for f in _py_files("paper_2404_09531_amd"):
        m = _imports(f)
        assert "oracle" not in m and "scenegen" not in m, f


def test_generators_hold_no_renderer_code():
    for f in _py_files("scenegen"):
        m = _imports(f)
        assert "oracle" not in m and "paper_2404_09531_amd" not in m, f


def test_product_sources_do_not_reference_oracle():
    csrc = os.path.join(ROOT, "paper_2404_09531_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower(), f
