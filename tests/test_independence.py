"""The oracle and the HIP path share no code: neither imports, includes or
links the other; only the seeded input module serves both, and the product
package never loads the oracle."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
IMPORT = re.compile(r"^\s*(?:from\s+(\S+)\s+import\s+(.+)|import\s+(\S+))", re.M)
INCLUDE = re.compile(r'^\s*#\s*include\s+[<"]([^>"]+)[>"]', re.M)


def _files(sub, exts):
    out = []
    for d, _, fs in os.walk(os.path.join(ROOT, sub)):
        for f in fs:
            if f.endswith(exts):
                out.append(os.path.join(d, f))
    return out


def _imports(src):
    mods = []
    for a, b, c in IMPORT.findall(src):
        if a:
            mods += [a] + [a + "." + x.strip() for x in b.split(",")]
        else:
            mods.append(c)
    return mods


def test_product_never_touches_the_oracle():
    for f in _files("paper_1311_0182_amd", (".py",)):
        for m in _imports(open(f).read()):
            assert not m.startswith("oracle"), (f, m)
        assert "liboracle" not in open(f).read(), f
    for f in _files("paper_1311_0182_amd", (".hip", ".hpp", ".h", ".cpp")):
        for inc in INCLUDE.findall(open(f).read()):
            assert "oracle" not in inc, (f, inc)


def test_oracle_never_touches_the_product():
    for f in _files("oracle", (".py",)):
        for m in _imports(open(f).read()):
            assert not m.startswith("paper_1311_0182_amd"), (f, m)
        assert "libtraphic_rt" not in open(f).read(), f
    for f in _files("oracle", (".c", ".h")):
        for inc in INCLUDE.findall(open(f).read()):
            assert "traphic_rt" not in inc and "csrc" not in inc, (f, inc)


def test_input_module_holds_no_method_arithmetic():
    src = open(os.path.join(ROOT, "paper_1311_0182_amd", "inputs.py")).read()
    for word in ("expm1", "philox", "in_cone", "merge", "knn"):
        assert word not in src.lower(), word
    assert not [m for m in _imports(src) if m not in ("__future__", "__future__.annotations", "math", "numpy")]
