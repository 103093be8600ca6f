"""The oracle and the HIP path share no code: neither imports, includes or
links the other; only the seeded input module serves both, and the product
package never loads the oracle."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _files(sub, exts):
    out = []
    for d, _, fs in os.walk(os.path.join(ROOT, sub)):
        for f in fs:
            if f.endswith(exts):
                out.append(os.path.join(d, f))
    return out


def test_product_never_touches_the_oracle():
    for f in _files("paper_1311_0182_amd", (".py", ".hip", ".hpp", ".h", ".cpp")):
        src = open(f).read()
        assert not re.search(r"\boracle\b", re.sub(r"#.*|//.*", "", src)), f
        assert "traphic_oracle" not in src, f


def test_oracle_never_touches_the_product():
    for f in _files("oracle", (".py", ".c", ".h")):
        src = open(f).read()
        assert "traphic_rt" not in src, f
        assert "paper_1311_0182_amd" not in src, f
        assert "csrc" not in src, f


def test_input_module_holds_no_method_arithmetic():
    src = open(os.path.join(ROOT, "paper_1311_0182_amd", "inputs.py")).read()
    for word in ("expm1", "exp(-", "in_cone", "alpha_A", "philox", "rotation", "argmax"):
        assert word not in src, word
