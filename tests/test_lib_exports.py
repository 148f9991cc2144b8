"""The C-ABI library loads and exports every symbol the headers in include/ declare (CPU only)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:mf_status|void|int|int64_t|const char\*)\s+(mf_\w+)\s*\(", text, re.M))
    return sorted(names)


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("mf_integrand", "mf_vegas_refine", "mf_integrate", "mf_grad"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2105_10529_amd as mf

    if not os.path.exists(mf.LIB_PATH):
        pytest.skip("libmf.so not built")
    L = mf.lib()
    for n in _declared():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", mf.LIB_PATH], capture_output=True, text=True).stdout
    for n in _declared():
        assert re.search(rf"\bT {n}\b", out), n
    assert set(_declared()) == set(mf.EXPORTS)


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2105_10529_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".h", ".hip", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
