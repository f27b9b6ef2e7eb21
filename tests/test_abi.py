"""The C-ABI library loads on the CPU and exports every symbol the public
header declares; the product path does not depend on the oracle."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(srm_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared_symbols()
    for required in ("srm_init", "srm_sweep", "srm_run_to_fraction", "srm_pairs", "srm_rdf"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2605_18254_amd as srm
    lib = ctypes.CDLL(srm.LIB_PATH)
    missing = [n for n in _declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows every exported entry point too
    assert set(_declared_symbols()) <= set(srm.SYMBOLS)


def test_library_does_not_link_the_oracle():
    import paper_2605_18254_amd as srm
    out = subprocess.run(["ldd", srm.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out
    nm = subprocess.run(["nm", "-D", "--defined-only", srm.LIB_PATH], capture_output=True,
                        text=True).stdout
    assert " o_" not in nm


def test_package_sources_never_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2605_18254_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", text, re.M), f
                assert "srm_oracle" not in text, f


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_2605_18254_amd as srm
    monkeypatch.setattr(srm, "_lib", None)
    monkeypatch.setattr(srm, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        srm.lib()
