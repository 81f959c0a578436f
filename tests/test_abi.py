"""The C-ABI library loads and exports every function include/vcsgc.h declares
(no GPU needed: symbols are resolved without calling into the device)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vcsgc.h")
LIB = os.path.join(ROOT, "paper_1012_5082_amd", "libvcsgc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("vcsgc_create", "vcsgc_destroy", "vcsgc_sweep", "eam_energy_forces",
                 "md_verlet_step", "vcsgc_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1012_5082_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_no_oracle_in_product_path():
    """The HIP library and the binding never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1012_5082_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "from oracle" not in text and "import oracle" not in text, f
                assert "liboracle" not in text and "or_sweep" not in text, f
