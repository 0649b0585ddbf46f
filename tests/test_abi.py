"""The C ABI library loads and exports every function include/gj.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "gj.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gj_[a-z_]+)\s*\(", txt)))


def test_exports_match_header():
    import paper_1802_03760_amd as gj
    lib = ctypes.CDLL(gj.LIB_PATH)
    names = declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(gj.EXPORTS) == names


def test_struct_layout():
    import paper_1802_03760_amd as gj
    # uint64 matches + 2 x 9 uint64 + 4 uint64 + 2 double
    assert ctypes.sizeof(gj.Stats) == 8 * (1 + 18 + 4 + 2)
    assert ctypes.sizeof(gj.Atom) == 2


def test_no_oracle_in_product():
    """The library and its binding never reach the oracle."""
    pkg = os.path.join(ROOT, "paper_1802_03760_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                t = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in t.replace("Oracle", ""), f
