"""The C-ABI library loads and exports every function include/soar.h declares (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "soar.h")
LIB = os.path.join(ROOT, "paper_2404_00774_amd", "libsoar.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:soar_status|void|size_t|const char\*)\s+(soar_\w+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("soar_assign", "soar_train_codebook", "soar_insert"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libsoar.so not built"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"


def test_status_strings():
    lib = ctypes.CDLL(LIB)
    lib.soar_status_string.restype = ctypes.c_char_p
    lib.soar_status_string.argtypes = [ctypes.c_int]
    for code in range(0, -8, -1):
        assert lib.soar_status_string(code).decode() not in ("", "unknown status")
