"""Host-side checks of the C ABI: the library loads and exports every entry
point declared in include/h2.h (no device work is started)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "h2.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(h2_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["h2_matrix_load", "h2_factor", "h2_solve", "h2_matvec", "h2_solve_ir",
              "h2_factor_batched", "h2_solve_batched"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2509_11152_amd", "libh2rss.so")
    assert os.path.exists(path), "build the library first (python paper_2509_11152_amd/build.py)"
    lib = ctypes.CDLL(path)
    for n in _declared():
        assert hasattr(lib, n), n


def test_status_strings_and_argument_errors():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2509_11152_amd", "libh2rss.so"))
    lib.h2_status_string.restype = ctypes.c_char_p
    assert lib.h2_status_string(0) == b"success"
    assert lib.h2_status_string(2).startswith(b"malformed")
    # null handles are rejected without touching a device
    assert lib.h2_context_destroy(None) == 1
    assert lib.h2_matrix_destroy(None) == 1
    assert lib.h2_factor_destroy(None) == 1
    assert lib.h2_context_create(None, None) == 1
