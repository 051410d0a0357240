"""The C-ABI library loads and exports every entry point the header declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ia355.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ia355_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2212_10550_amd", "libia355.so")
    assert os.path.exists(path), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(path)
    names = _declared()
    assert len(names) >= 17
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    lib.ia355_version.restype = ctypes.c_int32
    assert lib.ia355_version() >= 100
    lib.ia355_error_string.restype = ctypes.c_char_p
    assert lib.ia355_error_string(1)


def test_binding_names_match_header():
    from paper_2212_10550_amd import lib as K
    assert sorted("ia355_" + n for n in K._SIGS) == _declared()


def test_workspace_sizes_without_gpu():
    from paper_2212_10550_amd import lib as K
    assert K.march_workspace_size(291600, 128) >= 8 * (291600 // 4) + 16 * 291600 + 4 * 291600
    assert K.march_workspace_size(0, 0) > 0 and K.march_workspace_size(-1, 128) == 0
    assert K.deform_workspace_size(64, 64, 32) == 12 * 4 * 64 * 64 * 32
    assert K.mlp_bwd_workspace_size(1 << 20) >= 6532 * 4
