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
    # masks (16 B per ray at 128 steps), entry distances (4 B per ray) and one
    # 8-byte total per workgroup (16 rays per workgroup from 65536 rays, 4 below)
    assert K.march_workspace_size(291600, 128) >= 8 * (291600 // 16) + 16 * 291600 + 4 * 291600
    assert K.march_workspace_size(8192, 128) >= 8 * (8192 // 4) + 16 * 8192 + 4 * 8192
    assert K.march_workspace_size(0, 0) > 0 and K.march_workspace_size(-1, 128) == 0
    assert K.deform_workspace_size(64, 64, 32) == 12 * 4 * 64 * 64 * 32
    assert K.mlp_bwd_workspace_size(1 << 20) >= 6532 * 4


def test_status_codes_and_mlp_widths_without_gpu():
    """Every status code has its own text; the MLP entry points reject a
    decoder shape other than 32-64-64-4 (IA355_ERR_UNSUPPORTED) or a missing
    widths array (IA355_ERR_INVALID_ARG) before any device work."""
    path = os.path.join(ROOT, "paper_2212_10550_amd", "libia355.so")
    lib = ctypes.CDLL(path)
    lib.ia355_error_string.restype = ctypes.c_char_p
    texts = {lib.ia355_error_string(c) for c in range(7)}
    assert len(texts) == 7 and lib.ia355_error_string(99) == b"unknown status"
    hdr = open(os.path.join(ROOT, "include", "ia355.h")).read()
    codes = dict(re.findall(r"#define (IA355_(?:OK|ERR_[A-Z_]+)) (\d+)", hdr))
    assert codes["IA355_ERR_CAPACITY"] == "6" and codes["IA355_ERR_UNSUPPORTED"] == "3"
    assert codes["IA355_ERR_INVALID_ARG"] == "1"
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks return first
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    f = lib.ia355_mlp_fwd
    f.restype = i32
    f.argtypes = [ctypes.c_void_p, i32, ctypes.c_void_p, i64, ctypes.c_void_p, i64, ctypes.c_void_p, ctypes.c_void_p,
                  i32, i32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    ok = (i32 * 4)(32, 64, 64, 4)
    other = (i32 * 4)(32, 128, 64, 4)
    assert f(fake, 0, None, 16, None, 16, fake, other, 3, 0, fake, fake, None) == 3
    assert f(fake, 0, None, 16, None, 16, fake, ok, 2, 0, fake, fake, None) == 3
    assert f(fake, 0, None, 16, None, 16, fake, None, 3, 0, fake, fake, None) == 1
    assert f(fake, 0, None, -1, None, 16, fake, ok, 3, 0, fake, fake, None) == 1
    b = lib.ia355_mlp_bwd
    b.restype = i32
    vp = ctypes.c_void_p
    b.argtypes = [vp, vp, vp, i32, vp, i64, vp, i64, vp, vp, i32, i32, vp, vp, ctypes.c_uint32, vp, ctypes.c_size_t,
                  vp]
    assert b(fake, fake, fake, 0, None, 16, None, 16, fake, other, 3, 0, fake, None, 0, fake, 1 << 30, None) == 3


def test_batch_structs_match_the_header(tmp_path):
    """The ctypes mirrors of ia355_batch_pose / ia355_batch_model have the C
    layout (every field offset and the size), checked against a host program
    compiled from the header."""
    import subprocess
    from paper_2212_10550_amd import lib as K
    src = tmp_path / "layout.c"
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ia355.h"', "int main(void) {"]
    for cname, cls in (("ia355_batch_pose", K.BatchPose), ("ia355_batch_model", K.BatchModel)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l.strip())}
    for cname, cls in (("ia355_batch_pose", K.BatchPose), ("ia355_batch_model", K.BatchModel)):
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_batch_arguments_without_gpu():
    """Workspace and LDS sizes of the batched render, and the plan's argument
    checks, which return before any device work."""
    from paper_2212_10550_amd import lib as K
    L = K.lib()
    assert K.batch_workspace_size(16, 64, 64, 32, 24) >= 16 * 12 * 4 * 64 * 64 * 32
    assert K.batch_workspace_size(0, 64, 64, 32, 24) == 0
    assert K.batch_workspace_size(K.BATCH_MAX_POSES + 1, 64, 64, 32, 24) == 0
    assert K.batch_workspace_size(1, 64, 64, 32, 33) == 0
    assert 0 < K.batch_lds_bytes(32, 256) < K.batch_lds_bytes(64, 256) < K.batch_lds_bytes(64, 512)
    assert K.batch_lds_bytes(32, 256, 4) < K.batch_lds_bytes(32, 256, 8)
    assert K.batch_lds_bytes(0, 256) == 0 and K.batch_lds_bytes(65, 256) == 0 and K.batch_lds_bytes(16, 255) == 0
    assert K.batch_lds_bytes(16, 256, 2) == 0
    pose = K.BatchPose()
    model = K.BatchModel()
    assert L.ia355_batch_plan(ctypes.byref(pose), 0, ctypes.byref(model), None, 0, None) == 1
    assert L.ia355_batch_plan(ctypes.byref(pose), 1, ctypes.byref(model), None, 0, None) == 1  # nb = 0
    assert L.ia355_batch_render(None, 0, 32, 256, 4, 2, None) == 2
