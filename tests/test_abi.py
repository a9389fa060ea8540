"""The C-ABI library loads and exports every entry point declared in
include/hy.h, with a binding for each (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hy.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hy_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("hy_workspace_bytes", "hy_create", "hy_set_state", "hy_get_state", "hy_advance",
              "hy_batch_advance", "hy_query", "hy_destroy", "hy_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2409_16053_amd import hy
    if not os.path.exists(hy.LIB_PATH):
        pytest.fail("libhy.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(hy.LIB_PATH)
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(declared_functions()) == set(hy.SIGNATURES)


def test_workspace_bytes_and_validation_without_gpu():
    from paper_2409_16053_amd import hy
    from paper_2409_16053_amd import problems as P
    pb = P.turbulence(N=16, seed=1, kmax=4).with_(block=(8, 8, 8))
    n = hy.workspace_bytes(pb)
    assert n == 512 + 2 * ((16 ** 3 * 5 * 8 + 255) // 256 * 256)
    with pytest.raises(hy.HydroError):
        hy.workspace_bytes(pb.with_(block=(5, 8, 8)))
    with pytest.raises(hy.HydroError):
        hy.workspace_bytes(pb.with_(block=(8, 8, 8), recon=P.PPM4, n=(16, 16, 16)).with_(block=(2, 8, 8)))
    assert "ghost" in hy.last_error() or "divide" in hy.last_error()


def test_struct_layout_matches_header(tmp_path):
    # the ctypes mirror must match the C compiler's layout of hy_config
    import subprocess
    from paper_2409_16053_amd import hy
    fields = [f[0] for f in hy.HyConfig._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hy.h"\nint main(void){\n'
                   + 'printf("%zu\\n", sizeof(hy_config));\n'
                   + "".join(f'printf("%zu\\n", offsetof(hy_config, {f}));\n' for f in fields)
                   + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(hy.HyConfig)
    for f, off in zip(fields, vals[1:]):
        assert getattr(hy.HyConfig, f).offset == off, f
