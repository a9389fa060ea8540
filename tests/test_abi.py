"""The C-ABI library loads and exports every entry point declared in
include/hy.h, with a binding for each (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import numpy as np

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
    assert n == 1024 + 2 * ((16 ** 3 * 5 * 8 + 255) // 256 * 256)
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


# ------------------------------------------------------------- refined meshes
def _slab_faces(lv, nr, periodic):
    """Leaf faces whose neighbour region is at the other level, counted from
    the leaf list alone (coarse ones separately)."""
    have = {(int(L), int(x), int(y), int(z)) for L, x, y, z in lv}
    nvirt = ncf = 0
    for L, x, y, z in lv:
        for d in range(3):
            for s in (-1, 1):
                l = [int(x), int(y), int(z)]
                l[d] += s
                n = nr[d] << int(L)
                if not 0 <= l[d] < n:
                    if not periodic:
                        continue
                    l[d] %= n
                if (int(L), *l) not in have:
                    nvirt += 1
                    ncf += int(L) == 0
    return nvirt, ncf


@pytest.mark.parametrize("box,periodic", [(((1, 0, 1), (3, 2, 2)), True), (((0, 0, 0), (1, 1, 1)), False),
                                          (((0, 0, 0), (4, 3, 2)), True), (((2, 1, 0), (3, 3, 2)), False),
                                          ((((0, 0, 0), (2, 1, 1)), ((1, 1, 0), (2, 3, 1)),
                                            ((3, 2, 1), (4, 3, 2))), True),
                                          ((((0, 0, 0), (1, 1, 1)), ((1, 1, 1), (2, 2, 2)),
                                            ((2, 0, 0), (3, 1, 1)), ((3, 1, 1), (4, 2, 2))), False)])
def test_refined_leaves_and_workspace_without_gpu(box, periodic):
    import oracle
    from paper_2409_16053_amd import hy
    from paper_2409_16053_amd import problems as P
    pb = P.uniform(n=(32, 24, 16), rho=1.0, v=(0, 0, 0), p=1.0, bc=P.PERIODIC if periodic else P.OUTFLOW)
    pb = pb.with_(block=(8, 8, 8), refine=box, rk=3)
    lv = hy.leaves(pb)
    assert np.array_equal(lv, oracle.smr_leaves(pb))
    nvirt, ncf = _slab_faces(lv, (4, 3, 2), periodic)
    a = lambda b: (b + 255) // 256 * 256
    # the slabs' 2 ghost layers of a 64-cell face are packed 4 to a block
    # (512 cells per variable / 128 per slab)
    reg = a((len(lv) + (nvirt + 3) // 4) * 8 ** 3 * 5 * 8)
    tables = a(len(lv) * 12 * 4) + a(nvirt * 2 * 4 + 4) + a(24 * 2 * 4) + a(ncf * 2 * 4 + 4)
    assert hy.workspace_bytes(pb) == 1024 + 3 * reg + tables
    # FOFC adds one flag byte per leaf cell (none for the ghost slabs) and one
    # per plane of a leaf, and, per coarse face next to finer leaves, room for
    # one block face of states
    assert hy.workspace_bytes(pb.with_(fofc=1)) == (1024 + 3 * reg + a(len(lv) * 8 ** 3) + a(len(lv) * 8)
                                                    + tables + a(ncf * 64 * 5 * 8))


@pytest.mark.parametrize("block,recon,per_block", [((12, 8, 16), 1, 2), ((16, 16, 16), 0, 8),
                                                   ((6, 8, 10), 2, 2), ((12, 12, 12), 3, 4)])
def test_ghost_slabs_packed_per_block_without_gpu(block, recon, per_block):
    # a slab takes ghost depth x the largest block face cells per variable and
    # the slabs are packed into whole blocks after the leaves, the largest
    # power of two of them that fits: (12, 8, 16) with PPM4 holds 1536 cells
    # per variable and a slab 3 x 192 = 576, so 2 per block; (16, 16, 16) with
    # PLM 4096 / (2 x 256) = 8; (6, 8, 10) with WENO-Z 480 / (3 x 80) = 2;
    # (12, 12, 12) with PPMX 1728 / (3 x 144) = 4
    from paper_2409_16053_amd import hy
    from paper_2409_16053_amd import problems as P
    n = tuple(4 * b for b in block)
    pb = P.uniform(n=n, rho=1.0, v=(0, 0, 0), p=1.0, bc=P.PERIODIC).with_(
        block=block, recon=recon, refine=((1, 1, 1), (2, 2, 2)))
    lv = hy.leaves(pb)
    nvirt, ncf = _slab_faces(lv, (4, 4, 4), True)
    a = lambda x: (x + 255) // 256 * 256
    cells = block[0] * block[1] * block[2]
    reg = a((len(lv) + (nvirt + per_block - 1) // per_block) * cells * 5 * 8)
    tables = a(len(lv) * 12 * 4) + a(nvirt * 2 * 4 + 4) + a(64 * 2 * 4) + a(ncf * 2 * 4 + 4)
    assert hy.workspace_bytes(pb) == 1024 + 2 * reg + tables


@pytest.mark.parametrize("bad", [dict(block=(9, 8, 8), n=(36, 24, 16)),
                                 dict(refine=((0, 0, 0), (5, 1, 1))), dict(recon=3, block=(4, 8, 8)),
                                 dict(refine=(((0, 0, 0), (1, 1, 1)), ((1, 0, 0), (1, 1, 1)))),
                                 dict(refine=tuple(((0, 0, 0), (1, 1, 1)) for _ in range(9)))])
def test_refined_configuration_errors_without_gpu(bad):
    # each case is valid without refinement and invalid with it (odd block,
    # box outside the root grid, block below twice the ghost depth, an
    # empty box among several, more than 8 boxes)
    from paper_2409_16053_amd import hy
    from paper_2409_16053_amd import problems as P
    pb = P.uniform(n=(32, 24, 16), rho=1.0, v=(0, 0, 0), p=1.0, bc=P.PERIODIC)
    pb = pb.with_(block=(8, 8, 8), refine=((0, 0, 0), (1, 1, 1)))
    assert hy.workspace_bytes(pb) > 0
    if "refine" not in bad:
        assert hy.workspace_bytes(pb.with_(refine=None, **bad)) > 0
    with pytest.raises(hy.HydroError):
        hy.workspace_bytes(pb.with_(**bad))
