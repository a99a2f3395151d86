"""The C-ABI library loads and exports every entry point include/glint.h declares
(host-only checks: no kernel is launched here)."""
import ctypes as C
import os
import re

import pytest

from paper_2507_02674_amd import glint as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "glint.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(glint_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for required in ("glint_partition_env", "glint_prefilter", "glint_build_luts", "glint_shade",
                     "glint_create", "glint_destroy", "glint_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(G.library_path())
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(G.EXPORTS)


def test_host_side_queries():
    assert G.glint_version() == 1
    assert G.glint_pyramid_texels(256, 8) == sum(6 * (256 >> m) ** 2 for m in range(8)) == 524280
    assert G.glint_pyramid_texels(32, 6) == 8190
    assert G.glint_pyramid_texels(3, 1) == 0  # not a power of two
    assert G.glint_pyramid_texels(32, 7) == 0  # too many mips
    fp = G.PrefilterParams(8, 64, G.GLINT_F32)
    # chain levels 1..7 with a one-texel border per face, K+3 = 11 channels padded to 12 floats
    assert G.glint_prefilter_workspace_bytes(256, 8, fp) == sum(6 * ((256 >> s) + 2) ** 2 for s in range(1, 8)) * 12 * 4
    assert G.glint_partition_workspace_bytes(256) > 0
    assert G.glint_partition_workspace_bytes(100) == 0


def test_struct_layouts_match_header():
    # field order and sizes as declared in include/glint.h (LP64)
    assert C.sizeof(G.PartitionParams) == 24
    assert G.PartitionParams.ell.offset == 8
    assert C.sizeof(G.GBuffer) == 24 * 8
    assert C.sizeof(G.Env) == 5 * 8 + 4 * 4 + 8
    assert C.sizeof(G.ShadeParams) == 32
    assert C.sizeof(G.ShadeDebug) == 24


def test_struct_layouts_match_a_c_compiler(tmp_path):
    """sizeof/offsetof of every struct the binding mirrors, as a C compiler
    lays it out from include/glint.h, against the ctypes structures."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"glint_partition_params": G.PartitionParams, "glint_prefilter_params": G.PrefilterParams,
               "glint_gbuffer": G.GBuffer, "glint_env": G.Env, "glint_shade_params": G.ShadeParams,
               "glint_shade_debug": G.ShadeDebug, "glint_env_task": G.EnvTask, "glint_view": G.View}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "glint.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_calls_validate_before_touching_the_device():
    lib = G.lib()
    # a null context is rejected with EINVAL, not a crash
    rc = lib.glint_partition_env(None, None, 32, None, None, None, None, None, None)
    assert rc == G.GLINT_EINVAL
    assert "context" in lib.glint_last_error(None).decode()
    rc = lib.glint_shade(None, None, 10, None, None, None, None, None)
    assert rc == G.GLINT_EINVAL
    rc = lib.glint_sample_binomial(None, 0, 0, None, None, None, None, 10, None, None, None, None, None)
    assert rc == G.GLINT_EINVAL
