"""The C-ABI library loads and exports every entry point include/zf.h declares
(CPU only: no compute calls, no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zf.h")
LIB = os.path.join(ROOT, "paper_2404_19163_amd", "libzf.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zf_\w+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("zf_refine", "zf_refine_ex", "zf_residual", "zf_release", "zf_last_error"):
        assert must in names


@pytest.fixture(scope="module")
def libzf():
    if not os.path.exists(LIB):
        pytest.fail("libzf.so is not built (run python paper_2404_19163_amd/csrc/build.py)")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(libzf):
    missing = [n for n in _declared() if not hasattr(libzf, n)]
    assert not missing, missing


def test_exports_are_c_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    for n in _declared():
        assert n in exported, n


def test_binding_names_match_header():
    from paper_2404_19163_amd import zf
    assert set(zf.EXPORTS) <= set(_declared())
    assert set(_declared()) <= set(zf.EXPORTS)


def test_version_and_default_opts(libzf):
    # pure host functions: no device work
    from paper_2404_19163_amd import zf
    L = zf.lib()
    assert L.zf_version() >= 1
    o = zf.Opts()
    L.zf_default_opts(ctypes.byref(o))
    assert (o.order, o.precision, o.stop, o.max_sweeps, o.refine, o.max_refine) == (2, 1, 0, 100, 1, 10)
    assert o.z0 == zf.Z0_SCALED_IDENTITY  # opts.z0 takes the values of enum zf_z0_kind
    assert L.zf_last_error() == b""


def test_header_is_plain_c_and_links(tmp_path):
    """A C99 translation unit includes zf.h, takes the address of every declared entry
    point, links against libzf.so, and calls the two pure-host functions."""
    names = _declared()
    src = tmp_path / "abi.c"
    refs = ",\n  ".join(f"(void (*)(void)){n}" for n in names)
    src.write_text(
        "#include <stdio.h>\n#include \"zf.h\"\n"
        f"static void (*const table[])(void) = {{\n  {refs}\n}};\n"
        "int main(void) {\n"
        "  zf_opts o;\n  zf_default_opts(&o);\n"
        "  printf(\"%d %d %d %zu\\n\", zf_version(), o.order, o.precision, sizeof table / sizeof *table);\n"
        "  return 0;\n}\n")
    exe = tmp_path / "abi"
    cc = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                         str(src), LIB, f"-Wl,-rpath,{os.path.dirname(LIB)}", "-o", str(exe)],
                        capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, run.stderr
    version, order, precision, count = run.stdout.split()
    assert int(version) >= 1 and (int(order), int(precision)) == (2, 1)
    assert int(count) == len(names)
