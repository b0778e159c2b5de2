"""CPU checks of the C-ABI library: it is built for gfx950, loads, and exports every
function that include/iga.h declares (no compute calls: there may be no GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1811_06797_amd", "libiga.so")
HDR = os.path.join(ROOT, "include", "iga.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(iga_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_boundary_calls():
    names = declared_functions()
    for must in ("iga_assemble_factors", "iga_kkt_create", "iga_kkt_apply", "iga_amen_solve",
                 "iga_tt_wrap", "iga_btt_to_full", "iga_last_error", "iga_local_matvec"):
        assert must in names


def test_library_loads_and_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libiga.so missing: run __graft_entry__.build() first")
    from paper_1811_06797_amd import iga
    missing = [n for n in declared_functions() if not hasattr(iga.lib, n)]
    assert not missing, missing
    assert set(iga.EXPORTED) == set(declared_functions())


def test_library_embeds_gfx950_code_objects():
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data
    for other in (b"--gfx90a", b"--gfx942", b"--gfx1100"):
        assert other not in data


def test_error_path_without_device_context():
    from paper_1811_06797_amd import iga
    with pytest.raises(iga.IgaError):
        iga.ctx_create(device=10 ** 6)


def test_no_unresolved_library_symbols():
    import subprocess
    out = subprocess.run(["nm", "-D", "--undefined-only", LIB], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("nm unavailable")
    strong = [l for l in out.stdout.splitlines() if " U " in l and "iga" in l]
    assert not strong, strong


def test_noalloc_scratch_size_matches_header():
    from paper_1811_06797_amd import iga
    m = re.search(r"#define IGA_NOALLOC_SCRATCH_BYTES \((\d+)L << (\d+)\)", open(HDR).read())
    assert m and int(m.group(1)) << int(m.group(2)) == iga.NOALLOC_SCRATCH_BYTES


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the option and statistics structs have the C layout of iga.h
    (compiled here with the host C compiler: sizes and the offsets of the last fields)."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    from paper_1811_06797_amd import iga
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "iga.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu\\n", sizeof(iga_amen_stats), offsetof(iga_amen_stats, history_storage),\n'
        "         sizeof(iga_amen_opts), sizeof(iga_profile), sizeof(iga_local_problem));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(iga.AmenStats), iga.AmenStats.history_storage.offset, ctypes.sizeof(iga.AmenOpts),
            ctypes.sizeof(iga.Profile), ctypes.sizeof(iga.LocalProblem)]
    assert got == want
