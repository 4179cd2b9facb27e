"""The C ABI: the built library loads and exports every function that
include/ffmg.h declares (no GPU compute here), and the binding's structs match
the header's field order."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffmg.h")
LIB = os.path.join(ROOT, "paper_1211_4461_amd", "libffmg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s\*]+([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("mg_setup", "mg_vcycle", "mg_solve", "farfield_map", "mg_rhs_plane_wave", "mg_destroy"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libffmg.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if " T " in line)
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libffmg.so not built")
def test_library_loads_and_binding_resolves():
    from paper_1211_4461_amd import ffmg
    L = ffmg.lib()
    for n in declared_functions():
        assert hasattr(L, n)
    assert set(ffmg.EXPORTS) == set(declared_functions())
    o = ffmg.default_options()   # pure host code: fills the defaults
    assert (o.nu1, o.nu2, o.coarsest_n, o.max_cycles) == (2, 2, 8, 200)
    assert abs(o.omega - 0.8) < 1e-15
    assert L.ffmg_strerror(ffmg.FFMG_ENOCONV) == b"no convergence"


def test_struct_layout_matches_header():
    """Field order of the ctypes mirrors equals the header's."""
    from paper_1211_4461_amd import ffmg
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)

    def fields(struct):
        body = re.search(r"typedef struct %s \{(.*?)\}" % struct, text, flags=re.S).group(1)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):
                m = re.search(r"([A-Za-z_][A-Za-z0-9_]*)\s*(\[\d+\])?\s*$", part.strip())
                out.append(m.group(1))
        return out

    assert fields("ffmg_problem") == [f for f, _ in ffmg.Problem._fields_]
    assert fields("ffmg_options") == [f for f, _ in ffmg.Options._fields_]
    assert fields("ffmg_solve_info") == [f for f, _ in ffmg.SolveInfo._fields_]


def test_noalloc_limits_match_header():
    """The binding's limits of farfield_map_noalloc are the header's."""
    from paper_1211_4461_amd import ffmg
    text = open(HEADER).read()
    scratch = re.search(r"#define FFMG_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert int(scratch.group(1)) << int(scratch.group(2)) == ffmg.NOALLOC_SCRATCH_BYTES
    dirs = re.search(r"#define FFMG_NOALLOC_MAX_DIRS (\d+)", text)
    assert int(dirs.group(1)) == ffmg.NOALLOC_MAX_DIRS
