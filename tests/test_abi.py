"""The C-ABI library loads on a machine without a GPU and exports every function that
include/*.h declares (no GPU calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsa.h")


def declared_functions():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(fsa_[a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fsa_init", "fsa_destroy", "fsa_set_markers", "fsa_rhs", "fsa_rk3_step",
                     "fsa_ib_interp", "fsa_ib_spread", "fsa_probe_dp"):
        assert required in names
    assert len(names) >= 18


def test_library_exports_every_declared_symbol():
    from paper_1905_00182_amd import fsa

    if not os.path.exists(fsa.LIB_PATH):
        pytest.fail("libfsa.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(fsa.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert fsa.lib().fsa_abi_version() == 2
    assert fsa.lib().fsa_status_str(-4) == b"non-finite state"


def test_binding_signatures_cover_the_header():
    from paper_1905_00182_amd import fsa

    assert set(declared_functions()) == set(fsa._SIGS)


def test_descriptor_layouts_match_the_header():
    # field order of the ctypes mirrors must follow the C structs in include/fsa.h
    from paper_1905_00182_amd import fsa

    text = open(HEADER).read()
    body = re.search(r"typedef struct fsa_desc \{(.*?)\} fsa_desc;", text, flags=re.S).group(1)
    fields = re.findall(r"^\s*[a-z_0-9]+\s+([a-z_0-9]+)(?:\[|;)", body, flags=re.M)
    assert fields == [f[0] for f in fsa.FsaDesc._fields_]
    body = re.search(r"typedef struct fsa_stats \{(.*?)\} fsa_stats;", text, flags=re.S).group(1)
    fields = re.findall(r"^\s*[a-z_0-9]+\s+([a-z_0-9]+)(?:\[|;)", body, flags=re.M)
    assert fields == [f[0] for f in fsa.FsaStats._fields_]


def test_plate_descriptor_layout_matches_the_header():
    from paper_1905_00182_amd import fsa

    text = open(os.path.join(ROOT, "include", "fsa_plate.h")).read()
    body = re.search(r"typedef struct fsa_plate_desc \{(.*?)\} fsa_plate_desc;", text, flags=re.S).group(1)
    fields = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**([a-z_0-9]+)(?:\[|;)", body, flags=re.M)
    assert fields == [f[0] for f in fsa.FsaPlateDesc._fields_]
