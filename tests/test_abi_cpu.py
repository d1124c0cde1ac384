"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/btas.h, and its pure-host helpers agree
with the oracle.  No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

import oracle
import paper_1701_04733_amd as btas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared_symbols():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(btas_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("btas_create", "btas_destroy", "btas_tropical_gemm", "btas_tropical_gemv",
                     "btas_tropical_vadd", "btas_tropical_vmul", "btas_tropical_dot",
                     "btas_tropical_axpy", "btas_apsp_squaring"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = btas.lib()
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", btas.library_path], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (btas_\w+)", out))
    assert set(declared_symbols()) <= exported


def test_status_strings_and_version():
    L = btas.lib()
    for code, name in btas.STATUS.items():
        assert L.btas_status_string(code).decode() == name
    assert btas.version().startswith("btas-gfx950")


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 16, 17, 18, 256, 257, 258, 512, 16384, 100000])
def test_num_steps_matches_oracle(n):
    assert btas.apsp_num_steps(n) == oracle.apsp_steps(n)


def test_null_handle_and_bad_create_are_rejected_without_touching_a_device():
    L = btas.lib()
    assert L.btas_create(None, 0) == 1
    h = ctypes.c_void_p()
    assert L.btas_create(ctypes.byref(h), -1) == 1 and not h.value
    assert L.btas_tropical_gemm(None, 0, 0, 1, 1, 1, None, 1, None, 1, None, 1) == 1
    assert L.btas_apsp_squaring(None, 0, 4, None, 4, None, 4, 0, None) == 1
    assert L.btas_destroy(None) == 1
    assert L.btas_last_error(None) == b"null handle"
