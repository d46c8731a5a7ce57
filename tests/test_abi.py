"""CPU checks of the C-ABI boundary: the library loads, exports every declared
symbol, and its option/stat structs have the layout the Python binding uses."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(clr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("clr_create", "clr_gemm", "clr_sqrt_inv", "clr_compress", "clr_to_dense",
                     "clr_destroy", "clr_context_create", "clr_axpby"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1509_00309_amd import _abi
    lib = C.CDLL(_abi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(_abi.EXPORTS) == declared_functions()


def test_nm_lists_exports():
    from paper_1509_00309_amd import _abi
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (clr_\w+)", out))
    assert set(declared_functions()) <= exported


def _c_layout():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "clr.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(clr_gemm_opts), sizeof(clr_sqrtinv_opts),
         sizeof(clr_gemm_stats), sizeof(clr_sqrtinv_stats));
  printf("%zu %zu %zu\n", offsetof(clr_gemm_opts, alpha), offsetof(clr_sqrtinv_opts, conv_tol),
         offsetof(clr_gemm_stats, bytes_compulsory));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        return subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()


def test_struct_layout_matches_binding():
    from paper_1509_00309_amd import _abi
    vals = list(map(int, _c_layout()))
    assert vals[0] == C.sizeof(_abi.GemmOpts)
    assert vals[1] == C.sizeof(_abi.SqrtInvOpts)
    assert vals[2] == C.sizeof(_abi.GemmStats)
    assert vals[3] == C.sizeof(_abi.SqrtInvStats)
    assert vals[4] == _abi.GemmOpts.alpha.offset
    assert vals[5] == _abi.SqrtInvOpts.conv_tol.offset
    assert vals[6] == _abi.GemmStats.bytes_compulsory.offset


def test_status_strings_and_null_arguments():
    from paper_1509_00309_amd import _abi
    lib = _abi.lib
    assert lib.clr_status_string(0) == b"ok"
    assert lib.clr_status_string(2) == b"blockings do not conform"
    # null handles are rejected before any device work
    assert lib.clr_gemm(None, None, None, None, None, None) == _abi.CLR_ERR_INVALID_ARG
    assert lib.clr_destroy(None) == _abi.CLR_ERR_INVALID_ARG
    assert lib.clr_context_destroy(None) == _abi.CLR_ERR_INVALID_ARG
    assert lib.clr_last_error(None) == b""


def test_python_binding_has_no_cpu_fallback():
    """The package imports only the HIP library; it never reaches the oracle."""
    import paper_1509_00309_amd as pkg
    src = open(pkg.__file__).read() + open(os.path.join(os.path.dirname(pkg.__file__), "_abi.py")).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
