"""The C-ABI library loads and exports every function include/ifgf.h declares
(no compute calls: no GPU is needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2112_06316_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ifgf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ifgf_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares exactly the header's functions
    assert set(_lib.SIGNATURES) == set(names)


def test_status_strings_and_defaults_without_gpu():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    assert lib.ifgf_status_string(_lib.EDUPLICATE) == b"duplicate points"
    o = _lib.Options()
    lib.ifgf_options_default(ctypes.byref(o))
    assert (o.p_s, o.p_ang, o.ns0, o.nc0, o.depth, o.max_rhs) == (4, 6, 2, 4, 0, 1)
    assert o.leaf_h_lambda == 0.5
    assert (o.prop_kernel, o.target_kernel) == (_lib.PROP_AUTO, _lib.TARGET_AUTO)


def test_struct_layout_matches_header():
    # offsets of the C structs as laid out by a C compiler for x86-64
    assert ctypes.sizeof(_lib.Options) == 56
    assert _lib.Options.leaf_h_lambda.offset == 24
    assert _lib.Options.target_kernel.offset == 48
    assert _lib.Stats.boxes.offset == 64


def test_output_buffer_validation():
    # The library sees raw pointers only: a caller's output buffer must match
    # the input exactly, or the binding refuses it before any device call.
    import torch
    from paper_2112_06316_amd.api import _check_out
    s = torch.zeros(10, 2, dtype=torch.complex128)
    assert _check_out(torch.empty(10, 2, dtype=torch.complex128), s).shape == (10, 2)
    s1 = torch.zeros(10, 1, dtype=torch.complex64)
    assert _check_out(torch.empty(10, dtype=torch.complex64), s1).shape == (10, 1)
    with pytest.raises(TypeError):
        _check_out(torch.empty(10, 2, dtype=torch.complex64), s)
    with pytest.raises(ValueError):
        _check_out(torch.empty(9, 2, dtype=torch.complex128), s)
    with pytest.raises(ValueError):
        _check_out(torch.empty(2, 10, dtype=torch.complex128).t(), s)
    with pytest.raises(ValueError):
        _check_out(s, s)
    big = torch.zeros(20, 2, dtype=torch.complex128)
    with pytest.raises(ValueError):
        _check_out(big[5:15], big[:10])
    with pytest.raises(TypeError):
        _check_out(np.zeros((10, 2), dtype=np.complex128), s)
