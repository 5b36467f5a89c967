"""The C-ABI library loads and exports every entry point its header
declares; the Python layer rejects bad arguments before the ABI.  No GPU
compute here."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "nsp.h")).read()
    return sorted(set(re.findall(r"^(?:nsp_status|const char \*|int)\s*(nsp_\w+)\s*\(", hdr, re.M)))


def test_header_symbols_exported():
    from paper_1705_06149_amd import nsp
    L = nsp.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(nsp.EXPORTED)


def test_python_layer_rejects_bad_tensors():
    import torch
    from paper_1705_06149_amd import nsp
    t = torch.zeros((1, 4, 4, 5), dtype=torch.float64)
    with pytest.raises(ValueError):
        nsp._check(t, (1, 4, 4, 5), "u")          # CPU tensor: no CPU path
    with pytest.raises(TypeError):
        nsp._check(t.float(), (1, 4, 4, 5), "u")
    with pytest.raises(TypeError):
        nsp._check(np.zeros(3), (3,), "u")


def test_create_rejects_bad_grid_without_touching_gpu():
    import ctypes
    from paper_1705_06149_amd import nsp
    L = nsp.lib()
    h = ctypes.c_void_p()
    bad = nsp._Grid(0, 4, 4, 1.0, 1.0, 1.0, 100.0, 0, None, 1)
    assert L.nsp_create(ctypes.byref(bad), ctypes.byref(h)) == nsp.NSP_ERR_ARG
    flat = nsp._Grid(4, 4, 4, 1.0, 0.0, 1.0, 100.0, 1, None, 1)
    assert L.nsp_create(ctypes.byref(flat), ctypes.byref(h)) == nsp.NSP_ERR_ARG
    big = nsp._Grid(4, 4, 4, 1.0, 1.0, 1.0, 100.0, 0, None, 65)
    assert L.nsp_create(ctypes.byref(big), ctypes.byref(h)) == nsp.NSP_ERR_ARG
    slip = nsp._Grid(4, 4, 4, 1.0, 1.0, 1.0, 100.0, 0, None, 1, 2)
    assert L.nsp_create(ctypes.byref(slip), ctypes.byref(h)) == nsp.NSP_ERR_ARG
    assert L.nsp_destroy(None) == nsp.NSP_ERR_ARG
    assert L.nsp_last_error(None) == b"null handle"
