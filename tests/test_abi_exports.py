"""The built library loads and exports every function include/labs.h declares
(no GPU needed; nothing is computed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "labs.h")
LIB = os.path.join(ROOT, "paper_2409_07222_amd", "liblabs.so")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(labs_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for want in ("labs_energy", "labs_flip_deltas", "labs_walk_step1", "labs_pool_topk",
                 "labs_walk_step1_workspace", "labs_pool_topk_workspace"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name
    lib.labs_abi_version.restype = ctypes.c_int32
    assert lib.labs_abi_version() == 1
    lib.labs_words.restype = ctypes.c_int32
    assert [lib.labs_words(L) for L in (1, 32, 33, 501)] == [1, 1, 2, 16]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_arguments_are_rejected_without_a_gpu():
    lib = ctypes.CDLL(LIB)
    lib.labs_energy.restype = ctypes.c_int32
    lib.labs_energy.argtypes = [ctypes.c_int32, ctypes.c_int64] + [ctypes.c_void_p] * 4
    assert lib.labs_energy(0, 1, None, None, None, None) == -1
    assert lib.labs_energy(2000, 1, None, None, None, None) == -1
    assert lib.labs_energy(37, 5, None, None, None, None) == -1
    lib.labs_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.labs_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_mlp_layout_host_call():
    """labs_mlp_layout_of is host-only: the L = 501 network of 751 -> 256 -> 256 -> 251
    has 322,811 parameters, and the blob round-trips through the binding's placement."""
    import numpy as np
    from paper_2409_07222_amd import labs
    lay = labs.mlp_layout(501, 256)
    assert (lay.d_in, lay.d_out, lay.ld_in, lay.ld_out, lay.mask_words) == (751, 251, 768, 256, 8)
    used = lay.hidden * lay.d_in + lay.hidden + lay.hidden ** 2 + lay.hidden + \
        lay.d_out * lay.hidden + lay.d_out
    assert used == 322811
    offs = [lay.off_W1, lay.off_b1, lay.off_W2, lay.off_b2, lay.off_W3, lay.off_b3, lay.n_params]
    assert offs == sorted(offs) and all(o % 64 == 0 for o in offs)
    import labs_inputs as li
    P = li.mlp_init(55, lay.d_in, 256, lay.d_out)
    back = labs.mlp_dict_from_blob(lay, labs.mlp_blob_from_dict(lay, P))
    assert all(np.array_equal(back[k], P[k]) for k in P)
    with pytest.raises(labs.LabsError):
        labs.mlp_layout(500, 256)
    with pytest.raises(labs.LabsError):
        labs.mlp_layout(501, 100)
