"""The C-ABI library loads and exports every symbol declared in include/magpie.h.

No GPU work here: only host-side entry points (argument validation that
returns before touching a device, and the host permutation generator).
"""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2504_10118_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            with open(os.path.join(inc, fn)) as f:
                txt = f.read()
            names |= set(re.findall(r"^\s*(?:int|const char\*|void)\s+(magpie_\w+)\s*\(", txt, re.M))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("magpie_create", "magpie_set_probe", "magpie_set_positions", "magpie_load_intensities",
                 "magpie_run_epochs", "magpie_get_object", "magpie_get_probe", "magpie_objective"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = pkg.load_library()
    raw = ctypes.CDLL(pkg.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(raw, name), name
    assert lib is not None


def test_create_rejects_bad_arguments_before_touching_a_device():
    lib = pkg.load_library()
    h = ctypes.c_void_p()
    assert lib.magpie_create(ctypes.byref(h), 64, 64, 48, 2, 0.5, 0, None) == -6   # m unsupported
    assert b"m must be" in lib.magpie_last_error()
    assert lib.magpie_create(ctypes.byref(h), 64, 64, 32, 7, 0.5, 0, None) == -6   # too many levels
    assert lib.magpie_create(ctypes.byref(h), 16, 64, 32, 2, 0.5, 0, None) == -1   # object < probe
    assert lib.magpie_create(ctypes.byref(h), 64, 64, 32, 2, -1.0, 0, None) == -1  # alpha < 0
    assert lib.magpie_create(None, 64, 64, 32, 2, 0.5, 0, None) == -1
    # objects of 2^32 bytes or more (complex64) do not fit the kernels' 32-bit buffer ranges
    assert lib.magpie_create(ctypes.byref(h), 1 << 14, 1 << 15, 64, 3, 0.5, 0, None) == -6   # exactly 2^32 B
    assert b"2^32" in lib.magpie_last_error()
    assert lib.magpie_create(ctypes.byref(h), 23171, 23171, 128, 4, 0.5, 0, None) == -6      # just above
    assert not h.value
    # NULL context is rejected by every entry point that takes one
    assert lib.magpie_run_epochs(None, 1, 1, 0, None) == -1
    assert lib.magpie_run_minibatch(None, 1, None) == -1
    assert lib.magpie_destroy(None) == 0


@pytest.mark.parametrize("seed,epoch,n", [(0, 0, 1), (42, 3, 10), (2**63 + 5, 17, 1600), (7, 2**40, 6400)])
def test_permutation_matches_oracle(seed, epoch, n):
    got = pkg.permutation(seed, epoch, n)
    want = oracle.library_permutation(seed, epoch, n)
    np.testing.assert_array_equal(got, want)


def test_learned_entry_points_reject_bad_arguments_before_touching_a_device():
    lib = pkg.load_library()
    h = ctypes.c_void_p()
    assert lib.magpie_cnn_create(ctypes.byref(h), 2, 32, 64, 8, 0, 0, None) == -6    # in_ch
    assert lib.magpie_cnn_create(ctypes.byref(h), 3, 16, 64, 8, 0, 0, None) == -6    # width
    assert lib.magpie_cnn_create(ctypes.byref(h), 3, 32, 63, 8, 0, 0, None) == -1    # odd side
    assert lib.magpie_cnn_create(ctypes.byref(h), 3, 32, 64, 0, 0, 0, None) == -1    # max_batch
    assert lib.magpie_cnn_create(ctypes.byref(h), 3, 32, 64, 8, 5, 0, None) == -1    # weight dtype
    assert lib.magpie_cnn_create(None, 3, 32, 64, 8, 0, 0, None) == -1
    assert lib.magpie_cnn_forward(None, None, None, 1, 0) == -1
    assert lib.magpie_cnn_backward(None, None, 1, 0) == -1
    assert lib.magpie_cnn_adam_step(None, 1e-3, 0.9, 0.999, 1e-8) == -1
    assert lib.magpie_input_map(None, 64, None, 0) == -1
    assert lib.magpie_set_object_from_coarse(None, None, 64, 0, 0) == -1
    assert lib.magpie_learned_start(None, None, None, None, None) == -1
    assert lib.magpie_restrict_object(None, 64, 64, 1, None, None) == -1
    assert lib.magpie_cnn_destroy(None) == 0
