"""Host-side checks of libkx: it loads, exports every declared symbol, and its
host logic (FD weights, 1-D Laplacians, pair schedule, argument validation)
is right.  No device work is issued; these run without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_16998_amd import kx
import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
needs_lib = pytest.mark.skipif(not os.path.exists(kx.LIB_PATH), reason="libkx.so not built")


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "kx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kx_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_lists_binding_exports():
    assert sorted(kx.EXPORTS) == _declared_symbols()


@needs_lib
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(kx.LIB_PATH)
    for name in _declared_symbols():
        assert hasattr(L, name), name


@needs_lib
@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 16, 20, 24])
def test_fd_weights_match_oracle(order):
    w = kx.fd_weights(order)
    ref = np.array([float(x) for x in orc.fd_weights(order)])
    assert np.max(np.abs(w - ref)) <= 4e-16 * np.max(np.abs(ref))


@needs_lib
@pytest.mark.parametrize("n,h,order,bc", [(32, 0.3, 12, "dirichlet"), (96, 0.35, 12, "periodic"),
                                          (7, 0.4, 12, "periodic"), (5, 0.5, 12, "dirichlet"),
                                          (1, 0.3, 4, "periodic"), (60, 0.3, 2, "periodic")])
def test_laplacian_1d_matches_oracle(n, h, order, bc):
    L = kx.laplacian_1d(n, h, order, bc)
    ref = orc.laplacian_1d(n, h, order, bc)
    scale = abs(float(orc.fd_weights(order)[0])) / h ** 2
    assert np.max(np.abs(L - ref)) <= 1e-15 * scale * order
    assert np.array_equal(L, L.T)


@needs_lib
@pytest.mark.parametrize("norb,cap", [(1, 0), (2, 0), (5, 0), (8, 3), (128, 64), (33, 7), (0, 0)])
def test_pair_schedule_covers_every_pair_once_without_conflicts(norb, cap):
    pairs, offs = kx.pair_schedule(norb, cap)
    assert len(pairs) == norb * (norb + 1) // 2
    seen = {(int(i), int(j)) for i, j in pairs}
    assert len(seen) == len(pairs)
    assert all(0 <= i <= j < norb for i, j in seen)
    assert offs[0] == 0 and offs[-1] == len(pairs)
    for b in range(len(offs) - 1):
        batch = pairs[offs[b]:offs[b + 1]]
        assert len(batch) > 0
        if cap > 0:
            assert len(batch) <= cap
        touched = [int(v) for i, j in batch for v in ((i,) if i == j else (i, j))]
        assert len(touched) == len(set(touched)), "an orbital appears twice in one batch"


@needs_lib
def test_setup_validation_rejects_bad_arguments_before_device_work():
    L = kx.lib()
    good_n, good_h, good_bc = (16, 16, 16), (0.3, 0.3, 0.3), (0, 0, 0)

    def call(n=good_n, h=good_h, order=12, bc=good_bc, out=True):
        handle = ctypes.c_void_p()
        return L.kx_setup_laplacian((ctypes.c_int * 3)(*n), (ctypes.c_double * 3)(*h), order,
                                    (ctypes.c_int * 3)(*bc), None,
                                    ctypes.byref(handle) if out else None)

    bad = [dict(n=(0, 16, 16)), dict(n=(16, 161, 16)), dict(n=(16, 16, -3)),
           dict(h=(0.0, 0.3, 0.3)), dict(h=(0.3, float("nan"), 0.3)), dict(h=(0.3, 0.3, float("inf"))),
           dict(h=(0.3, -0.1, 0.3)), dict(order=0), dict(order=3), dict(order=26), dict(order=-2),
           dict(bc=(0, 2, 0)), dict(bc=(-1, 0, 0)), dict(out=False)]
    for kw in bad:
        assert call(**kw) == 1, kw


@needs_lib
def test_null_handle_and_host_helper_validation():
    L = kx.lib()
    w = np.zeros(16)
    dp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.kx_apply_fL(None, 0, 0.0, 1, 0, None, None, 0) == 1
    assert L.kx_apply_exchange(None, 0, 0.0, 1, 0, None, None, None, 0) == 1
    assert L.kx_exchange_energy(None, dp) == 1
    assert L.kx_pair_energies(None, 0, None, None) == 1
    assert L.kx_get_eigensystem(None, 0, None, None) == 1
    assert L.kx_ace_build(None, 4, 0, None, None, None) == 1
    assert L.kx_ace_apply(None, 4, 0, None, 1, None, None) == 1
    assert L.kx_profile_phases(None, 1) == 1
    assert L.kx_apply_fL_multipole(None, 1, 0, None, None, 0, 2, dp) == 1
    assert L.kx_reserve(None, 4, 0, 0) == 1
    assert L.kx_reserve_bloch(None, 1, 1) == 1
    assert L.kx_set_cell(None, dp) == 1
    assert L.kx_set_checks(None, 1) == 1
    assert L.kx_set_zero_mode(None, 1, 1.0) == 1
    assert L.kx_ace_build_complex(None, 2, None, None, None) == 1
    assert L.kx_ace_apply_complex(None, 2, None, 1, None, None) == 1
    assert L.kx_apply_exchange_multipole(None, 1, 0, None, None, None, 0, 2, dp) == 1
    assert L.kx_apply_fL_bloch(None, 1, 0.2, 1, dp, None, None, 0) == 1
    assert L.kx_apply_exchange_bloch(None, 1, 0.2, 1, 1, dp, dp, dp, None, None, 0) == 1
    assert L.kx_destroy(None) == 0
    assert L.kx_fd_weights(13, dp) == 1 and L.kx_fd_weights(12, None) == 1
    assert L.kx_laplacian_1d(0, 0.3, 12, 0, dp) == 1
    assert L.kx_laplacian_1d(4, 0.3, 12, 5, dp) == 1
    n1, n2 = ctypes.c_int(), ctypes.c_int()
    assert L.kx_pair_schedule(-1, 0, ctypes.byref(n1), ctypes.byref(n2), None, None) == 1
    for s in range(8):
        assert L.kx_status_string(s)
    assert L.kx_status_string(99) == b"unknown status"


@needs_lib
@pytest.mark.parametrize("norb,cap", [(128, 48), (128, 64), (33, 7), (256, 100), (9, 4)])
def test_pair_schedule_cuts_groups_evenly(norb, cap):
    # the diagonal group (norb pairs) and every tournament round (norb // 2
    # pairs) are cut into ceil(size / cap) batches whose sizes differ by at
    # most one, in launch order
    pairs, offs = kx.pair_schedule(norb, cap)
    sizes = list(np.diff(offs))
    groups = [norb] + [norb // 2] * (((norb + 1) & ~1) - 1)
    k = 0
    for size in groups:
        parts = -(-size // cap)
        got = sizes[k:k + parts]
        assert sum(got) == size and max(got) - min(got) <= 1 and max(got) <= cap, (size, got)
        k += parts
    assert k == len(sizes)
    # the diagonal pairs come first, in index order
    assert [tuple(p) for p in pairs[:norb]] == [(i, i) for i in range(norb)]
