"""The Python binding rejects bad tensors before any library call: a host
tensor, a wrong dtype, shape or device, a non-contiguous view, an output that
does not match its input or overlaps it, or a wrong number of occupations
would otherwise reach a kernel as a raw pointer.  Runs without a GPU: the
device-side attributes are imitated, and the library loader is replaced by
one that fails the test if it is reached."""
import numpy as np
import pytest
import torch

from paper_2406_16998_amd import kx

SHAPE3 = (6, 5, 4)  # (n3, n2, n1)


class FakeDev:
    """Just enough of a device tensor for the binding's checks."""

    def __init__(self, shape, dtype=torch.float64, device=0, contiguous=True, ptr=1 << 20):
        self.shape = torch.Size(shape)
        self.dtype = dtype
        self.is_cuda = True
        self.device = torch.device("cuda", device)
        self._contig = contiguous
        self._ptr = ptr

    def is_contiguous(self):
        return self._contig

    def dim(self):
        return len(self.shape)

    def numel(self):
        return int(np.prod(self.shape)) if len(self.shape) else 1

    def element_size(self):
        return 8 if self.dtype == torch.float64 else (4 if self.dtype == torch.float32 else 2)

    def data_ptr(self):
        return self._ptr


def _grid():
    g = kx.Grid.__new__(kx.Grid)
    g._h = None
    g.n = (SHAPE3[2], SHAPE3[1], SHAPE3[0])
    g.h = (0.3, 0.3, 0.3)
    g.shape3 = SHAPE3
    g.device = 0
    g.N = int(np.prod(SHAPE3))
    return g


@pytest.fixture
def no_library(monkeypatch):
    def refuse():
        raise AssertionError("the library was reached with a bad argument")
    monkeypatch.setattr(kx, "lib", refuse)


GOOD = (3,) + SHAPE3
BAD_INPUTS = {
    "host tensor": torch.zeros(GOOD, dtype=torch.float64),
    "float16": FakeDev(GOOD, dtype=torch.float16),
    "int64": FakeDev(GOOD, dtype=torch.int64),
    "non-contiguous": FakeDev(GOOD, contiguous=False),
    "3-D": FakeDev(SHAPE3),
    "wrong grid": FakeDev((3, 6, 4, 5)),
    "other device": FakeDev(GOOD, device=1),
    "not a tensor": np.zeros(GOOD),
}


@pytest.mark.parametrize("case", sorted(BAD_INPUTS))
def test_bad_input_tensor_is_rejected(no_library, case):
    g = _grid()
    x = BAD_INPUTS[case]
    with pytest.raises(ValueError):
        g.apply_exchange(x, [2.0] * 3, "erfc", 0.1)
    with pytest.raises(ValueError):
        g.apply_exchange_noalloc(x, [2.0] * 3, "erfc", 0.1)
    with pytest.raises(ValueError):
        g.apply_fL(x, "erfc", 0.1)
    with pytest.raises(ValueError):
        g.apply_fL_multipole(x, lmax=2)
    with pytest.raises(ValueError):
        g.ace_apply(x, FakeDev(GOOD, ptr=1 << 30), out=FakeDev(GOOD, ptr=1 << 31))


BAD_OUTPUTS = {
    "dtype": FakeDev(GOOD, dtype=torch.float32, ptr=1 << 30),
    "shape": FakeDev((2,) + SHAPE3, ptr=1 << 30),
    "device": FakeDev(GOOD, device=1, ptr=1 << 30),
    "non-contiguous": FakeDev(GOOD, contiguous=False, ptr=1 << 30),
    "same buffer": FakeDev(GOOD),
    "overlap": FakeDev(GOOD, ptr=(1 << 20) + 8 * 17),
}


@pytest.mark.parametrize("case", sorted(BAD_OUTPUTS))
def test_bad_output_tensor_is_rejected(no_library, case):
    g = _grid()
    psi = FakeDev(GOOD)
    out = BAD_OUTPUTS[case]
    with pytest.raises(ValueError):
        g.apply_exchange(psi, [2.0] * 3, "erfc", 0.1, out=out)
    with pytest.raises(ValueError):
        g.apply_fL(psi, "erfc", 0.1, out=out)


@pytest.mark.parametrize("occ", [[2.0, 2.0], [2.0] * 4, [2.0, float("nan"), 1.0], []])
def test_bad_occupations_are_rejected(no_library, occ):
    g = _grid()
    with pytest.raises(ValueError):
        g.apply_exchange(FakeDev(GOOD), occ, "erfc", 0.1, out=FakeDev(GOOD, ptr=1 << 30))


def test_ace_build_rejects_mismatched_fields(no_library):
    g = _grid()
    psi = FakeDev(GOOD)
    with pytest.raises(ValueError):
        g.ace_build(psi, FakeDev(GOOD, dtype=torch.float32, ptr=1 << 30))
    with pytest.raises(ValueError):
        g.ace_build(psi, FakeDev((2,) + SHAPE3, ptr=1 << 30))
    with pytest.raises(ValueError):  # xi written over W
        w = FakeDev(GOOD, ptr=1 << 30)
        g.ace_build(psi, w, out=w)


def test_batch_rejects_mismatched_lists(no_library):
    g = _grid()
    psi = FakeDev(GOOD)
    with pytest.raises(ValueError):
        kx.batch_apply_exchange([g], [psi], [[2.0] * 3, [2.0]], ["erfc"], [0.1])
    with pytest.raises(ValueError):
        kx.batch_apply_exchange([g], [torch.zeros(GOOD, dtype=torch.float64)], [[2.0] * 3],
                                ["erfc"], [0.1], outs=[FakeDev(GOOD, ptr=1 << 30)])
    with pytest.raises(ValueError):
        kx.batch_apply_exchange([g], [psi], [[2.0] * 2], ["erfc"], [0.1],
                                outs=[FakeDev(GOOD, ptr=1 << 30)])


def test_good_arguments_pass_the_checks():
    psi = FakeDev(GOOD)
    assert kx.check_fields(psi, SHAPE3, 0, "psi") == kx.DTYPE["f64"]
    assert kx.check_fields(FakeDev(GOOD, dtype=torch.float32), SHAPE3, 0, "psi") == kx.DTYPE["f32"]
    kx.check_out(FakeDev(GOOD, ptr=1 << 30), psi)
    assert kx.check_occ([2.0, 1.0, 0.5], 3).dtype == np.float64
