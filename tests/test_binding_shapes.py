"""The binding refuses wrongly shaped vectors before anything reaches the library.

The C ABI takes a batch count and derives every vector length from the operator's
point count, so a tensor whose trailing shape is not the operator's grid would be
read or written past its end on the device.  These tests run on the CPU: the
library loader is replaced by one that fails, so a check that came too late would
show up as that failure instead of the expected ValueError.
"""
import types

import pytest
import torch

from paper_1811_12378_amd import hfci


@pytest.fixture
def no_library(monkeypatch):
    def refuse(*a, **k):
        raise AssertionError("the library was reached before the shape check")
    monkeypatch.setattr(hfci, "load_library", refuse)
    monkeypatch.setattr(hfci, "_sync", refuse)


def fake_op(shape):
    n = 1
    for v in shape:
        n *= v
    return types.SimpleNamespace(shape=tuple(shape), n=n, h=None)


def c128(*shape):
    return torch.zeros(shape, dtype=torch.complex128)


OP = fake_op((6, 5, 4))
OP2 = fake_op((2, 6, 5, 4))  # a case-two operator: vectors [2, nz, ny, nx]
CONT = types.SimpleNamespace(J=4, h=None)


@pytest.mark.parametrize("f", [c128(6, 5, 4), c128(1, 6, 5, 5), c128(1, 120), c128(2, 4, 5, 6)])
def test_solve_fci_shifted_refuse_wrong_grid(no_library, f):
    for call in (lambda: hfci.solve(OP, CONT, f), lambda: hfci.fci_apply(OP, CONT, f),
                 lambda: hfci.shifted_solve(OP, CONT, f, steps=1)):
        with pytest.raises(ValueError):
            call()


def test_case_two_refuses_the_natural_rhs(no_library):
    # the natural right-hand side [nrhs, nz, ny, nx] is half the length of a case-two vector
    f = c128(1, 6, 5, 4)
    for call in (lambda: hfci.solve(OP2, CONT, f), lambda: hfci.fci_apply(OP2, CONT, f),
                 lambda: hfci.shifted_solve(OP2, CONT, f, steps=1)):
        with pytest.raises(ValueError):
            call()


def test_initial_guess_must_match_f(no_library):
    f = c128(2, 6, 5, 4)
    for u0 in (c128(1, 6, 5, 4), torch.zeros((2, 6, 5, 4), dtype=torch.complex64), c128(2, 6, 5, 4, 1)):
        with pytest.raises(ValueError):
            hfci.solve(OP, CONT, f, u0=u0)


def test_solve_and_fci_need_complex128(no_library):
    f = torch.zeros((1, 6, 5, 4), dtype=torch.complex64)
    with pytest.raises(TypeError):
        hfci.solve(OP, CONT, f)
    with pytest.raises(TypeError):
        hfci.fci_apply(OP, CONT, f)


def test_batches_refuse_mismatched_instances(no_library):
    opb = fake_op((4, 4, 4))
    good = [c128(6, 5, 4), c128(4, 4, 4)]
    with pytest.raises(ValueError):  # lists of different lengths
        hfci.solve_batch([OP, opb], [CONT], good)
    with pytest.raises(ValueError):  # second right-hand side on the wrong grid
        hfci.solve_batch([OP, opb], [CONT, CONT], [c128(6, 5, 4), c128(4, 4, 5)])
    with pytest.raises(ValueError):  # a batch dimension where none belongs
        hfci.solve_batch([OP, opb], [CONT, CONT], [c128(1, 6, 5, 4), c128(4, 4, 4)])
    with pytest.raises(ValueError):  # an initial guess of another grid
        hfci.solve_batch([OP, opb], [CONT, CONT], good, u0s=[c128(6, 5, 4), c128(6, 5, 4)])
    with pytest.raises(ValueError):
        hfci.shifted_solve_batch([OP, opb], [CONT, CONT], [c128(6, 5, 4), c128(4, 5, 4)])
    with pytest.raises(ValueError):
        hfci.shifted_solve_batch([], [], [])
    with pytest.raises(TypeError):  # mixed precisions in one batch
        hfci.shifted_solve_batch([OP, opb], [CONT, CONT],
                                 [c128(6, 5, 4), torch.zeros((4, 4, 4), dtype=torch.complex64)])


def test_net_apply_refuses_wrong_grid(no_library):
    net = hfci.Net.__new__(hfci.Net)
    with pytest.raises(ValueError):
        net.apply(OP, c128(1, 6, 5, 5))
