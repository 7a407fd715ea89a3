"""hfci_shifted_solve_noalloc against hfci_shifted_solve, through the C ABI (needs an MI355X).

The no-allocation entry point runs the same kernels with the same launch shapes as the
shifted solve, with its buffers in the library's static scratch array instead of the
workspace, so its iterates and step counts must equal the shifted solve's bit for bit.
Two calls in a row, the second on a smaller input (the array keeps the first call's
contents), then a solve too large for the array, which must be refused before any launch.
"""
import numpy as np
import pytest

from oracle import fci as OF
from oracle import fixed_point as OFP
from oracle import operator as OO
from tests.fp32_bounds import relmax

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hf = pytest.importorskip("paper_1811_12378_amd.hfci")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hf.load_library()
    c = hf.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def setup(ctx, shape, seed, q, J=4):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.0, 3.0, size=shape)
    h = 1.0 / shape[0]
    o = OO.Operator(c, 14.0, 3, 1.0, h=h)
    g = hf.Operator(ctx, dev(c), h, 14.0, 3, 1.0)
    poles = OF.pole_parameters(o, J, 1.0, 0.5, q)
    cg = hf.Contour(g, J, 1.0, 0.5, q, z=[p.z for p in poles], sigma=[p.sigma for p in poles],
                    delta=[p.delta for p in poles])
    return o, g, cg, poles, rng


@pytest.mark.parametrize("tune,q", [((1, 8, 2, 0, 1), 8), ((3, 8, 2, 0, 2, 1), 10)])
def test_noalloc_equals_shifted_solve_twice(ctx, tune, q):
    # call 1: complex64, two factors per pass (and, with kern 3 and fuse 2, the middle
    # factors three per pass), adaptive stopping, 4 poles x 3 sources
    o, g, cg, poles, rng = setup(ctx, (20, 24, 30), 81, q)
    g.set_tune(32, *tune)
    f = rng.standard_normal((3, 20, 24, 30)) + 1j * rng.standard_normal((3, 20, 24, 30))
    f[1] *= 1e-3
    fd = dev(f).to(torch.complex64)
    y_ref, st_ref = hf.shifted_solve(g, cg, fd, reduce=5.0, max_steps=60)
    y = torch.full_like(y_ref, float("nan"))
    st = hf.shifted_solve_noalloc(g, cg, fd, y, reduce=5.0, max_steps=60)
    assert np.array_equal(st, st_ref)
    assert torch.equal(y, y_ref)
    assert len(set(st.ravel().tolist())) > 1  # the systems stop at different steps

    # call 2, right after: a smaller grid, complex128, one factor per pass, fixed steps;
    # the array still holds call 1's buffers, which must not leak into this result
    o2, g2, cg2, poles2, rng2 = setup(ctx, (12, 10, 14), 82, 5)
    f2 = rng2.standard_normal((1, 12, 10, 14)) + 1j * rng2.standard_normal((1, 12, 10, 14))
    fd2 = dev(f2)
    y_ref2, st_ref2 = hf.shifted_solve(g2, cg2, fd2, steps=3)
    y2 = torch.full_like(y_ref2, float("nan"))
    st2 = hf.shifted_solve_noalloc(g2, cg2, fd2, y2, steps=3)
    assert np.all(st2 == 3) and np.array_equal(st2, st_ref2)
    assert torch.equal(y2, y_ref2)
    # and, as for the shifted solve, the oracle's iterates to the FP64 bar
    Am = lambda v, sh: o2.apply(v, sh)
    for j, p in enumerate(poles2):
        ref, _ = OFP.fixed_point_solve(Am, f2[0], p.z, p.z0, p.delta, 5, steps=3)
        assert relmax(y2[j, 0].cpu().numpy(), ref) <= 1e-12


def test_noalloc_refuses_a_solve_larger_than_its_array(ctx):
    # 8 poles x 4 sources at 64^3 in complex64 need about 3 x 32 x 2 MiB > 64 MiB
    o, g, cg, poles, rng = setup(ctx, (64, 64, 64), 83, 8, J=8)
    f = dev(np.ones((4, 64, 64, 64), dtype=np.complex64))
    y = torch.zeros((8, 4, 64, 64, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(hf.HfciError) as e:
        hf.shifted_solve_noalloc(g, cg, f, y, steps=2)
    assert e.value.status == -1
    assert "scratch" in str(e.value)
    assert torch.count_nonzero(y) == 0  # nothing was launched
    # a case-two operator is refused as well
    g2 = g.case_two()
    c2 = hf.Contour(g2, 4, 1.0, 0.5, 4)
    f2 = dev(np.ones((1, 2, 64, 64, 64), dtype=np.complex128))
    y2 = torch.zeros((4, 1, 2, 64, 64, 64), dtype=torch.complex128, device="cuda")
    with pytest.raises(hf.HfciError) as e:
        hf.shifted_solve_noalloc(g2, c2, f2, y2, steps=1)
    assert e.value.status == -6
