"""Jacobi/Laplace on the device against the FP64 oracle: bit-exact grids
(the sums are taken in the oracle's order, without fused multiply-add) and the
same last-iteration change, resident and per-iteration-transfer modes alike."""
import numpy as np
import pytest

import synth
from oracle import jacobi as oj
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    from paper_1811_03882_amd import dn as _dn
    G.torch_cuda()
    return _dn


def grid(n, m, tag):
    u = synth.make_tensor((n, m), synth.SEED_DETECT + 1, tag, -1.0, 1.0)
    u[1:-1, 1:-1] = 0.0
    return u


@pytest.mark.parametrize("n,m,iters", [(3, 3, 1), (37, 70, 5), (130, 257, 12), (1, 9, 2), (64, 2, 3), (300, 129, 0)])
def test_resident_matches_oracle_bitwise(dn, n, m, iters):
    torch = G.torch_cuda()
    u = grid(n, m, n * 1000 + m)
    ref, ref_ch = oj.solve(u, iters)
    du = torch.from_numpy(u.copy()).cuda()
    work = torch.empty_like(du)
    mc = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    dn.jacobi(du, work, n, m, iters, mc)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(du.cpu().numpy(), ref)
    assert mc.item() == ref_ch


def test_per_iteration_mode_equals_resident(dn):
    torch = G.torch_cuda()
    n, m, iters = 200, 300, 7
    u = grid(n, m, 7)
    ref, ref_ch = oj.solve(u, iters)
    host = u.copy()
    a = torch.empty((n, m), dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    ch = dn.jacobi_per_iteration(host, a, b, iters)
    np.testing.assert_array_equal(host, ref)
    assert ch == ref_ch


def test_large_grid_sampled(dn):
    """The bench grid (4096 x 4096): sampled rows recomputed by the oracle
    from the device's previous iterate."""
    torch = G.torch_cuda()
    n = m = 4096
    u = grid(n, m, 4096)
    du = torch.from_numpy(u.copy()).cuda()
    work = torch.empty_like(du)
    dn.jacobi(du, work, n, m, 9)
    prev = du.cpu().numpy()
    dn.jacobi(du, work, n, m, 1)
    got = du.cpu().numpy()
    for r in (1, 1000, 2047, 4094):
        band = prev[r - 1:r + 2].copy()
        step, _ = oj.step(band)
        np.testing.assert_array_equal(got[r, 1:-1], step[1, 1:-1])


def test_bad_arguments(dn):
    with pytest.raises(dn.DnError):
        dn.jacobi(None, None, 4, 4, 1)
    torch = G.torch_cuda()
    a = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(dn.DnError):
        dn.jacobi(a, a.clone(), 0, 4, 1)
