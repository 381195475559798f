"""GPU parity of bfgs_precond_diag (eq. 4's smoothed, median-damped diagonal B_0)
against the float64 oracle, and what it buys: fewer BFGS iterations than gamma I."""
import numpy as np
import pytest
import torch

from oracle import precond as oprecond
from workloads import quadratic as wq

pytestmark = pytest.mark.gpu

CASES = [
    # nx, nz, nparam, sigma, half, damping
    (600, 200, 3, 5.0, 20, 1.0),      # the 600 x 200 x 3 grid (n even)
    (37, 13, 3, 2.0, 40, 0.3),        # taps wider than the grid, n odd
    (1, 1, 1, 1.0, 3, 1.0),           # one point
    (129, 1, 2, 0.7, 2, 2.0),         # one grid row
    (5, 301, 1, 9.0, 30, 0.0),        # no damping
]


@pytest.mark.parametrize("nx,nz,npar,sigma,half,damping", CASES)
def test_precond_matches_oracle(nx, nz, npar, sigma, half, damping):
    import paper_2009_12663_amd as P
    n = nx * nz * npar
    rng = np.random.default_rng(n)
    h = np.exp(rng.standard_normal(n)).astype(np.float32)
    print(f"\n[precond] {nx}x{nz}x{npar} sigma={sigma} half={half} damping={damping}", flush=True)
    h0, hs, lam = P.precond_diag(torch.from_numpy(h).cuda(), nx, nz, npar, sigma, half, damping)
    hs_g = hs.double().cpu().numpy()
    h0_g = h0.double().cpu().numpy()
    # the smoothed field: float64 sums rounded to float32 on both sides
    hs_ref = oprecond.smooth(h.astype(np.float64), nx, nz, npar, sigma, half)
    ulp = np.spacing(np.abs(hs_ref).astype(np.float32)).astype(np.float64)
    assert (np.abs(hs_g - hs_ref) <= ulp).all()
    # the median is an order statistic of the GPU's own float32 field: exact
    assert lam == damping * float(np.median(hs_g))
    # h0 from the oracle's formula on the same hs and lambda: within half an ulp of float32
    want = 1.0 / (hs_g + lam)
    assert (np.abs(h0_g - want) <= 0.5 * np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)).all()
    # and end to end against the oracle run from the input alone
    h0_ref, _, lam_ref = oprecond.precond_diag(h.astype(np.float64), nx, nz, npar, sigma, half, damping)
    np.testing.assert_allclose(h0_g, h0_ref, rtol=3e-7)
    assert lam == pytest.approx(lam_ref, rel=1e-7)


def test_precond_argument_errors():
    import ctypes
    import paper_2009_12663_amd as P
    L = P.load()
    h = torch.ones(12, device="cuda")
    out = torch.empty(12, device="cuda")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    for nx, nz, npar, sigma, half, damping in [(0, 4, 3, 1.0, 2, 1.0), (4, 1, 3, 0.0, 2, 1.0), (4, 1, 3, 1.0, -1, 1.0),
                                               (4, 1, 3, 1.0, 2, -1.0), (4, 1, 3, 1.0, 513, 1.0)]:
        assert L.bfgs_precond_diag(nx, nz, npar, ptr(h), sigma, half, damping, ptr(out), None, None, None) == -1
    assert L.bfgs_precond_diag(4, 1, 3, None, 1.0, 2, 1.0, ptr(out), None, None, None) == -1
    assert L.bfgs_precond_diag(4, 1, 3, ptr(h), 1.0, 2, 1.0, ptr(out), None, None, None) == 0
    torch.cuda.synchronize()
    assert torch.allclose(out, torch.full_like(out, 0.5))


def test_precond_beats_gamma_identity():
    """On the 600 x 200 x 3 quadratic, preconditioned CG (= exact-line-search BFGS
    from that B_0) with the smoothed, damped diagonal of A needs fewer iterations to
    a relative gradient of 1e-6 than gamma I."""
    import paper_2009_12663_amd as P
    prob = wq.make_problem("grid2", device="cuda")
    h0, _, lam = P.precond_diag(prob.diag().float(), 600, 200, 3, 1.0, 3, 0.1)

    def iters(precond):
        _, _, gn = wq.cg_pairs(prob, 1000, precond=precond, rel_tol=1e-6)
        g = np.asarray(gn) / gn[0]
        return int(np.nonzero(g <= 1e-6)[0][0])

    it_gamma, it_diag = iters(None), iters(h0.double())
    print(f"\n[precond] iterations to 1e-6: gamma I {it_gamma}, smoothed damped diagonal {it_diag} "
          f"(lambda {lam:.3g})", flush=True)
    assert it_diag < it_gamma
