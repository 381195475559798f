"""GPU parity of the rSVD variants (bfgs_rsvd_ex): the B_0-whitened difference
B_0^-1/2 (B_k - B_0) B_0^-1/2 (eigenvalues of B_k B_0^-1 - I, the paper's "starts from
the identity" view) and Halko's two-pass Q^T A Q form, against the float64 oracle on
the same stored pairs and probes."""
import numpy as np
import pytest
import torch

from oracle import rsvd as orsvd, probes as oprobes, dense
from workloads import quadratic as wq
from tests.helpers import sigma_err, sigma_order_ok, gpu_input, oracle_input, h0_storage, make_pairs, gamma_of

pytestmark = pytest.mark.gpu
SIG_TOL = {"f64": 1e-11, "f32": 1e-6, "bf16": 1e-3}

CASES = [
    # storage, kind, nx, nz, k, rank, p, precond, two_pass
    ("f64", "secant", 12, 9, 12, 24, 6, True, False),
    ("f64", "cg", 20, 15, 30, 30, 10, True, True),
    ("f64", "secant", 12, 9, 12, 24, 6, False, True),
    ("f32", "cg", 40, 30, 30, 30, 10, True, False),
    ("f32", "secant", 33, 17, 20, 40, 8, False, True),
    ("f32", "cg", 61, 29, 60, 60, 20, True, True),
    ("bf16", "cg", 40, 30, 30, 30, 10, True, False),
    ("bf16", "secant", 45, 23, 25, 40, 12, True, True),
    ("bf16", "cg", 53, 19, 45, 45, 10, False, True),
]


@pytest.mark.parametrize("storage,kind,nx,nz,k,rank,p,precond,two_pass", CASES)
def test_rsvd_variant_parity(storage, kind, nx, nz, k, rank, p, precond, two_pass):
    import paper_2009_12663_amd as P
    print(f"\n[rsvd variant] {storage} {kind} n={3 * nx * nz} k={k} rank={rank} p={p} precond={precond} "
          f"two_pass={two_pass}", flush=True)
    prob, S, Y, h0 = make_pairs(kind, nx, nz, k, seed=k + 3, precond=True)   # a diagonal B_0 to whiten with
    n = prob.n
    H = P.Bfgs(n, S.shape[0], gpu_input(h0, storage), storage)
    for s, y in zip(S, Y):
        H.push_pair(gpu_input(s, storage), gpu_input(y, storage))
    seed = 13
    U, Sig = H.rsvd_ex(rank, p, seed, precond=precond, two_pass=two_pass)
    d = H.posterior_diag().double().cpu().numpy()
    assert H.get_status() == 0
    Ud = U.double().cpu().numpy()
    Sig = Sig.cpu().numpy()
    H.close()
    h = h0_storage(h0, storage)
    Sq, Yq = oracle_input(S, storage), oracle_input(Y, storage)
    X = oprobes.round_to(oprobes.normal_block(n, rank + p, seed), storage)
    if two_pass:
        ref = orsvd.rsvd_two_pass(h, Sq, Yq, X, rank, precond=precond)
    elif precond:
        ref = orsvd.rsvd_precond(h, Sq, Yq, X, rank)
    else:
        ref = orsvd.rsvd(h, Sq, Yq, X, rank)
    dref = (orsvd.posterior_diag_precond if precond else orsvd.posterior_diag)(h, ref["U"], ref["Sigma"])
    sig = sigma_err(Sig, ref["Sigma"])
    dmax = np.abs(d - dref).max() / np.abs(dref).max()
    orth = np.abs(Ud @ Ud.T - np.eye(rank)).max()
    print(f"  sigma {sig:.2e} diag_max {dmax:.2e} orth {orth:.2e}", flush=True)
    tol = SIG_TOL[storage]
    assert sigma_order_ok(Sig, tol)
    assert sig <= tol and dmax <= tol
    assert orth <= (1e-12 if storage == "f64" else 1e-5)


def test_precond_sigma_is_bk_b0inv_minus_identity_on_the_gpu():
    """Tiny float64 problem with rank = 2k >= rank(B_k - B_0) (a general diagonal B_0
    leaves the difference of rank up to 2k): the whitened Sigma are the eigenvalues of
    B_k B_0^-1 - I of the dense eq. (3) matrix, and both variants reconstruct B_k."""
    import paper_2009_12663_amd as P
    prob = wq.make_problem("tiny")
    k = 20
    S, Y, _ = wq.cg_pairs(prob, k)
    rng = np.random.default_rng(2)
    h0 = rng.uniform(0.5, 2.0, 300)
    Bk = dense.inverse_hessian(h0, S.numpy(), Y.numpy())
    ev = np.linalg.eigvals(Bk @ np.diag(1.0 / h0) - np.eye(300)).real
    ev = ev[np.argsort(-np.abs(ev))][:2 * k]
    for two_pass in (False, True):
        H = P.Bfgs(300, k, torch.from_numpy(h0).cuda(), "f64")
        for s, y in zip(S, Y):
            H.push_pair(s.cuda(), y.cuda())
        U, Sig = H.rsvd_ex(2 * k, 9, 0, precond=True, two_pass=two_pass)
        U, Sig = U.cpu().numpy(), Sig.cpu().numpy()
        d = H.posterior_diag().cpu().numpy()
        H.close()
        np.testing.assert_allclose(np.sort(Sig), np.sort(ev), rtol=0, atol=1e-11 * abs(ev[0]))
        W = np.sqrt(h0)[:, None] * U.T
        rec = np.diag(h0) + (W * Sig) @ W.T
        assert np.abs(rec - Bk).max() <= 1e-10 * np.abs(Bk).max()
        np.testing.assert_allclose(d, np.diag(Bk), rtol=1e-10)


def test_rsvd_ex_rejects_unknown_flags():
    import paper_2009_12663_amd as P
    prob, S, Y, h0 = make_pairs("cg", 8, 8, 4, seed=3)
    H = P.Bfgs(prob.n, 4, None, "f32")
    for s, y in zip(S, Y):
        H.push_pair(s.float().cuda(), y.float().cuda())
    U = torch.empty(4, prob.n, device="cuda")
    Sg = torch.empty(4, dtype=torch.float64, device="cuda")
    assert H.L.bfgs_rsvd_ex(H.h, 4, 2, 0, 4, U.data_ptr(), Sg.data_ptr()) == P.BFGS_ERR_ARG
    H.close()
