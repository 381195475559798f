"""The GPU-resident BFGS driver (bfgs_minimize_quadratic) and its grid operator
(bfgs_gridop_apply) against the float64 oracle: the operator against the problem's
own definition, the iterates and gradient norms against the oracle's full-history
BFGS with exact line search (Alg. 1, eq. 1) on the same quadratic."""
import numpy as np
import pytest
import torch

from oracle import bfgs as obfgs
from workloads import quadratic as wq

pytestmark = pytest.mark.gpu


def gridop(prob):
    import paper_2009_12663_amd as P
    return P.GridOp(prob.nx, prob.nz, prob.nparam, prob.D.cuda(), prob.sigma, wq.SMOOTH_HALF, prob.coupling)


@pytest.mark.parametrize("nx,nz", [(20, 15), (7, 3), (45, 50), (1, 9)])
def test_gridop_matches_problem(nx, nz):
    prob = wq.make_grid(nx, nz, seed=nx + nz)
    op = gridop(prob)
    X = wq.normal_block(prob.n, 3, seed=1)
    got = op.apply(X.cuda()).cpu().numpy()
    want = prob.matvec(X).numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"\n[gridop] {nx}x{nz}x3: max rel err {err:.2e}", flush=True)
    assert err <= 1e-14
    op.close()


@pytest.mark.parametrize("precond", [False, True])
def test_minimize_matches_oracle_bfgs(precond):
    import paper_2009_12663_amd as P
    prob = wq.make_grid(20, 15, seed=4)
    n = prob.n
    A = prob.matvec(torch.eye(n, dtype=torch.float64)).numpy()          # dense, for the oracle
    b = prob.b.numpy()
    h0 = (1.0 / prob.diag()).numpy() if precond else None
    k = 25
    op = gridop(prob)
    H = P.Bfgs(n, k, None if h0 is None else torch.from_numpy(h0).cuda(), "f64")
    m, gn = P.minimize_quadratic(H, op, prob.b.cuda(), k, 0.0)
    assert len(gn) == k + 1 and H.k == k
    S_o, Y_o, _, m_o, gn_o = obfgs.bfgs_quadratic(A, b, k, h0=h0)
    rel = np.abs(np.array(gn) - np.array(gn_o)) / np.array(gn_o)
    m_err = np.abs(m.cpu().numpy() - m_o).max() / np.abs(m_o).max()
    S_g, Y_g = (t.cpu().numpy() for t in H.get_pairs())
    s_err = np.abs(S_g - S_o).max() / np.abs(S_o).max()
    print(f"\n[driver] precond={precond}: |g| rel err max {rel.max():.2e} (|g_k|/|g_0| = {gn[-1] / gn[0]:.2e}), "
          f"m {m_err:.2e}, pairs {s_err:.2e}", flush=True)
    assert rel[:15].max() <= 1e-9 and rel.max() <= 1e-6
    assert m_err <= 1e-9 and s_err <= 1e-8
    H.close()
    op.close()


def test_minimize_converges_and_stops():
    """float32 storage reaches a relative gradient of 1e-6 on the 600 x 200 x 3 grid in
    about as many iterations as the float64 oracle's conjugate-gradient equivalent, and
    stops there; argument and state errors are refused."""
    import paper_2009_12663_amd as P
    prob = wq.make_problem("grid2", device="cuda")
    op = gridop(prob)
    H = P.Bfgs(prob.n, 200, None, "f32")
    m, gn = P.minimize_quadratic(H, op, prob.b, 200, 1e-6)
    _, _, gn_cg = wq.cg_pairs(prob, 200, rel_tol=1e-6)
    it, it_cg = len(gn) - 1, len(gn_cg) - 1
    print(f"\n[driver] grid2 f32: {it} iterations to 1e-6 (float64 CG: {it_cg})", flush=True)
    assert gn[-1] <= 1e-6 * gn[0] and abs(it - it_cg) <= 2 and H.k == it
    r = prob.matvec(m) - prob.b
    assert float(torch.linalg.vector_norm(r)) <= 2e-6 * gn[0]
    with pytest.raises(P.BfgsError) as e:
        P.minimize_quadratic(H, op, prob.b, 5, 0.0)          # history not empty
    assert e.value.code == P.BFGS_ERR_STATE
    Hb = P.Bfgs(prob.n, 4, None, "bf16")
    with pytest.raises(P.BfgsError) as e:
        P.minimize_quadratic(Hb, op, prob.b, 5, 0.0)
    assert e.value.code == P.BFGS_ERR_ARG
    Hb.close()
    H.close()
    op.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_pop_oldest_is_the_shorter_history(storage):
    """bfgs_pop_oldest: after forgetting the two oldest of seven pairs the handle applies
    the inverse Hessian of the last five (against the eq. (3) recursion over them and
    against a handle that only ever held them, same B_0); with B_0 = gamma I the gamma of
    the first pair stays; popping every pair leaves B_0; errors."""
    import paper_2009_12663_amd as P
    from oracle import recursion
    from tests.helpers import TOL, col_max_rel, gpu_input, oracle_input, h0_storage, make_pairs, gamma_of
    prob, S, Y, h0 = make_pairs("secant", 17, 11, 7, seed=3, precond=True)
    n = prob.n
    V = wq.normal_block(n, 9, seed=2)
    Vg = gpu_input(V, storage)
    Sq, Yq, Vq = oracle_input(S, storage), oracle_input(Y, storage), oracle_input(V, storage)
    for gamma in (False, True):
        hg = None if gamma else gpu_input(h0, storage)
        H = P.Bfgs(n, 7, hg, storage)
        for s, y in zip(S, Y):
            H.push_pair(gpu_input(s, storage), gpu_input(y, storage))
        H.pop_oldest()
        H.pop_oldest()
        assert H.k == 5
        h = (np.full(n, gamma_of(Sq, Yq) if storage == "f64" else float(np.float32(gamma_of(Sq, Yq))))
             if gamma else h0_storage(h0, storage))
        got = H.apply_Hinv(Vg).double().cpu().numpy()
        want = recursion.apply_hk(h, Sq[2:], Yq[2:], Vq)
        err = col_max_rel(got, want)
        print(f"\n[pop] {storage} gamma={gamma}: after two pops elem err {err:.2e}", flush=True)
        assert err <= TOL[storage]
        if not gamma:
            R = P.Bfgs(n, 5, hg, storage)
            for s, y in zip(S[2:], Y[2:]):
                R.push_pair(gpu_input(s, storage), gpu_input(y, storage))
            assert col_max_rel(got, R.apply_Hinv(Vg).double().cpu().numpy()) <= TOL[storage]
            R.close()
        # a pushed pair lands after the window, then everything can be forgotten
        H.push_pair(gpu_input(S[0], storage), gpu_input(Y[0], storage))
        got = H.apply_Hinv(Vg).double().cpu().numpy()
        want = recursion.apply_hk(h, np.concatenate([Sq[2:], Sq[:1]]), np.concatenate([Yq[2:], Yq[:1]]), Vq)
        assert col_max_rel(got, want) <= TOL[storage]
        for _ in range(6):
            H.pop_oldest()
        assert H.k == 0
        got = H.apply_Hinv(Vg).double().cpu().numpy()
        assert col_max_rel(got, h[None, :] * Vq) <= TOL[storage]
        with pytest.raises(P.BfgsError) as e:
            H.pop_oldest()
        assert e.value.code == P.BFGS_ERR_STATE
        H.close()
    Hb = P.Bfgs(n, 4, None, "bf16")
    Hb.push_pair(S[0].float().cuda(), Y[0].float().cuda())
    with pytest.raises(P.BfgsError) as e:
        Hb.pop_oldest()
    assert e.value.code == P.BFGS_ERR_ARG
    Hb.close()


def test_minimize_limited_memory_matches_oracle():
    """bfgs_minimize_quadratic_ex with the last five pairs and half steps: the gradient
    norms, the iterate and the stored window against the oracle's limited-memory BFGS
    (same fixed B_0, same damped line search); full memory with the same steps differs.
    Out-of-range memory and damping are refused."""
    import paper_2009_12663_amd as P
    prob = wq.make_grid(20, 15, seed=4)
    n = prob.n
    A = prob.matvec(torch.eye(n, dtype=torch.float64)).numpy()
    b = prob.b.numpy()
    h0 = (1.0 / prob.diag()).numpy()
    k, mem, damp = 30, 5, 0.5
    op = gridop(prob)
    H = P.Bfgs(n, mem, torch.from_numpy(h0).cuda(), "f64")
    m, gn = P.minimize_quadratic(H, op, prob.b.cuda(), k, 0.0, memory=mem, damping=damp)
    assert len(gn) == k + 1 and H.k == mem
    S_o, Y_o, _, m_o, gn_o = obfgs.bfgs_quadratic(A, b, k, h0=h0, damping=damp, memory=mem)
    rel = np.abs(np.array(gn) - np.array(gn_o)) / np.array(gn_o)
    m_err = np.abs(m.cpu().numpy() - m_o).max() / np.abs(m_o).max()
    S_g, _ = (t.cpu().numpy() for t in H.get_pairs())
    s_err = np.abs(S_g - S_o[-mem:]).max() / np.abs(S_o[-mem:]).max()
    _, _, _, _, gn_full = obfgs.bfgs_quadratic(A, b, k, h0=h0, damping=damp)
    print(f"\n[driver L-BFGS({mem}), steps x{damp}] |g| rel err max {rel.max():.2e}, m {m_err:.2e}, window {s_err:.2e}; "
          f"|g_k|/|g_0| {gn[-1] / gn[0]:.2e} (full memory {gn_full[-1] / gn_full[0]:.2e})", flush=True)
    assert rel.max() <= 1e-8 and m_err <= 1e-9 and s_err <= 1e-8
    assert abs(gn_full[-1] - gn_o[-1]) > 1e-3 * gn_o[-1]
    H.close()
    H = P.Bfgs(n, 3, None, "f64")
    for mem_bad, damp_bad in ((4, 1.0), (-1, 1.0), (2, 0.0), (2, 1.5)):
        with pytest.raises(P.BfgsError) as e:
            P.minimize_quadratic(H, op, prob.b.cuda(), 3, 0.0, memory=mem_bad, damping=damp_bad)
        assert e.value.code == P.BFGS_ERR_ARG
    H.close()
    op.close()
