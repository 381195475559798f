"""GPU parity of bfgs_apply_Hinv / bfgs_apply_Hdiff against the float64 oracle
(the eq. (3) recursion on the same stored inputs), plus the ABI's error behaviour."""
import numpy as np
import pytest
import torch

from oracle import recursion, dense
from oracle.probes import round_to
from workloads import quadratic as wq
from tests.helpers import TOL, rel_f, gpu_input, oracle_input, h0_storage, make_pairs, gamma_of

pytestmark = pytest.mark.gpu


def lib():
    import paper_2009_12663_amd as P
    return P


def build_handle(storage, S, Y, h0=None, k_max=None):
    P = lib()
    n = S.shape[1]
    H = P.Bfgs(n, k_max or max(1, S.shape[0]), None if h0 is None else gpu_input(h0, storage), storage)
    for s, y in zip(S, Y):
        H.push_pair(gpu_input(s, storage), gpu_input(y, storage))
    return H


def oracle_apply(storage, S, Y, V, h0=None, diff=False):
    Sq, Yq, Vq = oracle_input(S, storage), oracle_input(Y, storage), oracle_input(V, storage)
    if h0 is None:
        g = gamma_of(Sq, Yq)
        h = np.full(S.shape[1], g if storage == "f64" else float(np.float32(g)))
    else:
        h = h0_storage(h0, storage)
    return recursion.apply_hk(h, Sq, Yq, Vq, subtract_b0=diff), h


CASES = [
    # storage, pair kind, nx, nz, k, ncols, precond
    ("f64", "cg", 10, 10, 40, 50, False),
    ("f64", "secant", 13, 7, 17, 33, True),
    ("f32", "secant", 40, 30, 23, 70, True),
    ("f32", "cg", 37, 21, 31, 129, False),
    ("bf16", "secant", 40, 30, 23, 70, True),
    ("bf16", "cg", 53, 19, 45, 220, False),
]


@pytest.mark.parametrize("storage,kind,nx,nz,k,c,precond", CASES)
def test_apply_parity(storage, kind, nx, nz, k, c, precond):
    print(f"\n[apply parity] {storage} {kind} n={3*nx*nz} k={k} c={c}", flush=True)
    prob, S, Y, h0 = make_pairs(kind, nx, nz, k, seed=k, precond=precond)
    H = build_handle(storage, S, Y, h0)
    assert H.k == S.shape[0]
    V = wq.normal_block(prob.n, c, seed=c)
    out = H.apply_Hinv(gpu_input(V, storage)).double().cpu().numpy()
    want, h = oracle_apply(storage, S, Y, V, h0)
    err = rel_f(out, want)
    corr_err = rel_f(out - h * oracle_input(V, storage), want - h * oracle_input(V, storage))
    print(f"  rel_F={err:.3e}  correction rel_F={corr_err:.3e}", flush=True)
    assert err <= TOL[storage]
    outd = H.apply_Hdiff(gpu_input(V, storage)).double().cpu().numpy()
    wantd, _ = oracle_apply(storage, S, Y, V, h0, diff=True)
    assert rel_f(outd, wantd) <= 10 * TOL[storage]
    assert H.get_status() == 0
    H.close()


def test_apply_f64_matches_dense_eq3():
    prob = wq.make_problem("tiny")
    S, Y, _ = wq.cg_pairs(prob, 40)
    H = build_handle("f64", S, Y)
    g = float(S[0] @ Y[0] / (Y[0] @ Y[0]))
    B = dense.inverse_hessian(np.full(300, g), S.numpy(), Y.numpy())
    eye = torch.eye(300, dtype=torch.float64, device="cuda")
    out = torch.cat([H.apply_Hinv(eye[:150]), H.apply_Hinv(eye[150:])]).cpu().numpy()
    assert np.abs(out - B).max() <= 1e-12 * np.abs(B).max()
    # secant and symmetry of the GPU operator itself
    assert np.abs(out - out.T).max() <= 1e-13 * np.abs(B).max()
    Hy = H.apply_Hinv(Y[-1:].cuda()).cpu().numpy()[0]
    assert np.abs(Hy - S[-1].numpy()).max() <= 1e-12 * np.abs(S[-1].numpy()).max()
    H.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_edge_shapes(storage):
    """k = 0, a single column, the maximum column count and a ragged n."""
    P = lib()
    prob, S, Y, h0 = make_pairs("secant", 7, 11, 5, seed=1, precond=True)
    n = prob.n                                              # 231: ragged against every tile
    H = P.Bfgs(n, 8, gpu_input(h0, storage), storage)
    V = wq.normal_block(n, 256, seed=3)
    out0 = H.apply_Hinv(gpu_input(V, storage)).double().cpu().numpy()
    np.testing.assert_allclose(out0, oracle_input(V, storage) * h0_storage(h0, storage), rtol=1e-7)
    assert np.abs(H.apply_Hdiff(gpu_input(V[:3], storage)).double().cpu().numpy()).max() == 0.0
    for s, y in zip(S, Y):
        H.push_pair(gpu_input(s, storage), gpu_input(y, storage))
    for c in (1, 256):
        out = H.apply_Hinv(gpu_input(V[:c], storage)).double().cpu().numpy()
        want, _ = oracle_apply(storage, S, Y, V[:c], h0)
        assert rel_f(out, want) <= TOL[storage]
    H.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_stored_pairs_are_rne_and_gamma(storage):
    P = lib()
    prob, S, Y, _ = make_pairs("cg", 9, 8, 3, seed=2)
    H = build_handle(storage, S, Y)
    for j in range(3):
        s, y = H.get_pair(j)
        want_s = torch.from_numpy(S[j].numpy()).float()
        if storage == "bf16":
            want_s = want_s.to(torch.bfloat16).float()
        assert torch.equal(s.cpu(), want_s)
    g = gamma_of(oracle_input(S, storage), oracle_input(Y, storage))
    h0 = H.get_h0().cpu()
    assert torch.all(h0 == torch.tensor(np.float32(g)))
    H.close()


def test_errors_and_recovery():
    P = lib()
    prob, S, Y, _ = make_pairs("cg", 8, 8, 4, seed=3)
    H = P.Bfgs(prob.n, 3, None, "f32")
    x = torch.zeros(2, prob.n, device="cuda")
    with pytest.raises(P.BfgsError) as e:
        H.apply_Hinv(x)                          # gamma not known before the first pair
    assert e.value.code == -3
    with pytest.raises(P.BfgsError) as e:
        H.push_pair(gpu_input(S[0], "f32"), gpu_input(-Y[0], "f32"))
    assert e.value.code == -4 and H.k == 0
    bad = gpu_input(S[0], "f32").clone()
    bad[5] = float("nan")
    with pytest.raises(P.BfgsError) as e:
        H.push_pair(bad, gpu_input(Y[0], "f32"))
    assert e.value.code == -5 and H.k == 0
    for j in range(3):
        H.push_pair(gpu_input(S[j], "f32"), gpu_input(Y[j], "f32"))
    with pytest.raises(P.BfgsError) as e:
        H.push_pair(gpu_input(S[3], "f32"), gpu_input(Y[3], "f32"))
    assert e.value.code == -2 and H.k == 3
    V = torch.randn(4, prob.n, device="cuda")
    out_buf = torch.empty(257, prob.n, device="cuda")
    for c in (0, 257, -1):
        assert H.L.bfgs_apply_Hinv(H.h, V.data_ptr(), c, out_buf.data_ptr()) == -1
    assert H.L.bfgs_apply_Hinv(H.h, V.data_ptr(), 2, V.data_ptr()) == -1       # out aliases V
    assert H.L.bfgs_apply_Hinv(H.h, None, 2, out_buf.data_ptr()) == -1
    with pytest.raises(P.BfgsError) as e:
        H.posterior_diag()
    assert e.value.code == -3
    # the handle still works and matches the oracle after the rejected pushes
    out = H.apply_Hinv(V).double().cpu().numpy()
    want, _ = oracle_apply("f32", S[:3], Y[:3], V.double().cpu())
    assert rel_f(out, want) <= 1e-6
    Vn = V.clone()
    Vn[1, 7] = float("inf")
    H.apply_Hinv(Vn)
    assert H.get_status() == -5
    assert H.get_status() == 0
    H.close()
    with pytest.raises(P.BfgsError):
        P.Bfgs(0, 3)
    with pytest.raises(P.BfgsError):
        P.Bfgs(10, 0)


def test_apply_is_deterministic():
    prob, S, Y, h0 = make_pairs("secant", 30, 20, 20, seed=4, precond=True)
    H = build_handle("bf16", S, Y, h0)
    V = gpu_input(wq.normal_block(prob.n, 64, seed=1), "bf16")
    a = H.apply_Hinv(V)
    b = H.apply_Hinv(V)
    assert torch.equal(a, b)
    H.close()
