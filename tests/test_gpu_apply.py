"""GPU parity of bfgs_apply_Hinv / bfgs_apply_Hdiff against the float64 oracle
(the eq. (3) recursion on the same stored inputs), plus the ABI's error behaviour."""
import numpy as np
import pytest
import torch

from oracle import recursion, dense
from oracle.probes import round_to
from workloads import quadratic as wq
from tests.helpers import TOL, rel_f, col_max_rel, gpu_input, oracle_input, h0_storage, make_pairs, gamma_of

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
    elem = col_max_rel(out, want)
    corr_err = rel_f(out - h * oracle_input(V, storage), want - h * oracle_input(V, storage))
    outd = H.apply_Hdiff(gpu_input(V, storage)).double().cpu().numpy()
    wantd, _ = oracle_apply(storage, S, Y, V, h0, diff=True)
    errd, elemd = rel_f(outd, wantd), col_max_rel(outd, wantd)
    print(f"  rel_F={err:.3e} elem={elem:.3e} correction rel_F={corr_err:.3e} diff rel_F={errd:.3e} "
          f"diff elem={elemd:.3e}", flush=True)
    assert err <= TOL[storage] and elem <= TOL[storage]
    assert errd <= TOL[storage] and elemd <= 10 * TOL[storage]
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
        assert rel_f(out, want) <= TOL[storage] and col_max_rel(out, want) <= TOL[storage]
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


def test_f32_full_size_all_columns():
    """Float32 storage on the 1700 x 350 x 3 grid (k = 200 exact-line-search pairs,
    gamma I) with 220 probe columns: every column against the oracle, element-wise."""
    print("\n[f32 full size] generating pairs", flush=True)
    P = lib()
    prob = wq.make_problem("grid3", device="cuda")
    S, Y, _ = wq.cg_pairs(prob, 200)
    n = prob.n
    del prob
    H = P.Bfgs(n, 200, None, "f32")
    for s, y in zip(S, Y):
        H.push_pair(s.float(), y.float())
    Sq = S.float().double().cpu().numpy()
    Yq = Y.float().double().cpu().numpy()
    del S, Y
    V = H.generate_probes(2, 220)
    out = H.apply_Hinv(V).double().cpu().numpy()
    assert H.get_status() == 0
    H.close()
    g = float(np.float32(gamma_of(Sq, Yq)))
    h = np.full(n, g)
    Vq = V.double().cpu().numpy()
    del V
    print("[f32 full size] oracle over 220 columns", flush=True)
    want = recursion.apply_hk(h, Sq, Yq, Vq)
    err, elem = rel_f(out, want), col_max_rel(out, want)
    corr = rel_f(out - h * Vq, want - h * Vq)
    print(f"  rel_F={err:.3e} elem={elem:.3e} correction={corr:.3e}", flush=True)
    assert err <= TOL["f32"] and elem <= TOL["f32"]


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_zero_pairs_nonfinite_is_reported(storage):
    """With no pairs the apply is B_0 V; a non-finite input still sets the deferred status."""
    P = lib()
    n = 300
    H = P.Bfgs(n, 2, gpu_input(torch.ones(n, dtype=torch.float64), storage), storage)
    V = torch.randn(3, n, dtype=torch.float64)
    out = H.apply_Hinv(gpu_input(V, storage))
    assert H.get_status() == 0
    np.testing.assert_allclose(out.double().cpu().numpy(), oracle_input(V, storage), rtol=1e-7)
    V[2, 17] = float("nan")
    H.apply_Hinv(gpu_input(V, storage))
    assert H.get_status() == P.BFGS_ERR_NONFINITE
    assert H.get_status() == 0
    H.close()


def _bf16_rne_exact(x: float) -> float:
    """Nearest bfloat16 to x (ties to even) by integer arithmetic on the exact float64
    value (normal range): x = m 2^e with 0.5 <= |m| < 1 keeps 8 significant bits."""
    import math
    if x == 0.0:
        return 0.0
    m, e = math.frexp(x)
    scaled = m * 256.0                     # exact: a power-of-two scaling
    r = round(scaled)                      # Python rounds exact halves to even
    return math.ldexp(r, e - 8)


def test_f64_input_to_bf16_storage_rounds_once():
    """float64 pairs pushed into bfloat16 storage are rounded once, to nearest-even:
    values just above a bfloat16 midpoint that a float32 intermediate would round down
    onto the midpoint (and then to even) must round up."""
    P = lib()
    n = 64
    rng = np.random.default_rng(5)
    base = rng.uniform(1.0, 2.0, n)
    base = np.floor(base * 64.0) / 64.0    # bfloat16 values with an even last bit
    # midpoint between base and the next bfloat16 up, plus a nudge below float32's resolution:
    # through float32 it lands on the midpoint and ties to the even neighbour, base
    s = base + 2.0 ** -8 + 2.0 ** -30
    s[::2] = rng.standard_normal(n // 2)
    y = s * 3.0
    H = P.Bfgs(n, 2, torch.ones(n, device="cuda"), "bf16")
    H.push_pair(torch.from_numpy(s).cuda(), torch.from_numpy(y).cuda())
    got_s, got_y = (t.double().cpu().numpy() for t in H.get_pair(0))
    want_s = np.array([_bf16_rne_exact(v) for v in s])
    want_y = np.array([_bf16_rne_exact(v) for v in y])
    np.testing.assert_array_equal(got_s, want_s)
    np.testing.assert_array_equal(got_y, want_y)
    # the double rounding would differ on the nudged entries: the test sees that case
    via_f32 = torch.from_numpy(s).float().to(torch.bfloat16).double().numpy()
    assert (via_f32 != want_s).sum() == n // 2
    H.close()


def test_apply_with_ill_conditioned_r():
    """Pairs whose scales span six orders of magnitude (s_i scaled by 10^u, u uniform in
    [-3, 3], y_i = A s_i), so R = triu(S^T Y) has curvatures from about 1e-6 to 1e6 of
    each other and a condition number near 1e12.  The inner solve goes through the
    R^-1 kept at push time; the oracle (the eq. (3) recursion) never forms R.  Float64
    storage, every column element-wise."""
    prob = wq.make_problem("tiny")
    n = prob.n
    rng = np.random.default_rng(17)
    k = 24
    S = torch.from_numpy(rng.standard_normal((k, n)) * 10.0 ** rng.uniform(-3, 3, (k, 1)))
    Y = prob.matvec(S).contiguous()
    H = build_handle("f64", S, Y)
    V = wq.normal_block(n, 31, seed=4)
    out = H.apply_Hinv(gpu_input(V, "f64")).double().cpu().numpy()
    want, _ = oracle_apply("f64", S, Y, V)
    R = np.triu(S.numpy() @ Y.numpy().T)
    err, elem = rel_f(out, want), col_max_rel(out, want)
    print(f"\n[ill-conditioned R] cond(R) {np.linalg.cond(R):.2e}: rel_F {err:.2e} elem {elem:.2e}", flush=True)
    assert np.linalg.cond(R) > 1e10
    assert elem <= TOL["f64"]          # measured 2e-15 at cond(R) = 9e11
    assert H.get_status() == 0
    H.close()
