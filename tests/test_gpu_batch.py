"""Batched form: independent problems of uneven n and k driven together (persistent
work-queue passes for float32/float64 storage, fork/join over side streams otherwise,
pairs pushed by bfgs_batch_push_pairs, captured hipGraph), every problem checked
against the float64 oracle; the persistent apply equals the per-problem apply bit for
bit; the captured graph refuses to replay once a handle has changed."""
import numpy as np
import pytest
import torch

from oracle import recursion, rsvd as orsvd, probes as oprobes
from workloads import quadratic as wq
from tests.helpers import sigma_err, sigma_order_ok, rel_f, col_max_rel, gpu_input, oracle_input, h0_storage, make_pairs, gamma_of

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-12, "f32": 1e-6, "bf16": 1e-3}
SIG_TOL = {"f64": 1e-11, "f32": 1e-6, "bf16": 1e-3}

SMALL = [  # kind, nx, nz, k, diagonal B0
    ("cg", 20, 9, 12, True),
    ("secant", 33, 14, 25, False),
    ("cg", 17, 30, 40, True),
    ("secant", 45, 11, 7, False),
    ("cg", 28, 28, 33, False),
    ("secant", 13, 40, 19, True),
]


def oracle_h(storage, S, Y, h0):
    if h0 is None:
        g = gamma_of(oracle_input(S, storage), oracle_input(Y, storage))
        return np.full(S.shape[1], g if storage == "f64" else float(np.float32(g)))
    return h0_storage(h0, storage)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_persistent_apply_equals_per_problem_apply(storage):
    """The persistent passes run the per-problem kernels' tiles with the same chunking
    and fixed-order sums: the batch result is the per-problem result, bit for bit, and
    both match the oracle.  Uneven problems, including k and c past one 128 tile."""
    import paper_2009_12663_amd as P
    shapes = SMALL + [("secant", 61, 29, 150, False), ("cg", 9, 7, 3, True)]
    print(f"\n[persistent apply {storage}] {len(shapes)} problems", flush=True)
    probs = [make_pairs(kind, nx, nz, k, seed=i + 11, precond=pre) for i, (kind, nx, nz, k, pre) in enumerate(shapes)]
    ns = [p[0].n for p in probs]
    ks = [p[1].shape[0] for p in probs]
    h0s = [None if p[3] is None else gpu_input(p[3], storage) for p in probs]
    B = P.BfgsBatch(ns, ks, h0s, storage)
    assert B.push_pairs([gpu_input(p[1], storage) for p in probs], [gpu_input(p[2], storage) for p in probs]) == 0
    cs = [min(ns[i], k + 10 + 3 * i) for i, k in enumerate(ks)]
    V = [gpu_input(wq.normal_block(n, c, seed=40 + i), storage) for i, (n, c) in enumerate(zip(ns, cs))]
    out = B.apply_Hinv(V)
    torch.cuda.synchronize()
    for i, (prob, S, Y, h0) in enumerate(probs):
        single = B.problems[i].apply_Hinv(V[i])
        torch.cuda.synchronize()
        assert torch.equal(out[i], single), i
        h = oracle_h(storage, S, Y, h0)
        want = recursion.apply_hk(h, oracle_input(S, storage), oracle_input(Y, storage),
                                  oracle_input(V[i].double().cpu(), storage))
        got = out[i].double().cpu().numpy()
        err, elem = rel_f(got, want), col_max_rel(got, want)
        print(f"  problem {i}: n={ns[i]} k={ks[i]} c={cs[i]} rel_F {err:.2e} elem {elem:.2e}", flush=True)
        assert err <= TOL[storage] and elem <= TOL[storage]
    assert all(H.get_status() == 0 for H in B.problems)
    B.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_batch_parity_and_graph(storage):
    import paper_2009_12663_amd as P
    print(f"\n[batch small {storage}]", flush=True)
    probs = [make_pairs(kind, nx, nz, k, seed=i + 3, precond=pre) for i, (kind, nx, nz, k, pre) in enumerate(SMALL)]
    ns = [p[0].n for p in probs]
    ks = [p[1].shape[0] for p in probs]
    h0s = [None if p[3] is None else gpu_input(p[3], storage) for p in probs]
    B = P.BfgsBatch(ns, ks, h0s, storage)
    rc = B.push_pairs([gpu_input(p[1], storage) for p in probs], [gpu_input(p[2], storage) for p in probs])
    assert rc == 0 and [H.k for H in B.problems] == ks
    cs = [k + 10 for k in ks]
    V = [gpu_input(wq.normal_block(n, c, seed=i), storage) for i, (n, c) in enumerate(zip(ns, cs))]
    out = B.apply_Hinv(V)
    U, Sig = B.rsvd(ks, 10, seed=5)
    torch.cuda.synchronize()
    for i, (prob, S, Y, h0) in enumerate(probs):
        h = oracle_h(storage, S, Y, h0)
        Sq, Yq = oracle_input(S, storage), oracle_input(Y, storage)
        want = recursion.apply_hk(h, Sq, Yq, oracle_input(V[i].double().cpu(), storage))
        got = out[i].double().cpu().numpy()
        err, elem = rel_f(got, want), col_max_rel(got, want)
        X = oprobes.round_to(oprobes.normal_block(ns[i], cs[i], 5 + i), storage)
        ref = orsvd.rsvd(h, Sq, Yq, X, ks[i])
        sig = sigma_err(Sig[i].cpu().numpy(), ref["Sigma"])
        assert sigma_order_ok(Sig[i].cpu().numpy(), SIG_TOL[storage])
        d = B.problems[i].posterior_diag().double().cpu().numpy()
        dref = orsvd.posterior_diag(h, ref["U"], ref["Sigma"])
        derr = np.abs(d - dref).max() / np.abs(dref).max()
        print(f"  problem {i}: n={ns[i]} k={ks[i]} apply {err:.2e} elem {elem:.2e} sigma {sig:.2e} diag {derr:.2e}",
              flush=True)
        assert err <= TOL[storage] and elem <= TOL[storage]
        assert sig <= SIG_TOL[storage] and derr <= SIG_TOL[storage]
    # graph: capture apply + rsvd once, replay with eager work in between, compare every replay
    eager_out = [o.clone() for o in out]
    eager_U = [u.clone() for u in U]
    eager_S = [s.clone() for s in Sig]
    out2 = [torch.empty_like(o) for o in out]
    U2 = [torch.empty_like(u) for u in U]
    S2 = [torch.empty_like(s) for s in Sig]
    B.graph_build(V, out2, ks, 10, 5, U2, S2)

    def replay_and_compare():
        for rep in range(3):
            for o in out2:
                o.zero_()
            B.graph_launch()
            torch.cuda.synchronize()
            for a, b in zip(out2, eager_out):
                assert torch.equal(a, b)
            for a, b in zip(U2, eager_U):
                assert torch.equal(a, b)
            for a, b in zip(S2, eager_S):
                assert torch.equal(a, b)
            B.apply_Hinv(V)                    # eager work between replays
            torch.cuda.synchronize()

    replay_and_compare()
    # retuning changes launch shapes (and may grow workspaces): the graph must refuse to run
    tun = B.autotune(V, ks, 10)
    assert all(t["g1_rows"] > 0 for t in tun)
    for o in out2:
        o.fill_(7.0)
    with pytest.raises(P.BfgsError) as e:
        B.graph_launch()
    assert e.value.code == P.BFGS_ERR_STATE
    torch.cuda.synchronize()
    assert all(bool((o == 7.0).all()) for o in out2)           # nothing was launched
    with pytest.raises(P.BfgsError):
        B.graph_launch()                                      # discarded until rebuilt
    out3 = B.apply_Hinv(V)
    torch.cuda.synchronize()
    for a, b in zip(out3, eager_out):
        assert rel_f(a.double().cpu().numpy(), b.double().cpu().numpy()) <= TOL[storage]
    # rebuilt after tuning: replays match the eager results of the tuned shapes
    eager_out = [o.clone() for o in out3]
    Ue, Se = B.rsvd(ks, 10, seed=5)
    torch.cuda.synchronize()
    eager_U = [u.clone() for u in Ue]
    eager_S = [s.clone() for s in Se]
    B.graph_build(V, out2, ks, 10, 5, U2, S2)
    replay_and_compare()
    # a larger rSVD on one problem grows its workspaces: the graph must refuse to run
    H0 = B.problems[0]
    H0.rsvd(min(ns[0] - 20, 200), 20, 9)
    torch.cuda.synchronize()
    with pytest.raises(P.BfgsError) as e:
        B.graph_launch()
    assert e.value.code == P.BFGS_ERR_STATE
    B.close()


def _batch_fixture(storage):
    import paper_2009_12663_amd as P
    shapes = wq.batch_shapes()
    ns, ks = [s["n"] for s in shapes], [s["k"] for s in shapes]
    print(f"\n[batch full {storage}] building 64 problems", flush=True)
    B = P.BfgsBatch(ns, ks, None, storage)
    Ss, Ys = [], []
    for sh in shapes:
        prob = wq.make_grid(sh["nx"], sh["nz"], sh["seed"], device="cuda")
        S, Y, _ = wq.cg_pairs(prob, sh["k"], rel_tol=1e-13)
        Ss.append(S.float())
        Ys.append(Y.float())
        del prob, S, Y
    rc = B.push_pairs(Ss, Ys)
    del Ss, Ys
    assert rc == 0
    ks = [H.k for H in B.problems]          # a history ends early if the gradient reaches rounding level
    cs = [k + 10 for k in ks]
    V = [B.problems[i].generate_probes(100 + i, cs[i]) for i in range(64)]
    out = B.apply_Hinv(V)
    U, Sig = B.rsvd(ks, 10, seed=7)
    diags = [H.posterior_diag() for H in B.problems]
    torch.cuda.synchronize()
    assert all(H.get_status() == 0 for H in B.problems)
    # graph replay reproduces the eager results bit for bit
    out2 = [torch.empty_like(o) for o in out]
    U2 = [torch.empty_like(u) for u in U]
    S2 = [torch.empty_like(s) for s in Sig]
    B.graph_build(V, out2, ks, 10, 7, U2, S2)
    B.graph_launch()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(out2, out))
    assert all(torch.equal(a, b) for a, b in zip(S2, Sig))
    res = [dict(n=ns[i], k=ks[i], c=cs[i], V=V[i][[0, cs[i] - 1]].double().cpu().numpy(),
                out=out[i][[0, cs[i] - 1]].double().cpu().numpy(), Sig=Sig[i].cpu().numpy(),
                d=diags[i].double().cpu().numpy()) for i in range(64)]
    del V, out, U, Sig, diags, out2, U2, S2
    print(f"[batch full {storage}] k from {min(ks)} to {max(ks)}", flush=True)
    return B, res


@pytest.fixture(scope="module")
def batch_bf16():
    B, res = _batch_fixture("bf16")
    yield B, res
    B.close()


@pytest.fixture(scope="module")
def batch_f32():
    B, res = _batch_fixture("f32")
    yield B, res
    B.close()


def _check_quarter(fix, storage, q):
    B, res = fix
    for i in range(16 * q, 16 * q + 16):
        r = res[i]
        H = B.problems[i]
        S, Y = H.get_pairs()                     # the stored values, upcast exactly
        S, Y = S.double().cpu().numpy(), Y.double().cpu().numpy()
        h0 = H.get_h0().double().cpu().numpy()
        X = oprobes.round_to(oprobes.normal_block(r["n"], r["c"], 7 + i), storage)
        ref = orsvd.rsvd(h0, S, Y, X, r["k"])
        sig = sigma_err(r["Sig"], ref["Sigma"])
        assert sigma_order_ok(r["Sig"], SIG_TOL[storage])
        dref = orsvd.posterior_diag(h0, ref["U"], ref["Sigma"])
        derr = np.abs(r["d"] - dref).max() / np.abs(dref).max()
        want = recursion.apply_hk(h0, S, Y, r["V"])
        elem = col_max_rel(r["out"], want)
        cond_t = float(np.linalg.cond(ref["T"]))
        del S, Y, ref
        # On the bfloat16 path E carries the apply's float32-accumulation error (the
        # element-wise error just measured), which the Omega solve amplifies by up to
        # cond(Q^T X).  Histories that run past convergence leave some sketches
        # ill-conditioned; there that bound is the gate, elsewhere the path's tolerance
        # is.  The float32 path keeps E and Q in float64 and is held to 1e-6 throughout.
        gate = max(SIG_TOL[storage], 4.0 * elem * cond_t) if storage == "bf16" else SIG_TOL[storage]
        print(f"  problem {i}: n={r['n']} k={r['k']} apply elem {elem:.2e} sigma {sig:.2e} diag {derr:.2e} "
              f"cond(Q^T X) {cond_t:.3g} gate {gate:.2e}", flush=True)
        assert elem <= TOL[storage] and sig <= gate and derr <= gate


@pytest.mark.parametrize("q", range(4))
def test_batch_full_shapes_bf16(batch_bf16, q):
    """The 64-problem batch (n log-uniform in [5e4, 1e6], k in [20, 150], rank k + 10
    oversampling) in bfloat16: Sigma and the posterior diagonal of every problem, and
    two apply columns of each, against the oracle on the stored values (16 problems
    per test)."""
    _check_quarter(batch_bf16, "bf16", q)


@pytest.mark.parametrize("q", range(4))
def test_batch_full_shapes_f32(batch_f32, q):
    """The same 64-problem batch with float32 storage."""
    _check_quarter(batch_f32, "f32", q)
