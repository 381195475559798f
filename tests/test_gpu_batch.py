"""Batched form: independent problems of uneven n and k driven together (fork/join over
side streams, captured hipGraph), each problem checked against the float64 oracle."""
import numpy as np
import pytest
import torch

from oracle import recursion, rsvd as orsvd, probes as oprobes
from workloads import quadratic as wq
from tests.helpers import rel_f, gpu_input, oracle_input, h0_storage, make_pairs, gamma_of

pytestmark = pytest.mark.gpu
TOL = {"f32": 1e-6, "bf16": 1e-3}
SIG_TOL = {"f32": 1e-5, "bf16": 1e-3}

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
        return np.full(S.shape[1], float(np.float32(g)))
    return h0_storage(h0, storage)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_batch_parity_and_graph(storage):
    import paper_2009_12663_amd as P
    probs = [make_pairs(kind, nx, nz, k, seed=i + 3, precond=pre) for i, (kind, nx, nz, k, pre) in enumerate(SMALL)]
    ns = [p[0].n for p in probs]
    ks = [p[1].shape[0] for p in probs]
    h0s = [None if p[3] is None else gpu_input(p[3], storage) for p in probs]
    B = P.BfgsBatch(ns, ks, h0s, storage)
    for (prob, S, Y, h0), H in zip(probs, B.problems):
        for s, y in zip(S, Y):
            H.push_pair(gpu_input(s, storage), gpu_input(y, storage))
    cs = [k + 10 for k in ks]
    V = [gpu_input(wq.normal_block(n, c, seed=i), storage) for i, (n, c) in enumerate(zip(ns, cs))]
    out = B.apply_Hinv(V)
    U, Sig = B.rsvd(ks, 10, seed=5)
    torch.cuda.synchronize()
    for i, (prob, S, Y, h0) in enumerate(probs):
        h = oracle_h(storage, S, Y, h0)
        Sq, Yq = oracle_input(S, storage), oracle_input(Y, storage)
        want = recursion.apply_hk(h, Sq, Yq, oracle_input(V[i].double().cpu(), storage))
        err = rel_f(out[i].double().cpu().numpy(), want)
        X = oprobes.round_to(oprobes.normal_block(ns[i], cs[i], 5 + i), storage)
        ref = orsvd.rsvd(h, Sq, Yq, X, ks[i])
        sig = np.abs(Sig[i].cpu().numpy() - ref["Sigma"]).max() / abs(ref["Sigma"][0])
        d = B.problems[i].posterior_diag().double().cpu().numpy()
        dref = orsvd.posterior_diag(h, ref["U"], ref["Sigma"])
        derr = np.abs(d - dref).max() / np.abs(dref).max()
        print(f"\n[batch {storage}] problem {i}: n={ns[i]} k={ks[i]} apply {err:.2e} sigma {sig:.2e} diag {derr:.2e}",
              flush=True)
        assert err <= TOL[storage] and sig <= SIG_TOL[storage] and derr <= SIG_TOL[storage]
    # graph: capture apply + rsvd once, replay with eager work in between, compare every replay
    eager_out = [o.clone() for o in out]
    eager_U = [u.clone() for u in U]
    eager_S = [s.clone() for s in Sig]
    out2 = [torch.empty_like(o) for o in out]
    U2 = [torch.empty_like(u) for u in U]
    S2 = [torch.empty_like(s) for s in Sig]
    B.graph_build(V, out2, ks, 10, 5, U2, S2)
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
    # autotuning keeps results within tolerance
    tun = B.autotune(V, ks, 10)
    out3 = B.apply_Hinv(V)
    torch.cuda.synchronize()
    for a, b in zip(out3, eager_out):
        assert rel_f(a.double().cpu().numpy(), b.double().cpu().numpy()) <= TOL[storage]
    assert all(t["g1_rows"] > 0 for t in tun)
    B.close()


def test_batch_full_shapes_sampled():
    """The 64-problem batch (n log-uniform in [5e4, 1e6], k in [20, 150], rank k + 10
    oversampling) in bfloat16: apply and rSVD of every problem, graph replay, and
    oracle checks on sampled columns of four problems."""
    import paper_2009_12663_amd as P
    shapes = wq.batch_shapes()
    check = {0: None, 21: None, 42: None, 63: None}
    ns, ks = [s["n"] for s in shapes], [s["k"] for s in shapes]
    B = P.BfgsBatch(ns, ks, None, "bf16")
    for i, sh in enumerate(shapes):
        prob = wq.make_grid(sh["nx"], sh["nz"], sh["seed"], device="cuda")
        S, Y, _ = wq.cg_pairs(prob, sh["k"], rel_tol=1e-13)
        H = B.problems[i]
        for s, y in zip(S, Y):
            H.push_pair(s.float(), y.float())
        if i in check:
            check[i] = (S.float().to(torch.bfloat16).double().cpu().numpy(),
                        Y.float().to(torch.bfloat16).double().cpu().numpy())
        del S, Y
    ks = [H.k for H in B.problems]          # a history ends early if the gradient reaches rounding level
    print(f"\n[batch full] pairs pushed: k from {min(ks)} to {max(ks)}", flush=True)
    cs = [k + 10 for k in ks]
    V = [B.problems[i].generate_probes(100 + i, cs[i]) for i in range(64)]
    out = B.apply_Hinv(V)
    U, Sig = B.rsvd(ks, 10, seed=7)
    torch.cuda.synchronize()
    for i, (Sq, Yq) in check.items():
        g = float(np.float32(gamma_of(Sq, Yq)))
        cols = [0, cs[i] - 1]
        Vq = V[i][cols].double().cpu().numpy()
        want = recursion.apply_hk(np.full(ns[i], g), Sq, Yq, Vq)
        err = rel_f(out[i][cols].double().cpu().numpy(), want)
        print(f"  problem {i}: n={ns[i]} k={ks[i]} sampled apply rel_F {err:.2e}", flush=True)
        assert err <= 1e-3
    assert all(torch.isfinite(s).all() for s in Sig)
    out2 = [torch.empty_like(o) for o in out]
    U2 = [torch.empty_like(u) for u in U]
    S2 = [torch.empty_like(s) for s in Sig]
    B.graph_build(V, out2, ks, 10, 7, U2, S2)
    B.graph_launch()
    torch.cuda.synchronize()
    for a, b in zip(out2, out):
        assert torch.equal(a, b)
    for a, b in zip(S2, Sig):
        assert torch.equal(a, b)
    B.close()
