"""Out-of-core histories (bfgs_create_streamed): pairs in pinned host memory, streamed
to the device in row slices for every pass.  Apply, difference, rSVD and posterior
variance against the float64 oracle on the same stored values, and against a
device-resident handle of the same pairs; slice sizes that leave a ragged last slice,
one slice, and slices of a single row block."""
import numpy as np
import pytest
import torch

from oracle import recursion, rsvd as orsvd, probes as oprobes
from workloads import quadratic as wq
from tests.helpers import (TOL, rel_f, col_max_rel, sigma_err, sigma_order_ok, gpu_input, oracle_input, h0_storage,
                           make_pairs, gamma_of)

pytestmark = pytest.mark.gpu
SIG_TOL = {"f64": 1e-11, "f32": 1e-6}


def build(storage, S, Y, h0, slice_rows):
    import paper_2009_12663_amd as P
    n = S.shape[1]
    H = P.Bfgs(n, S.shape[0], None if h0 is None else gpu_input(h0, storage), storage, slice_rows=slice_rows)
    for s, y in zip(S, Y):
        H.push_pair(gpu_input(s, storage), gpu_input(y, storage))
    return H


def oracle_h(storage, S, Y, h0):
    if h0 is None:
        g = gamma_of(oracle_input(S, storage), oracle_input(Y, storage))
        return np.full(S.shape[1], g if storage == "f64" else float(np.float32(g)))
    return h0_storage(h0, storage)


CASES = [
    # storage, kind, nx, nz, k, ncols, precond, slice_rows
    ("f64", "cg", 20, 15, 30, 41, True, 250),       # 900 rows: 4 slices, last 150
    ("f64", "secant", 13, 9, 12, 17, False, 10**6),  # one slice
    ("f32", "cg", 40, 30, 25, 70, False, 1000),     # 3600 rows: 4 slices, last 600
    ("f32", "secant", 33, 17, 20, 33, True, 128),   # 1683 rows: 14 slices of one row block
]


@pytest.mark.parametrize("storage,kind,nx,nz,k,c,precond,slice_rows", CASES)
def test_streamed_apply_and_rsvd(storage, kind, nx, nz, k, c, precond, slice_rows):
    print(f"\n[streamed] {storage} {kind} n={3 * nx * nz} k={k} c={c} slice_rows={slice_rows}", flush=True)
    prob, S, Y, h0 = make_pairs(kind, nx, nz, k, seed=k + 5, precond=precond)
    n = prob.n
    H = build(storage, S, Y, h0, slice_rows)
    R = build(storage, S, Y, h0, None)
    assert H.k == R.k == S.shape[0]
    h = oracle_h(storage, S, Y, h0)
    Sq, Yq = oracle_input(S, storage), oracle_input(Y, storage)
    # the stored pairs read back from host memory are the device handle's
    for j in (0, H.k - 1):
        a, b = H.get_pair(j), R.get_pair(j)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    V = wq.normal_block(n, c, seed=c)
    Vg = gpu_input(V, storage)
    out = H.apply_Hinv(Vg).double().cpu().numpy()
    outd = H.apply_Hdiff(Vg).double().cpu().numpy()
    ref_dev = R.apply_Hinv(Vg).double().cpu().numpy()
    want = recursion.apply_hk(h, Sq, Yq, oracle_input(V, storage))
    wantd = recursion.apply_hk(h, Sq, Yq, oracle_input(V, storage), subtract_b0=True)
    err, elem = rel_f(out, want), col_max_rel(out, want)
    errd, elemd = rel_f(outd, wantd), col_max_rel(outd, wantd)
    dev = col_max_rel(out, ref_dev)
    print(f"  apply rel_F {err:.2e} elem {elem:.2e}; diff rel_F {errd:.2e} elem {elemd:.2e}; "
          f"vs device-resident {dev:.2e}", flush=True)
    assert err <= TOL[storage] and elem <= TOL[storage]
    assert errd <= TOL[storage] and elemd <= 10 * TOL[storage]
    assert dev <= TOL[storage]
    # rSVD and the posterior variance through the streamed range sample
    rank, p, seed = min(k + 5, n // 4), 8, 21
    U, Sig = H.rsvd(rank, p, seed)
    d = H.posterior_diag().double().cpu().numpy()
    assert H.get_status() == 0
    Sig = Sig.cpu().numpy()
    U = U.double().cpu().numpy()
    X = oprobes.round_to(oprobes.normal_block(n, rank + p, seed), storage)
    ref = orsvd.rsvd(h, Sq, Yq, X, rank)
    dref = orsvd.posterior_diag(h, ref["U"], ref["Sigma"])
    sig = sigma_err(Sig, ref["Sigma"])
    dmax = np.abs(d - dref).max() / np.abs(dref).max()
    orth = np.abs(U @ U.T - np.eye(rank)).max()
    print(f"  rsvd sigma {sig:.2e} diag_max {dmax:.2e} orth {orth:.2e}", flush=True)
    assert sigma_order_ok(Sig, SIG_TOL[storage])
    assert sig <= SIG_TOL[storage] and dmax <= SIG_TOL[storage]
    assert orth <= (1e-12 if storage == "f64" else 1e-5)
    H.close()
    R.close()


def test_streamed_gamma_mode_and_errors():
    import paper_2009_12663_amd as P
    prob, S, Y, _ = make_pairs("cg", 12, 11, 9, seed=4)
    n = prob.n
    H = build("f32", S, Y, None, 100)            # B_0 = gamma I from the first pair
    R = build("f32", S, Y, None, None)
    assert torch.equal(H.get_h0(), R.get_h0())
    V = gpu_input(wq.normal_block(n, 5, seed=3), "f32")
    a = H.apply_Hinv(V).double().cpu().numpy()
    b = R.apply_Hinv(V).double().cpu().numpy()
    assert col_max_rel(a, b) <= TOL["f32"]
    # no workspace-free apply on a streamed handle
    from paper_2009_12663_amd._lib import _ptr
    out = torch.empty_like(V)
    assert H.L.bfgs_apply_Hinv_noalloc(H.h, _ptr(V), 5, _ptr(out)) == P.BFGS_ERR_STATE
    H.close()
    R.close()
    with pytest.raises(P.BfgsError) as e:
        P.Bfgs(n, 4, None, "bf16", slice_rows=64)
    assert e.value.code == P.BFGS_ERR_ARG
    with pytest.raises(P.BfgsError) as e:
        P.Bfgs(n, 4, None, "f32", slice_rows=0)
    assert e.value.code == P.BFGS_ERR_ARG
