"""The allocation-free apply (bfgs_apply_Hinv_noalloc) against bfgs_apply_Hinv through
the C ABI: two calls in a row on one handle, the second with a smaller block, for
every storage type, to the tolerance of each storage's path."""
import ctypes

import numpy as np
import pytest
import torch

from workloads import quadratic as wq
from tests.helpers import TOL, rel_f, col_max_rel, gpu_input, make_pairs

pytestmark = pytest.mark.gpu


def _noalloc(H, V, out):
    return H.L.bfgs_apply_Hinv_noalloc(H.h, ctypes.c_void_p(V.data_ptr()), V.shape[0],
                                       ctypes.c_void_p(out.data_ptr()))


CASES = [
    # storage, kind, nx, nz, k, c1, c2, diagonal B0
    ("bf16", "cg", 60, 40, 200, 220, 37, False),
    ("bf16", "secant", 41, 23, 47, 128, 1, True),
    ("f32", "secant", 40, 30, 60, 256, 100, True),
    ("f64", "cg", 20, 15, 30, 50, 7, False),
]


@pytest.mark.parametrize("storage,kind,nx,nz,k,c1,c2,precond", CASES)
def test_noalloc_matches_apply(storage, kind, nx, nz, k, c1, c2, precond):
    import paper_2009_12663_amd as P
    print(f"\n[noalloc] {storage} {kind} n={3 * nx * nz} k={k} c={c1} then {c2}", flush=True)
    prob, S, Y, h0 = make_pairs(kind, nx, nz, k, seed=k + 2, precond=precond)
    H = P.Bfgs(prob.n, S.shape[0], None if h0 is None else gpu_input(h0, storage), storage)
    for s, y in zip(S, Y):
        H.push_pair(gpu_input(s, storage), gpu_input(y, storage))
    for c in (c1, c2):
        V = H._block(gpu_input(wq.normal_block(prob.n, c, seed=c), storage))
        want = H.apply_Hinv(V)
        got = torch.full_like(want, float("nan"))
        assert _noalloc(H, V, got) == 0
        torch.cuda.synchronize()
        g, w = got.double().cpu().numpy(), want.double().cpu().numpy()
        err, elem = rel_f(g, w), col_max_rel(g, w)
        print(f"  c={c}: rel_F {err:.2e} elem {elem:.2e}", flush=True)
        assert err <= TOL[storage] and elem <= TOL[storage]
    assert H.get_status() == 0
    # argument errors are refused before anything runs
    V = torch.zeros((2, prob.n), dtype=H.sdt, device="cuda")
    assert _noalloc(H, V, V) == P.BFGS_ERR_ARG
    H.close()
