"""Seeded synthetic quadratic problems and the inputs derived from them.

The paper obtains its (s_i, y_i) pairs from elastic full-waveform inversion of
the Marmousi model (Numerical examples, 2D elastic Marmousi benchmark).  That
model, the wave solver and the data are not available, so every input here is
a seeded synthetic stand-in with the same structure: a model vector made of
three parameter fields on a 2-D grid, an SPD operator A playing the Hessian,
and an optimizer trajectory on f(m) = 1/2 m^T A m - b^T m.

Layout conventions (shared with the GPU binding and the oracle):
  * a model vector has index (param * nz + iz) * nx + ix (field-major);
  * a block of ncols vectors is a torch tensor of shape (ncols, n), i.e. a
    column-major n x ncols matrix whose column j is row j of the tensor.

Everything is float64 and works on any torch device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

# ----------------------------------------------------------------------------
# Configurations.  Grid sizes, pair counts, ranks and oversampling follow the
# five workload descriptions (tiny dense problem; 600x200x3 grid; 1700x350x3
# grid; 64-problem batch; learned-preconditioner study).
# ----------------------------------------------------------------------------
CONFIGS = {
    "tiny": dict(kind="dense", n=300, nlow=8, k=40, rank=40, oversample=10, seed=0),
    "grid2": dict(kind="grid", nx=600, nz=200, k=100, rank=100, oversample=20, seed=0),
    "grid3": dict(kind="grid", nx=1700, nz=350, k=200, rank=200, oversample=20, seed=1),
}

SMOOTH_SIGMA = 5.0      # cells
SMOOTH_HALF = 20        # taps on each side of the centre
DIAG_LOG_STD = 0.5      # D = exp(N(0, 0.5^2))
COUPLING = 0.1          # off-diagonal cross-parameter coupling


def gaussian_taps(sigma: float = SMOOTH_SIGMA, half: int = SMOOTH_HALF) -> np.ndarray:
    """Normalised (sum 1) truncated Gaussian smoothing kernel."""
    x = np.arange(-half, half + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return w / w.sum()


@dataclass
class GridQuadratic:
    """A = diag(D) + P (x) (G_z (x) G_x) on nparam fields of an nz x nx grid.

    D is lognormal, G_x / G_z are truncated Gaussian smoothers with zero
    boundary, P = I + c (11^T - I) couples the parameter fields.  A is SPD.
    """

    nx: int
    nz: int
    D: torch.Tensor            # (n,) float64
    b: torch.Tensor            # (n,) float64
    nparam: int = 3
    sigma: float = SMOOTH_SIGMA
    coupling: float = COUPLING
    _taps: torch.Tensor = field(default=None, repr=False)

    def __post_init__(self):
        t = torch.as_tensor(gaussian_taps(self.sigma), dtype=torch.float64, device=self.D.device)
        self._taps = t.view(1, 1, -1)
        p = torch.full((self.nparam, self.nparam), self.coupling, dtype=torch.float64, device=self.D.device)
        p.fill_diagonal_(1.0)
        self.P = p
        self._Gx = self._banded(self.nx)
        self._Gz = self._banded(self.nz)

    def _banded(self, m: int) -> torch.Tensor:
        """Dense m x m matrix of the truncated smoother with zero boundary (symmetric Toeplitz)."""
        taps = self._taps.view(-1)
        half = taps.numel() // 2
        idx = torch.arange(m, device=taps.device)
        off = idx.view(-1, 1) - idx.view(1, -1)
        G = torch.zeros(m, m, dtype=torch.float64, device=taps.device)
        band = off.abs() <= half
        G[band] = taps[(off[band] + half)]
        return G

    @property
    def n(self) -> int:
        return self.nparam * self.nz * self.nx

    @property
    def device(self):
        return self.D.device

    def _smooth(self, x: torch.Tensor) -> torch.Tensor:
        """x: (B, nparam, nz, nx) -> separable Gaussian smoothing of each field
        (G_z X G_x with the symmetric banded smoothers)."""
        y = torch.matmul(x, self._Gx)
        return torch.matmul(self._Gz, y)

    def matvec(self, x: torch.Tensor) -> torch.Tensor:
        """A x for x of shape (n,) or (ncols, n)."""
        single = x.dim() == 1
        xb = x.reshape(-1, self.nparam, self.nz, self.nx).to(torch.float64)
        g = self._smooth(xb)
        coupled = torch.einsum("pq,bqzx->bpzx", self.P, g)
        out = coupled.reshape(xb.shape[0], -1) + self.D * xb.reshape(xb.shape[0], -1)
        return out[0] if single else out

    def diag(self) -> torch.Tensor:
        """Exact diagonal of A: D + P_pp * g_0^2-weighted smoother diagonal."""
        taps = self._taps.view(-1)
        half = taps.numel() // 2
        centre = float(taps[half])
        # smoother diagonal is centre_x * centre_z everywhere (zero boundary keeps it)
        return self.D + centre * centre

    def depth_index(self) -> torch.Tensor:
        iz = torch.arange(self.nz, device=self.device, dtype=torch.float64)
        return iz.view(1, self.nz, 1).expand(self.nparam, self.nz, self.nx).reshape(-1)


@dataclass
class DenseQuadratic:
    """A = diag(D) + U U^T, held densely (small n only)."""

    A: torch.Tensor
    b: torch.Tensor
    D: torch.Tensor

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def device(self):
        return self.A.device

    def matvec(self, x: torch.Tensor) -> torch.Tensor:
        return x.to(torch.float64) @ self.A  # A symmetric: (ncols, n) @ A == (A X)^T

    def diag(self) -> torch.Tensor:
        return torch.diagonal(self.A).clone()


def make_dense(n: int = 300, nlow: int = 8, seed: int = 0, device="cpu") -> DenseQuadratic:
    """A = D + U U^T with D = exp(N(0,1)), U_ij ~ N(0, 1/8), b ~ N(0,1); draws in that order."""
    rng = np.random.default_rng(seed)
    D = np.exp(rng.standard_normal(n))
    U = rng.standard_normal((n, nlow)) * math.sqrt(1.0 / 8.0)
    b = rng.standard_normal(n)
    A = np.diag(D) + U @ U.T
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)
    return DenseQuadratic(A=t(A), b=t(b), D=t(D))


def make_grid(nx: int, nz: int, seed: int, device="cpu", nparam: int = 3) -> GridQuadratic:
    """Lognormal-diagonal + smoothed-and-coupled grid operator; draws D then b."""
    n = nparam * nz * nx
    rng = np.random.default_rng(seed)
    D = np.exp(DIAG_LOG_STD * rng.standard_normal(n))
    b = rng.standard_normal(n)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)
    return GridQuadratic(nx=nx, nz=nz, D=t(D), b=t(b), nparam=nparam)


def make_problem(name: str, device="cpu", seed: int | None = None):
    cfg = CONFIGS[name]
    s = cfg["seed"] if seed is None else seed
    if cfg["kind"] == "dense":
        return make_dense(cfg["n"], cfg["nlow"], s, device)
    return make_grid(cfg["nx"], cfg["nz"], s, device)


def batch_shapes(nprob: int = 64, seed: int = 4):
    """Shapes of the 64-problem batch: n log-uniform in [5e4, 1e6] on 3-field
    grids of aspect a ~ U[2, 6] (nz = round(sqrt(n / 3a)), nx = round(a nz)),
    k uniform on {20..150}; problem i uses seed 1000 + i.  Draw order per
    problem: log n, a, k."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nprob):
        n_target = math.exp(rng.uniform(math.log(5e4), math.log(1e6)))
        a = rng.uniform(2.0, 6.0)
        k = int(rng.integers(20, 151))
        nz = max(1, int(round(math.sqrt(n_target / (3.0 * a)))))
        nx = max(1, int(round(a * nz)))
        out.append(dict(nx=nx, nz=nz, n=3 * nx * nz, k=k, rank=k, oversample=10, seed=1000 + i))
    return out


# ----------------------------------------------------------------------------
# Pair generators
# ----------------------------------------------------------------------------
def cg_pairs(problem, k: int, precond: torch.Tensor | None = None, rel_tol: float = 0.0):
    """Steps of preconditioned conjugate gradients from m_0 = 0 on 1/2 m^T A m - b^T m.

    With an exact line search on a strongly convex quadratic, BFGS started from
    a fixed diagonal initial inverse Hessian H0 produces the same iterates as
    conjugate gradients preconditioned by H0 (a scalar H0 does not change the
    iterates), so these are the pairs a full-memory BFGS run emits.  y_i = A s_i
    is formed directly rather than as a gradient difference, which is the same
    quantity without the cancellation of differencing tiny gradients.

    Returns (S, Y, gnorms) with S, Y of shape (kk, n), kk <= k (stops early if
    the gradient vanishes below rel_tol * |g_0|), gnorms the gradient norms
    |g_0| .. |g_kk|.
    """
    b = problem.b
    n = b.numel()
    M = precond if precond is not None else torch.ones(n, dtype=torch.float64, device=b.device)
    g = -b.clone()                       # gradient at m = 0
    z = M * g
    p = -z
    gz = torch.dot(g, z)
    S, Y, gn = [], [], [float(torch.linalg.vector_norm(g))]
    for _ in range(k):
        Ap = problem.matvec(p)
        pAp = torch.dot(p, Ap)
        alpha = -torch.dot(g, p) / pAp
        s = alpha * p
        y = alpha * Ap
        S.append(s)
        Y.append(y)
        g = g + y
        gn.append(float(torch.linalg.vector_norm(g)))
        if gn[-1] <= rel_tol * gn[0]:
            break
        z = M * g
        gz_new = torch.dot(g, z)
        beta = gz_new / gz
        gz = gz_new
        p = -z + beta * p
    return torch.stack(S), torch.stack(Y), gn


def random_secant_pairs(problem, k: int, seed: int = 0):
    """k secant pairs along independent random directions: s_i ~ N(0, I), y_i = A s_i.

    Every pair has s^T y = s^T A s > 0, and S^T Y is dense, unlike the nearly
    diagonal S^T Y of conjugate directions."""
    S = normal_block(problem.n, k, seed, problem.device)
    return S, problem.matvec(S)


def normal_block(n: int, ncols: int, seed: int, device="cpu") -> torch.Tensor:
    """ncols independent N(0, I_n) vectors, shape (ncols, n), float64."""
    rng = np.random.default_rng(seed)
    return torch.as_tensor(rng.standard_normal((ncols, n)), dtype=torch.float64, device=device)
