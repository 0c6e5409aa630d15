"""Preconditioned conjugate gradients and the Lanczos condition estimate
(oracle; test infrastructure).

Section 5 runs PCG on the full system and stops on a reduction of the
residual 2-norm.  Readings used here: start from x0 = 0; stop when the
recurrence residual satisfies ||r_k||_2 <= rtol ||b||_2; the iteration count
is the number of operator applications inside the loop.

The condition number is estimated from the CG coefficients (the Lanczos
tridiagonal matrix of the preconditioned operator; Saad, Iterative Methods
for Sparse Linear Systems, Section 6.7.3): diagonal 1/alpha_0, then
1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_{j-1})/alpha_{j-1}.
Theorem 3 bounds the spectrum of BA below by 1.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List

import numpy as np
import scipy.linalg as sla


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    resnorms: List[float]
    alphas: List[float]
    betas: List[float]

    def lanczos(self):
        return lanczos_matrix(self.alphas, self.betas)

    def eig_extremes(self):
        T = self.lanczos()
        if T.size == 0:
            return 1.0, 1.0
        ev = sla.eigvalsh(T)
        return float(ev[0]), float(ev[-1])

    @property
    def kappa(self) -> float:
        lo, hi = self.eig_extremes()
        return hi / lo


def lanczos_matrix(alphas, betas) -> np.ndarray:
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j]
        if j > 0:
            T[j, j] += betas[j - 1] / alphas[j - 1]
            off = np.sqrt(betas[j - 1]) / alphas[j - 1]
            T[j, j - 1] = T[j - 1, j] = off
    return T


def pcg(apply_A: Callable, apply_B: Callable, b: np.ndarray, rtol: float = 1e-8,
        maxit: int = 1000, fixed_iters: int = 0) -> PCGResult:
    """Hestenes-Stiefel PCG from x0 = 0.

    ``fixed_iters > 0`` runs exactly that many iterations (no residual test),
    which lets two implementations be compared at equal iterates.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return PCGResult(x, 0, True, [0.0], [], [])
    r = b.copy()
    z = apply_B(r)
    p = z.copy()
    rz = float(r @ z)
    resn = [bnorm]
    alphas, betas = [], []
    limit = fixed_iters if fixed_iters > 0 else maxit
    converged = False
    it = 0
    for k in range(limit):
        q = apply_A(p)
        pq = float(p @ q)
        alpha = rz / pq
        alphas.append(alpha)
        x += alpha * p
        r -= alpha * q
        it = k + 1
        rn = float(np.linalg.norm(r))
        resn.append(rn)
        if fixed_iters == 0 and rn <= rtol * bnorm:
            converged = True
            break
        if it == limit:
            break
        z = apply_B(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    if fixed_iters:
        converged = resn[-1] <= rtol * bnorm
    return PCGResult(x, it, converged, resn, alphas, betas)


def solve(bddc, b, rtol=1e-8, maxit=1000, fixed_iters=0) -> PCGResult:
    """PCG on the assembled global matrix with the BDDC-SO preconditioner."""
    return pcg(lambda v: bddc.A @ v, bddc.apply, b, rtol, maxit, fixed_iters)
