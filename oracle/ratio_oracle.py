"""Plain CPU FP64 oracle of the constant-photometric-ratio variant of the fit.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

The subtraction of pipeline step 6 ("Pipeline steps") fits a kernel whose
shape follows the PSF across the frame ("Statement of need").  Left free, the
kernel's sum -- the flux ratio between template and science image that a point
source sees -- may vary across the frame too.  The constrained variant keeps
that ratio constant: with the kernel written as

    K(z, u) = sum_a k_{a,u} m_a(z - u)      (the subtraction's coefficient layout),

a point source of flux f at z0 in the template puts f sum_a m_a(z0) s_a,
s_a = sum_u k_{a,u}, into the model.  The monomials m_a are linearly
independent, so the ratio is the same at every z0 exactly when

    s_a = sum_u k_{a,u} = 0   for every a >= 1,

nK - 1 linear equality constraints C theta = 0 (row a - 1 of C holds ones on
the L^2 coefficients of monomial a).  The constrained least-squares solution is
the plain definition of an equality-constrained quadratic minimum: the KKT
system

    [ Omega  C^T ] [ theta  ]   [ beta ]
    [ C      0   ] [ lambda ] = [ 0    ]

solved here as one dense LU solve (numpy.linalg.solve, FP64).  The background
coefficients are not constrained.
"""
from __future__ import annotations

import numpy as np

from .sfft_oracle import monomials, num_basis, num_coeffs

__all__ = ["ratio_constraints", "solve_const_ratio", "ratio_map", "kernel_sums"]


def ratio_constraints(w, dk, db):
    """C (nK - 1 rows, n columns): row a - 1 sums the kernel coefficients of monomial a."""
    L2 = (2 * w + 1) ** 2
    nk = num_basis(dk)
    n = num_coeffs(w, dk, db)
    C = np.zeros((nk - 1, n))
    for a in range(1, nk):
        C[a - 1, a * L2:(a + 1) * L2] = 1.0
    return C


def solve_const_ratio(omega, beta, w, dk, db):
    """theta minimising theta^T Omega theta - 2 beta^T theta subject to C theta = 0
    (the KKT system above).  Returns (theta, lambda)."""
    omega = np.asarray(omega, np.float64)
    beta = np.asarray(beta, np.float64)
    C = ratio_constraints(w, dk, db)
    nc, n = C.shape
    if nc == 0:
        return np.linalg.solve(omega, beta), np.zeros(0)
    kkt = np.zeros((n + nc, n + nc))
    kkt[:n, :n] = omega
    kkt[:n, n:] = C.T
    kkt[n:, :n] = C
    rhs = np.concatenate([beta, np.zeros(nc)])
    sol = np.linalg.solve(kkt, rhs)
    return sol[:n], sol[n:]


def kernel_sums(theta, w, dk):
    """s_a = sum_u k_{a,u} for every monomial a."""
    L2 = (2 * w + 1) ** 2
    nk = num_basis(dk)
    return np.asarray(theta[:nk * L2], np.float64).reshape(nk, L2).sum(axis=1)


def ratio_map(theta, w, dk, ny, nx):
    """Flux ratio a point source at each pixel sees: sum_a m_a(z) s_a (ny x nx)."""
    s = kernel_sums(theta, w, dk)
    m = monomials(ny, nx, dk)
    return np.tensordot(s, m, axes=1)
