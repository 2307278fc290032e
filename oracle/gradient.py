"""Gradient of the differentiable-optics loss (oracle; test infrastructure only).

L(rho) = 1/2 sum(rho * phi) + sum((phi - phi_t)^2),  phi = A rho,

where A is the discrete pipe operator (Eq. 4 pattern with Eq. 8).  A is
symmetric on the mesh: G is unchanged by swapping (x, y, z) with (x', y', z')
because R is even in each argument (Eq. 9) and the sum terms x + x', y + y'
are symmetric.  Hence dL/drho = A rho + 2 A (phi - phi_t) = phi + 2 A (phi - phi_t).
"""
import numpy as np


def loss(rho, phi, phi_t):
    return 0.5 * float(np.sum(rho * phi)) + float(np.sum((phi - phi_t) ** 2))


def grad(apply_A, rho, phi_t):
    """apply_A: callable mapping an (nx, ny, nz) FP64 array to A @ it (O2 or O3)."""
    phi = apply_A(rho)
    return phi + 2.0 * apply_A(phi - phi_t)
