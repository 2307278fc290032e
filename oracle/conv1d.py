"""1-D zero-padded FFT convolution and correlation of the Appendix (oracle; test infrastructure only).

Convolution, Eq. A.1:  p_j = sum_{k=0}^{K-1} r_k x_{j-k},  j = 0..J-1,
with x indexed m = -(K-1)..J-1 (M = J + K - 1 values).
Correlation, Eq. A.9:  p_j = sum_{k=0}^{K-1} r_k x_{j+k},  j = 0..J-1,
with x indexed m = 0..J+K-2 (the printed index line for A.9 repeats the one
of A.1; the range that the sum actually visits is j + k = 0..J+K-2).

``x`` is passed as a Python callable of the integer index so that both the
direct sums and the padded FFT build their sequences from the same values.
"""
import numpy as np


def conv_direct(r, x, J):
    K = len(r)
    return np.array([sum(r[k] * x(j - k) for k in range(K)) for j in range(J)])


def corr_direct(r, x, J):
    K = len(r)
    return np.array([sum(r[k] * x(j + k) for k in range(K)) for j in range(J)])


def conv_fft(r, x, J, N):
    """Eq. A.2-A.4: zero-padded r, N-periodic xi (zero on m = J..N-K), forward
    transforms of both, product, backward transform with the 1/N."""
    K = len(r)
    if N < J + K - 1:
        raise ValueError("N must be at least J + K - 1")
    rho = np.zeros(N)
    rho[:K] = r
    xi = np.zeros(N)
    for m in range(-(K - 1), J):
        xi[m % N] = x(m)
    W = np.exp(-2j * np.pi / N)
    n = np.arange(N)
    F = W ** np.outer(n, n)                  # forward:  sum_n a_n W^{nk}
    B = W ** (-np.outer(n, n))               # backward: sum_n a_n W^{-nk}
    phi = (B @ ((F @ rho) * (F @ xi))) / N
    return phi[:J]


def corr_fft(r, x, J, N):
    """A.9: the same zero padding, with the Green transform and the final
    transform taken in the backward and forward directions respectively."""
    K = len(r)
    if N < J + K - 1:
        raise ValueError("N must be at least J + K - 1")
    rho = np.zeros(N)
    rho[:K] = r
    xi = np.zeros(N)
    for m in range(0, J + K - 1):
        xi[m] = x(m)
    W = np.exp(-2j * np.pi / N)
    n = np.arange(N)
    F = W ** np.outer(n, n)
    B = W ** (-np.outer(n, n))
    phi = (F @ ((F @ rho) * (B @ xi))) / N
    return phi[:J]
