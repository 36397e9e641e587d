"""Pin of the theta-grid product rule the HIP kernels use for the axion source
and current (Sec. 3.3): sampling two fields of modes 0..M-1 on N = 3M - 2
equispaced angles, multiplying pointwise and projecting back gives the
oracle's direct convolution C_m (Eq. mode_convolution) for every output mode
0..M-1 once the complex mode-0 product is restored; one point fewer aliases."""
import math

import numpy as np
import pytest
import torch

from oracle import qds as Q


def _theta_product(A, B, N):
    th = 2 * math.pi * np.arange(N) / N
    M = A.shape[0]
    m = np.arange(M)
    e = np.exp(-1j * np.outer(th, m))                    # [N, M]
    a = np.real(e @ A)                                   # Re sum A^(m) e^{-i m theta}
    b = np.real(e @ B)
    p = a * b
    out = (np.exp(1j * np.outer(m, th)) @ p) / N
    out[1:] *= 2
    # the literal convolution's mode 0 uses the complex product A^(0) B^(0)
    out[0] += A[0] * B[0] - A[0].real * B[0].real
    return out


@pytest.mark.parametrize("M", [2, 3, 4, 6, 8])
def test_theta_grid_of_3M_minus_2_points_is_exact(M):
    rng = np.random.default_rng(M)
    A = rng.normal(size=(M, 5)) + 1j * rng.normal(size=(M, 5))   # complex mode 0 too
    B = rng.normal(size=(M, 5)) + 1j * rng.normal(size=(M, 5))
    ref = Q.mode_conv(torch.from_numpy(A), torch.from_numpy(B)).numpy()
    got = _theta_product(A, B, 3 * M - 2)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    if M >= 2:
        bad = _theta_product(A, B, 3 * M - 3)
        assert np.abs(bad - ref).max() > 1e-3 * np.abs(ref).max()
