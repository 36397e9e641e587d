"""Algebraic identities the GPU kernels rely on, checked in FP64 with the
oracle's mode convolution on random mode coefficients (CPU only).

The single-precision kernels form the transverse part of the axion source and
the theta / r components of the axion current from the transport variables
T^+- = E +- B (and T_a^+- = d_t phi -+ d_x phi) instead of from E and B: the
same bilinear form, written so that co-propagating waves do not subtract two
large products (Eqs. source_mode_zero/_m, jar_mode, jat_mode)."""
import torch

from oracle.qds import mode_conv


def _rand(M, shape, g):
    return torch.randn((M,) + shape, dtype=torch.complex128, generator=g)


def test_axion_source_transport_form():
    g = torch.Generator().manual_seed(3)
    for M in (1, 2, 3, 4):
        Tp, Tm, Sp, Sm = (_rand(M, (5, 7), g) for _ in range(4))     # T_r^+-, T_th^+-
        br = torch.zeros_like(Tp)
        bt = torch.zeros_like(Tp)
        if M > 1:
            br[1] = 0.3 - 0.2j
            bt[1] = -0.1 + 0.4j
        Er, Bt = 0.5 * (Tp + Tm), 0.5 * (Tp - Tm) + bt
        Et, Br = 0.5 * (Sp + Sm), 0.5 * (Sp - Sm) + br
        lhs = mode_conv(Er, Br) + mode_conv(Et, Bt)
        rhs = 0.5 * mode_conv(Tp + bt, Sp + br) - 0.5 * mode_conv(Tm - bt, Sm - br)
        assert torch.allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_axion_current_transport_forms():
    g = torch.Generator().manual_seed(4)
    for M in (1, 2, 3):
        Tp, Tm, Sp, Sm, Ap, Am = (_rand(M, (4, 6), g) for _ in range(6))
        b = torch.zeros_like(Tp)
        if M > 1:
            b[1] = 0.2 + 0.1j
        dt, dx = 0.5 * (Ap + Am), 0.5 * (Am - Ap)       # T_a^+- = d_t phi -+ d_x phi
        Er, Bt = 0.5 * (Tp + Tm), 0.5 * (Tp - Tm) + b
        lhs = mode_conv(Bt, dt) + mode_conv(Er, dx)
        rhs = 0.5 * mode_conv(Tp + b, Am) - 0.5 * mode_conv(Tm - b, Ap)
        assert torch.allclose(lhs, rhs, rtol=0, atol=1e-13)
        Et, Br = 0.5 * (Sp + Sm), 0.5 * (Sp - Sm) + b
        lhs = mode_conv(Br, dt) - mode_conv(Et, dx)
        rhs = 0.5 * mode_conv(Sp + b, Ap) - 0.5 * mode_conv(Sm - b, Am)
        assert torch.allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_transport_form_removes_the_single_precision_cancellation():
    """A co-propagating pair (T^- = 0 up to 1e-4): the E/B form in complex64
    loses digits, the transport form keeps them."""
    g = torch.Generator().manual_seed(5)
    M = 2
    Tp, Sm = _rand(M, (8, 8), g), _rand(M, (8, 8), g)
    Tm, Sp = 1e-4 * _rand(M, (8, 8), g), 1e-4 * _rand(M, (8, 8), g)
    ref = 0.5 * mode_conv(Tp, Sp) - 0.5 * mode_conv(Tm, Sm)
    c = lambda t: t.to(torch.complex64)
    Er, Bt, Et, Br = 0.5 * (c(Tp) + c(Tm)), 0.5 * (c(Tp) - c(Tm)), 0.5 * (c(Sp) + c(Sm)), 0.5 * (c(Sp) - c(Sm))
    eb = mode_conv(Er, Br) + mode_conv(Et, Bt)
    tf = 0.5 * mode_conv(c(Tp), c(Sp)) - 0.5 * mode_conv(c(Tm), c(Sm))
    err = lambda x: float((x.to(torch.complex128) - ref).norm() / ref.norm())
    assert err(tf) < 1e-6 < err(eb)
