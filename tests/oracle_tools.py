"""Test-side tools around the oracle: dense one-step matrices, k-blocks,
energies and centroids.  Test infrastructure only."""
import math

import numpy as np
import torch

from oracle import qds as Q

HALF_X = {"Ex0", "Bx0", "jx0", "phi", "Ex1", "Bx1", "jx1"}


def copy_state(st):
    return {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in st.items()}


def dense_real(g, ph, keys, st0=None):
    """One-step matrix of the oracle over ``keys`` as a real 2N x 2N map
    (real and imaginary parts interleaved).  Only for linear configurations."""
    if st0 is None:
        st0 = Q.zero_state(g, ph)
    idx = [(k, i) for k in keys for i in range(st0[k].numel())]
    N = len(idx)
    A = np.zeros((2 * N, 2 * N))
    for c, (k, i) in enumerate(idx):
        for part, val in ((0, 1.0), (1, 1j)):
            st = copy_state(st0)
            a = st[k].clone().reshape(-1)
            a[i] = val
            st[k] = a.reshape(st0[k].shape)
            out = Q.step(st, g, ph)
            vec = torch.cat([out[kk].reshape(-1) for kk in keys])
            A[0::2, 2 * c + part] = vec.real.numpy()
            A[1::2, 2 * c + part] = vec.imag.numpy()
    return A


def kblock(g, ph, keys, m, k):
    """Complex one-step matrix restricted to fields of mode ``m`` proportional
    to exp(i k x) (periodic x, C-linear configurations only)."""
    st0 = Q.zero_state(g, ph)
    rows = {key: st0[key].shape[1] for key in keys}
    idx = [(key, j) for key in keys for j in range(rows[key])]
    N = len(idx)
    A = np.zeros((N, N), complex)
    xi = torch.arange(g.nx, dtype=torch.float64)
    for c, (key, j) in enumerate(idx):
        st = copy_state(st0)
        off = 0.5 if key in HALF_X else 0.0
        a = st[key].clone()
        a[m, j] = torch.exp(1j * k * (xi + off) * g.h)
        st[key] = a
        out = Q.step(st, g, ph)
        for r, (key2, j2) in enumerate(idx):
            off2 = 0.5 if key2 in HALF_X else 0.0
            A[r, c] = complex(out[key2][m, j2, 0].item()) / complex(np.exp(1j * k * off2 * g.h))
    return A


def mu_from_eigs(lam, k, h):
    """mu implied by each eigenvalue lam = exp(-i w h) through
    sin^2(w h/2) = sin^2(k h/2) + (h/2)^2 mu cos^2(k h/2)."""
    om = -np.angle(lam) / h
    s = np.sin(om * h / 2) ** 2
    return (s - np.sin(k * h / 2) ** 2) / ((h / 2) ** 2 * np.cos(k * h / 2) ** 2)


def mode_weights(M):
    return torch.tensor([2 * math.pi] + [math.pi] * (M - 1), dtype=torch.float64).view(-1, 1, 1)


def transverse_energy_x(st, g, s=0):
    """U(x_i) of the transverse fields of set s (Sec. 4.1 diagnostic):
    mode weight 2 pi (m=0) or pi (m>0), area r dr (axis row: dr^2/8)."""
    w = mode_weights(g.nmodes)
    rK = ((torch.arange(g.nr) + 0.5) * g.dr).view(1, -1, 1)
    rJ = (torch.arange(g.nr + 1) * g.dr).view(1, -1, 1).clone()
    rJ[0, 0, 0] = g.dr / 8
    uK = 0.25 * (st[f"Trp{s}"].abs() ** 2 + st[f"Trm{s}"].abs() ** 2) * rK * g.dr * w
    uJ = 0.25 * (st[f"Ttp{s}"].abs() ** 2 + st[f"Ttm{s}"].abs() ** 2) * rJ * g.dr * w
    return uK.sum((0, 1)) + uJ.sum((0, 1))


def em_energy(st, g, s=0):
    """Transverse + longitudinal field energy of set s (x-summed)."""
    w = mode_weights(g.nmodes)
    rK = ((torch.arange(g.nr) + 0.5) * g.dr).view(1, -1, 1)
    rJ = (torch.arange(g.nr + 1) * g.dr).view(1, -1, 1).clone()
    rJ[0, 0, 0] = g.dr / 8
    ut = transverse_energy_x(st, g, s).sum()
    ul = (0.5 * (st[f"Ex{s}"].abs() ** 2) * rJ * g.dr * w).sum() + \
         (0.5 * (st[f"Bx{s}"][:, :g.nr].abs() ** 2) * rK * g.dr * w).sum()
    return (ut + ul).item()


def axion_energy(st, g):
    """Axion energy from the transport variables, 1/4 (|T_a^+|^2 + |T_a^-|^2)
    = 1/2 (phi_t^2 + phi_x^2), plus the radial-gradient part."""
    w = mode_weights(g.nmodes)
    rK = ((torch.arange(g.nr) + 0.5) * g.dr).view(1, -1, 1)
    u = (0.25 * (st["Tap"].abs() ** 2 + st["Tam"].abs() ** 2) * rK * g.dr * w).sum()
    rJ = (torch.arange(1, g.nr) * g.dr).view(1, -1, 1)
    dphi = (st["phi"][:, 1:] - st["phi"][:, :-1]) / g.dr
    u = u + (0.5 * dphi.abs() ** 2 * rJ * g.dr * w).sum()
    return u.item()


def loss_energy(st, g, s=1, mode=1, x0=None, x1=None):
    """Energy of one mode of set s over columns [x0, x1): transverse fields at
    t^N, E_x and B_x at t^{N-1/2}, mode weight 2 pi (m=0) or pi, area r dr
    (axis row dr^2/8), times dx.  A differentiable torch scalar."""
    x0 = max(0, g.nx - 256) if x0 is None else x0
    x1 = g.nx if x1 is None else x1
    w = (2 * math.pi if mode == 0 else math.pi) * g.h * g.dr
    rK = ((torch.arange(g.nr, dtype=torch.float64) + 0.5) * g.dr).view(-1, 1)
    rJ = (torch.arange(g.nr + 1, dtype=torch.float64) * g.dr).clone()
    rJ[0] = g.dr / 8
    rJ = rJ.view(-1, 1)
    sl = slice(x0, x1)
    e = lambda t: (t.real ** 2 + t.imag ** 2)
    L = (0.25 * (e(st[f"Trp{s}"][mode, :, sl]) + e(st[f"Trm{s}"][mode, :, sl])) * rK).sum()
    L = L + (0.25 * (e(st[f"Ttp{s}"][mode, :, sl]) + e(st[f"Ttm{s}"][mode, :, sl])) * rJ).sum()
    L = L + (0.5 * e(st[f"Ex{s}"][mode, :, sl]) * rJ).sum()
    L = L + (0.5 * e(st[f"Bx{s}"][mode, : g.nr, sl]) * rK).sum()
    return w * L
