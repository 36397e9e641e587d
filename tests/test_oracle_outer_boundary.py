"""Pin of the oracle's outer radial electromagnetic boundary (Sec. 3.2, Eqs.
em_r_characteristic, em_r_open_bx, em_r_open_bt) against exact outgoing
cylindrical waves.

A mode-m TM wave (E_x = H_m^(1)(k_perp r) e^{i(k x - w t)}, B_x = 0) or TE wave
(B_x = H_m^(1)(k_perp r) e^{i(k x - w t)}, E_x = 0) with w^2 = k^2 + k_perp^2
solves Maxwell's equations exactly and leaves the domain through r = R_max.
Its fields are sampled at the staggered positions of one oracle step (the
exterior ghosts B_x at r_{nr+1/2}, t^{-1/2} and B_theta at r_{nr+1/2}, t^0
included) and the step's new ghosts are compared with the exact wave.

The outflow condition assumes a locally transverse wave (E_theta = B_x,
E_x = -B_theta); for the exact wave, Maxwell's equations give its residual:
    (d_t + d_r) B_x     - rhs_x = -1/2 (d_t + d_r)(E_theta - B_x)
    (d_t + d_r) B_theta - rhs_t =  1/2 (d_t + d_r)(E_x + B_theta)
so a consistent discretisation centred at (r_nr, t^n) with step factor
c_R = 2 dt dr / (dr + dt) yields  ghost_exact + c_R * (rhs - (d_t + d_r) B)
to O(dt dr).  The pin requires that to second order (a factor >= 3.5 per
halving of dx = c dt and dr), and shows that each right-hand-side term
(the axial derivative, the curvature terms) weighs far more than what is
left, so a dropped term or a flipped sign fails it.
"""
import math

import numpy as np
import pytest
import sympy as sp
import torch

from oracle import qds as Q

XS, RS, TS = sp.symbols("x r t", real=True)
M = 3
L_X = 8.0          # periodic x length
R_MAX = 8.0
K_X = 2 * math.pi / L_X
K_P = 1.1


class Wave:
    """Exact mode-m wave (Maxwell with c = 1, e^{-i m theta} convention):
    TM: E_r = i k f'/kp^2, E_theta = m k f/(r kp^2), B_r = -m w f/(r kp^2), B_theta = i w f'/kp^2
    TE: by E -> B, B -> -E."""

    def __init__(self, m, kind, amp=1.0):
        w = math.sqrt(K_X ** 2 + K_P ** 2)
        f = amp * sp.hankel1(m, K_P * RS) * sp.exp(sp.I * (K_X * XS - w * TS))
        fp = sp.diff(f, RS)
        Er, Et = sp.I * K_X * fp / K_P ** 2, m * K_X * f / (RS * K_P ** 2)
        Br, Bt = -m * w * f / (RS * K_P ** 2), sp.I * w * fp / K_P ** 2
        if kind == "TM":
            e = {"Ex": f, "Er": Er, "Et": Et, "Bx": 0 * f, "Br": Br, "Bt": Bt}
        else:
            e = {"Bx": f, "Br": Er, "Bt": Et, "Ex": 0 * f, "Er": -Br, "Et": -Bt}
        # residuals of the two outflow equations
        e["res_x"] = -sp.Rational(1, 2) * (sp.diff(e["Et"] - e["Bx"], TS) + sp.diff(e["Et"] - e["Bx"], RS))
        e["res_t"] = sp.Rational(1, 2) * (sp.diff(e["Ex"] + e["Bt"], TS) + sp.diff(e["Ex"] + e["Bt"], RS))
        # the right-hand sides' terms, for the sensitivity check
        e["dxBr"] = sp.Rational(1, 2) * sp.diff(e["Br"], XS)
        e["curv_x"] = -(e["Et"] + sp.I * m * e["Er"]) / (2 * RS)
        e["dxEr"] = -sp.Rational(1, 2) * sp.diff(e["Er"], XS)
        e["curv_t"] = -(e["Bt"] + sp.I * m * e["Br"]) / (2 * RS)
        self.m = m
        self.f = {k: sp.lambdify((XS, RS, TS), v, modules=["scipy", "numpy"]) for k, v in e.items()}

    def __call__(self, name, x, r, t):
        X, R = np.meshgrid(np.asarray(x, float), np.asarray(r, float))
        return np.broadcast_to(self.f[name](X, R, t), X.shape).astype(complex)


def _state(wave, nx, nr, h, dr):
    """Oracle state at t^0 (transverse fields) and t^{-1/2} (E_x, B_x), the
    wave in mode ``wave.m`` on the rows r >= R_MAX / 2 (the Hankel function is
    singular on the axis; one step only reaches a few rows back from the edge)."""
    g = Q.Grid(nx, nr, M, h, dr, "periodic", "open")
    st = Q.zero_state(g, Q.Physics())
    xI = np.arange(nx) * h
    xH = xI + 0.5 * h
    rK = (np.arange(nr + 1) + 0.5) * dr
    rJ = np.arange(nr + 1) * dr
    m = wave.m

    def put(key, name, xs, rs, t, rows):
        v = np.zeros((len(rs), len(xs)), complex)
        keep = rs >= R_MAX / 2
        v[keep] = wave(name, xs, rs[keep], t)
        a = st[key].clone()
        a[m, rows] = torch.from_numpy(v)
        st[key] = a

    Er = np.zeros((nr, nx), complex)
    Bt = np.zeros((nr, nx), complex)
    keep = rK[:nr] >= R_MAX / 2
    Er[keep] = wave("Er", xI, rK[:nr][keep], 0.0)
    Bt[keep] = wave("Bt", xI, rK[:nr][keep], 0.0)
    Et = np.zeros((nr + 1, nx), complex)
    Br = np.zeros((nr + 1, nx), complex)
    keepJ = rJ >= R_MAX / 2
    Et[keepJ] = wave("Et", xI, rJ[keepJ], 0.0)
    Br[keepJ] = wave("Br", xI, rJ[keepJ], 0.0)
    for key, val in (("Trp0", Er + Bt), ("Trm0", Er - Bt), ("Ttp0", Et + Br), ("Ttm0", Et - Br)):
        a = st[key].clone()
        a[m] = torch.from_numpy(val)
        st[key] = a
    put("Ex0", "Ex", xH, rJ, -0.5 * h, slice(None))
    put("Bx0", "Bx", xH, rK, -0.5 * h, slice(None))           # row nr: the exterior ghost
    bg = st["Bg0"].clone()
    bg[m] = torch.from_numpy(wave("Bt", xI, np.array([rK[nr]]), 0.0)[0])
    st["Bg0"] = bg
    return g, st


LEVELS = [(32, 16), (64, 32), (128, 64)]     # nx, nr: dx = L_X / nx, dr = R_MAX / nr


TERMS = {"x": ("dxBr", "curv_x"), "t": ("dxEr", "curv_t")}


def _ghost_errors(wave, mutate=None):
    """Per level: (B_x ghost error, B_theta ghost error), each relative to the
    largest exact ghost value.  ``mutate`` = (term, factor) changes the
    ghost the step produced by factor * c_R * that right-hand-side term
    (factor -1: the term dropped; -2: its sign flipped), as a slip in the
    oracle's update would."""
    out = []
    for nx, nr in LEVELS:
        h, dr = L_X / nx, R_MAX / nr
        g, st = _state(wave, nx, nr, h, dr)
        new = Q.step(st, g, Q.Physics())
        cR = 2 * h * dr / (dr + h)
        xI = np.arange(nx) * h
        xH = xI + 0.5 * h
        rG = np.array([(nr + 0.5) * dr])
        rN = np.array([nr * dr])
        m = wave.m
        bx_ex = wave("Bx", xH, rG, 0.5 * h)[0]
        bx_pred = bx_ex - cR * wave("res_x", xH, rN, 0.0)[0]
        bt_ex = wave("Bt", xI, rG, h)[0]
        bt_pred = bt_ex - cR * wave("res_t", xI, rN, 0.5 * h)[0]
        gx = new["Bx0"][m, nr].numpy().copy()
        gt = new["Bg0"][m].numpy().copy()
        if mutate is not None:
            term, fac = mutate
            if term in TERMS["x"]:
                gx = gx + fac * cR * wave(term, xH, rN, 0.0)[0]
            else:
                gt = gt + fac * cR * wave(term, xI, rN, 0.5 * h)[0]
        sx = max(np.abs(bx_ex).max(), np.abs(bt_ex).max())
        out.append((np.abs(gx - bx_pred).max() / sx, np.abs(gt - bt_pred).max() / sx))
    return out


def pin_failures(errs):
    """Second order (>= 3.5 per halving) for each ghost the wave excites."""
    bad = []
    for q, name in ((0, "B_x ghost"), (1, "B_theta ghost")):
        e = [lev[q] for lev in errs]
        if max(e) < 1e-12:
            continue        # this field is zero for this wave (B_x of TM / m = 0)
        if not (e[0] / e[1] >= 3.5 and e[1] / e[2] >= 3.5):
            bad.append((name, e))
    return bad


WAVES = [(0, "TM"), (0, "TE"), (1, "TM"), (1, "TE"), (2, "TM"), (2, "TE")]


@pytest.mark.parametrize("m,kind", WAVES)
def test_outer_ghosts_are_consistent_with_the_outflow_equations(m, kind):
    assert pin_failures(_ghost_errors(Wave(m, kind))) == []


@pytest.mark.parametrize("term", ["dxBr", "curv_x", "dxEr", "curv_t"])
@pytest.mark.parametrize("fac", [-1.0, -2.0])
def test_a_dropped_or_flipped_term_fails_the_pin(term, fac):
    """Each right-hand-side term of the two outflow equations, dropped or with
    its sign flipped, fails the pin for some mode-0..2 TM or TE wave that
    exercises it."""
    failed = [(m, kind) for m, kind in WAVES if pin_failures(_ghost_errors(Wave(m, kind), (term, fac)))]
    assert failed, (term, fac)
