"""Pin of the oracle's axion current j_a (Eqs. jax_mode, jar_mode, jat_mode and
their interpolation to the source points of the regenerated set, with the axis
limits of the paper's regularity rules, Sec. 2.3).

Smooth analytic fields, regular on the axis, are sampled at the staggered
positions and time levels the oracle's state holds; the oracle's discrete j_a
at every source point (x_{i+1/2}, r_j, t^n) for j_a,x, (x_{i+1/2}, r_{j+1/2},
t^{n+1/2}) for j_a,r and (x_{i+1/2}, r_j, t^{n+1/2}) for j_a,theta is compared
with the continuous j_a = B d_t phi - E x grad phi evaluated at the same point
by theta quadrature of the Cartesian product (exact derivatives, no mode
algebra).  Refining dx = c dt and dr together, the error must fall at second
order on every row, the axis row and the first rows included; sampling any
input half a cell off its position breaks that.
"""
import math

import numpy as np
import pytest
import sympy as sp
import torch

from oracle import qds as Q

M = 4
XS, RS, TS = sp.symbols("x r t", real=True)


def _gauss(c, x0, v, w, s):
    return c * sp.exp(-((XS - x0 - v * TS) / w) ** 2 - (RS / s) ** 2)


def _rand_c(rng, m):
    re, im = rng.normal(size=2)
    return complex(re, 0.0 if m == 0 else im)   # the m = 0 mode of a real field is real


class Fields:
    """Mode functions F^(m)(x, r, t) of a regular field configuration.

    Scalars (phi, E_x, B_x): F^(m) = r^m alpha(x, r^2, t).  Transverse vectors
    from two regular potentials a, b (E = grad_perp a + x_hat x grad_perp b):
    E_r^(m) = d_r a^(m) + i m b^(m)/r, E_theta^(m) = -i m a^(m)/r + d_r b^(m),
    which obey the axis rules (E_r^(1) = i E_theta^(1) at r = 0)."""

    def __init__(self, seed):
        rng = np.random.default_rng(seed)
        self.expr = {}

        def alpha(m):
            return _gauss(_rand_c(rng, m), 8.0 + rng.uniform(-1, 1), rng.uniform(-0.5, 0.9),
                          rng.uniform(2.2, 3.0), rng.uniform(1.6, 2.2))

        for name in ("phi", "Ex", "Bx"):
            self.expr[name] = [RS ** m * alpha(m) for m in range(M)]
        # phi^(m)/r (regular for m >= 1; it enters only as m phi^(m)/r)
        self.expr["phi_r"] = [sp.simplify(self.expr["phi"][m] / RS) if m >= 1 else sp.Integer(0) for m in range(M)]
        for v in ("E", "B"):
            a = [RS ** m * alpha(m) for m in range(M)]
            b = [RS ** m * alpha(m) for m in range(M)]
            a_r = [sp.simplify(a[m] / RS) for m in range(M)]
            b_r = [sp.simplify(b[m] / RS) for m in range(M)]
            self.expr[v + "r"] = [sp.diff(a[m], RS) + sp.I * m * b_r[m] for m in range(M)]
            self.expr[v + "t"] = [-sp.I * m * a_r[m] + sp.diff(b[m], RS) for m in range(M)]
        phi = self.expr["phi"]
        self.expr["dtphi"] = [sp.diff(phi[m], TS) for m in range(M)]
        self.expr["dxphi"] = [sp.diff(phi[m], XS) for m in range(M)]
        self.expr["drphi"] = [sp.diff(phi[m], RS) for m in range(M)]
        self.f = {k: [sp.lambdify((XS, RS, TS), e, "numpy") for e in v] for k, v in self.expr.items()}

    def modes(self, name, x, r, t):
        """[M, len(r), len(x)] complex samples of the mode functions."""
        X, R = np.meshgrid(np.asarray(x, float), np.asarray(r, float))
        out = np.zeros((M,) + X.shape, complex)
        for m in range(M):
            out[m] = np.broadcast_to(self.f[name][m](X, R, t), X.shape)
        return torch.from_numpy(out)

    def real(self, name, x, r, t, th):
        """Real field on the theta grid [T, len(r), len(x)]."""
        F = self.modes(name, x, r, t).numpy()
        e = np.exp(-1j * np.outer(th, np.arange(M)))          # [T, M]
        return np.real(np.einsum("tm,mrx->trx", e, F))


def continuous_ja(F, x, r, t):
    """Mode coefficients of j_a = B d_t phi - E x grad phi at (x, r, t): the
    Cartesian product on an equispaced theta grid, projected (T = 16 resolves
    the modes up to 6 of a product of modes up to 3)."""
    Tn = 16
    th = 2 * math.pi * np.arange(Tn) / Tn
    c, s = np.cos(th)[:, None, None], np.sin(th)[:, None, None]
    g = {k: F.real(k, x, r, t, th) for k in ("Ex", "Er", "Et", "Bx", "Br", "Bt", "dtphi", "dxphi", "drphi")}
    # (1/r) d_theta phi = Re sum (-i m phi^(m) / r) e^{-i m theta}, with phi^(m)/r regular
    Pr = F.modes("phi_r", x, r, t).numpy()
    mm = np.arange(M)[:, None, None]
    e = np.exp(-1j * np.outer(th, np.arange(M)))
    gth = np.real(np.einsum("tm,mrx->trx", e, -1j * mm * Pr))
    Ey, Ez = g["Er"] * c - g["Et"] * s, g["Er"] * s + g["Et"] * c
    By, Bz = g["Br"] * c - g["Bt"] * s, g["Br"] * s + g["Bt"] * c
    Gx, Gy, Gz = g["dxphi"], g["drphi"] * c - gth * s, g["drphi"] * s + gth * c
    Ex = g["Ex"]
    jx = g["Bx"] * g["dtphi"] - (Ey * Gz - Ez * Gy)
    jy = By * g["dtphi"] - (Ez * Gx - Ex * Gz)
    jz = Bz * g["dtphi"] - (Ex * Gy - Ey * Gx)
    jr, jt = jy * c + jz * s, -jy * s + jz * c

    def proj(P):
        ee = np.exp(1j * np.outer(np.arange(M), th))             # [M, T]
        out = np.einsum("mt,trx->mrx", ee, P) / Tn
        out[1:] *= 2
        return out
    return proj(jx), proj(jr), proj(jt)


def discrete_ja(F, nx, nr, h, dr, shift=None, form="transport"):
    """The oracle's j_a from samples of F at the staggered positions of one
    step n = 0 -> 1 (t^n = 0).  ``shift`` = (field, axis) samples that input
    half a cell off its position (x or r) to show the pin's sensitivity."""
    g = Q.Grid(nx, nr, M, h, dr, "open", "open")
    c = Q._Ctx(g)
    xI = np.arange(nx) * h
    xH = xI + 0.5 * h
    rK = (np.arange(nr + 1) + 0.5) * dr
    rJ = np.arange(nr + 1) * dr

    def off(name, xs, rs):
        if shift and shift[0] == name:
            if shift[1] == "x":
                return xs + 0.5 * h, rs
            return xs, rs + 0.5 * dr
        return xs, rs

    def smp(name, xs, rs, t, key=None):
        xs2, rs2 = off(key or name, xs, rs)
        return F.modes(name, xs2, rs2, t)

    def state(t, te):
        """Background set with the transverse fields at t, E_x, B_x at te."""
        Er, Bt = smp("Er", xI, rK[:nr], t), smp("Bt", xI, rK[:nr], t)
        Et, Br = smp("Et", xI, rJ, t), smp("Br", xI, rJ, t)
        return {"Trp0": Er + Bt, "Trm0": Er - Bt, "Ttp0": Et + Br, "Ttm0": Et - Br,
                "Ex0": smp("Ex", xH, rJ, te), "Bx0": smp("Bx", xH, rK, te)}

    def axion(t, ta):
        tap = smp("dtphi", xI, rK[:nr], ta, "Ta") - smp("dxphi", xI, rK[:nr], ta, "Ta")
        tam = smp("dtphi", xI, rK[:nr], ta, "Ta") + smp("dxphi", xI, rK[:nr], ta, "Ta")
        return {"phi": smp("phi", xH, rK[:nr], t), "Tap": tap, "Tam": tam}

    st = state(0.0, -0.5 * h)
    new = state(h, 0.5 * h)
    st.update(axion(0.0, -0.5 * h))
    kg = axion(h, 0.5 * h)
    f = Q._bg_fields(c, st, new, (0j, 0j, 0j))
    return Q.axion_current(c, f, st, kg, (0j, 0j, 0j), form)


LEVELS = [(64, 24, 0.25, 0.25), (128, 48, 0.125, 0.125), (256, 96, 0.0625, 0.0625)]
R_BAND = 1.0     # rows at r >= R_BAND: a band at a fixed physical radius


def _errors(F, shift=None, form="transport"):
    """Per level and component (x, r, theta), errors relative to the largest
    reference value, over interior columns and rows below the outer row:
    [0] the r-weighted L2 norm over all rows (area r dr, the axis row dr/8),
    [1] the axis row (r = 0; r_{1/2} for j_a,r), [2] the largest error at
    r >= R_BAND, [3] the first row off the axis (r = dr; r_{3/2} for j_a,r)."""
    out = []
    for nx, nr, h, dr in LEVELS:
        jx, jr, jt = discrete_ja(F, nx, nr, h, dr, shift, form)
        xH = (np.arange(nx) + 0.5) * h
        rJ = np.arange(nr + 1) * dr
        rK = (np.arange(nr) + 0.5) * dr
        cx_, _, _ = continuous_ja(F, xH, rJ[:nr], 0.0)
        _, cr_, _ = continuous_ja(F, xH, rK, 0.5 * h)
        _, _, ct_ = continuous_ja(F, xH, rJ[:nr], 0.5 * h)
        sl = slice(3, nx - 3)
        lev = {}
        for name, d, ref, rr in (("x", jx, cx_, rJ[:nr]), ("r", jr, cr_, rK), ("t", jt, ct_, rJ[:nr])):
            d = d.numpy()[:, : nr - 1, sl]
            ref = ref[:, : nr - 1, sl]
            rr = rr[: nr - 1]
            scale = np.abs(ref).max()
            err = np.abs(d - ref) / scale
            w = np.where(rr > 0, rr, dr / 8) * dr * h
            l2 = np.sqrt((err ** 2 * w[None, :, None]).sum() / (w.sum() * err.shape[0] * err.shape[2]))
            lev[name] = (l2, err[:, 0].max(), err[:, rr >= R_BAND].max(), err[:, 1].max())
        out.append(lev)
    return out


@pytest.fixture(scope="module")
def fields():
    return Fields(2609)


def _ratios(errs, comp, which):
    e = [lev[comp][which] for lev in errs]
    return e, e[0] / e[1], e[1] / e[2]


def pin_failures(errs):
    """The convergence pin's criteria, returned as the list of those that
    fail: second order (>= 3.5 per halving) in the r-weighted norm, on the
    axis row and at a fixed radius for every component, and on the first row
    off the axis for j_a,r and j_a,theta (>= 3.0 from the coarsest grid, which
    is not yet asymptotic there); the first row of j_a,x at first order: the
    paper's rule averages the field and then divides by r_j (as for
    B_theta / r in Gamma_x), which leaves an O(dr^2 / r_j) error, O(dr) at
    r_j = dr."""
    bad = []
    for comp in ("x", "r", "t"):
        for which in range(3):
            e, q1, q2 = _ratios(errs, comp, which)
            if not (q1 >= 3.5 and q2 >= 3.5 and e[2] < 2e-3):
                bad.append((comp, ["r-weighted L2", "axis row", "r >= 1"][which], e))
        e, q1, q2 = _ratios(errs, comp, 3)
        ok = (q1 >= 1.8 and q2 >= 1.8) if comp == "x" else (q1 >= 3.0 and q2 >= 3.5)
        if not ok:
            bad.append((comp, "first row", e))
    return bad


@pytest.mark.parametrize("form", ["transport", "eb"])
def test_axion_current_converges_at_second_order(fields, form):
    assert pin_failures(_errors(fields, form=form)) == []


@pytest.mark.parametrize("shift", [("Er", "r"), ("Et", "r"), ("Br", "r"), ("Bt", "x"), ("Ex", "r"),
                                   ("Bx", "x"), ("phi", "x"), ("phi", "r"), ("Ta", "x")])
def test_half_cell_shift_breaks_second_order(fields, shift):
    """Each input sampled half a cell off its position makes the pin above fail."""
    assert pin_failures(_errors(fields, shift=shift)) != [], shift


def test_odd_ghost_for_every_mode_fails_the_pin(fields, monkeypatch):
    """Ghosts taken odd for every m >= 1 (a regular mode-2 scalar is even in r)
    leave an O(dr) error in d_r phi on the axis: the pin fails."""
    orig = Q._Ctx.__init__

    def init(self, g):
        orig(self, g)
        self.par = torch.tensor([1.0] + [-1.0] * (g.nmodes - 1), dtype=Q.RDT).view(-1, 1)
        self.tpar = torch.tensor([-1.0] * g.nmodes, dtype=Q.RDT).view(-1, 1)
    monkeypatch.setattr(Q._Ctx, "__init__", init)
    assert pin_failures(_errors(fields)) != []


def _source_errors(F, form="transport", shift=None):
    """Per level: r-weighted L2, axis-row and fixed-radius errors of the
    oracle's S_a = E.B at (x_{i+1/2}, r_{j+1/2}, t^n) against the Cartesian
    dot product of the analytic fields."""
    out = []
    for nx, nr, h, dr in LEVELS:
        g = Q.Grid(nx, nr, M, h, dr, "open", "open")
        c = Q._Ctx(g)
        xI = np.arange(nx) * h
        xH = xI + 0.5 * h
        rK = (np.arange(nr + 1) + 0.5) * dr
        rJ = np.arange(nr + 1) * dr

        def smp(name, xs, rs, t):
            if shift and shift[0] == name:
                xs, rs = (xs + 0.5 * h, rs) if shift[1] == "x" else (xs, rs + 0.5 * dr)
            return F.modes(name, xs, rs, t)

        def state(t, te):
            Er, Bt = smp("Er", xI, rK[:nr], t), smp("Bt", xI, rK[:nr], t)
            Et, Br = smp("Et", xI, rJ, t), smp("Br", xI, rJ, t)
            return {"Trp0": Er + Bt, "Trm0": Er - Bt, "Ttp0": Et + Br, "Ttm0": Et - Br,
                    "Ex0": smp("Ex", xH, rJ, te), "Bx0": smp("Bx", xH, rK, te)}
        f = Q._bg_fields(c, state(0.0, -0.5 * h), state(h, 0.5 * h), (0j, 0j, 0j))
        S = Q.axion_source(c, f, (0j, 0j, 0j), form).numpy()
        Tn = 16
        th = 2 * math.pi * np.arange(Tn) / Tn
        g_ = {k: F.real(k, xH, rK[:nr], 0.0, th) for k in ("Ex", "Er", "Et", "Bx", "Br", "Bt")}
        dot = g_["Ex"] * g_["Bx"] + g_["Er"] * g_["Br"] + g_["Et"] * g_["Bt"]
        ee = np.exp(1j * np.outer(np.arange(M), th))
        ref = np.einsum("mt,trx->mrx", ee, dot) / Tn
        ref[1:] *= 2
        sl = slice(3, nx - 3)
        d, ref = S[:, : nr - 1, sl], ref[:, : nr - 1, sl]
        rr = rK[: nr - 1]
        err = np.abs(d - ref) / np.abs(ref).max()
        w = rr * dr * h
        l2 = np.sqrt((err ** 2 * w[None, :, None]).sum() / (w.sum() * err.shape[0] * err.shape[2]))
        out.append((l2, err[:, 0].max(), err[:, rr >= R_BAND].max()))
    return out


def _source_failures(errs):
    bad = []
    for which in range(3):
        e = [lev[which] for lev in errs]
        if not (e[0] / e[1] >= 3.5 and e[1] / e[2] >= 3.5 and e[2] < 2e-3):
            bad.append((["r-weighted L2", "first half row", "r >= 1"][which], e))
    return bad


@pytest.mark.parametrize("form", ["transport", "eb"])
def test_axion_source_converges_at_second_order(fields, form):
    """S_a (Eqs. source_mode_zero, source_mode_m: E.B of the background set
    brought to (x_{i+1/2}, r_{j+1/2}) at t^n) converges at second order to
    the Cartesian dot product of the analytic fields, in both product orders."""
    assert _source_failures(_source_errors(fields, form)) == []


@pytest.mark.parametrize("shift", [("Er", "r"), ("Et", "r"), ("Br", "x"), ("Bt", "x"), ("Ex", "r"), ("Bx", "x")])
def test_source_half_cell_shift_breaks_second_order(fields, shift):
    assert _source_failures(_source_errors(fields, shift=shift)) != [], shift
