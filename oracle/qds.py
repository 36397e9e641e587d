"""CPU oracle for the quasi-cylindrical direction-splitting (QDS) field advance.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the HIP product path
never calls it and shares no code with it.

A plain, slow, float64 / complex128 implementation written from the paper's
update equations with PyTorch CPU tensor operations (functional style, so that
autograd can differentiate a run for the adjoint checks).  Every array of one
set of fields has shape [M, rows, nx] (mode, radial row, axial column).

Staggering (inferred from the subscripts of Sec. 2.1-2.3, the staggering figure
itself is missing):
  T_r^+-, E_r, B_theta, j_r : (x_i,      r_{j+1/2}, t^n)       "I,K" arrays, nr rows
  T_th^+-, E_theta, B_r, j_th: (x_i,     r_j,       t^n)       "I,J" arrays, nr+1 rows
  E_x, j_x                  : (x_{i+1/2}, r_j,       t^{n-1/2}) "H,J" arrays, nr+1 rows
  B_x                       : (x_{i+1/2}, r_{j+1/2}, t^{n-1/2}) "H,K" arrays, + ghost row
  phi                       : (x_{i+1/2}, r_{j+1/2}, t^n)       "H,K"
  T_a^+-                    : (x_i,      r_{j+1/2}, t^{n-1/2})  "I,K"
H ("half-x") arrays hold cell i at x_{i+1/2}; with open or window x boundaries
the last column (i = nx-1) lies outside the domain and is kept at zero.
Row nr of the K arrays is the exterior ghost row r_{nr+1/2} used by the outer
radial boundary.

Pins hold it to what the paper and the mathematics fix (tests/test_oracle_pins.py,
test_oracle_axion_current_convergence.py, test_oracle_outer_boundary.py,
test_stability_bound.py, test_theta_grid_pin.py, test_identities.py): dispersion
relations, waveguide spectra, exact one-cell transport, the theta-product form
of the mode convolutions, photon-axion conversion and its reverse through j_a,
plasma oscillation, second-order convergence of S_a and of j_a at every source
point (axis rows included) to the continuous E.B and B d_t phi - E x grad phi,
the exterior ghosts of the open radial boundary against exact outgoing Hankel
waves at second order, outgoing shells, white lab-frame drive noise, and more.
No function here is parity-unpinned.

State keys (s = 0 background set, s = 1 axion-regenerated set):
  Trp{s} Trm{s} [M,nr,nx]   Ttp{s} Ttm{s} [M,nr+1,nx]   Ex{s} [M,nr+1,nx]
  Bx{s} [M,nr+1,nx] (row nr = ghost)   Bg{s} [M,nx] ghost B_theta at r_{nr+1/2}
  jx{s} [M,nr+1,nx] (t^{n-1})  jr{s} [M,nr,nx] (t^{n-1/2})  jt{s} [M,nr+1,nx] (t^{n-1/2})
  phi [M,nr,nx]  Tap Tam [M,nr,nx]  phig [M,nx] (ghost phi^n at r_{nr+1/2})
  n (step counter), w (moving-window offset in cells)
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, Optional, Tuple

import torch

from oracle import rng as orng

CDT = torch.complex128
RDT = torch.float64


@dataclass(frozen=True)
class Grid:
    nx: int
    nr: int
    nmodes: int
    h: float            # dx = c dt
    dr: float
    x_bc: str = "open"  # open | periodic | window
    r_bc: str = "open"  # open | pec


@dataclass(frozen=True)
class Physics:
    wp2: float = 0.0
    axion: bool = False
    arem: bool = False
    ma2: float = 0.0
    s_phi: float = 1.0
    s_j: float = 1.0
    bext: Tuple[complex, complex, complex] = (0j, 0j, 0j)
    drive: Optional[object] = None   # inputs.Drive
    axion_rbc: str = "mur"           # mur | three_level (the latter only for its instability test)
    # evaluation order of the transverse products in S_a and in the theta and r
    # components of j_a: "transport" collects them in the transport variables
    # (see axion_source), "eb" forms the literal E and B products
    product_form: str = "transport"


def grid_physics(wl) -> Tuple[Grid, Physics]:
    g = Grid(wl.nx, wl.nr, wl.nmodes, wl.h, wl.dr, wl.x_bc, wl.r_bc)
    p = Physics(wl.wp2, wl.axion, wl.arem, wl.ma2, wl.s_phi, wl.s_j, tuple(wl.bext), wl.drive)
    return g, p


# ----------------------------------------------------------------------------
# small helpers
# ----------------------------------------------------------------------------

def _sx(a: torch.Tensor, s: int, periodic: bool) -> torch.Tensor:
    """result[..., i] = a[..., i + s]; zero beyond the ends unless periodic."""
    if periodic:
        return torch.roll(a, -s, dims=-1)
    nx = a.shape[-1]
    z = torch.zeros_like(a[..., : abs(s)])
    if s > 0:
        return torch.cat([a[..., s:], z], dim=-1)
    return torch.cat([z, a[..., : nx + s]], dim=-1)


class _Ctx:
    """Geometry shared by the stages of one step."""

    def __init__(self, g: Grid):
        self.g = g
        self.M, self.nr, self.nx = g.nmodes, g.nr, g.nx
        self.h, self.dr = g.h, g.dr
        self.per = g.x_bc == "periodic"
        self.open_r = g.r_bc == "open"
        live = torch.ones(g.nx, dtype=RDT)
        if not self.per:
            live[g.nx - 1] = 0.0
        self.live = live                                            # H-cell mask
        self.m = torch.arange(g.nmodes, dtype=RDT).view(-1, 1, 1)   # [M,1,1]
        self.im = 1j * self.m.to(CDT)
        self.rJ = (g.dr * torch.arange(g.nr + 1, dtype=RDT)).view(1, -1, 1)
        self.rK = (g.dr * (torch.arange(g.nr, dtype=RDT) + 0.5)).view(1, -1, 1)
        # ghost parity across the axis (Sec. 2.3 regularity): a scalar or
        # longitudinal mode m (B_x, phi, T_a) behaves as r^m near the axis, so
        # its ghost at r_{-1/2} is (-1)^m times the value at r_{1/2}; a
        # transverse component (E_r, B_theta) of mode m != 1 as r^|m-1|,
        # parity (-1)^(m-1) (mode 1 takes the axis relation instead)
        self.par = torch.tensor([(-1.0) ** m for m in range(g.nmodes)], dtype=RDT).view(-1, 1)
        self.tpar = torch.tensor([(-1.0) ** (m - 1) for m in range(g.nmodes)], dtype=RDT).view(-1, 1)

    def xp(self, a):   # value at i+1
        return _sx(a, 1, self.per)

    def xm(self, a):   # value at i-1
        return _sx(a, -1, self.per)

    def xavg(self, a):  # I positions (i, i+1) -> H cell i
        return 0.5 * (a + self.xp(a))


# ----------------------------------------------------------------------------
# azimuthal mode convolution  C_m{A, B}  (Sec. 2.2, Eqs. source_mode_zero,
# source_mode_m, mode_convolution)
# ----------------------------------------------------------------------------

def mode_conv(A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """C_m{A,B} for m = 0..M-1 written as the paper's three sums; a negative
    mode index means the complex conjugate, F^(-k) = conj(F^(k)) (Eq.
    fourier_decomp), for k = 0 too."""
    M = A.shape[0]

    def neg(F, k):
        return F[k].conj()

    out = []
    s0 = A[0] * B[0]
    for k in range(1, M):
        s0 = s0 + 0.5 * (A[k] * neg(B, k)).real
    out.append(s0)
    for m in range(1, M):
        acc = torch.zeros_like(A[0])
        for k in range(M):
            for l in range(M):
                if k + l == m:
                    acc = acc + A[k] * B[l]
                if k - l == m:
                    acc = acc + A[k] * neg(B, l)
                if l - k == m:
                    acc = acc + neg(A, k) * B[l]
        out.append(0.5 * acc)
    return torch.stack(out)


# ----------------------------------------------------------------------------
# prescribed drive (stand-in for deposited current)
# ----------------------------------------------------------------------------

def drive_jx(c: _Ctx, drv, n: int, w: int) -> torch.Tensor:
    """j_x^(0) at (x_{i+1/2}, r_j, t^n), lab frame x = (i + 1/2 + w) h."""
    out = torch.zeros(c.M, c.nr + 1, c.nx, dtype=CDT)
    if drv is None:
        return out
    i = torch.arange(c.nx, dtype=RDT)
    x = (i + 0.5 + w) * c.h
    t = n * c.h
    gx = torch.exp(-((x - drv.x0 - drv.v * t) ** 2) / (2.0 * drv.sx ** 2))
    r = c.rJ.view(-1)
    gr = torch.exp(-((r - drv.r0) ** 2) / (2.0 * drv.sr ** 2))
    xi = orng.normal_field(drv.seed, n, c.nx, c.nr + 1, w)
    val = drv.amp * gr.view(-1, 1) * gx.view(1, -1) * (1.0 + drv.noise * xi)
    out = out.clone()
    out[0] = val.to(CDT) * c.live
    return out


# ----------------------------------------------------------------------------
# one electromagnetic set (Sec. 2.1, 2.3, 3.2)
# ----------------------------------------------------------------------------

def em_set(c: _Ctx, st: Dict, s: int, wp2: float, jx_add, jr_add, jt_add) -> Dict:
    """Advance set ``s`` from (T^n, E_x^{n-1/2}, B_x^{n-1/2}) to
    (T^{n+1}, E_x^{n+1/2}, B_x^{n+1/2}).

    jx_add [M,nr+1,nx] at (x_{i+1/2}, r_j, t^n), jr_add [M,nr,nx] at
    (x_{i+1/2}, r_{j+1/2}, t^{n+1/2}), jt_add [M,nr+1,nx] at
    (x_{i+1/2}, r_j, t^{n+1/2}) are extra currents already at the source points.
    """
    M, nr, h, dr = c.M, c.nr, c.h, c.dr
    live = c.live
    Trp, Trm, Ttp, Ttm = st[f"Trp{s}"], st[f"Trm{s}"], st[f"Ttp{s}"], st[f"Ttm{s}"]
    Ex, Bx, Bg = st[f"Ex{s}"], st[f"Bx{s}"], st[f"Bg{s}"]
    jx, jr, jt = st[f"jx{s}"], st[f"jr{s}"], st[f"jt{s}"]

    # field reconstruction at t^n (Eq. reconstruct_fields)
    Er, Bth = 0.5 * (Trp + Trm), 0.5 * (Trp - Trm)
    Eth, Br = 0.5 * (Ttp + Ttm), 0.5 * (Ttp - Ttm)

    # cold linear plasma response, leapfrogged with the fields it responds to
    jx_n = jx + h * wp2 * Ex          # t^n
    jr_h = jr + h * wp2 * Er          # t^{n+1/2}
    jt_h = jt + h * wp2 * Eth         # t^{n+1/2}

    # total currents at the source points; r and theta currents averaged from
    # their integer-x positions to x_{i+1/2} (Sec. 3.1, last paragraph)
    JX = (jx_n + jx_add) * live
    JR = (c.xavg(jr_h) + jr_add) * live
    JT = (c.xavg(jt_h) + jt_add) * live

    # ---- longitudinal fields: E_x, B_x leapfrog (Eqs. Ex_update, Gammax/Phix_explicit)
    BthF = torch.cat([Bth, Bg.unsqueeze(1)], dim=1)          # K rows 0..nr (row nr = ghost)
    lo, hi = BthF[:, 0:nr], BthF[:, 1:nr + 1]                # K rows j-1, j for J row j=1..nr
    Bth_avg = 0.25 * (lo + hi + c.xp(lo) + c.xp(hi))
    dBth = ((hi + c.xp(hi)) - (lo + c.xp(lo))) / (2.0 * dr)
    Br_avg = c.xavg(Br[:, 1:])
    rj = c.rJ[:, 1:]
    Gx = Bth_avg / rj + dBth + c.im * Br_avg / rj - JX[:, 1:]
    Ex_rows = Ex[:, 1:] + h * Gx
    # on-axis E_x: Gauss form for m = 0 (Eq. axis_Ex), zero for m >= 1
    Gx0 = (4.0 / dr) * c.xavg(Bth[0, 0]) - JX[0, 0]
    ax = torch.zeros(M, 1, c.nx, dtype=CDT)
    ax = torch.cat([(Ex[0, 0] + h * Gx0).view(1, 1, -1), ax[1:]], dim=0)
    Ex_new = torch.cat([ax, Ex_rows], dim=1) * live
    if not c.open_r:
        Ex_new = torch.cat([Ex_new[:, :nr], torch.zeros_like(Ex_new[:, nr:])], dim=1)

    lo, hi = Eth[:, 0:nr], Eth[:, 1:nr + 1]
    Eth_avg = 0.25 * (lo + hi + c.xp(lo) + c.xp(hi))
    dEth = ((hi + c.xp(hi)) - (lo + c.xp(lo))) / (2.0 * dr)
    Er_avg = c.xavg(Er)
    rk = c.rK
    Fx = -(Eth_avg / rk + dEth) - c.im * Er_avg / rk
    Bx_int = (Bx[:, :nr] + h * Fx) * live

    kap = (dr - h) / (dr + h)
    cR = 2.0 * h * dr / (dr + h)
    rN = nr * dr
    imv = c.im.view(M, 1)
    if c.open_r:
        # outflow at r = R_max for B_x (Eq. em_r_open_bx), centred at (r_nr, t^n)
        # on the ghost row r_{nr+1/2} with a Mur-type average
        Rx = (0.5 * (c.xp(Br[:, nr]) - Br[:, nr]) / h
              - (c.xavg(Eth[:, nr]) + imv * c.xavg(Er[:, nr - 1])) / (2.0 * rN)
              - 0.5 * JT[:, nr])
        Bx_gh = (Bx[:, nr - 1] + kap * (Bx[:, nr] - Bx_int[:, nr - 1]) + cR * Rx) * live
    else:
        Bx_gh = torch.zeros_like(Bx[:, nr])
    Bx_new = torch.cat([Bx_int, Bx_gh.unsqueeze(1)], dim=1)

    # ---- transverse transport: shift by one cell plus dt * source at t^{n+1/2}
    # (Eqs. Trp/Trm/Ttp/Ttm_update and the source terms that follow them)
    Gr = -c.im * Bx_int / rk - JR
    Pr = (Ex_new[:, 1:] - Ex_new[:, :nr]) / dr
    Sp = h * (Gr + Pr) * live
    Sm = h * (Gr - Pr) * live
    Trp_new = c.xm(Trp + Sp)            # T_r^+(i+1) <- T_r^+(i) + dt (G_r + P_r)(i+1/2)
    Trm_new = c.xp(Trm) + Sm            # T_r^-(i)   <- T_r^-(i+1) + dt (G_r - P_r)(i+1/2)

    Gt = -(Bx_new[:, 1:nr + 1] - Bx_new[:, 0:nr]) / dr - JT[:, 1:]
    Pt = c.im * Ex_new[:, 1:] / rj
    # on-axis T_theta for m = 1 (Eq. axis_Ttheta); other modes vanish there
    Gt0 = torch.zeros(M, 1, c.nx, dtype=CDT)
    Pt0 = torch.zeros(M, 1, c.nx, dtype=CDT)
    if M > 1:
        g1 = (-(2.0 / dr) * Bx_int[1, 0] - JT[1, 0]).view(1, 1, -1)
        p1 = (1j * Ex_new[1, 1] / dr).view(1, 1, -1)
        Gt0 = torch.cat([Gt0[:1], g1, Gt0[2:]], dim=0)
        Pt0 = torch.cat([Pt0[:1], p1, Pt0[2:]], dim=0)
    Gt = torch.cat([Gt0, Gt], dim=1)
    Pt = torch.cat([Pt0, Pt], dim=1)
    Sp = h * (Gt + Pt) * live
    Sm = h * (Gt - Pt) * live
    Ttp_new = c.xp(Ttp) + Sp            # left mover
    Ttm_new = c.xm(Ttm + Sm)            # right mover
    axis_keep = torch.zeros(M, 1, 1, dtype=RDT)
    if M > 1:
        axis_keep[1] = 1.0
    rowmask = torch.ones(1, nr + 1, 1, dtype=RDT)
    Ttp_new = torch.cat([Ttp_new[:, :1] * axis_keep, Ttp_new[:, 1:]], dim=1)
    Ttm_new = torch.cat([Ttm_new[:, :1] * axis_keep, Ttm_new[:, 1:]], dim=1)
    if not c.open_r:
        rowmask[0, nr, 0] = 0.0
        Ttp_new = Ttp_new * rowmask
        Ttm_new = Ttm_new * rowmask

    # outflow for B_theta (Eq. em_r_open_bt) on the ghost row, RHS at t^n
    if c.open_r:
        Bth_new_top = 0.5 * (Trp_new[:, nr - 1] - Trm_new[:, nr - 1])
        I0 = Bth[:, nr - 1]
        dxEr = (c.xp(Er[:, nr - 1]) - c.xm(Er[:, nr - 1])) / (2.0 * h)
        jx_I = 0.5 * (JX[:, nr] + c.xm(JX[:, nr]))
        Rt = -0.5 * dxEr - (0.5 * (I0 + Bg) + imv * Br[:, nr]) / (2.0 * rN) + 0.5 * jx_I
        Bg_new = I0 + kap * (Bg - Bth_new_top) + cR * Rt
    else:
        Bg_new = torch.zeros_like(Bg)

    out = {f"Trp{s}": Trp_new, f"Trm{s}": Trm_new, f"Ttp{s}": Ttp_new, f"Ttm{s}": Ttm_new,
           f"Ex{s}": Ex_new, f"Bx{s}": Bx_new, f"Bg{s}": Bg_new}
    if wp2 != 0.0:
        out.update({f"jx{s}": jx_n, f"jr{s}": jr_h, f"jt{s}": jt_h * rowmask})
    else:
        out.update({f"jx{s}": jx, f"jr{s}": jr, f"jt{s}": jt})
    return out


# ----------------------------------------------------------------------------
# axion: source, Klein-Gordon transport, regenerated-field current (Sec. 2.2, 3.2)
# ----------------------------------------------------------------------------

def _bg_fields(c: _Ctx, st: Dict, new: Dict, bext):
    """Background (set 0) fields at t^n, t^{n+1} and the longitudinal ones at
    t^{n-1/2}, t^{n+1/2}; the uniform external field is kept separately."""
    f = {}
    f["Er0"] = 0.5 * (st["Trp0"] + st["Trm0"])
    f["Bt0"] = 0.5 * (st["Trp0"] - st["Trm0"])
    f["Et0"] = 0.5 * (st["Ttp0"] + st["Ttm0"])
    f["Br0"] = 0.5 * (st["Ttp0"] - st["Ttm0"])
    f["Er1"] = 0.5 * (new["Trp0"] + new["Trm0"])
    f["Bt1"] = 0.5 * (new["Trp0"] - new["Trm0"])
    f["Et1"] = 0.5 * (new["Ttp0"] + new["Ttm0"])
    f["Br1"] = 0.5 * (new["Ttp0"] - new["Ttm0"])
    for k in ("Trp0", "Trm0", "Ttp0", "Ttm0"):
        f[k.replace("0", "") + "_o"] = st[k]
        f[k.replace("0", "") + "_n"] = new[k]
    f["Exo"], f["Exh"] = st["Ex0"], new["Ex0"]
    f["Bxo"], f["Bxh"] = st["Bx0"][:, : c.nr], new["Bx0"][:, : c.nr]
    return f


def _ext(c: _Ctx, bext, comp: int) -> torch.Tensor:
    """Uniform external magnetic field as a [M,1,1] mode vector: component 0 is
    B_x^(0), 1 is B_r^(1), 2 is B_theta^(1)."""
    v = torch.zeros(c.M, 1, 1, dtype=CDT)
    val = complex(bext[comp])
    mode = 0 if comp == 0 else 1
    if mode < c.M and val != 0:
        v = v.clone()
        v[mode] = val
    return v


def axion_source(c: _Ctx, f: Dict, bext, form: str = "transport") -> torch.Tensor:
    """S_a^n = sum_alpha C_m{E_alpha, B_alpha} at (x_{i+1/2}, r_{j+1/2}, t^n)
    (Eqs. source_mode_zero, source_mode_m).

    With E_r, B_theta = (T_r^+ +- T_r^-)/2 and E_theta, B_r = (T_theta^+ +-
    T_theta^-)/2 (Eq. Tdefs), and C_m bilinear and symmetric, the transverse
    products collect exactly into
        C{E_r, B_r} + C{E_theta, B_theta}
            = 1/2 C{T_r^+ + b_theta, T_theta^+ + b_r} - 1/2 C{T_r^- - b_theta, T_theta^- - b_r}
    (b = the uniform external field).  ``form="transport"`` evaluates this
    collected form, whose products pair a large factor with a small one for
    co-propagating waves; ``form="eb"`` the literal products, which cancel to a
    few parts in 10^13 there."""
    nr = c.nr
    Exn = 0.5 * (f["Exo"] + f["Exh"])
    Ex = 0.5 * (Exn[:, :nr] + Exn[:, 1:])
    Bx = 0.5 * (f["Bxo"] + f["Bxh"]) + _ext(c, bext, 0)
    x4 = lambda F: 0.25 * (F[:, :nr] + F[:, 1:] + c.xp(F[:, :nr]) + c.xp(F[:, 1:]))
    if form == "transport":
        bt, br = _ext(c, bext, 2), _ext(c, bext, 1)
        Pp, Pm = c.xavg(f["Trp_o"]), c.xavg(f["Trm_o"])
        Qp, Qm = x4(f["Ttp_o"]), x4(f["Ttm_o"])
        S = mode_conv(Ex, Bx) + 0.5 * mode_conv(Pp + bt, Qp + br) - 0.5 * mode_conv(Pm - bt, Qm - br)
        return S * c.live
    Er = c.xavg(f["Er0"])
    Bt = c.xavg(f["Bt0"]) + _ext(c, bext, 2)
    Et = x4(f["Et0"])
    Br = x4(f["Br0"]) + _ext(c, bext, 1)
    S = mode_conv(Ex, Bx) + mode_conv(Er, Br) + mode_conv(Et, Bt)
    return S * c.live


def kg_update(c: _Ctx, st: Dict, S: torch.Tensor, ph: Physics) -> Dict:
    """Klein-Gordon transport: T_a^{n-1/2} -> T_a^{n+1/2} (Eqs. Ta_plus_update,
    Ta_minus_update), phi^n -> phi^{n+1} (Eq. phi_update), zero inflow at the x
    ends (Eq. axion_x_open).

    Outer radial boundary: the outgoing-wave condition (d_t + c d_r) phi = 0
    (Eq. axion_r_sommerfeld) fixes the exterior ghost phi at r_{nr+1/2}, which
    enters Gamma_a of the outermost row.  The ghost is advanced with the
    two-level (Mur) centring of that condition at (r_{nr}, t^{n+1/2}); the
    paper's three-level update of the outermost row (Eq. axion_r_update) is
    kept in ``kg_update_three_level`` only to show that at c dt = dx it is
    unstable for the x-Nyquist mode.
    """
    if ph.axion_rbc == "three_level" and c.open_r:
        return kg_update_three_level(c, st, S, ph)
    nr, h, dr = c.nr, c.h, c.dr
    phi, Tap, Tam, G = st["phi"], st["Tap"], st["Tam"], st["phig"]
    msq = c.m * c.m
    rk = c.rK
    src = ph.s_phi * S
    if not c.open_r:
        G = torch.zeros_like(G)
    up = torch.cat([phi[:, 1:], G.unsqueeze(1)], dim=1)
    dn = torch.cat([torch.zeros_like(phi[:, :1]), phi[:, :-1]], dim=1)  # axis ghost has zero weight
    # Gamma_a at (x_{i+1/2}, r_{j+1/2}, t^n): radial Laplacian of mode m by
    # centred differences, mass term and source
    Ga = ((up - 2.0 * phi + dn) / dr ** 2 + (up - dn) / (2.0 * dr * rk)
          - (msq / rk ** 2 + ph.ma2) * phi + src) * c.live
    Tap_new = c.xm(Tap + h * Ga)     # T_a^+(i+1) <- T_a^+(i) + c dt Gamma_a(i+1/2)
    Tam_new = c.xp(Tam) + h * Ga     # T_a^-(i)   <- T_a^-(i+1) + c dt Gamma_a(i+1/2)
    phi_new = (phi + (h / 4.0) * (Tap_new + c.xp(Tap_new) + Tam_new + c.xp(Tam_new))) * c.live
    if c.open_r:
        kap = (dr - h) / (dr + h)
        G_new = (phi[:, nr - 1] + kap * (G - phi_new[:, nr - 1])) * c.live
    else:
        G_new = G
    return {"phi": phi_new, "Tap": Tap_new, "Tam": Tam_new, "phig": G_new}


def kg_update_three_level(c: _Ctx, st: Dict, S: torch.Tensor, ph: Physics) -> Dict:
    """The paper's literal outer-row treatment (Eqs. axion_r_ghost,
    axion_r_update): the outermost phi row takes the three-level value and the
    ghost follows from the centred outgoing condition.  Here ``phig`` holds
    phi^{n-1} of the outermost row.  Not used by the advance (unstable at
    c dt = dx); kept for the test that shows it."""
    nr, h, dr = c.nr, c.h, c.dr
    phi, Tap, Tam, phim = st["phi"], st["Tap"], st["Tam"], st["phig"]
    msq = c.m * c.m
    src = ph.s_phi * S
    rk = c.rK
    N = nr - 1
    rN = (N + 0.5) * dr
    mN = msq.view(-1, 1)
    A = 1.0 / h ** 2 + 1.0 / (dr * h) + 1.0 / (2.0 * rN * h)
    Rb = ((c.xp(phi[:, N]) - 2.0 * phi[:, N] + c.xm(phi[:, N])) / h ** 2
          - mN / rN ** 2 * phi[:, N]
          + (2.0 / dr ** 2) * (phi[:, N - 1] - phi[:, N])
          - ph.ma2 * phi[:, N] + src[:, N])
    phiN = (-(1.0 / h ** 2 - 1.0 / (dr * h) - 1.0 / (2.0 * rN * h)) * phim
            + (2.0 / h ** 2) * phi[:, N] + Rb) / A
    phiN = phiN * c.live
    ghost = phi[:, N - 1] - (dr / h) * (phiN - phim)
    up = torch.cat([phi[:, 1:], ghost.unsqueeze(1)], dim=1)
    dn = torch.cat([torch.zeros_like(phi[:, :1]), phi[:, :-1]], dim=1)
    Ga = ((up - 2.0 * phi + dn) / dr ** 2 + (up - dn) / (2.0 * dr * rk)
          - (msq / rk ** 2 + ph.ma2) * phi + src) * c.live
    Tap_new = c.xm(Tap + h * Ga)
    Tam_new = c.xp(Tam) + h * Ga
    phi_new = (phi + (h / 4.0) * (Tap_new + c.xp(Tap_new) + Tam_new + c.xp(Tam_new))) * c.live
    phi_new = torch.cat([phi_new[:, :nr - 1], phiN.unsqueeze(1)], dim=1)
    return {"phi": phi_new, "Tap": Tap_new, "Tam": Tam_new, "phig": phi[:, N]}


def ja_x_modes(Bx, dtphi, Er, dth_phi_r, Et, drphi):
    """Mode m of j_a,x = B_x d_t phi - (1/r) E_r d_theta phi + E_theta d_r phi
    (Eq. jax_mode, scaled units); ``dth_phi_r`` is (d_theta phi)/r."""
    return mode_conv(Bx, dtphi) - mode_conv(Er, dth_phi_r) + mode_conv(Et, drphi)


def ja_r_modes(Br, dtphi, Et, dxphi, Ex, dth_phi_r):
    """j_a,r = B_r d_t phi - E_theta d_x phi + (1/r) E_x d_theta phi (Eq. jar_mode)."""
    return mode_conv(Br, dtphi) - mode_conv(Et, dxphi) + mode_conv(Ex, dth_phi_r)


def ja_t_modes(Bt, dtphi, Ex, drphi, Er, dxphi):
    """j_a,theta = B_theta d_t phi - E_x d_r phi + E_r d_x phi (Eq. jat_mode)."""
    return mode_conv(Bt, dtphi) - mode_conv(Ex, drphi) + mode_conv(Er, dxphi)


def _k2j(c: _Ctx, F: torch.Tensor, g0: torch.Tensor) -> torch.Tensor:
    """K rows -> J rows 0..nr-1 by the mean of r_{j-1/2} and r_{j+1/2};
    ``g0`` is the ghost value at r_{-1/2}."""
    lo = torch.cat([g0.unsqueeze(1), F[:, :-1]], dim=1)
    return 0.5 * (lo + F)


def _ghost_par(c: _Ctx, F: torch.Tensor) -> torch.Tensor:
    return c.par.to(F.dtype) * F[:, 0]


def _ghost_Er(c: _Ctx, Er: torch.Tensor, Et: torch.Tensor) -> torch.Tensor:
    """E_r at r_{-1/2}: the m = 1 reflection through the axis relation
    T_r^+-(-1/2) = 2i T_th^-+(0) - T_r^+-(1/2) (Eq. axis_Tr), parity
    (-1)^(m-1) otherwise."""
    g = c.tpar.to(Er.dtype) * Er[:, 0]
    if c.M > 1:
        g = torch.cat([g[:1], (2j * Et[1, 0] - Er[1, 0]).view(1, -1), g[2:]], dim=0)
    return g


def _ghost_Bt(c: _Ctx, Bt: torch.Tensor, Br: torch.Tensor) -> torch.Tensor:
    """B_theta at r_{-1/2} from the same reflection: -2i B_r(0) - B_theta(1/2)
    for m = 1, parity (-1)^(m-1) otherwise."""
    g = c.tpar.to(Bt.dtype) * Bt[:, 0]
    if c.M > 1:
        g = torch.cat([g[:1], (-2j * Br[1, 0] - Bt[1, 0]).view(1, -1), g[2:]], dim=0)
    return g


def axion_current(c: _Ctx, f: Dict, st: Dict, kg: Dict, bext, form: str = "transport") -> Tuple[torch.Tensor, ...]:
    """Mode expansion of j_a = B_0 d_t phi - E_0 x grad phi (Eqs. jax_mode,
    jar_mode, jat_mode), each component evaluated directly at the source point
    of the regenerated set: j_a,x at (x_{i+1/2}, r_j, t^n), j_a,r at
    (x_{i+1/2}, r_{j+1/2}, t^{n+1/2}), j_a,theta at (x_{i+1/2}, r_j, t^{n+1/2}).
    Off-grid values are centred means of the nearest samples; d_t phi and d_x phi
    come from T_a (Eq. phi_update); d_theta phi^(l) = -i l phi^(l).  The
    components on the outer integer row r_nr are set to zero.

    ``form="transport"`` collects the theta and r components in the transport
    variables (T_a^+- = d_t phi -+ d_x phi, Eq. T_axion_def; Eq. Tdefs):
        C{B_theta, d_t phi} + C{E_r, d_x phi} = 1/2 C{T_r^+ + b_theta, T_a^-} - 1/2 C{T_r^- - b_theta, T_a^+}
        C{B_r, d_t phi} - C{E_theta, d_x phi} = 1/2 C{T_theta^+ + b_r, T_a^+} - 1/2 C{T_theta^- - b_r, T_a^-}
    with every factor brought to the source point by the same means (the axis
    ghosts combine likewise: T_r^+- at r_{-1/2} = 2i T_theta^-+(0) - T_r^+-(1/2)
    for m = 1)."""
    M, nr, dr = c.M, c.nr, c.dr
    mv = c.m.to(CDT)
    phi0, phi1 = st["phi"], kg["phi"]
    phih = 0.5 * (phi0 + phi1)
    dt_o = 0.5 * (st["Tap"] + st["Tam"])
    dt_h = 0.5 * (kg["Tap"] + kg["Tam"])
    dx_h = 0.5 * (kg["Tam"] - kg["Tap"])
    rJ = c.rJ[:, :nr]
    r_half = 0.5 * dr

    def k2j_par(F):
        return _k2j(c, F, _ghost_par(c, F))

    def dr_par(F):   # (F_{j+1/2} - F_{j-1/2}) / dr at J rows 0..nr-1
        lo = torch.cat([_ghost_par(c, F).unsqueeze(1), F[:, :-1]], dim=1)
        return (F - lo) / dr

    def dth_over_r_J(F):   # (d_theta F)/r at J rows, axis by its r_{1/2} value
        FJ = k2j_par(F)
        rows = -1j * mv * FJ[:, 1:] / rJ[:, 1:]
        ax = torch.zeros(M, 1, c.nx, dtype=CDT)
        if M > 1:
            ax = torch.cat([ax[:1], (-1j * F[1, 0] / r_half).view(1, 1, -1), ax[2:]], dim=0)
        return torch.cat([ax, rows], dim=1)

    def zrow(a):
        return torch.cat([a, torch.zeros_like(a[:, :1])], dim=1) * c.live

    # ---- j_a,x at t^n
    Bxn = 0.5 * (f["Bxo"] + f["Bxh"])
    BxJ = k2j_par(Bxn) + _ext(c, bext, 0)
    dtn = 0.5 * (dt_o + dt_h)                       # I,K at t^n
    dtJ = c.xavg(k2j_par(dtn))
    ErJ = c.xavg(_k2j(c, f["Er0"], _ghost_Er(c, f["Er0"], f["Et0"])))
    EtJ = c.xavg(f["Et0"][:, :nr])
    drJ = dr_par(phi0)
    pthJ = dth_over_r_J(phi0)
    jax = ja_x_modes(BxJ, dtJ, ErJ, pthJ, EtJ, drJ)

    # ---- j_a,r at t^{n+1/2}
    x4 = lambda F: 0.25 * (F[:, :nr] + F[:, 1:] + c.xp(F[:, :nr]) + c.xp(F[:, 1:]))
    ExK = 0.5 * (f["Exh"][:, :nr] + f["Exh"][:, 1:])
    pthK = -1j * mv * phih / c.rK
    br, bt = _ext(c, bext, 1), _ext(c, bext, 2)
    if form == "transport":
        Qp = x4(0.5 * (f["Ttp_o"] + f["Ttp_n"]))
        Qm = x4(0.5 * (f["Ttm_o"] + f["Ttm_n"]))
        ApK, AmK = c.xavg(kg["Tap"]), c.xavg(kg["Tam"])
        jar = (0.5 * mode_conv(Qp + br, ApK) - 0.5 * mode_conv(Qm - br, AmK) + mode_conv(ExK, pthK))
    else:
        Brh = 0.5 * (f["Br0"] + f["Br1"])
        Eth = 0.5 * (f["Et0"] + f["Et1"])
        BrK = x4(Brh) + br
        EtK = x4(Eth)
        dtK = c.xavg(dt_h)
        dxK = c.xavg(dx_h)
        jar = ja_r_modes(BrK, dtK, EtK, dxK, ExK, pthK)

    # ---- j_a,theta at t^{n+1/2}
    ExJ = f["Exh"][:, :nr]
    drJh = dr_par(phih)
    if form == "transport":
        Ph = 0.5 * (f["Trp_o"] + f["Trp_n"])
        Nh = 0.5 * (f["Trm_o"] + f["Trm_n"])
        Tph = 0.5 * (f["Ttp_o"] + f["Ttp_n"])
        Tmh = 0.5 * (f["Ttm_o"] + f["Ttm_n"])
        # axis ghosts at r_{-1/2}: parity (-1)^(m-1) for m != 1, the axis
        # relation for m = 1
        tp = c.tpar.to(Ph.dtype)
        gP, gN = tp * Ph[:, 0], tp * Nh[:, 0]
        if M > 1:
            gP = torch.cat([gP[:1], (2j * Tmh[1, 0] - Ph[1, 0]).view(1, -1), gP[2:]], dim=0)
            gN = torch.cat([gN[:1], (2j * Tph[1, 0] - Nh[1, 0]).view(1, -1), gN[2:]], dim=0)
        PJ = c.xavg(_k2j(c, Ph, gP)) + bt
        NJ = c.xavg(_k2j(c, Nh, gN)) - bt
        AmJ = c.xavg(k2j_par(kg["Tam"]))
        ApJ = c.xavg(k2j_par(kg["Tap"]))
        jat = 0.5 * mode_conv(PJ, AmJ) - 0.5 * mode_conv(NJ, ApJ) - mode_conv(ExJ, drJh)
    else:
        Brh = 0.5 * (f["Br0"] + f["Br1"])
        Eth = 0.5 * (f["Et0"] + f["Et1"])
        Bth = 0.5 * (f["Bt0"] + f["Bt1"])
        Erh = 0.5 * (f["Er0"] + f["Er1"])
        BtJ = c.xavg(_k2j(c, Bth, _ghost_Bt(c, Bth, Brh))) + bt
        dtJh = c.xavg(k2j_par(dt_h))
        ErJh = c.xavg(_k2j(c, Erh, _ghost_Er(c, Erh, Eth)))
        dxJh = c.xavg(k2j_par(dx_h))
        jat = ja_t_modes(BtJ, dtJh, ExJ, drJh, ErJh, dxJh)

    return zrow(jax), jar * c.live, zrow(jat)


# ----------------------------------------------------------------------------
# one full step and runs
# ----------------------------------------------------------------------------

def step(st: Dict, g: Grid, ph: Physics, ext: Optional[Tuple[torch.Tensor, ...]] = None) -> Dict:
    """One step n -> n+1 of the whole advance: background set, axion, regenerated set.
    ``ext`` = (j_x at t^n [M,nr+1,nx], j_r at t^{n+1/2} [M,nr,nx], j_theta at
    t^{n+1/2} [M,nr+1,nx]), already at the source points x_{i+1/2}, is an
    extra current of the background set (the particle currents of the PIC
    coupling)."""
    c = _Ctx(g)
    n, w = st["n"], st["w"]
    zJ = torch.zeros(c.M, c.nr + 1, c.nx, dtype=CDT)
    zK = torch.zeros(c.M, c.nr, c.nx, dtype=CDT)
    jx_drive = drive_jx(c, ph.drive, n, w) if ph.drive is not None else zJ
    if ext is None:
        new = em_set(c, st, 0, ph.wp2, jx_drive, zK, zJ)
    else:
        new = em_set(c, st, 0, ph.wp2, jx_drive + ext[0], ext[1], ext[2])
    if ph.axion:
        f = _bg_fields(c, st, new, ph.bext)
        S = axion_source(c, f, ph.bext, ph.product_form)
        kg = kg_update(c, st, S, ph)
        new.update(kg)
        if ph.arem:
            jax, jar, jat = axion_current(c, f, st, kg, ph.bext, ph.product_form)
            new.update(em_set(c, st, 1, ph.wp2, ph.s_j * jax, ph.s_j * jar, ph.s_j * jat))
    for k, v in st.items():
        if k not in new and k not in ("n", "w"):
            new[k] = v
    new["n"] = n + 1
    new["w"] = w
    if g.x_bc == "window":
        for k, v in list(new.items()):
            if isinstance(v, torch.Tensor):
                new[k] = _sx(v, 1, False)
        new["w"] = w + 1
    return new


def run(st: Dict, g: Grid, ph: Physics, nsteps: int) -> Dict:
    for _ in range(nsteps):
        st = step(st, g, ph)
    return st


# ----------------------------------------------------------------------------
# state construction
# ----------------------------------------------------------------------------

def zero_state(g: Grid, ph: Physics) -> Dict:
    M, nr, nx = g.nmodes, g.nr, g.nx
    st = {"n": 0, "w": 0}
    sets = [0, 1] if ph.arem else [0]
    for s in sets:
        st[f"Trp{s}"] = torch.zeros(M, nr, nx, dtype=CDT)
        st[f"Trm{s}"] = torch.zeros(M, nr, nx, dtype=CDT)
        st[f"Ttp{s}"] = torch.zeros(M, nr + 1, nx, dtype=CDT)
        st[f"Ttm{s}"] = torch.zeros(M, nr + 1, nx, dtype=CDT)
        st[f"Ex{s}"] = torch.zeros(M, nr + 1, nx, dtype=CDT)
        st[f"Bx{s}"] = torch.zeros(M, nr + 1, nx, dtype=CDT)
        st[f"Bg{s}"] = torch.zeros(M, nx, dtype=CDT)
        st[f"jx{s}"] = torch.zeros(M, nr + 1, nx, dtype=CDT)
        st[f"jr{s}"] = torch.zeros(M, nr, nx, dtype=CDT)
        st[f"jt{s}"] = torch.zeros(M, nr + 1, nx, dtype=CDT)
    if ph.axion:
        st["phi"] = torch.zeros(M, nr, nx, dtype=CDT)
        st["Tap"] = torch.zeros(M, nr, nx, dtype=CDT)
        st["Tam"] = torch.zeros(M, nr, nx, dtype=CDT)
        st["phig"] = torch.zeros(M, nx, dtype=CDT)
    return st


def pulse_modes(pol: str, f):
    """Mode amplitudes (m, E_r, E_theta, B_r, B_theta) of a forward pulse whose
    polarised field is ``f`` (Eq. fourier_decomp with B = x_hat x E):
      E_y = f: E_r^(1) = f, E_th^(1) = -i f, B_r^(1) = i f, B_th^(1) = f
      E_z = f: E_r^(1) = i f, E_th^(1) = f, B_r^(1) = -f, B_th^(1) = i f
      radial E_r^(0) = f with B_th^(0) = f; azimuthal E_th^(0) = f with B_r^(0) = -f."""
    if pol == "y":
        return 1, f, -1j * f, 1j * f, f
    if pol == "z":
        return 1, 1j * f, f, -f, 1j * f
    if pol == "r":
        return 0, f, 0 * f, 0 * f, f
    if pol == "t":
        return 0, 0 * f, f, -f, 0 * f
    raise ValueError(pol)


def init_state(wl, basis: Optional[Tuple[int, int]] = None) -> Dict:
    """State at t = 0 from the workload's pulses sampled at the staggered points.
    E_x = B_x = 0, currents and axion fields zero.  ``basis`` = (pulse, q)
    instead returns the derivative of the state with respect to that pulse's
    envelope coefficient q (the state is linear in it)."""
    g, ph = grid_physics(wl)
    st = zero_state(g, ph)
    import numpy as np
    xI = np.arange(g.nx) * g.h
    rK = (np.arange(g.nr) + 0.5) * g.dr
    rJ = np.arange(g.nr + 1) * g.dr
    pulses = wl.pulses if basis is None else (wl.pulses[basis[0]],)
    for p in pulses:
        if basis is None:
            fK = torch.from_numpy(p.field(xI[None, :], rK[:, None]))
            fJ = torch.from_numpy(p.field(xI[None, :], rJ[:, None]))
        else:
            fK = torch.from_numpy(p.field_basis(xI[None, :], rK[:, None], basis[1]))
            fJ = torch.from_numpy(p.field_basis(xI[None, :], rJ[:, None], basis[1]))
        m, Er, _, _, Bt = pulse_modes(p.pol, fK.to(CDT))
        _, _, Et, Br, _ = pulse_modes(p.pol, fJ.to(CDT))
        if m >= g.nmodes:
            continue
        Trp = st["Trp0"].clone(); Trm = st["Trm0"].clone()
        Ttp = st["Ttp0"].clone(); Ttm = st["Ttm0"].clone()
        Trp[m] += Er + Bt
        Trm[m] += Er - Bt
        Ttp[m] += Et + Br
        Ttm[m] += Et - Br
        st["Trp0"], st["Trm0"], st["Ttp0"], st["Ttm0"] = Trp, Trm, Ttp, Ttm
    # fields on the axis obey the regularity constraints (Sec. 2.3)
    keep = torch.zeros(g.nmodes, 1, dtype=RDT)
    if g.nmodes > 1:
        keep[1] = 1.0
    for k in ("Ttp0", "Ttm0"):
        a = st[k].clone()
        a[:, 0] = a[:, 0] * keep
        st[k] = a
    if g.r_bc == "pec":
        for k in ("Ttp0", "Ttm0"):
            a = st[k].clone()
            a[:, g.nr] = 0
            st[k] = a
    # the outer ghost B_theta at r_{nr+1/2} samples the pulse there too
    if g.r_bc == "open":
        rG = np.array([(g.nr + 0.5) * g.dr])
        Bg = st["Bg0"].clone()
        for p in pulses:
            if basis is None:
                fG = torch.from_numpy(p.field(xI[None, :], rG[:, None]))[0]
            else:
                fG = torch.from_numpy(p.field_basis(xI[None, :], rG[:, None], basis[1]))[0]
            m, _, _, _, Bt = pulse_modes(p.pol, fG.to(CDT))
            if m < g.nmodes:
                Bg[m] += Bt
        st["Bg0"] = Bg
    return st
