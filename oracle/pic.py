"""CPU oracle of the particle side of the cylindrical PIC coupling (Sec. 3.1):
field gather, relativistic Boris push and the charge-conserving modal current
deposition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the HIP product path
never calls it and shares no code with it.

Plain float64 numpy, one particle at a time in Python loops (small cases
only), following the paper's equations in their order.  Readings taken where
the paper is silent (listed with the others in the design notes):

* Grids.  Charge and j_theta at (x_i, r_j); j_x at (x_{i+1/2}, r_j); j_r at
  (x_i, r_{j+1/2}) (the positions of Eqs. face_current_x, face_current_r and
  the staggering of the field solver).  x_i = i dx, r_j = j dr.
* Shape.  The triangular particle shape: its cell-integrated weights on a
  grid of spacing d are the three quadratic-spline weights
  1/2 (1/2 - t)^2, 3/4 - t^2, 1/2 (1/2 + t)^2 around the nearest node,
  t = (s - s_node)/d.  Near the axis a weight that falls on a row below the
  axis (r_{-1} for integer rows, r_{-1/2} for half rows) is added to its
  mirror row (r_1, r_{1/2}): the shape is reflected at the axis, the same for
  every mode and component, so the radial weights still sum to one.
* Axis cell.  Areas and volumes of row j = 0 use r_0 -> dr/8 (the cell
  0 <= r <= dr/2 has volume pi (dr/2)^2 dx = 2 pi (dr/8) dr dx).
* Azimuthal current.  Eq. particle_azimuthal_current with v_theta,p taken
  as r_j dtheta_p / dt at each deposition row (the angular displacement of
  the deposition path), i.e. j_theta = Q dtheta <g_x g_r>_m / (2 pi dx dr dt):
  with this the angular term of Eq. particle_charge_identity is cancelled
  exactly, and Eq. discrete_continuity holds to rounding for every mode as
  the paper states.
* Time levels.  Particles hold x^n and u^{n-1/2}.  The push gathers the
  transverse fields at t^n (from T^n) and E_x, B_x at t^n extrapolated from
  their two latest levels, 3/2 F^{n-1/2} - 1/2 F^{n-3/2} (or F^{n-1/2} alone
  when no earlier level is given); the deposit along x^n -> x^{n+1} is the
  current at t^{n+1/2}.
* Magnetic-field centring.  The QDS B_x, B_r, B_theta are first averaged
  along x onto the positions the standard staggered (Yee) interpolation uses
  for them, (x_i, r_{j+1/2}), (x_{i+1/2}, r_j), (x_{i+1/2}, r_{j+1/2}), and
  gathered with the shape weights of those grids; E_x, E_r, E_theta are
  gathered at their own positions.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# shape weights (Sec. 3.1: cell-integrated weights of the triangular shape)
# ---------------------------------------------------------------------------

def tsc_weights(s: float, d: float, offset: float) -> Tuple[int, np.ndarray]:
    """Weights of a particle at coordinate ``s`` on the grid s_k = (k + offset) d:
    the nearest node k0 and the weights of k0-1, k0, k0+1."""
    u = s / d - offset
    k0 = int(math.floor(u + 0.5))
    t = u - k0
    w = np.array([0.5 * (0.5 - t) ** 2, 0.75 - t * t, 0.5 * (0.5 + t) ** 2])
    return k0, w


def radial_weights(r: float, dr: float, half: bool) -> Dict[int, float]:
    """Row -> weight on the integer rows (half=False) or the half rows
    (half=True, row k at r_{k+1/2}), rows below the axis reflected onto their
    mirror (r_{-1} -> r_1, r_{-1/2} -> r_{1/2})."""
    k0, w = tsc_weights(r, dr, 0.5 if half else 0.0)
    out: Dict[int, float] = {}
    for a in range(3):
        k = k0 - 1 + a
        if k < 0:
            k = -k - 1 if half else -k
        out[k] = out.get(k, 0.0) + w[a]
    return out


def axial_weights(x: float, dx: float, half: bool) -> Dict[int, float]:
    """Column -> weight on the integer (x_i) or half (x_{i+1/2}, index i) columns."""
    k0, w = tsc_weights(x, dx, 0.5 if half else 0.0)
    return {k0 - 1 + a: w[a] for a in range(3)}


# ---------------------------------------------------------------------------
# field gather (Eq. particle_field_gather)
# ---------------------------------------------------------------------------

def _modes_at(F: np.ndarray, i: int, j: int, emi: np.ndarray) -> float:
    """Re sum_m F^(m)_{j,i} e^{-i m theta} (emi[m] = e^{-i m theta})."""
    return float(np.real(np.sum(F[:, j, i] * emi)))


def gather(fields: Dict[str, np.ndarray], x: float, r: float, theta: float, dx: float, dr: float
           ) -> Tuple[np.ndarray, np.ndarray]:
    """Cylindrical (E_x, E_r, E_theta), (B_x, B_r, B_theta) at the particle.

    ``fields`` holds complex arrays [M, rows, nx] at their native positions:
    Ex (x_{i+1/2}, r_j), Er (x_i, r_{j+1/2}), Et (x_i, r_j), and the QDS
    Bx (x_{i+1/2}, r_{j+1/2}), Br (x_i, r_j), Bt (x_i, r_{j+1/2})."""
    M = fields["Ex"].shape[0]
    emi = np.exp(-1j * np.arange(M) * theta)
    xI, xH = axial_weights(x, dx, False), axial_weights(x, dx, True)
    rJ, rK = radial_weights(r, dr, False), radial_weights(r, dr, True)

    def g(F, wx, wr):
        return sum(ax * ar * _modes_at(F, i, j, emi) for i, ax in wx.items() for j, ar in wr.items())

    def xavg_left(F):
        # value at x_i from the half columns x_{i-1/2}, x_{i+1/2}
        G = np.zeros_like(F)
        G[:, :, 1:] = 0.5 * (F[:, :, :-1] + F[:, :, 1:])
        G[:, :, 0] = 0.5 * F[:, :, 0]
        return G

    def xavg_right(F):
        # value at x_{i+1/2} from the integer columns x_i, x_{i+1}
        G = np.zeros_like(F)
        G[:, :, :-1] = 0.5 * (F[:, :, :-1] + F[:, :, 1:])
        G[:, :, -1] = 0.5 * F[:, :, -1]
        return G

    E = np.array([g(fields["Ex"], xH, rJ), g(fields["Er"], xI, rK), g(fields["Et"], xI, rJ)])
    B = np.array([g(xavg_left(fields["Bx"]), xI, rK), g(xavg_right(fields["Br"]), xH, rJ),
                  g(xavg_right(fields["Bt"]), xH, rK)])
    return E, B


def to_cartesian(Fcyl: np.ndarray, theta: float) -> np.ndarray:
    """(F_x, F_r, F_theta) -> (F_x, F_y, F_z) (Sec. 3.1)."""
    c, s = math.cos(theta), math.sin(theta)
    return np.array([Fcyl[0], Fcyl[1] * c - Fcyl[2] * s, Fcyl[1] * s + Fcyl[2] * c])


# ---------------------------------------------------------------------------
# relativistic Boris push (Eqs. boris_parameters, boris_update)
# ---------------------------------------------------------------------------

def boris(u: np.ndarray, E: np.ndarray, B: np.ndarray, qm: float, dt: float) -> np.ndarray:
    """u = p/(m c) advanced by dt in the Cartesian fields E, B (c = 1, charge
    to mass ratio qm in code units)."""
    um = u + 0.5 * qm * dt * E
    gm = math.sqrt(1.0 + float(um @ um))
    t = 0.5 * qm * dt * B / gm
    s = 2.0 * t / (1.0 + float(t @ t))
    up = um + np.cross(um, t)
    uplus = um + np.cross(up, s)
    return uplus + 0.5 * qm * dt * E


# ---------------------------------------------------------------------------
# trajectory averages of the mode weight (Eq. particle_mode_weight)
# ---------------------------------------------------------------------------

def xi_moments(phi: float) -> np.ndarray:
    """E_k(phi) = int_0^1 xi^k e^{i phi xi} dxi, k = 0, 1, 2.

    The closed forms E_0 = (e^{i phi} - 1)/(i phi), E_{k+1} = (e^{i phi} -
    (k+1) E_k)/(i phi) lose about eps / |phi|^(k+1) to cancellation as phi -> 0
    (the paper switches to series below |m dtheta| = 1e-4 for the e^{i phi} - 1
    terms; the xi-weighted moments need more).  Below |phi| = 0.5 the series
    sum_n (i phi)^n / (n! (n + k + 1)) is summed to 16 terms (truncation
    < 1e-18), the closed forms above it."""
    if abs(phi) < 0.5:
        out = np.zeros(3, complex)
        for k in range(3):
            term = 1.0 + 0j
            for n in range(16):
                out[k] += term / (n + k + 1)
                term *= 1j * phi / (n + 1)
        return out
    e = complex(math.cos(phi), math.sin(phi))
    ip = 1j * phi
    E0 = (e - 1.0) / ip
    E1 = e / ip - E0 / ip
    E2 = e / ip - 2.0 * E1 / ip
    return np.array([E0, E1, E2])


def mode_factor(m: int, theta0: float) -> complex:
    """C_m(theta0) of Eq. particle_mode_weight: 1 for m = 0, 2 e^{i m theta0}."""
    return 1.0 + 0j if m == 0 else 2.0 * complex(math.cos(m * theta0), math.sin(m * theta0))


def traj_avg(poly: Tuple[float, ...], m: int, theta0: float, dtheta: float) -> complex:
    """<W>_m for W(xi) = poly[0] + poly[1] xi + poly[2] xi^2."""
    Ek = xi_moments(m * dtheta)
    return mode_factor(m, theta0) * sum(c * Ek[k] for k, c in enumerate(poly))


# ---------------------------------------------------------------------------
# charge-conserving modal deposition (Eqs. particle_deposition_path ..
# face_current_r)
# ---------------------------------------------------------------------------

def cell_area_x(j: int, dr: float) -> float:
    """A_{r theta, j} = 2 pi r_j dr (r_0 -> dr/8)."""
    return 2.0 * math.pi * (dr / 8.0 if j == 0 else j * dr) * dr


def cell_area_r(j: int, dx: float, dr: float) -> float:
    """A_{x theta, j+1/2} = 2 pi r_{j+1/2} dx."""
    return 2.0 * math.pi * (j + 0.5) * dr * dx


def wrap_angle(a: float) -> float:
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def deposit(x0: Tuple[float, float, float], x1: Tuple[float, float, float], Q: float, M: int,
            dx: float, dr: float, dt: float, jx: np.ndarray, jr: np.ndarray, jt: np.ndarray) -> None:
    """Add one particle's modal currents for the step x0 -> x1 (Cartesian) to
    jx [M, nr+1, nx] (x_{i+1/2}, r_j), jr [M, nr+1, nx] (x_i, r_{j+1/2}),
    jt [M, nr+1, nx] (x_i, r_j)."""
    r0, r1 = math.hypot(x0[1], x0[2]), math.hypot(x1[1], x1[2])
    th0 = math.atan2(x0[2], x0[1])
    dth = wrap_angle(math.atan2(x1[2], x1[1]) - th0)
    gx0, gx1 = axial_weights(x0[0], dx, False), axial_weights(x1[0], dx, False)
    gr0, gr1 = radial_weights(r0, dr, False), radial_weights(r1, dr, False)
    cols = sorted(set(gx0) | set(gx1))
    rows = sorted(set(gr0) | set(gr1))
    gx = {i: (gx0.get(i, 0.0), gx1.get(i, 0.0) - gx0.get(i, 0.0)) for i in cols}   # (g^0, h)
    gr = {j: (gr0.get(j, 0.0), gr1.get(j, 0.0) - gr0.get(j, 0.0)) for j in rows}
    for m in range(M):
        # net currents I_x, I_r (Eq. particle_modal_currents) and j_theta
        # (Eq. particle_azimuthal_current, with v_theta = r_j dtheta / dt)
        Ix = {(i, j): Q / dt * gx[i][1] * traj_avg((gr[j][0], gr[j][1]), m, th0, dth) for i in cols for j in rows}
        Ir = {(i, j): Q / dt * gr[j][1] * traj_avg((gx[i][0], gx[i][1]), m, th0, dth) for i in cols for j in rows}
        for i in cols:
            for j in rows:
                a, b = gx[i]
                c, d = gr[j]
                avg = traj_avg((a * c, a * d + b * c, b * d), m, th0, dth)
                jt[m, j, i] += Q * dth * avg / (2.0 * math.pi * dx * dr * dt)
        # face currents: A_{r theta, j} (j_x(i+1/2) - j_x(i-1/2)) = -I_x
        # (Eq. face_current_x), summed from the face left of the support
        for j in rows:
            acc = 0.0 + 0j
            for i in cols:
                acc = acc - Ix[(i, j)] / cell_area_x(j, dr)
                jx[m, j, i] += acc          # j_x at x_{i+1/2}
        # A_{x theta, j+1/2} j_r(j+1/2) - A_{x theta, j-1/2} j_r(j-1/2) = -I_r
        # (Eq. face_current_r), summed outward from the axis
        for i in cols:
            flux = 0.0 + 0j
            for j in range(0, max(rows) + 1):
                flux = flux - Ir.get((i, j), 0.0)
                jr[m, j, i] += flux / cell_area_r(j, dx, dr)


def charge_modes(pos: np.ndarray, Q: np.ndarray, M: int, nx: int, nr: int, dx: float, dr: float) -> np.ndarray:
    """Modal charge q^(m)_{j,i} = sum_p Q_p g_x g_r C_m(theta_p) at (x_i, r_j)
    (Eq. particle_modal_charge; not divided by the cell volume)."""
    q = np.zeros((M, nr + 1, nx), complex)
    for p in range(pos.shape[0]):
        x, y, z = pos[p]
        r, th = math.hypot(y, z), math.atan2(z, y)
        for i, ax in axial_weights(x, dx, False).items():
            for j, ar in radial_weights(r, dr, False).items():
                for m in range(M):
                    q[m, j, i] += Q[p] * ax * ar * mode_factor(m, th)
    return q


def continuity_residual(q0: np.ndarray, q1: np.ndarray, jx: np.ndarray, jr: np.ndarray, jt: np.ndarray,
                        dx: float, dr: float, dt: float) -> np.ndarray:
    """Eq. discrete_continuity multiplied by the cell volume V_ij dt:
    (q^{n+1} - q^n) + dt [A_{r theta,j} (j_x(i+1/2) - j_x(i-1/2))
    + A_{x theta,j+1/2} j_r(j+1/2) - A_{x theta,j-1/2} j_r(j-1/2)] - i m dt (V_ij / r_j) j_theta,
    with V_ij / r_j = 2 pi dx dr."""
    M, rows, nx = q0.shape
    res = (q1 - q0).astype(complex)
    Ax = np.array([cell_area_x(j, dr) for j in range(rows)]).reshape(1, -1, 1)
    jx_left = np.concatenate([np.zeros_like(jx[..., :1]), jx[..., :-1]], axis=-1)
    res += dt * Ax * (jx - jx_left)
    Ar = np.array([cell_area_r(j, dx, dr) for j in range(rows)]).reshape(1, -1, 1)
    flux = Ar * jr
    flux_below = np.concatenate([np.zeros_like(flux[:, :1]), flux[:, :-1]], axis=1)
    res += dt * (flux - flux_below)
    m = np.arange(M).reshape(-1, 1, 1)
    res -= 1j * m * dt * 2.0 * math.pi * dx * dr * jt
    return res


# ---------------------------------------------------------------------------
# one particle step
# ---------------------------------------------------------------------------

def particle_step(fields: Dict[str, np.ndarray], long_prev: Optional[Dict[str, np.ndarray]],
                  pos: np.ndarray, u: np.ndarray, Q: np.ndarray, qm: float, dx: float, dr: float,
                  dt: float) -> Tuple[np.ndarray, np.ndarray, Tuple[np.ndarray, np.ndarray, np.ndarray]]:
    """Advance particles (x^n, u^{n-1/2}) -> (x^{n+1}, u^{n+1/2}) in the fields
    of ``fields`` (Er, Et, Br, Bt at t^n; Ex, Bx at t^{n-1/2}) and return the
    deposited j^{n+1/2} (jx, jr, jt, each [M, nr+1, nx]).  ``long_prev`` holds
    Ex, Bx at t^{n-3/2} for the extrapolation of the longitudinal fields to
    t^n, or None."""
    f = dict(fields)
    if long_prev is not None:
        f["Ex"] = 1.5 * fields["Ex"] - 0.5 * long_prev["Ex"]
        f["Bx"] = 1.5 * fields["Bx"] - 0.5 * long_prev["Bx"]
    M, rows, nx = fields["Et"].shape
    jx = np.zeros((M, rows, nx), complex)
    jr = np.zeros((M, rows, nx), complex)
    jt = np.zeros((M, rows, nx), complex)
    new_pos = pos.copy()
    new_u = u.copy()
    for p in range(pos.shape[0]):
        x, y, z = pos[p]
        r, th = math.hypot(y, z), math.atan2(z, y)
        Ec, Bc = gather(f, x, r, th, dx, dr)
        Eg, Bg = to_cartesian(Ec, th), to_cartesian(Bc, th)
        un = boris(u[p], Eg, Bg, qm, dt)
        gam = math.sqrt(1.0 + float(un @ un))
        xn = pos[p] + dt * un / gam
        deposit(tuple(pos[p]), tuple(xn), Q[p], M, dx, dr, dt, jx, jr, jt)
        new_pos[p] = xn
        new_u[p] = un
    return new_pos, new_u, (jx, jr, jt)


# ---------------------------------------------------------------------------
# the coupled PIC step: particles, then the field advance with their current
# ---------------------------------------------------------------------------

def source_currents(jx_prev, jx_new, jr, jt):
    """The deposits brought to the source points of the field step: j_x^n as
    the mean of the deposits of the steps ending at t^{n-1/2} (jx_prev, or
    None) and t^{n+1/2}; j_r, j_theta of the latter averaged along x from x_i,
    x_{i+1} onto x_{i+1/2} (Sec. 3.1, last paragraph), zero beyond the last
    column."""
    def xavg(a):
        b = np.zeros_like(a)
        b[..., :-1] = 0.5 * (a[..., :-1] + a[..., 1:])
        b[..., -1] = 0.5 * a[..., -1]
        return b
    jx = 0.5 * jx_new if jx_prev is None else 0.5 * (jx_prev + jx_new)
    return jx, xavg(jr)[:, :-1], xavg(jt)


def fields_of(st):
    """The gather's inputs from an oracle state: background set only."""
    return {"Ex": st["Ex0"].numpy(), "Bx": st["Bx0"].numpy(),
            "Er": (0.5 * (st["Trp0"] + st["Trm0"])).numpy(), "Bt": (0.5 * (st["Trp0"] - st["Trm0"])).numpy(),
            "Et": (0.5 * (st["Ttp0"] + st["Ttm0"])).numpy(), "Br": (0.5 * (st["Ttp0"] - st["Ttm0"])).numpy()}


def coupled_steps(st, g, ph, pos, u, Q, qm, nsteps):
    """``nsteps`` PIC steps on the oracle: particle step in the state's fields
    (E_x, B_x extrapolated from the previous state from the second step on),
    then one field step (oracle.qds.step) with the particle currents."""
    import torch
    from oracle import qds as OQ
    prev_state, prev_jx = None, None
    for _ in range(nsteps):
        lp = None if prev_state is None else {"Ex": prev_state["Ex0"].numpy(), "Bx": prev_state["Bx0"].numpy()}
        pos, u, (jx, jr, jt) = particle_step(fields_of(st), lp, pos, u, Q, qm, g.h, g.dr, g.h)
        ext = tuple(torch.from_numpy(np.ascontiguousarray(a)) for a in source_currents(prev_jx, jx, jr, jt))
        prev_state = st
        st = OQ.step(st, g, ph, ext)
        prev_jx = jx
    return st, pos, u
