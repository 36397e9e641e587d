"""Pins of the particle oracle (Sec. 3.1) against what the paper and the
mathematics fix: the discrete continuity equation holds to rounding for every
retained mode (Eq. discrete_continuity), the analytic trajectory averages
(Eq. particle_mode_weight) equal Gauss-Legendre quadrature of their integrals
(the series branch for |m dtheta| < 1e-4 included), the Boris rotation keeps
|u| and turns it by 2 atan|t| (Eqs. boris_parameters, boris_update), and the
gather reproduces uniform Cartesian fields and fields linear in x and r at
their own staggered positions (Eq. particle_field_gather)."""
import math

import numpy as np
import pytest

from oracle import pic as P

DX, DR, DT = 0.39, 1.3, 0.39


def _particles(n, nx, nr, seed, r_max=None, speed=0.9):
    rng = np.random.default_rng(seed)
    x = rng.uniform(3 * DX, (nx - 4) * DX, n)
    rmax = (nr - 3) * DR if r_max is None else r_max
    r = rmax * np.sqrt(rng.uniform(0, 1, n))
    th = rng.uniform(-math.pi, math.pi, n)
    pos = np.stack([x, r * np.cos(th), r * np.sin(th)], axis=1)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    v = speed * rng.uniform(0.2, 1.0, n)[:, None] * d
    u = v / np.sqrt(1 - (v ** 2).sum(axis=1, keepdims=True))
    return pos, u


@pytest.mark.parametrize("M", [1, 3, 5])
@pytest.mark.parametrize("near_axis", [False, True])
def test_deposition_satisfies_discrete_continuity(M, near_axis):
    """Particles moving up to 0.9 c in every direction (near the axis: all
    within 1.5 dr of it, crossing it), deposited over one step: the residual
    of Eq. discrete_continuity (charge form) vanishes to rounding in every
    cell and mode, the axis cell included."""
    nx, nr = 16, 8
    pos, u = _particles(40, nx, nr, 11 + M, r_max=1.5 * DR if near_axis else None)
    Q = np.random.default_rng(3).uniform(0.5, 2.0, len(pos))
    jx = np.zeros((M, nr + 1, nx), complex)
    jr = np.zeros_like(jx)
    jt = np.zeros_like(jx)
    gam = np.sqrt(1 + (u ** 2).sum(axis=1, keepdims=True))
    new = pos + DT * u / gam
    for p in range(len(pos)):
        P.deposit(tuple(pos[p]), tuple(new[p]), Q[p], M, DX, DR, DT, jx, jr, jt)
    q0 = P.charge_modes(pos, Q, M, nx, nr, DX, DR)
    q1 = P.charge_modes(new, Q, M, nx, nr, DX, DR)
    res = P.continuity_residual(q0, q1, jx, jr, jt, DX, DR, DT)
    scale = np.abs(q1 - q0).max()
    assert scale > 0.1
    assert np.abs(res).max() < 1e-13 * max(scale, np.abs(q0).max())
    # every retained mode carries current, and the angular current matters
    for m in range(M):
        assert np.abs(jx[m]).max() > 1e-3 and np.abs(jr[m]).max() > 1e-3
    if M > 1:
        assert np.abs(jt[1:]).max() > 1e-3


def test_continuity_fails_with_the_cartesian_azimuthal_velocity():
    """The literal v_theta,p / V_ij weighting (v_theta from the Cartesian
    velocity) leaves an O(1) residual in the modes m >= 1: the angular current
    must carry the path's angular displacement for Eq. discrete_continuity."""
    nx, nr, M = 16, 8, 3
    pos, u = _particles(20, nx, nr, 5)
    Q = np.ones(len(pos))
    jx = np.zeros((M, nr + 1, nx), complex)
    jr = np.zeros_like(jx)
    jt = np.zeros_like(jx)
    gam = np.sqrt(1 + (u ** 2).sum(axis=1, keepdims=True))
    new = pos + DT * u / gam
    for p in range(len(pos)):
        P.deposit(tuple(pos[p]), tuple(new[p]), Q[p], M, DX, DR, DT, jx, jr, jt)
    # the azimuthal velocity at the midpoint of the straight path
    mid = 0.5 * (pos + new)
    thm = np.arctan2(mid[:, 2], mid[:, 1])
    vth = (-(new - pos)[:, 1] * np.sin(thm) + (new - pos)[:, 2] * np.cos(thm)) / DT
    jt2 = np.zeros_like(jt)
    # build the literal form directly
    for p in range(len(pos)):
        th0 = math.atan2(pos[p, 2], pos[p, 1])
        dth = P.wrap_angle(math.atan2(new[p, 2], new[p, 1]) - th0)
        gx0, gx1 = P.axial_weights(pos[p, 0], DX, False), P.axial_weights(new[p, 0], DX, False)
        gr0 = P.radial_weights(math.hypot(pos[p, 1], pos[p, 2]), DR, False)
        gr1 = P.radial_weights(math.hypot(new[p, 1], new[p, 2]), DR, False)
        for m in range(M):
            for i in set(gx0) | set(gx1):
                for j in set(gr0) | set(gr1):
                    a, b = gx0.get(i, 0.0), gx1.get(i, 0.0) - gx0.get(i, 0.0)
                    c_, d = gr0.get(j, 0.0), gr1.get(j, 0.0) - gr0.get(j, 0.0)
                    rj = DR / 8 if j == 0 else j * DR
                    avg = P.traj_avg((a * c_, a * d + b * c_, b * d), m, th0, dth)
                    jt2[m, j, i] += Q[p] * vth[p] * avg / (2 * math.pi * rj * DX * DR)
    q0 = P.charge_modes(pos, Q, M, nx, nr, DX, DR)
    q1 = P.charge_modes(new, Q, M, nx, nr, DX, DR)
    res = P.continuity_residual(q0, q1, jx, jr, jt2, DX, DR, DT)
    assert np.abs(res[1:]).max() > 1e-4 * np.abs(q1 - q0).max()


@pytest.mark.parametrize("phi", [0.0, 3e-9, 2e-6, 9e-5, 1.1e-4, 0.3, 0.4999, 0.5001, 2.0, -3.0, 6.0])
def test_trajectory_moments_equal_quadrature(phi):
    """E_k(phi) = int_0^1 xi^k e^{i phi xi} dxi by 40-point Gauss-Legendre
    (exact for these smooth integrands up to its own rounding, ~40 eps), on both sides of the
    paper's series switch at 1e-4 and of the switch at 0.5 used here."""
    xg, wg = np.polynomial.legendre.leggauss(40)
    xi, w = 0.5 * (xg + 1), 0.5 * wg
    got = P.xi_moments(phi)
    for k in range(3):
        ref = np.sum(w * xi ** k * np.exp(1j * phi * xi))
        assert abs(got[k] - ref) < 1e-14, (phi, k, got[k], ref)


def test_trajectory_average_equals_quadrature_of_the_definition():
    """<W>_m = int W(xi) C_m(theta0 + xi dtheta) dxi for quadratic W."""
    xg, wg = np.polynomial.legendre.leggauss(40)
    xi, w = 0.5 * (xg + 1), 0.5 * wg
    for m, th0, dth in ((0, 0.4, 0.7), (1, -2.0, 0.3), (3, 1.0, -0.9), (2, 0.2, 4e-5)):
        poly = (0.3, -0.2, 0.05)
        W = poly[0] + poly[1] * xi + poly[2] * xi ** 2
        C = np.ones_like(xi) if m == 0 else 2 * np.exp(1j * m * (th0 + xi * dth))
        ref = np.sum(w * W * C)
        assert abs(P.traj_avg(poly, m, th0, dth) - ref) < 1e-14


def test_boris_rotation_in_a_uniform_magnetic_field():
    """E = 0: |u| is kept exactly and u turns about B by 2 atan(|t|),
    t = (q dt / 2 m gamma) B."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        u = rng.normal(size=3) * 3
        B = rng.normal(size=3) * 2
        qm, dt = -1.0, 0.39
        un = P.boris(u, np.zeros(3), B, qm, dt)
        assert abs(np.linalg.norm(un) / np.linalg.norm(u) - 1) < 1e-15
        bh = B / np.linalg.norm(B)
        upar, npar = u @ bh, un @ bh
        assert abs(npar - upar) < 1e-13 * np.linalg.norm(u)
        a, b = u - upar * bh, un - npar * bh
        ang = math.atan2(np.cross(a, b) @ bh, a @ b)
        gam = math.sqrt(1 + u @ u)
        t = abs(0.5 * qm * dt * np.linalg.norm(B) / gam)
        assert abs(abs(ang) - 2 * math.atan(t)) < 1e-13
        # a negative charge turns counter-clockwise about B (du/dt = q/m u x B / gamma)
        assert ang > 0


def test_boris_electric_kick():
    """B = 0: u^{n+1} = u^n + q dt E / m exactly."""
    u = np.array([0.3, -1.2, 0.5])
    E = np.array([0.7, 0.1, -0.4])
    assert np.allclose(P.boris(u, E, np.zeros(3), -1.0, 0.39), u - 0.39 * E, rtol=0, atol=1e-15)


def _fields(M, nr, nx):
    z = np.zeros((M, nr + 1, nx), complex)
    return {k: z.copy() for k in ("Ex", "Er", "Et", "Bx", "Br", "Bt")}


def test_gather_reproduces_uniform_cartesian_fields():
    """A uniform E_y, B_z (mode 1: E_r = E_y, E_theta = -i E_y; B_r = i B_z,
    B_theta = B_z) and uniform E_x, B_x (mode 0) come back exactly at every
    particle position, the axis region included."""
    M, nr, nx = 3, 8, 16
    f = _fields(M, nr, nx)
    f["Ex"][0] = 0.7
    f["Bx"][0] = -0.2
    f["Er"][1], f["Et"][1] = 1.3, -1.3j
    f["Br"][1], f["Bt"][1] = 0.4j, 0.4
    pos, _ = _particles(50, nx, nr, 2)
    pos[:10, 1:] *= 0.05
    for x, y, z in pos:
        r, th = math.hypot(y, z), math.atan2(z, y)
        E, B = P.gather(f, x, r, th, DX, DR)
        Ec, Bc = P.to_cartesian(E, th), P.to_cartesian(B, th)
        assert np.allclose(Ec, [0.7, 1.3, 0.0], atol=1e-14)
        assert np.allclose(Bc, [-0.2, 0.0, 0.4], atol=1e-14)


@pytest.mark.parametrize("comp,half_x,half_r", [("Ex", True, False), ("Er", False, True), ("Et", False, False),
                                                ("Bx", True, True), ("Br", False, False), ("Bt", False, True)])
def test_gather_reproduces_linear_fields_at_their_positions(comp, half_x, half_r):
    """A mode-0 component a + b x + c r sampled at its own staggered
    positions is gathered exactly at any particle farther than 2 dr from the
    axis (the shape reproduces linear functions; a half-cell slip in a
    position would leave b dx/2 or c dr/2)."""
    M, nr, nx = 1, 10, 20
    f = _fields(M, nr, nx)
    xs = (np.arange(nx) + (0.5 if half_x else 0.0)) * DX
    rs = (np.arange(nr + 1) + (0.5 if half_r else 0.0)) * DR
    a, b, c = 0.3, 0.11, -0.07
    f[comp][0] = a + b * xs[None, :] + c * rs[:, None]
    idx = {"Ex": 0, "Er": 1, "Et": 2, "Bx": 0, "Br": 1, "Bt": 2}[comp]
    rng = np.random.default_rng(1)
    for _ in range(30):
        x = rng.uniform(4 * DX, (nx - 5) * DX)
        r = rng.uniform(2.1 * DR, (nr - 3) * DR)
        E, B = P.gather(f, x, r, 0.3, DX, DR)
        v = (E if comp[0] == "E" else B)[idx]
        assert abs(v - (a + b * x + c * r)) < 1e-13, (comp, x, r, v)
