"""The radial stability bound of qds_init against the oracle's own one-step map.

With c dt = dx the step of one mode and axial wavenumber k factorises as
sin^2(w dt/2) = sin^2(k dx/2) + (dt/2)^2 mu cos^2(k dx/2) (pinned in
test_oracle_pins), so it is stable exactly when dt^2 mu_max <= 4.  The
library's mu_max (largest eigenvalue of the radial operators, from Sturm
bisection) must equal the largest mu of the oracle's k-block spectrum with a
conducting wall, and the bound must be sharp: a grid it refuses has an
eigenvalue of modulus > 1 in the oracle's step, a grid it accepts none.
Host only (no device work)."""
import ctypes
import math

import numpy as np
import pytest

from oracle import qds as Q
from paper_2609_03550_amd import inputs as I
import oracle_tools as T

H = I.H
EM_KEYS = ["Trp0", "Trm0", "Ttp0", "Ttm0", "Ex0", "Bx0"]
KG_KEYS = ["phi", "Tap", "Tam"]


@pytest.fixture(scope="module")
def lib():
    from paper_2609_03550_amd import qds
    return qds.lib()


def _lib_mu(lib, nr, dr, M, r_bc):
    a, b = ctypes.c_double(), ctypes.c_double()
    assert lib.qds_radial_mu_max(nr, dr, M, r_bc, ctypes.byref(a), ctypes.byref(b)) == 0
    return a.value, b.value


def _oracle_block(g, ph, keys, m, kidx=1):
    k = 2 * math.pi * kidx / (g.nx * g.h)
    lam = np.linalg.eigvals(T.kblock(g, ph, keys, m, k))
    lam = lam[np.abs(lam) > 1e-9]
    return lam, T.mu_from_eigs(lam, k, g.h).real


@pytest.mark.parametrize("nr,ratio,M", [(10, 4.0, 3), (8, 4.2, 5), (12, 2.5, 2), (7, 7.2, 8)])
def test_bound_equals_the_oracle_spectrum(lib, nr, ratio, M):
    """Conducting wall, periodic x: mu_max of the electromagnetic step and
    m_a^2 + mu_max of the Klein-Gordon step, over all modes."""
    dr = ratio * H
    g = Q.Grid(8, nr, M, H, dr, "periodic", "pec")
    ma2 = 0.013
    mu_em, mu_kg = _lib_mu(lib, nr, dr, M, 1)
    em = max(_oracle_block(g, Q.Physics(), EM_KEYS, m)[1].max() for m in range(M))
    kg = max(_oracle_block(g, Q.Physics(axion=True, ma2=ma2), KG_KEYS, m)[1].max() for m in range(M))
    assert abs(mu_em / em - 1) < 1e-9, (mu_em, em)
    assert abs((mu_kg + ma2) / kg - 1) < 1e-9, (mu_kg + ma2, kg)


@pytest.mark.parametrize("M,ratio,stable", [(4, 4.0, True), (5, 4.0, False), (5, 4.2, True),
                                            (8, 7.0, False), (8, 7.2, True), (6, 6.0, True)])
def test_bound_is_sharp(lib, M, ratio, stable):
    """qds_init accepts exactly the grids whose oracle step has no growing
    mode.  (5 modes at dr = 4.2 dx were refused by the earlier row-sum
    bound (8 + 4 m^2)/dr^2, which is not sharp.)"""
    from paper_2609_03550_amd import qds
    nr, dr = 8, ratio * H
    h = ctypes.c_void_p()
    grid = qds.Grid(64, nr, qds.F64, qds.X_BC["periodic"], qds.R_BC["pec"], 0, dr)
    st = lib.qds_init(ctypes.byref(grid), M, H, H, ctypes.byref(h))
    assert st == (qds.QDS_OK if stable else qds.QDS_ECFL), (M, ratio, st)
    if st == qds.QDS_OK:
        lib.qds_destroy(h)
    g = Q.Grid(8, nr, M, H, dr, "periodic", "pec")
    rho = max(np.abs(_oracle_block(g, Q.Physics(), EM_KEYS, m)[0]).max() for m in range(M))
    if stable:
        assert rho < 1 + 1e-12, rho
    else:
        assert rho > 1 + 1e-3, rho


def test_axion_mass_enters_the_bound_at_step(lib):
    """The Klein-Gordon step adds m_a^2: qds_step refuses an axion mass that
    makes dt^2 (mu_kg + m_a^2) exceed 4 before touching the device."""
    from paper_2609_03550_amd import qds
    nr, M, dr = 8, 3, 4.0 * H
    mu_em, mu_kg = _lib_mu(lib, nr, dr, M, 0)
    h = ctypes.c_void_p()
    grid = qds.Grid(64, nr, qds.F64, 0, 0, qds.HAS_AXION, dr)
    assert lib.qds_init(ctypes.byref(grid), M, H, H, ctypes.byref(h)) == qds.QDS_OK
    st = qds.State()
    st.buf[0], st.buf[1] = 64, 128
    ax = qds.Axion()
    ax.s_phi = ax.s_j = 1.0
    ax.ma2 = 4.0 / H ** 2 - mu_kg + 1e-6
    assert lib.qds_step(h, ctypes.byref(st), None, ctypes.byref(ax), 1, None) == qds.QDS_ECFL
    assert b"axion stability" in lib.qds_last_error(h)
    lib.qds_destroy(h)
