"""Seeded synthetic inputs for the QDS field advance.

This module only describes *inputs*: analytic laser pulses as real functions of
(x, r), the prescribed-current drive parameters, the workload configurations
(grid sizes, step counts, physics switches, seeds) and the seeded generator of
batched instances.  It holds none of the field-advance arithmetic: no staggering,
no mode decomposition of a pulse, no transport variables, no counter-based noise.
Both the CPU oracle and the HIP path sample these functions at their own
staggered coordinates and build their own state from them.

Units (code units, c = eps0 = mu0 = 1): lengths in c/omega1, times in 1/omega1,
fields in m_e c omega1 / e, currents in e n_c c, with omega1 the angular
frequency of the 0.8 um laser.  The grid spacing along x equals the time step
(c dt = dx, the condition the transport update relies on, Sec. 2.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

LAMBDA = 2.0 * math.pi            # laser wavelength (0.8 um) in c/omega1
CELLS_PER_LAMBDA = 16
H = LAMBDA / CELLS_PER_LAMBDA     # dx = c dt
DR = 4.0 * H                      # radial cell
UM = LAMBDA / 0.8                 # one micrometre in c/omega1
FS = 0.299792458 * UM             # c * 1 fs in c/omega1
NC_CM3 = 1.7419597e21             # critical density at 0.8 um, cm^-3
J_UNIT_A_M2 = 1.602176634e-19 * NC_CM3 * 1e6 * 2.99792458e8   # e n_c c in A/m^2


@dataclass(frozen=True)
class Pulse:
    """A polarised Gaussian pulse, forward propagating along +x.

    ``field(x, r)`` is the real field E_pol at t = 0: pol = 'y' or 'z' is a
    linear Cartesian polarisation, pol = 'r' or 't' a radial or azimuthal one
    (these carry an extra factor r / w0 so that they vanish on the axis);
    the magnetic field is the forward-wave partner (|B| = |E|).  The envelope is
    Gaussian in x with the given intensity FWHM and Gaussian in r with 1/e field
    radius ``w0``; ``coeffs`` = (a_1..a_K, b_1..b_K) optionally modulate the
    longitudinal envelope by 1 + sum_k a_k cos(2 pi k xi / P) + b_k sin(2 pi k xi / P)
    with P = ``period`` (the adjoint workload's 64 envelope coefficients).
    """
    pol: str
    a0: float
    omega: float
    w0: float
    fwhm: float
    x0: float
    coeffs: Tuple[float, ...] = ()
    period: float = 0.0

    @property
    def e_peak(self) -> float:
        return self.a0 * self.omega

    def envelope(self, xi: np.ndarray) -> np.ndarray:
        sigma = self.fwhm / (2.0 * math.sqrt(math.log(2.0)))
        g = np.exp(-xi * xi / (2.0 * sigma * sigma))
        if self.coeffs:
            k = len(self.coeffs) // 2
            mod = np.ones_like(xi)
            for q in range(1, k + 1):
                ph = 2.0 * math.pi * q * xi / self.period
                mod = mod + self.coeffs[q - 1] * np.cos(ph) + self.coeffs[k + q - 1] * np.sin(ph)
            g = g * mod
        return g

    def envelope_basis(self, xi: np.ndarray, q: int) -> np.ndarray:
        """d(envelope)/d(coeffs[q]) — the pulse is linear in its coefficients."""
        sigma = self.fwhm / (2.0 * math.sqrt(math.log(2.0)))
        g = np.exp(-xi * xi / (2.0 * sigma * sigma))
        k = len(self.coeffs) // 2
        if q < k:
            return g * np.cos(2.0 * math.pi * (q + 1) * xi / self.period)
        return g * np.sin(2.0 * math.pi * (q - k + 1) * xi / self.period)

    def _transverse(self, r: np.ndarray) -> np.ndarray:
        rr = np.asarray(r, dtype=np.float64)
        prof = np.exp(-rr * rr / (self.w0 * self.w0))
        if self.pol in ("r", "t"):
            # radially / azimuthally polarised pulses vanish on the axis
            prof = prof * (rr / self.w0)
        return prof

    def field(self, x: np.ndarray, r: np.ndarray) -> np.ndarray:
        xi = np.asarray(x, dtype=np.float64) - self.x0
        return self.e_peak * self.envelope(xi) * self._transverse(r) * np.cos(self.omega * xi)

    def field_basis(self, x: np.ndarray, r: np.ndarray, q: int) -> np.ndarray:
        xi = np.asarray(x, dtype=np.float64) - self.x0
        return (self.e_peak * self.envelope_basis(xi, q) * self._transverse(r)
                * np.cos(self.omega * xi))


@dataclass(frozen=True)
class Drive:
    """Prescribed longitudinal current j_x^(0), a stand-in for particle deposition.

    j_x = amp * exp(-(x - x0 - v t)^2 / (2 sx^2)) * exp(-(r - r0)^2 / (2 sr^2)) * (1 + noise * xi)
    with xi a standard normal drawn per (step, cell, row) from the seed.  The
    formula and the generator are implemented separately by each side.
    """
    amp: float
    x0: float
    v: float
    sx: float
    r0: float
    sr: float
    noise: float
    seed: int


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    nr: int
    nmodes: int
    steps: int
    h: float = H
    dr: float = DR
    x_bc: str = "open"       # open | periodic | window
    r_bc: str = "open"       # open | pec
    wp2: float = 0.0         # cold-plasma response d_t j = wp2 E on every set
    axion: bool = False
    arem: bool = False
    ma2: float = 0.0
    s_phi: float = 1.0       # KG source scale (1 in scaled units, g for physical)
    s_j: float = 1.0         # axion-current scale (1 in scaled units, g for physical)
    bext: Tuple[complex, complex, complex] = (0j, 0j, 0j)
    pulses: Tuple[Pulse, ...] = ()
    drive: Optional[Drive] = None
    g: float = 1.0           # physical coupling, for reporting physical fields only

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)

    @property
    def cell_modes(self) -> int:
        return self.nx * self.nr * self.nmodes


def _fwhm_fs(fs: float) -> float:
    return fs * FS


# omega_p^2 / omega1^2 for n_e = 1e17 cm^-3
WP2_1E17 = 1e17 / NC_CM3


def resonant_ma2(omega1: float, omega2: float, wp2: float) -> float:
    """Axion mass^2 that phase-matches the sum-frequency mixing of two
    co-propagating lasers in a cold plasma (energy and momentum conservation,
    Sec. 4.3): m_a^2 = (w1 + w2)^2 - (k1 + k2)^2 with k = sqrt(w^2 - wp^2)."""
    k1 = math.sqrt(omega1 * omega1 - wp2)
    k2 = math.sqrt(omega2 * omega2 - wp2)
    return (omega1 + omega2) ** 2 - (k1 + k2) ** 2


def vacuum_em(nx: int = 512, nr: int = 64, steps: int = 200) -> Workload:
    """Plain QDS Maxwell, vacuum, modes m=0,1; m=1 LP-y Gaussian a0=0.01,
    waist 8 lambda, 10 fs intensity FWHM, centred at cell 128."""
    p = Pulse("y", 0.01, 1.0, 8 * LAMBDA, _fwhm_fs(10.0), 128 * H)
    return Workload("vacuum_em_512x64x2", nx, nr, 2, steps, pulses=(p,))


def driven_window(nx: int = 4096, nr: int = 256, steps: int = 4000) -> Workload:
    """QDS Maxwell with a prescribed moving current in a moving window, modes 0..2."""
    p = Pulse("y", 2.0, 1.0, 10 * LAMBDA, _fwhm_fs(30.0), 0.75 * nx * H)
    d = Drive(amp=1e12 / J_UNIT_A_M2, x0=0.5 * nx * H, v=0.999, sx=3 * UM, r0=0.0,
              sr=5 * UM, noise=1e-3, seed=2)
    return Workload(f"driven_window_{nx}x{nr}x3", nx, nr, 3, steps, x_bc="window",
                    pulses=(p,), drive=d)


def axion_two_colour(nx: int = 8192, nr: int = 256, steps: int = 6000, nmodes: int = 3) -> Workload:
    """QDS + Klein-Gordon + regenerated fields, two-colour drive (omega1 LP-y,
    omega2 = 0.8 omega1 LP-z, a0 = 0.5 each, waist 12 lambda, 50 fs), uniform
    plasma 1e17 cm^-3 as a cold linear response on both sets, sum-frequency
    resonant axion mass, scaled coupling."""
    w1, w2 = 1.0, 0.8
    p1 = Pulse("y", 0.5, w1, 12 * LAMBDA, _fwhm_fs(50.0), 1100 * H)
    p2 = Pulse("z", 0.5, w2, 12 * LAMBDA, _fwhm_fs(50.0), 1100 * H)
    return Workload(f"axion_{nx}x{nr}x{nmodes}", nx, nr, nmodes, steps, wp2=WP2_1E17,
                    axion=True, arem=True, ma2=resonant_ma2(w1, w2, WP2_1E17),
                    pulses=(p1, p2), g=1e-6)


def adjoint_workload(nx: int = 4096, nr: int = 128, steps: int = 2000, seed: int = 5,
                     ncoef: int = 64) -> Workload:
    """Forward + adjoint workload: axion physics, modes 0..1, the omega1
    envelope carries ``ncoef`` seeded Fourier coefficients."""
    rng = np.random.default_rng(seed)
    coeffs = tuple(float(c) for c in rng.normal(0.0, 0.02, size=ncoef))
    fwhm = _fwhm_fs(50.0)
    x0 = (nx - 128 - steps) * H
    p1 = Pulse("y", 0.5, 1.0, 12 * LAMBDA, fwhm, x0, coeffs=coeffs, period=4 * fwhm)
    p2 = Pulse("z", 0.5, 0.8, 12 * LAMBDA, fwhm, x0)
    return Workload(f"adjoint_{nx}x{nr}x2", nx, nr, 2, steps, wp2=WP2_1E17, axion=True,
                    arem=True, ma2=resonant_ma2(1.0, 0.8, WP2_1E17), pulses=(p1, p2), g=1e-6)


def batched_instances(count: int = 64, seed: int = 4, scale: float = 1.0):
    """Seeded uneven instances for the batched forward: nx in {1024..8192}
    (multiples of 256), nr in [64, 256], 1-3 modes, a0 log-uniform in
    [0.01, 2], waist in [6, 15] lambda, steps in [500, 3000]; otherwise the
    two-colour axion physics.  ``scale`` < 1 shrinks grids and steps for tests."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx = int(rng.integers(4, 33)) * 256
        nr = int(rng.integers(64, 257))
        nm = int(rng.integers(1, 4))
        a0 = float(math.exp(rng.uniform(math.log(0.01), math.log(2.0))))
        w0 = float(rng.uniform(6.0, 15.0)) * LAMBDA
        steps = int(rng.integers(500, 3001))
        if scale != 1.0:
            nx = max(64, int(nx * scale) // 64 * 64)
            nr = max(8, int(nr * scale))
            steps = max(4, int(steps * scale))
        fw = _fwhm_fs(30.0)
        x0 = min(0.5 * nx * H, 3 * fw)
        p1 = Pulse("y", a0, 1.0, w0, fw, x0)
        p2 = Pulse("z", a0, 0.8, w0, fw, x0)
        # a single retained mode (m = 0) cannot carry a linearly polarised
        # pulse; such instances carry radially (E_r) and azimuthally (E_theta)
        # polarised m = 0 pulses instead
        if nm == 1:
            p1 = replace(p1, pol="r")
            p2 = replace(p2, pol="t")
        out.append(Workload(f"inst{k}", nx, nr, nm, steps, wp2=WP2_1E17, axion=True, arem=True,
                            ma2=resonant_ma2(1.0, 0.8, WP2_1E17), pulses=(p1, p2), g=1e-6))
    return out
