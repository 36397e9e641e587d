"""Single precision over a long horizon: 2000 steps of the full physics
(background set with cold plasma, Klein-Gordon axion, regenerated set) on a
periodic 384 x 24 x 3 grid, so the two-colour pulse keeps crossing the
domain and the axion and regenerated fields keep growing.  Every physical
field and mode (E_r, B_theta, E_theta, B_r, E_x, B_x, the currents, phi,
d_t phi, d_x phi of each set) is compared with the FP64 oracle against its
own norm (at least 1e-3 of its field set's norm) and must stay within 1e-5 or within 4x the
deviation of the oracle run whose state is rounded to single precision after
every step (the error of single-precision storage alone), at 250, 1000 and
2000 steps."""
import pytest
import torch

from oracle import qds as Q
from paper_2609_03550_amd import inputs as I
import parity_tools as P

pytestmark = pytest.mark.gpu
H = I.H
MARKS = (250, 1000, 2000)


def _wl():
    p1 = I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 30 * H, 150 * H)
    p2 = I.Pulse("z", 0.5, 0.8, 3 * I.LAMBDA, 30 * H, 150 * H)
    return I.Workload("horizon", 384, 24, 3, 0, wp2=I.WP2_1E17, axion=True, arem=True, x_bc="periodic",
                      ma2=I.resonant_ma2(1.0, 0.8, I.WP2_1E17), pulses=(p1, p2))


def _oracle_marks(wl, dtype=None):
    """The oracle's states at MARKS; with ``dtype`` the state passes through
    storage rounding of that precision before the first step and after every
    step."""
    g, ph = Q.grid_physics(wl)
    gen = torch.Generator().manual_seed(0)
    rnd = (lambda st: P.storage_rounded(st, dtype, gen)) if dtype else (lambda st: st)
    st = rnd(Q.init_state(wl))
    out, done = {}, 0
    for n in MARKS:
        for _ in range(n - done):
            st = rnd(Q.step(st, g, ph))
        done = n
        out[n] = dict(st)
    return out


@pytest.fixture(scope="module")
def oracle_marks():
    """The plain and the storage-rounded oracle runs, shared by both kernel
    arrangements."""
    wl = _wl()
    return _oracle_marks(wl), _oracle_marks(wl, "f32")


@pytest.mark.parametrize("kernel_ax", [0, 1])
def test_single_precision_over_2000_steps(oracle_marks, kernel_ax):
    """The split kernels (kernel A, the axion kernel, kernel B) and kernel AX
    (the background set, the axion and its current in one march) alike."""
    from paper_2609_03550_amd import qds
    wl = _wl()
    ref, emu = oracle_marks
    s = qds.Solver(wl, dtype="f32")
    s.set_option(qds.OPT_KERNEL_AX, kernel_ax)
    s.load_pulses()
    done = 0
    for n in MARKS:
        s.step(n - done)
        done = n
        torch.cuda.synchronize()
        w = P.compare_band(s.fields(), ref[n], emu[n], 1e-5)
        print(f"step {n}: worst per-field single-precision relative L2 {w[3]:.2e} ({w[1]}[{w[2]}]), "
              f"storage rounding there {w[4]:.2e}", flush=True)
