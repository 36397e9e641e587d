"""The two-step march (QDS_OPT_PAIR): one launch advances a set through two
steps, the first step's rows handed to the second through an LDS ring.  Each
step's arithmetic is the one-step march's, so a paired run must equal single
steps bit for bit: the regenerated set with the axion (kernel A and the axion
kernel writing the pair buffer in between), and the background set alone, at
tile heights from one row up (the two-row lag, the ghost chunk, ragged last
chunks), odd step counts (a single step after the pairs), 58-column strips
over widths that leave ragged strips, periodic and open x, conducting and open
outer walls; and against the oracle per field."""
import ctypes

import pytest
import torch

from paper_2609_03550_amd import inputs as I
import parity_tools as P
from test_gpu_parity import _full, _random_reachable_state

pytestmark = pytest.mark.gpu
H = I.H


def _random_state_no_plasma(wl, seed):
    """As _random_reachable_state, for a set without the plasma: its state
    has no current planes, so the oracle's (which it would keep as fixed
    sources) start at zero."""
    from oracle import qds as Q
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    gen = torch.Generator().manual_seed(seed)
    for k, v in st.items():
        if isinstance(v, torch.Tensor) and v.is_complex():
            st[k] = torch.zeros_like(v) if k[0] == "j" else torch.randn(v.shape, dtype=torch.complex128, generator=gen)
    return Q.step(st, g, ph), g, ph


def _em(nx, nr, M, **kw):
    p = I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 0.4 * nx * H)
    return I.Workload("em", nx, nr, M, 0, wp2=0.02, pulses=(p,)).with_(**kw)


def _run(wl, dtype, st, nsteps, pair, rows, tune=False):
    from paper_2609_03550_amd import qds
    s = qds.Solver(wl, dtype=dtype)
    s.set_option(qds.OPT_PAIR, pair)
    s.set_option(qds.OPT_ROWS, rows)
    if tune:
        s.set_option(qds.OPT_TUNE, 1)
    s.load_fields(st)
    assert s.fused
    s.step(nsteps)
    torch.cuda.synchronize()
    return s


def _equal(a, b):
    fa, fb = a.fields(), b.fields()
    assert (a.n, a.window) == (b.n, b.window)
    bad = {}
    for k in fa:
        if not torch.equal(fa[k], fb[k]):
            d = (fa[k] - fb[k]).abs().max().item()
            bad[k] = (d, fa[k].abs().max().item())
    assert not bad, bad


@pytest.mark.parametrize("dtype,M,x_bc,r_bc,rows,nx", [
    ("f64", 3, "open", "open", 1, 190), ("f64", 3, "open", "open", 2, 190), ("f64", 3, "open", "open", 5, 190),
    ("f64", 3, "periodic", "pec", 3, 175), ("f64", 3, "open", "pec", 24, 117), ("f64", 1, "open", "open", 4, 59),
    ("f64", 2, "periodic", "open", 7, 58), ("f64", 4, "open", "open", 6, 240), ("f64", 6, "open", "open", 5, 131),
    ("f32", 3, "open", "open", 4, 190), ("f32", 2, "open", "pec", 1, 100), ("f32", 4, "periodic", "pec", 9, 121)])
def test_pair_with_regenerated_set_equals_single_steps(dtype, M, x_bc, r_bc, rows, nx):
    from oracle import qds as Q
    kw = dict(x_bc=x_bc, r_bc=r_bc)
    if M > 4:
        kw["dr"] = M * H
    wl = _full(nx, 23, M, **kw)
    st, g, ph = _random_reachable_state(wl, 70 + rows + M)
    a = _run(wl, dtype, st, 7, 1, rows)
    b = _run(wl, dtype, st, 7, 0, rows)
    _equal(a, b)
    if dtype == "f64" and M == 3:
        ref = Q.run(st, g, ph, 7)
        P.compare_states(a.fields(), ref, 1e-12, 1e-14, set_floor=P.SET_FLOOR, phys=True)


@pytest.mark.parametrize("dtype,M,x_bc,r_bc,rows,nx", [
    ("f64", 3, "open", "open", 2, 190), ("f64", 2, "periodic", "pec", 5, 121), ("f32", 3, "open", "open", 4, 190),
    ("f32", 1, "open", "pec", 3, 64)])
def test_pair_with_regenerated_set_without_plasma_equals_single_steps(dtype, M, x_bc, r_bc, rows, nx):
    """The axion physics without the cold plasma: the march's instantiation
    without plasma currents (fewer registers) equals single steps bit for
    bit, and the oracle per field."""
    from oracle import qds as Q
    wl = _full(nx, 23, M, x_bc=x_bc, r_bc=r_bc, wp2=0.0)
    st, g, ph = _random_state_no_plasma(wl, 110 + rows + M)
    a = _run(wl, dtype, st, 7, 1, rows)
    b = _run(wl, dtype, st, 7, 0, rows)
    _equal(a, b)
    if dtype == "f64":
        ref = Q.run(st, g, ph, 7)
        P.compare_states(a.fields(), ref, 1e-12, 1e-14, set_floor=P.SET_FLOOR, phys=True)


@pytest.mark.parametrize("dtype,M,x_bc,r_bc,rows,nx,wp2", [
    ("f64", 3, "open", "open", 1, 190, 0.02), ("f64", 3, "open", "open", 3, 190, 0.0),
    ("f64", 3, "periodic", "pec", 4, 175, 0.02), ("f64", 2, "open", "pec", 26, 117, 0.0),
    ("f64", 1, "periodic", "open", 2, 61, 0.02), ("f64", 8, "open", "pec", 5, 131, 0.02),
    ("f32", 3, "open", "open", 6, 190, 0.02), ("f32", 4, "periodic", "open", 2, 130, 0.0)])
def test_pair_background_set_alone_equals_single_steps(dtype, M, x_bc, r_bc, rows, nx, wp2):
    """With and without the cold plasma (whose currents the ring carries)."""
    from oracle import qds as Q
    kw = dict(x_bc=x_bc, r_bc=r_bc, wp2=wp2)
    if M > 4:
        kw["dr"] = M * H
    wl = _em(nx, 19, M, **kw)
    st, g, ph = (_random_reachable_state if wp2 else _random_state_no_plasma)(wl, 90 + rows + M)
    a = _run(wl, dtype, st, 9, 1, rows)
    b = _run(wl, dtype, st, 9, 0, rows)
    _equal(a, b)
    if dtype == "f64":
        ref = Q.run(st, g, ph, 9)
        P.compare_states(a.fields(), ref, 1e-12, 1e-14, set_floor=P.SET_FLOOR, phys=True)


@pytest.mark.parametrize("arem", [True, False])
def test_pair_autotuner_trials_change_nothing(arem):
    """The tuner times its first 8 pairs over four heights of each kernel
    (the two-step march in place of kernel B): 21 tuned paired steps equal
    21 single steps at fixed heights."""
    wl = _full(190, 23, 3) if arem else _em(190, 23, 3)
    st, _, _ = _random_reachable_state(wl, 5)
    a = _run(wl, "f64", st, 21, 1, 8, tune=True)
    assert a.tiles()[1]
    b = _run(wl, "f64", st, 21, 0, 8)
    _equal(a, b)


def test_pair_calls_in_a_row_and_uneven_counts():
    """Calls of 1, 2, 3, 4 and 6 steps in a row (the pair buffer allocated on
    the first call that pairs, the table rebuilt for it) equal one call of 16
    single steps; the state's buffer index follows the pairs."""
    from paper_2609_03550_amd import qds
    wl = _full(150, 21, 3)
    st, _, _ = _random_reachable_state(wl, 11)
    a = qds.Solver(wl, dtype="f64")
    a.set_option(qds.OPT_PAIR, 1)
    a.set_option(qds.OPT_ROWS, 6)
    a.load_fields(st)
    for n in (1, 2, 3, 4, 6):
        a.step(n)
    torch.cuda.synchronize()
    b = _run(wl, "f64", st, 16, 0, 6)
    _equal(a, b)


def _window_wl(nx, wp2, noise):
    d = I.Drive(amp=50.0, x0=60 * H, v=0.999, sx=10 * H, r0=0.0, sr=4 * I.DR, noise=noise, seed=3)
    return I.Workload("pair_window", nx, 17, 3, 0, x_bc="window", wp2=wp2,
                      pulses=(I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 50 * H),), drive=d)


@pytest.mark.parametrize("dtype,nx,wp2,noise,rows,random", [
    ("f64", 200, 0.01, 1e-3, 5, False), ("f64", 116, 0.0, 0.0, 3, False), ("f64", 117, 0.01, 1e-3, 1, True),
    ("f64", 232, 0.01, 1e-3, 26, True), ("f32", 175, 0.01, 1e-3, 7, False), ("f32", 174, 0.0, 1e-3, 2, True)])
def test_pair_moving_window_with_drive_equals_single_steps(dtype, nx, wp2, noise, rows, random):
    """The moving window with the prescribed drive, in pairs: the second
    step's strips start one column left (its lane k reads the first step's
    result of lane k), the first step puts the column the window brings in
    into the ring as zeros, and the drive is evaluated for both steps (the
    second one column on).  Widths at and beside multiples of the 58-column
    strip (the second step covers one more column), with and without the
    plasma: 9 steps equal single steps bit for bit, counters included, and
    the oracle in FP64."""
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    wl = _window_wl(nx, wp2, noise)
    out = []
    for pair in (1, 0):
        s = qds.Solver(wl, dtype=dtype)
        s.set_option(qds.OPT_PAIR, pair)
        s.set_option(qds.OPT_ROWS, rows)
        if random:
            st, g, ph = (_random_reachable_state if wp2 else _random_state_no_plasma)(wl, 50 + nx)
            s.load_fields(st)
        else:
            s.load_pulses()
        assert s.fused
        w0 = s.window
        s.step(9)
        torch.cuda.synchronize()
        assert s.window == w0 + 9
        out.append(s)
    _equal(out[0], out[1])
    if dtype == "f64":
        if random:
            ref = Q.run(st, g, ph, 9)
        else:
            ref = P.oracle_run(wl, 9)
        P.compare_states(out[0].fields(), ref, 1e-12, 1e-14, set_floor=P.SET_FLOOR, phys=True)


@pytest.mark.parametrize("dtype,M,x_bc,r_bc,rows,nx", [
    ("f64", 3, "open", "open", 1, 190), ("f64", 3, "open", "open", 5, 190), ("f64", 3, "periodic", "pec", 3, 175),
    ("f64", 3, "open", "pec", 24, 117), ("f64", 1, "open", "open", 4, 59), ("f64", 2, "periodic", "open", 7, 58),
    ("f64", 4, "open", "open", 6, 130), ("f32", 3, "open", "open", 4, 190), ("f32", 4, "periodic", "pec", 9, 121),
    ("f32", 2, "open", "pec", 2, 100)])
def test_pair_with_background_set_march_equals_single_steps(dtype, M, x_bc, r_bc, rows, nx):
    """QDS_OPT_PAIR_A: the background set's two-step march with the axion
    source of both steps (2M waves per tile, each group forming S_a through
    its own exchange area), the first step's field planes to the pair buffer
    for the axion kernel.  7 steps from random reachable states equal single
    steps bit for bit (FP64 with 4 modes does not fit its LDS and pairs with
    kernel A instead); the oracle per field in FP64."""
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    wl = _full(nx, 23, M, x_bc=x_bc, r_bc=r_bc)
    st, g, ph = _random_reachable_state(wl, 30 + rows + M)
    out = []
    for pair, pa in ((1, 1), (0, 0)):
        s = qds.Solver(wl, dtype=dtype)
        s.set_option(qds.OPT_PAIR, pair)
        s.set_option(qds.OPT_PAIR_A, pa)
        s.set_option(qds.OPT_ROWS, rows)
        s.load_fields(st)
        s.step(7)
        torch.cuda.synchronize()
        out.append(s)
    _equal(out[0], out[1])
    if dtype == "f64" and M == 3:
        ref = Q.run(st, g, ph, 7)
        P.compare_states(out[0].fields(), ref, 1e-12, 1e-14, set_floor=P.SET_FLOOR, phys=True)


@pytest.mark.parametrize("arem", [True, False])
def test_pair_with_particle_currents_equals_single_steps(arem):
    """Deposited particle currents (QDS_J_PARTICLES, the same deposit for every
    step of the call) over one call of 5 steps: in pairs (the fused sources
    formed once per call, read by both steps of a pair) equal to single steps
    bit for bit, and to the staged kernels (which form the sums themselves) to
    rounding, with and without the regenerated set."""
    from paper_2609_03550_amd import qds
    wl = _full(150, 21, 3) if arem else _em(150, 21, 3)
    st, _, _ = _random_reachable_state(wl, 17)
    gen = torch.Generator().manual_seed(5)
    planes = None
    out = []
    for pair, path in ((1, qds.PATH_AUTO), (0, qds.PATH_AUTO), (0, qds.PATH_STAGED)):
        s = qds.Solver(wl, dtype="f64", path=path)
        s.set_option(qds.OPT_PAIR, pair)
        s.set_option(qds.OPT_ROWS, 6)
        s.load_fields(st)
        if planes is None:
            planes = [p.copy_(torch.randn(p.shape, dtype=p.dtype, generator=gen).to(p.device))
                      for p in s.current_planes() + s.current_planes()[:1]]
        J = qds.Current()
        ctypes.memmove(ctypes.byref(J), ctypes.byref(s.cur), ctypes.sizeof(qds.Current))
        J.kind = qds.J_PARTICLES
        J.pjx_prev = planes[3].data_ptr()
        J.pjx_next, J.pjr, J.pjt = planes[0].data_ptr(), planes[1].data_ptr(), planes[2].data_ptr()
        qds._check(qds.lib().qds_step(s.h, ctypes.byref(s.state), ctypes.byref(J), ctypes.byref(s.ax), 5,
                                      qds._stream_ptr()), s.h)
        torch.cuda.synchronize()
        out.append(s)
    assert out[0].fused and not out[2].fused
    _equal(out[0], out[1])
    P.compare_states(out[0].fields(), out[2].fields(), 1e-13, 1e-15)


@pytest.mark.parametrize("nx,nr,M,kind", [(8, 4, 1, "full"), (8, 4, 3, "full"), (9, 5, 2, "full"), (8, 4, 3, "em"),
                                          (12, 4, 2, "window"), (8, 6, 3, "full_a2")])
def test_pair_on_the_smallest_grids(nx, nr, M, kind):
    """The smallest grids the library accepts (nx >= 8, nr >= 4): a single
    strip with most lanes beyond the grid, chunks shorter than the two-row
    lag, the exterior ghost row in the first chunk; pairs equal single steps
    bit for bit over 7 steps."""
    from paper_2609_03550_amd import qds
    dr = M * H if M > 1 else I.DR
    if kind.startswith("full"):
        wl = _full(nx, nr, M, dr=dr)
    elif kind == "em":
        wl = _em(nx, nr, M, dr=dr)
    else:
        d = I.Drive(amp=50.0, x0=4 * H, v=0.999, sx=2 * H, r0=0.0, sr=dr, noise=1e-3, seed=3)
        wl = I.Workload("pair_tiny_window", nx, nr, M, 0, x_bc="window", wp2=0.01, dr=dr,
                        pulses=(I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 2 * H, 4 * H),), drive=d)
    st, _, _ = _random_reachable_state(wl, 3 + nx + nr)
    out = []
    for pair in (1, 0):
        for rows in (1, 3):
            s = qds.Solver(wl, dtype="f64")
            s.set_option(qds.OPT_PAIR, pair)
            s.set_option(qds.OPT_PAIR_A, 1 if kind == "full_a2" else 0)
            s.set_option(qds.OPT_ROWS, rows)
            s.load_fields(st)
            assert s.fused
            s.step(7)
            torch.cuda.synchronize()
            out.append(s)
    for s in out[1:]:
        _equal(out[0], s)
