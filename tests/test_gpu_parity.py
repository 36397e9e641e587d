"""GPU parity: the HIP step (through the C ABI) against the CPU oracle, element
by element on the same seeded inputs.  Relative L2 per field and mode against
the field's own norm (fields below 1e-3 of their field set's norm against that
fraction of the set's norm): FP64 <= 1e-12, FP32 <= 1e-5."""
import os

import pytest
import torch

from paper_2609_03550_amd import inputs as I
import parity_tools as P

pytestmark = pytest.mark.gpu
H, DR = I.H, I.DR
TOL = {"f64": (1e-12, 1e-13), "f32": (1e-5, 1e-6)}


def _solver(wl, dtype, path=0, rows=None):
    from paper_2609_03550_amd import qds
    s = qds.Solver(wl, dtype=dtype, path=path, rows=rows)
    s.load_pulses()
    return s


def _check(wl, nsteps, dtype, chunks=1, path=0, rows=None):
    s = _solver(wl, dtype, path, rows)
    for _ in range(chunks):
        s.step(nsteps // chunks)
    torch.cuda.synchronize()
    ora = P.oracle_run(wl, nsteps)
    tol, floor = TOL[dtype]
    P.compare_states(s.fields(), ora, tol, floor, set_floor=P.SET_FLOOR, phys=True)
    assert s.n == nsteps
    return s


def _vac(nx, nr, M, **kw):
    p = I.Pulse("y", 0.05, 1.0, 3 * I.LAMBDA, 20 * H, 0.4 * nx * H)
    return I.Workload("vac", nx, nr, M, 0, pulses=(p,)).with_(**kw)


def _full(nx, nr, M, **kw):
    p1 = I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 0.4 * nx * H)
    p2 = I.Pulse("z", 0.5, 0.8, 3 * I.LAMBDA, 20 * H, 0.4 * nx * H)
    if M == 1:
        p1 = I.Pulse("r", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 0.4 * nx * H)
        p2 = I.Pulse("t", 0.5, 0.8, 3 * I.LAMBDA, 20 * H, 0.4 * nx * H)
    wl = I.Workload("full", nx, nr, M, 0, wp2=0.01, axion=True, arem=True, ma2=0.02, pulses=(p1, p2))
    return wl.with_(**kw)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("x_bc,r_bc", [("open", "open"), ("periodic", "pec"), ("open", "pec"), ("periodic", "open")])
def test_vacuum_em(dtype, x_bc, r_bc):
    _check(_vac(130, 14, 3, x_bc=x_bc, r_bc=r_bc), 25, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_config1_vacuum_pulse_full_length(dtype):
    """512 x 64 x 2 modes, 200 steps: the small EM workload in full."""
    _check(I.vacuum_em(), 200, dtype, chunks=4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_driven_moving_window(dtype):
    wl = I.driven_window(nx=200, nr=20, steps=0)
    d = wl.drive
    wl = wl.with_(drive=d.__class__(d.amp * 1e4, 90 * H, d.v, 10 * H, 0.0, 4 * DR, d.noise, d.seed),
                  pulses=(wl.pulses[0].__class__("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 140 * H),))
    _check(wl, 30, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_full_physics_modes(dtype, M):
    _check(_full(97, 13, M), 14, dtype)


@pytest.mark.parametrize("dtype", ["f64"])
@pytest.mark.parametrize("x_bc,r_bc", [("periodic", "pec"), ("periodic", "open"), ("open", "pec")])
def test_full_physics_boundaries(dtype, x_bc, r_bc):
    _check(_full(96, 12, 3, x_bc=x_bc, r_bc=r_bc), 14, dtype)


def test_full_physics_external_field_and_scales():
    wl = _full(100, 12, 3, bext=(0.3 + 0j, 0.7 - 0.2j, -0.2 - 0.7j), s_phi=0.5, s_j=2.0)
    _check(wl, 10, "f64")


def test_full_physics_longer_run():
    _check(_full(160, 24, 3), 120, "f64", chunks=3)


# ---- both paths: the staged kernels and the fused single-pass kernels


@pytest.mark.parametrize("path,rows", [(1, 16), (2, 1), (2, 3), (2, 7), (2, 16), (2, 64)])
def test_fused_and_staged_chunk_seams(path, rows):
    """Every radial chunk size (seams between workgroups at every row) gives
    the oracle's result; path 1 = staged kernels (one chunk size: it only
    affects the fused kernels), 2 = fused kernels."""
    s = _check(_full(131, 15, 3), 12, "f64", path=path, rows=rows)
    assert s.fused == (path == 2)


@pytest.mark.parametrize("M", [1, 2, 4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_modes(M, dtype):
    s = _check(_full(70, 9, M), 10, dtype, path=2, rows=4)
    assert s.fused


@pytest.mark.parametrize("x_bc,r_bc", [("periodic", "pec"), ("periodic", "open"), ("open", "pec")])
def test_fused_boundaries(x_bc, r_bc):
    _check(_full(128, 12, 3, x_bc=x_bc, r_bc=r_bc), 12, "f64", path=2, rows=5)


@pytest.mark.parametrize("dtype,M,rows", [("f64", 3, 5), ("f64", 1, 3), ("f32", 3, 4), ("f64", 4, 1)])
def test_window_with_regenerated_set_runs_kernel_ax(dtype, M, rows):
    """The moving window with the regenerated set runs kernel AX (the axion
    current from the background set's old columns, held in registers, while
    every new value lands one column left): it matches the oracle and the
    staged kernels (which shift after the whole step) to rounding; beyond 4
    modes the fused path refuses the combination."""
    from paper_2609_03550_amd import qds
    wl = _full(128, 12, M, x_bc="window")
    s = _check(wl, 12, dtype, rows=rows)
    assert s.fused
    st = qds.Solver(wl, dtype=dtype, path=qds.PATH_STAGED)
    st.load_pulses()
    st.step(12)
    torch.cuda.synchronize()
    close = (1e-13, 1e-15) if dtype == "f64" else (2e-6, 1e-7)
    P.compare_states(s.fields(), st.fields(), *close)
    with pytest.raises(qds.QDSError):
        qds.Solver(_full(128, 12, 5, x_bc="window", dr=5 * H), path=qds.PATH_FUSED)


def test_window_axion_without_regenerated_set_fused():
    s = _check(_full(128, 12, 3, x_bc="window", arem=False), 12, "f64", path=2, rows=5)
    assert s.fused


@pytest.mark.parametrize("rows", [2, 9])
def test_fused_em_only_window_drive(rows):
    wl = I.driven_window(nx=200, nr=20, steps=0)
    d = wl.drive
    wl = wl.with_(drive=d.__class__(d.amp * 1e4, 90 * H, d.v, 10 * H, 0.0, 4 * DR, d.noise, d.seed),
                  pulses=(wl.pulses[0].__class__("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 140 * H),))
    _check(wl, 30, "f64", path=2, rows=rows)


def test_fused_matches_staged_on_a_long_run():
    """The two paths agree with each other to rounding after many steps."""
    from paper_2609_03550_amd import qds
    wl = _full(250, 30, 3, bext=(0.1 + 0j, 0.2 + 0.1j, -0.1 + 0.2j))
    a = _solver(wl, "f64", path=1)
    b = _solver(wl, "f64", path=2, rows=8)
    a.step(300)
    b.step(300)
    torch.cuda.synchronize()
    P.compare_states(b.fields(), a.fields(), 1e-11, 1e-12)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("pair", [0, 1])
def test_autotuned_tiles_change_no_result(dtype, pair):
    """qds_step with the autotuner on: its 8 trials (four tile heights, twice;
    single steps, or pairs of steps with the two-step march of the
    regenerated set in place of kernel B) and the chosen tiles give
    bit-identical states to the default tiling, and the chosen heights are
    candidates (for the two-step march, whose candidates follow the GPU's
    occupancy: 20 rows or a height that tiles the 21 rows)."""
    from paper_2609_03550_amd import qds
    wl = _full(70, 20, 3)
    a = qds.Solver(wl, dtype=dtype)
    a.load_pulses()
    b = qds.Solver(wl, dtype=dtype)
    b.load_pulses()
    for s in (a, b):
        s.set_option(qds.OPT_PAIR, pair)
    b.set_option(qds.OPT_TUNE, 1)
    a.step(18)
    b.step(18)
    torch.cuda.synchronize()
    rows, tuned = b.tiles()
    assert tuned and rows[0] in (8, 16, 24, 32) and rows[1] in (4, 6, 8, 16)
    if pair:
        assert rows[2] == 16 and 4 <= rows[3] <= 21
    else:
        assert rows[2] in (16, 32, 52, 64) and rows[3] == 11
    assert a.tiles() == ([16, 16, 16, 11], False)
    assert torch.equal(a.bufs[a.state.cur], b.bufs[b.state.cur])


@pytest.mark.parametrize("pair", [0, 1])
def test_autotuned_tiles_with_a_drive_change_no_result(pair):
    """With a prescribed drive (moving window, no axion; the drive plane is
    filled before every step, both planes before every pair) the autotuner's
    choice is one of the candidates of the background set alone (single
    steps) or of the two-step march (pairs: 20 rows or a height that tiles
    the 21 rows), and the states are bit-identical to the default tiling."""
    from paper_2609_03550_amd import qds
    wl = I.driven_window(nx=200, nr=20, steps=0)
    d = wl.drive
    wl = wl.with_(drive=d.__class__(d.amp * 1e4, 90 * H, d.v, 10 * H, 0.0, 4 * DR, d.noise, d.seed))
    a = _solver(wl, "f64")
    b = _solver(wl, "f64")
    for s in (a, b):
        s.set_option(qds.OPT_PAIR, pair)
    b.set_option(qds.OPT_TUNE, 1)
    a.step(18)
    b.step(18)
    torch.cuda.synchronize()
    rows, tuned = b.tiles()
    assert tuned
    assert 4 <= rows[3] <= 21 if pair else rows[0] in (8, 16, 26, 52)
    assert torch.equal(a.bufs[a.state.cur], b.bufs[b.state.cur])


@pytest.mark.parametrize("dtype,M,x_bc,r_bc", [("f64", 3, "open", "open"), ("f32", 3, "open", "open"),
                                               ("f64", 4, "periodic", "pec"), ("f64", 1, "open", "pec")])
def test_overlapped_steps_change_no_result(dtype, M, x_bc, r_bc):
    """QDS_OPT_OVERLAP runs kernel A of step k+1 on a second stream beside the
    regenerated set of step k: calls of 1, 2 and 7 steps (the last with the
    per-kernel timing events on) give bit-identical states to the serial
    order, and the overlapped solver still matches the oracle."""
    from paper_2609_03550_amd import qds
    wl = _full(190, 20, M, x_bc=x_bc, r_bc=r_bc)
    a = qds.Solver(wl, dtype=dtype)
    a.load_pulses()
    b = qds.Solver(wl, dtype=dtype)
    b.load_pulses()
    b.set_option(qds.OPT_OVERLAP, 1)
    for n in (1, 2, 7):
        if n == 7:
            b.set_option(qds.OPT_TIMING, 1)
        a.step(n)
        b.step(n)
        torch.cuda.synchronize()
        assert torch.equal(a.bufs[a.state.cur], b.bufs[b.state.cur]), n
    assert b.n == 10
    tol, floor = TOL[dtype]
    P.compare_states(b.fields(), P.oracle_run(wl, 10), tol, floor, set_floor=P.SET_FLOOR, phys=True)


def test_per_kernel_tile_heights_change_no_result():
    """QDS_OPT_ROWS_A / _CUR / _B / _PAIR set one kernel's tile height each
    (used to replay the autotuner's choice): uneven heights that leave ragged
    last chunks give bit-identical states (9 steps: four pairs, then a single
    step with kernel B); out-of-range heights are rejected."""
    from paper_2609_03550_amd import qds
    wl = _full(131, 21, 3)
    a = qds.Solver(wl, dtype="f64")
    a.load_pulses()
    b = qds.Solver(wl, dtype="f64")
    b.load_pulses()
    for opt, v in ((qds.OPT_ROWS_A, 5), (qds.OPT_ROWS_CUR, 3), (qds.OPT_ROWS_B, 13), (qds.OPT_ROWS_PAIR, 7)):
        b.set_option(opt, v)
    assert b.tiles() == ([5, 3, 13, 7], False)
    a.step(9)
    b.step(9)
    torch.cuda.synchronize()
    assert torch.equal(a.bufs[a.state.cur], b.bufs[b.state.cur])
    for bad in (0, 4097):
        with pytest.raises(qds.QDSError):
            b.set_option(qds.OPT_ROWS_CUR, bad)
        with pytest.raises(qds.QDSError):
            b.set_option(qds.OPT_ROWS_PAIR, bad)
    assert b.tiles() == ([5, 3, 13, 7], False)


@pytest.mark.parametrize("dtype,x_bc,r_bc,arem,M", [("f64", "open", "open", True, 3), ("f64", "periodic", "pec", True, 3),
                                                    ("f32", "open", "open", True, 3), ("f64", "window", "open", False, 3),
                                                    ("f64", "window", "pec", True, 3), ("f64", "open", "open", True, 1),
                                                    ("f64", "open", "open", True, 4), ("f64", "open", "pec", True, 5),
                                                    ("f64", "periodic", "open", False, 2)])
def test_random_full_state(dtype, x_bc, r_bc, arem, M):
    """Every plane of both sets, the plasma currents and the axion start at
    O(1) seeded random values (so every term of the step, the couplings
    included, weighs as much as the transport): one oracle step makes it a
    state the scheme can reach (fixed axis rows, ghosts), then GPU and oracle
    take 4 steps from it over three x strips and several radial chunks (the
    staged kernels for the moving window with the regenerated set)."""
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    # (more modes need a coarser dr for the radial stability bound)
    wl = _full(131, 21, M, x_bc=x_bc, r_bc=r_bc, arem=arem, **({"dr": 5 * H} if M > 4 else {}))
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    gen = torch.Generator().manual_seed(2609)
    for k, v in st.items():
        if isinstance(v, torch.Tensor) and v.is_complex():
            st[k] = torch.randn(v.shape, dtype=torch.complex128, generator=gen)
    st = Q.step(st, g, ph)
    s = qds.Solver(wl, dtype=dtype)
    s.load_fields(st)
    assert s.fused
    s.step(4)
    torch.cuda.synchronize()
    ref = Q.run(st, g, ph, 4)
    tol, floor = (1e-12, 1e-14) if dtype == "f64" else (1e-5, 1e-7)
    P.compare_states(s.fields(), ref, tol, floor, set_floor=P.SET_FLOOR, phys=True)


def _random_reachable_state(wl, seed):
    """O(1) seeded random values in every complex plane, then one oracle step
    (fixed axis rows, ghosts): a state the scheme can reach."""
    from oracle import qds as Q
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    gen = torch.Generator().manual_seed(seed)
    for k, v in st.items():
        if isinstance(v, torch.Tensor) and v.is_complex():
            st[k] = torch.randn(v.shape, dtype=torch.complex128, generator=gen)
    return Q.step(st, g, ph), g, ph


@pytest.mark.parametrize("kernel_ax", [0, 1])
@pytest.mark.parametrize("x_bc,r_bc", [("open", "open"), ("periodic", "pec")])
def test_axion_advance_in_current_march_equals_kernel_a(x_bc, r_bc, kernel_ax):
    """Placements of the axion advance on one random full state: with the
    regenerated set, the marched axion kernel after kernel A (kernel_ax 0) or
    the one-pass kernel AX (kernel_ax 1) advances T_a and phi; without it kernel A advances them
    itself.  The background set and the axion do not depend on the
    regenerated set, so after 6 steps the runs agree on them bit for bit."""
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    wl = _full(131, 21, 3, x_bc=x_bc, r_bc=r_bc)
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    gen = torch.Generator().manual_seed(7)
    for k, v in st.items():
        if isinstance(v, torch.Tensor) and v.is_complex():
            st[k] = torch.randn(v.shape, dtype=torch.complex128, generator=gen)
    st = Q.step(st, g, ph)
    a = qds.Solver(wl, dtype="f64")
    a.set_option(qds.OPT_KERNEL_AX, kernel_ax)
    a.load_fields(st)
    a.step(6)
    b = qds.Solver(wl.with_(arem=False), dtype="f64")
    b.load_fields(st)
    b.step(6)
    torch.cuda.synchronize()
    assert a.fused and b.fused
    fa, fb = a.fields(), b.fields()
    assert set(fb) and set(fb) < set(fa)
    for k in fb:
        assert torch.equal(fa[k], fb[k]), k


def test_random_state_with_drive():
    """The prescribed drive (with its noise) on a random full state in the
    moving window: the drive plane of each step, read by the background set,
    against the oracle."""
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    wl = I.driven_window(nx=200, nr=20, steps=0)
    d = wl.drive
    wl = wl.with_(drive=d.__class__(d.amp * 1e4, 90 * H, d.v, 10 * H, 0.0, 4 * DR, d.noise, d.seed), pulses=())
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    s = qds.Solver(wl)
    held = set(s.fields())        # no plasma here: the current planes stay zero
    gen = torch.Generator().manual_seed(1)
    for k, v in st.items():
        if k in held:
            st[k] = torch.randn(v.shape, dtype=torch.complex128, generator=gen)
    st = Q.step(st, g, ph)
    s.load_fields(st)
    s.step(5)
    torch.cuda.synchronize()
    ref = Q.run(st, g, ph, 5)
    P.compare_states(s.fields(), ref, 1e-12, 1e-14)


@pytest.mark.parametrize("dtype,x_bc", [("f64", "open"), ("f32", "open"), ("f64", "window"), ("f32", "window")])
def test_random_state_with_drive_and_regenerated_set(dtype, x_bc):
    """The prescribed drive together with the plasma, the axion and the
    regenerated set: the drive plane feeds the background set while the axion
    and kernel B run as without a drive (open x: kernel A and the marched
    axion kernel; the moving window: kernel AX); a random full state, 4
    steps, against the oracle."""
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    d = I.Drive(amp=50.0, x0=60 * H, v=0.999, sx=10 * H, r0=0.0, sr=4 * DR, noise=1e-3, seed=3)
    wl = _full(131, 21, 3, x_bc=x_bc).with_(drive=d)
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    gen = torch.Generator().manual_seed(11)
    for k, v in st.items():
        if isinstance(v, torch.Tensor) and v.is_complex():
            st[k] = torch.randn(v.shape, dtype=torch.complex128, generator=gen)
    st = Q.step(st, g, ph)
    s = qds.Solver(wl, dtype=dtype)
    s.load_fields(st)
    assert s.fused
    s.step(4)
    torch.cuda.synchronize()
    ref = Q.run(st, g, ph, 4)
    tol, floor = (1e-12, 1e-14) if dtype == "f64" else (1e-5, 1e-7)
    P.compare_states(s.fields(), ref, tol, floor, set_floor=P.SET_FLOOR, phys=True)


def test_stop_save_reload_continue_is_bitwise():
    """Checkpoint and resume: 5 steps, the state saved through fields() and
    loaded into a fresh solver (counters included), 6 more steps, equals 11
    uninterrupted steps bit for bit (FP64; the moving window with the drive,
    whose lab position and noise depend on the counters)."""
    from paper_2609_03550_amd import qds
    wl = I.driven_window(nx=200, nr=20, steps=0)
    d = wl.drive
    wl = wl.with_(drive=d.__class__(d.amp * 1e4, 90 * H, d.v, 10 * H, 0.0, 4 * DR, d.noise, d.seed),
                  pulses=(wl.pulses[0].__class__("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 140 * H),))
    a = _solver(wl, "f64")
    a.step(11)
    b = _solver(wl, "f64")
    b.step(5)
    saved = dict(b.fields(), n=b.n, w=b.window)
    c = qds.Solver(wl, dtype="f64")
    c.load_fields(saved)
    c.step(6)
    torch.cuda.synchronize()
    assert (c.n, c.window) == (a.n, a.window)
    fa, fc = a.fields(), c.fields()
    for k in fa:
        assert torch.equal(fa[k], fc[k]), k


@pytest.mark.parametrize("dtype,M,x_bc,r_bc,rows", [
    ("f64", 3, "open", "open", 1), ("f64", 3, "open", "open", 2), ("f64", 3, "open", "open", 5),
    ("f64", 3, "periodic", "pec", 3), ("f64", 3, "open", "pec", 24), ("f64", 1, "open", "open", 4),
    ("f64", 2, "periodic", "open", 7), ("f64", 4, "open", "open", 6), ("f32", 3, "open", "open", 4),
    ("f32", 2, "open", "pec", 1), ("f32", 4, "periodic", "pec", 9)])
def test_kernel_ax_equals_split_kernels_and_oracle(dtype, M, x_bc, r_bc, rows):
    """Kernel AX (the background set, the axion source, the axion advance and
    the axion current in one r-march, j_a,r rows owned one row down) against
    the split kernels (kernel A writing S_a, the marched axion kernel
    re-reading the background set) on a random full state, at chunk heights
    from one row up (the two lower halo rows, the ghost chunk, ragged last
    chunks): every plane agrees to rounding after 5 steps, and both match the
    oracle per field."""
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    wl = _full(190, 23, M, x_bc=x_bc, r_bc=r_bc)
    st, g, ph = _random_reachable_state(wl, 31 + rows)
    out = []
    for kernel_ax in (1, 0):
        s = qds.Solver(wl, dtype=dtype)
        s.set_option(qds.OPT_KERNEL_AX, kernel_ax)
        s.set_option(qds.OPT_ROWS, rows)
        s.load_fields(st)
        assert s.fused
        s.step(5)
        torch.cuda.synchronize()
        out.append(s.fields())
    ref = Q.run(st, g, ph, 5)
    tol, floor = (1e-12, 1e-14) if dtype == "f64" else (1e-5, 1e-7)
    for f in out:
        P.compare_states(f, ref, tol, floor, set_floor=P.SET_FLOOR, phys=True)
    close = (1e-14, 1e-15) if dtype == "f64" else (2e-6, 1e-7)
    P.compare_states(out[0], out[1], *close)


@pytest.mark.parametrize("dtype,M,arem,rows", [("f64", 5, True, 7), ("f64", 6, True, 4), ("f64", 7, True, 9),
                                              ("f64", 8, True, 5), ("f64", 6, False, 6), ("f32", 6, True, 5),
                                              ("f32", 8, True, 3)])
def test_fused_kernels_beyond_four_modes(dtype, M, arem, rows):
    """5 to 8 modes on the fused kernels (one wavefront per mode, workgroups of
    up to 512 threads, the mode convolutions reading their factors from LDS as
    needed; dr = M dx, what the radial stability bound allows): a random full
    state against the oracle, and against the staged kernels (one thread per
    point and every mode) to rounding, over 4 steps and several chunks."""
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    wl = _full(131, 21, M, arem=arem, dr=M * H)
    st, g, ph = _random_reachable_state(wl, 40 + M)
    out = {}
    for path in (qds.PATH_FUSED, qds.PATH_STAGED):
        s = qds.Solver(wl, dtype=dtype, path=path)
        s.set_option(qds.OPT_ROWS, rows)
        s.load_fields(st)
        assert s.fused == (path == qds.PATH_FUSED)
        s.step(4)
        torch.cuda.synchronize()
        out[path] = s.fields()
    ref = Q.run(st, g, ph, 4)
    tol, floor = (1e-12, 1e-14) if dtype == "f64" else (1e-5, 1e-7)
    P.compare_states(out[qds.PATH_FUSED], ref, tol, floor, set_floor=P.SET_FLOOR, phys=True)
    close = (1e-13, 1e-15) if dtype == "f64" else (2e-6, 1e-7)
    P.compare_states(out[qds.PATH_FUSED], out[qds.PATH_STAGED], *close)
