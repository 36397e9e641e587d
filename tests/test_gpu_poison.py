"""Stale-read check: the buffer a step writes is filled with NaN before every
step.  Every value the step later reads must have been written by it (the
transport's output offsets, the halo rows and columns, the exterior ghosts,
the dead last column, the moving window's zero-filled column), so the run must
equal, bit for bit, a run on zero-initialised buffers."""
import pytest
import torch

from paper_2609_03550_amd import inputs as I

pytestmark = pytest.mark.gpu
H = I.H


def _full(nx, nr, M, **kw):
    p1 = I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 0.4 * nx * H)
    p2 = I.Pulse("z", 0.5, 0.8, 3 * I.LAMBDA, 20 * H, 0.4 * nx * H)
    wl = I.Workload("poison", nx, nr, M, 0, wp2=0.01, axion=True, arem=True, ma2=0.02, pulses=(p1, p2))
    return wl.with_(**kw)


def _run(wl, dtype, opts, poison, nsteps=6, per_call=1):
    from paper_2609_03550_amd import qds
    path = opts.pop("path", qds.PATH_AUTO)
    s = qds.Solver(wl, dtype=dtype, path=path)
    for k, v in opts.items():
        s.set_option(k, v)
    s.load_pulses()
    for _ in range(nsteps // per_call):
        if poison:
            s.bufs[1 - s.state.cur].fill_(0xFF)      # every word a NaN
        s.step(per_call)
    torch.cuda.synchronize()
    return s


@pytest.mark.parametrize("case", ["split", "kernel_ax", "window_kernel_ax", "staged", "eight_modes", "em_window"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_poisoned_output_buffer_changes_nothing(case, dtype):
    from paper_2609_03550_amd import qds
    opts = {qds.OPT_ROWS: 5}
    wl = _full(130, 17, 3)
    if case == "kernel_ax":
        opts[qds.OPT_KERNEL_AX] = 1
    elif case == "window_kernel_ax":
        wl = _full(130, 17, 3, x_bc="window")
    elif case == "staged":
        opts["path"] = qds.PATH_STAGED
        wl = _full(130, 17, 3, x_bc="window")
    elif case == "eight_modes":
        wl = _full(130, 17, 8, dr=8 * H, r_bc="pec")
    elif case == "em_window":
        d = I.Drive(amp=50.0, x0=60 * H, v=0.999, sx=10 * H, r0=0.0, sr=4 * I.DR, noise=1e-3, seed=3)
        wl = I.Workload("poison_em", 130, 17, 3, 0, x_bc="window", wp2=0.01,
                        pulses=(I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 50 * H),), drive=d)
    a = _run(wl, dtype, dict(opts), poison=False)
    b = _run(wl, dtype, dict(opts), poison=True)
    assert a.state.cur == b.state.cur
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert torch.isfinite(fb[k]).all(), k
        assert torch.equal(fa[k], fb[k]), k


@pytest.mark.parametrize("case", ["regenerated", "em", "em_window"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_poisoned_output_buffer_changes_nothing_in_pairs(case, dtype):
    """The same for pairs of steps: the buffer a pair writes (the state's other
    buffer, as for a single step) is filled with NaN before every call of two
    steps, so everything the two-step march (and, with the regenerated set,
    the second half of kernel A and the axion kernel) leaves must be written
    by it: 8 steps in 4 calls equal a run on zero-initialised buffers."""
    from paper_2609_03550_amd import qds
    opts = {qds.OPT_ROWS: 5, qds.OPT_PAIR: 1}
    if case == "regenerated":
        wl = _full(130, 17, 3)
    elif case == "em":
        wl = I.Workload("poison_em2", 130, 17, 3, 0, wp2=0.01,
                        pulses=(I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 50 * H),))
    else:
        d = I.Drive(amp=50.0, x0=60 * H, v=0.999, sx=10 * H, r0=0.0, sr=4 * I.DR, noise=1e-3, seed=3)
        wl = I.Workload("poison_em", 117, 17, 3, 0, x_bc="window", wp2=0.01,
                        pulses=(I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 50 * H),), drive=d)
    a = _run(wl, dtype, dict(opts), poison=False, nsteps=8, per_call=2)
    b = _run(wl, dtype, dict(opts), poison=True, nsteps=8, per_call=2)
    assert a.state.cur == b.state.cur
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert torch.isfinite(fb[k]).all(), k
        assert torch.equal(fa[k], fb[k]), k
