"""qds_loss_eval_noalloc (the entry point that allocates nothing) against
qds_loss_eval (which takes a temporary gradient buffer) through the C ABI:
two calls in a row, the second on a smaller grid and a narrower loss window,
in double and single precision."""
import ctypes

import pytest
import torch

from paper_2609_03550_amd import inputs as I

pytestmark = pytest.mark.gpu
H = I.H


def _solver(nx, nr, M, dtype):
    from paper_2609_03550_amd import qds
    p1 = I.Pulse("y", 0.5, 1.0, 2 * I.LAMBDA, 10 * H, 0.5 * nx * H)
    p2 = I.Pulse("z", 0.4, 0.8, 2 * I.LAMBDA, 10 * H, 0.5 * nx * H)
    wl = I.Workload("noalloc", nx, nr, M, 0, wp2=0.02, axion=True, arem=True, ma2=0.03, pulses=(p1, p2))
    s = qds.Solver(wl, dtype=dtype)
    s.load_pulses()
    s.step(6)
    return s


def _both(s, lset, mode, x0, x1):
    from paper_2609_03550_amd import qds
    L = qds.lib()
    lo = qds.Loss(lset, mode, x0, x1)
    out = torch.zeros(2, dtype=torch.float64, device=s.device)
    buf = s.bufs[s.state.cur].data_ptr()
    stream = torch.cuda.current_stream().cuda_stream
    assert L.qds_loss_eval(s.h, buf, ctypes.byref(lo), out.data_ptr(), None, stream) == qds.QDS_OK
    st = L.qds_loss_eval_noalloc(s.h, buf, ctypes.byref(lo), out.data_ptr() + 8, stream)
    assert st == qds.QDS_OK, L.qds_last_error(s.h)
    torch.cuda.synchronize()
    return float(out[0]), float(out[1])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_loss_equals_allocating_loss(dtype):
    big = _solver(300, 37, 3, dtype)
    small = _solver(96, 9, 2, dtype)
    cases = [(big, 1, 1, 0, 300), (small, 0, 1, 10, 70)]
    for s, lset, mode, x0, x1 in cases:
        ref, got = _both(s, lset, mode, x0, x1)
        assert ref > 0
        # the two sum the same per-point terms in different orders
        tol = 1e-12 if dtype == "f64" else 1e-12
        assert abs(got / ref - 1) < tol, (dtype, s.wl.nx, got, ref)
    # the first handle again after the smaller call: nothing left over
    ref, got = _both(big, 0, 1, 5, 290)
    assert abs(got / ref - 1) < 1e-12
    big.close()
    small.close()


def test_noalloc_full_width_window_after_other_calls():
    """A full-width window on a fresh handle after the calls above (the
    refusal of a window beyond the scratch is checked on the CPU)."""
    from paper_2609_03550_amd import qds
    s = _solver(300, 37, 3, "f64")
    ref, got = _both(s, 0, 1, 0, 300)
    assert ref > 0 and abs(got / ref - 1) < 1e-12
    s.close()
