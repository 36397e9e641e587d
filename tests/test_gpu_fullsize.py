"""Parity at the benchmark sizes.

The full-size grids run on the GPU in the launch configuration bench.py
times (the autotuner's trial steps first, then its tiles).  The oracle cannot
step a full grid in seconds, so it runs the same initial data on an x-crop:
the transport moves information exactly one cell per step and the
longitudinal updates read one neighbouring column, so after n steps the crop
agrees with the full grid at every column more than n + 2 columns from the
crop edges (the moving window adds n more at the right edge).  The crop keeps
the lab column of its first cell as the window offset, so the prescribed
drive and its noise are those of the full grid.

Each physical field and mode is compared against its own norm (fields below
1e-3 of their field set's norm against that fraction of the set's norm: their
last digits follow the rounding of the set's dominant values).  The axion and
regenerated fields follow from nearly cancelling sources (the E.B of
co-propagating waves; the T^- sources Gamma -+ Phi of a forward beam), so
storage rounding alone moves them by far more than the unit roundoff: in
single precision by up to ~1e-4 of their norm over these steps, in double
precision by up to ~5e-12.  Every field is therefore held to 1e-5 (single) or
1e-12 (double), or to 4x the deviation of the oracle run whose state passes
through storage rounding of that precision after every step, whichever is
larger.

The adjoint at its full size (2000 steps, checkpoints every 45) is checked by
properties that hold at any size: the scaled-unit sensitivities equal 2L, and
the gradient along an envelope coefficient equals the central difference of
the GPU forward loss.
"""
from dataclasses import replace

import pytest
import torch

from oracle import qds as Q
from paper_2609_03550_amd import inputs as I
import parity_tools as P

pytestmark = pytest.mark.gpu
TOL = {"f64": (1e-12, 1e-13), "f32": (1e-5, 1e-6)}


def _gpu_full(wl, dtype, nsteps):
    from paper_2609_03550_amd import qds
    s = qds.Solver(wl, dtype=dtype)
    s.load_pulses()
    s.set_option(qds.OPT_TUNE, 1)
    s.step(nsteps)
    torch.cuda.synchronize()
    # the autotuner has run on the first 8 steps (with or without a drive)
    assert s.tiles()[1]
    return s.fields()


def _crop(wl, x0, width, product_form=None):
    """Initial state, grid and physics of the x-crop starting at lab column x0."""
    pulses = tuple(replace(p, x0=p.x0 - x0 * wl.h) for p in wl.pulses)
    wc = wl.with_(nx=width, pulses=pulses)
    g, ph = Q.grid_physics(wc)
    if product_form:
        ph = replace(ph, product_form=product_form)
    st = Q.init_state(wc)
    st["w"] = x0          # lab column of crop column 0
    return st, g, ph


def _oracle_crop(wl, x0, width, nsteps, product_form=None):
    st, g, ph = _crop(wl, x0, width, product_form)
    return Q.run(st, g, ph, nsteps)


def _oracle_crop_rounded(wl, x0, width, nsteps, dtype):
    """The crop run with its state passed through storage rounding of
    ``dtype`` after every step (the arithmetic stays FP64)."""
    st, g, ph = _crop(wl, x0, width)
    return P.run_rounded(st, g, ph, nsteps, dtype)


def _compare(gpu, ref, x0, lo, hi, dtype):
    """Per physical field and mode on the crop's exact columns [lo, hi): within
    the precision's tolerance or 4x the storage-rounding deviation."""
    a = {k: v[..., x0 + lo:x0 + hi] for k, v in gpu.items()}
    b = {k: ref["plain"][k][..., lo:hi] for k in gpu}
    e = {k: ref[dtype][k][..., lo:hi] for k in gpu}
    return P.compare_band(a, b, e, TOL[dtype][0])


AX_N, AX_X0, AX_W = 128, 900, 600      # the crop holds the two-colour pulse (centre 1100 -> 1228)
WIN_N, WIN_X0, WIN_W = 128, 1800, 600  # the crop holds the drive (centre 2048)


def _oracle_set(wl, x0, width, nsteps):
    return {"plain": _oracle_crop(wl, x0, width, nsteps),
            "f64": _oracle_crop_rounded(wl, x0, width, nsteps, "f64"),
            "f32": _oracle_crop_rounded(wl, x0, width, nsteps, "f32")}


@pytest.fixture(scope="module")
def axion_oracle():
    """The FP64 oracle run of the axion crop and its two storage-rounded
    twins, shared by both precisions and the literal-order test."""
    return _oracle_set(I.axion_two_colour(8192, 256, 6000, 3), AX_X0, AX_W, AX_N)


@pytest.fixture(scope="module")
def window_oracle():
    return _oracle_set(I.driven_window(4096, 256, 4000), WIN_X0, WIN_W, WIN_N)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_axion_two_colour_full_size(dtype, axion_oracle):
    """8192 x 256 x 3 modes, full physics, 128 steps (8 autotuner trials +
    120), against a 600-column crop of the oracle (exact away from its edges)."""
    wl = I.axion_two_colour(8192, 256, 6000, 3)
    gpu = _gpu_full(wl, dtype, AX_N)
    w = _compare(gpu, axion_oracle, AX_X0, AX_N + 2, AX_W - AX_N - 2, dtype)
    print(f"{dtype}: worst per-field relative L2 {w[3]:.2e} ({w[1]}[{w[2]}]), storage rounding there {w[4]:.2e}")


def test_axion_full_size_against_the_literal_product_order(axion_oracle):
    """The literal E/B order of the products (Eqs. source_mode_m, jax_mode ..
    jat_mode as written) on the same 128-step crop: the oracle's two product
    orders, and the GPU (which uses the collected transport order) against the
    literal one, agree per physical field within 1e-12 or 4x the FP64
    storage-rounding deviation (the cancellation of the products sets how far
    any two FP64 evaluation orders drift apart)."""
    wl = I.axion_two_colour(8192, 256, 6000, 3)
    eb = _oracle_crop(wl, AX_X0, AX_W, AX_N, product_form="eb")
    gpu = _gpu_full(wl, "f64", AX_N)
    lo, hi = AX_N + 2, AX_W - AX_N - 2
    crop = lambda st: {k: st[k][..., lo:hi] for k in gpu}
    emu = crop(axion_oracle["f64"])
    w_ora = P.compare_band(crop(axion_oracle["plain"]), crop(eb), emu, 1e-12)
    w_gpu = P.compare_band({k: v[..., AX_X0 + lo:AX_X0 + hi] for k, v in gpu.items()}, crop(eb), emu, 1e-12)
    print(f"literal vs transport product order over 128 steps: oracle {w_ora[3]:.2e} ({w_ora[1]}[{w_ora[2]}]), "
          f"GPU {w_gpu[3]:.2e} ({w_gpu[1]}[{w_gpu[2]}])")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_driven_window_full_size(dtype, window_oracle):
    """4096 x 256 x 3 modes, prescribed drive with noise, moving window, 128 steps."""
    wl = I.driven_window(4096, 256, 4000)
    gpu = _gpu_full(wl, dtype, WIN_N)
    w = _compare(gpu, window_oracle, WIN_X0, WIN_N + 2, WIN_W - 2 * WIN_N - 2, dtype)
    print(f"{dtype}: worst per-field relative L2 {w[3]:.2e} ({w[1]}[{w[2]}]), storage rounding there {w[4]:.2e}")


def test_adjoint_full_size_properties():
    """4096 x 128 x 2 modes, 2000 steps, checkpoints every 45 (FP64)."""
    from paper_2609_03550_amd import qds
    wl = I.adjoint_workload()
    s = qds.Solver(wl)
    s.load_pulses()
    L, lam, dlds = s.backward(2000, 45)
    assert L > 0
    assert abs(dlds[0] / (2 * L) - 1) < 1e-9
    assert abs(dlds[1] / (2 * L) - 1) < 1e-9
    q = 3
    b = qds.Solver(wl)
    b.load_pulses(basis=(0, q))
    torch.cuda.synchronize()
    grad = s.dot(lam, b.bufs[b.state.cur])
    eps = 1e-4
    vals = []
    for sgn in (1, -1):
        c = list(wl.pulses[0].coeffs)
        c[q] += sgn * eps
        w2 = wl.with_(pulses=(replace(wl.pulses[0], coeffs=tuple(c)),) + tuple(wl.pulses[1:]))
        f = qds.Solver(w2)
        f.load_pulses()
        f.step(2000)
        vals.append(f.loss())
        f.close()
    fd = (vals[0] - vals[1]) / (2 * eps)
    assert abs(grad - fd) <= 1e-6 * abs(fd) + 1e-9 * L, (grad, fd)
