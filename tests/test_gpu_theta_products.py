"""The theta-grid products (QDS_PRODUCTS_THETA: the axion source and current
through a transform pair on 3M - 2 theta points, Sec. 3.3) against the
oracle, whose mode products are the direct convolution C_m (Eq.
mode_convolution), on random full states of 2..8 modes, and against the
direct convolution of the same staged kernels."""
import pytest
import torch

from paper_2609_03550_amd import inputs as I
import parity_tools as P

pytestmark = pytest.mark.gpu
H = I.H


def _wl(M, x_bc="open", r_bc="open"):
    p1 = I.Pulse("y", 0.5, 1.0, 3 * I.LAMBDA, 20 * H, 0.4 * 150 * H)
    p2 = I.Pulse("z", 0.5, 0.8, 3 * I.LAMBDA, 20 * H, 0.4 * 150 * H)
    # 8 modes need dr >= 7.2 dx for the radial stability bound
    return I.Workload("theta", 150, 13, M, 0, wp2=0.01, axion=True, arem=True, ma2=0.02, pulses=(p1, p2),
                      dr=8 * H, x_bc=x_bc, r_bc=r_bc)


def _random_state(wl, seed=3550):
    from oracle import qds as Q
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    gen = torch.Generator().manual_seed(seed)
    for k, v in st.items():
        if isinstance(v, torch.Tensor) and v.is_complex():
            st[k] = torch.randn(v.shape, dtype=torch.complex128, generator=gen)
    return Q.step(st, g, ph), g, ph


def _gpu(wl, st, dtype, products, nsteps):
    from paper_2609_03550_amd import qds
    s = qds.Solver(wl, dtype=dtype)
    s.set_option(qds.OPT_PRODUCTS, products)
    s.load_fields(st)
    assert s.fused == (products == qds.PRODUCTS_DIRECT)
    s.step(nsteps)
    torch.cuda.synchronize()
    return s.fields()


@pytest.mark.parametrize("dtype,M,x_bc,r_bc", [("f64", 6, "open", "open"), ("f64", 8, "open", "open"),
                                               ("f64", 8, "periodic", "pec"), ("f64", 3, "open", "open"),
                                               ("f64", 2, "periodic", "open"), ("f32", 8, "open", "open"),
                                               ("f32", 6, "open", "pec")])
def test_theta_products_match_the_oracle(dtype, M, x_bc, r_bc):
    from oracle import qds as Q
    from paper_2609_03550_amd import qds
    wl = _wl(M, x_bc, r_bc)
    st, g, ph = _random_state(wl)
    got = _gpu(wl, st, dtype, qds.PRODUCTS_THETA, 4)
    ref = Q.run(st, g, ph, 4)
    tol, floor = (1e-12, 1e-14) if dtype == "f64" else (1e-5, 1e-7)
    P.compare_states(got, ref, tol, floor, set_floor=P.SET_FLOOR, phys=True)


@pytest.mark.parametrize("M", [6, 8])
def test_theta_products_equal_the_direct_convolution(M):
    """Both product forms on the staged kernels, 6 steps, double precision:
    they differ only by rounding."""
    from paper_2609_03550_amd import qds
    wl = _wl(M)
    st, _, _ = _random_state(wl, seed=7)
    a = _gpu(wl, st, "f64", qds.PRODUCTS_THETA, 6)
    s = qds.Solver(wl, dtype="f64", path=qds.PATH_STAGED)
    s.load_fields(st)
    s.step(6)
    torch.cuda.synchronize()
    P.compare_states(a, s.fields(), 1e-13, 1e-14)
