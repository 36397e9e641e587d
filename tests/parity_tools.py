"""Comparison helpers for GPU-vs-oracle parity tests (test infrastructure)."""
import torch

from oracle import qds as Q


def rel_err(a: torch.Tensor, b: torch.Tensor, floor: float) -> float:
    d = float((a - b).abs().pow(2).sum().sqrt())
    nb = float(b.abs().pow(2).sum().sqrt())
    return d / max(nb, floor)


def group_of(key: str) -> str:
    """Field set a state key belongs to: electromagnetic set 0 or 1, its plasma
    currents, or the axion."""
    if key in ("phi", "phig", "Tap", "Tam"):
        return "axion"
    s = key[-1]
    return ("j" if key.startswith("j") else "em") + s


def compare_states(gpu: dict, ora: dict, tol: float, floor_rel: float, skip=(), by_group=False):
    """Relative L2 per field and mode.  The denominator is the field's own norm
    for that mode, floored at floor_rel x the field's norm over all modes; with
    ``by_group`` it is the norm of the whole field set the key belongs to (used
    for single precision, whose rounding of the dominant fields sets the error
    of fields far smaller than them).  Returns the worst (error, key, mode)."""
    gnorm = {}
    for k in gpu:
        gg = group_of(k)
        gnorm[gg] = gnorm.get(gg, 0.0) + float(ora[k].abs().pow(2).sum())
    worst = (0.0, None, None)
    for k, a in gpu.items():
        if k in skip:
            continue
        b = ora[k]
        assert a.shape == b.shape, (k, a.shape, b.shape)
        fnorm = float(b.abs().pow(2).sum().sqrt())
        floor = max(floor_rel * fnorm, 1e-300)
        if by_group:
            floor = max(gnorm[group_of(k)] ** 0.5, 1e-300)
        for m in range(a.shape[0]):
            e = rel_err(a[m], b[m], floor)
            if e > worst[0]:
                worst = (e, k, m)
    assert worst[0] <= tol, f"worst relative L2 {worst[0]:.3e} in {worst[1]} mode {worst[2]} (tol {tol:g})"
    return worst


def oracle_run(wl, nsteps):
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    return Q.run(st, g, ph, nsteps)
