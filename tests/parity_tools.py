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
    if key in ("phi", "phig", "Tap", "Tam", "dtphi", "dxphi"):
        return "axion"
    s = key[-1]
    return ("j" if key.startswith("j") else "em") + s


def physical(st: dict) -> dict:
    """The physical fields of a state (Eq. reconstruct_fields, Eq.
    T_axion_def): per set E_r, B_theta, E_theta, B_r from the transport
    variables, E_x, B_x, the exterior ghost B_theta and the plasma currents;
    phi, its exterior ghost, d_t phi = (T_a^+ + T_a^-)/2 and
    d_x phi = (T_a^- - T_a^+)/2."""
    out = {}
    for s in (0, 1):
        if f"Trp{s}" not in st:
            continue
        trp, trm, ttp, ttm = st[f"Trp{s}"], st[f"Trm{s}"], st[f"Ttp{s}"], st[f"Ttm{s}"]
        out[f"Er{s}"], out[f"Bt{s}"] = 0.5 * (trp + trm), 0.5 * (trp - trm)
        out[f"Et{s}"], out[f"Br{s}"] = 0.5 * (ttp + ttm), 0.5 * (ttp - ttm)
        for k in ("Ex", "Bx", "Bg", "jx", "jr", "jt"):
            if f"{k}{s}" in st:
                out[f"{k}{s}"] = st[f"{k}{s}"]
    if "phi" in st:
        out["phi"], out["phig"] = st["phi"], st["phig"]
        out["dtphi"], out["dxphi"] = 0.5 * (st["Tap"] + st["Tam"]), 0.5 * (st["Tam"] - st["Tap"])
    return out


def compare_states(gpu: dict, ora: dict, tol: float, floor_rel: float, skip=(), by_group=False, set_floor=0.0,
                   phys=False):
    """Relative L2 per field and mode.  The denominator is the field's own norm
    for that mode, floored at floor_rel x the field's norm over all modes and
    at set_floor x the norm of the whole field set the key belongs to (a field
    far smaller than its set -- the tail of a pulse, a ghost row far outside
    the beam -- carries the rounding of the set's dominant values, not of its
    own); with ``by_group`` the denominator is the field set's norm.  With
    ``phys`` both states are first turned into their physical fields
    (``physical``).  Returns the worst (error, key, mode)."""
    if phys:
        gpu, ora = physical(gpu), physical({k: ora[k] for k in gpu})
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
        gn = gnorm[group_of(k)] ** 0.5
        for m in range(a.shape[0]):
            floor = max(floor_rel * fnorm, set_floor * gn, 1e-300)
            if by_group:
                floor = max(gn, 1e-300)
            e = rel_err(a[m], b[m], floor)
            if e > worst[0]:
                worst = (e, k, m)
    assert worst[0] <= tol, f"worst relative L2 {worst[0]:.3e} in {worst[1]} mode {worst[2]} (tol {tol:g})"
    return worst


SET_FLOOR = 1e-3    # per-field comparisons: fields below this fraction of their set use it
BAND = 4.0          # allowed multiple of the storage-rounding deviation
U64 = 2.0 ** -53    # unit roundoff of double precision


def storage_rounded(st: dict, dtype: str, gen: torch.Generator) -> dict:
    """A state as storage in ``dtype`` leaves it.  f32: every value rounded to
    single precision.  f64, where rounding a double to a double changes
    nothing: every real and imaginary part times 1 + d, d uniform in
    [-2^-53, 2^-53] (the relative error bound of rounding to double), drawn
    from ``gen``."""
    out = {}
    for k, v in st.items():
        if isinstance(v, torch.Tensor) and (v.is_complex() or v.is_floating_point()):
            if dtype == "f32":
                v = v.to(torch.complex64 if v.is_complex() else torch.float32).to(v.dtype)
            elif v.is_complex():
                d = (2 * torch.rand((2,) + tuple(v.shape), generator=gen, dtype=torch.float64) - 1) * U64
                v = torch.complex(v.real * (1 + d[0]), v.imag * (1 + d[1]))
            else:
                v = v * (1 + (2 * torch.rand(v.shape, generator=gen, dtype=torch.float64) - 1) * U64)
        out[k] = v
    return out


def run_rounded(st: dict, g, ph, nsteps: int, dtype: str, seed: int = 0) -> dict:
    """The oracle's run with its state passed through ``storage_rounded``
    before the first step and after every step; the arithmetic stays FP64.
    Its deviation from the plain run is what storage in ``dtype`` alone does
    to each field over these steps (large where a field follows from nearly
    cancelling products)."""
    gen = torch.Generator().manual_seed(seed)
    st = storage_rounded(st, dtype, gen)
    for _ in range(nsteps):
        st = storage_rounded(Q.step(st, g, ph), dtype, gen)
    return st


def oracle_run_rounded(wl, nsteps: int, dtype: str, seed: int = 0) -> dict:
    g, ph = Q.grid_physics(wl)
    return run_rounded(Q.init_state(wl), g, ph, nsteps, dtype, seed)


def compare_band(gpu: dict, ora: dict, emu: dict, tol: float, set_floor: float = SET_FLOOR,
                 factor: float = BAND):
    """Per physical field and mode, the denominator being the field's own norm
    for that mode floored at ``set_floor`` x its field set's norm: the GPU's
    deviation from the oracle ``ora`` is within ``tol`` or within ``factor`` x
    the deviation of the storage-rounded oracle run ``emu``, whichever is
    larger.  Returns the worst (deviation / allowed, key, mode, deviation,
    storage-rounding deviation)."""
    a = physical(gpu)
    b = physical({k: ora[k] for k in gpu})
    e = physical({k: emu[k] for k in gpu})
    gnorm = {}
    for k in b:
        gnorm[group_of(k)] = gnorm.get(group_of(k), 0.0) + float(b[k].abs().pow(2).sum())
    worst = (0.0, "", -1, 0.0, 0.0)
    for k in a:
        assert a[k].shape == b[k].shape, (k, a[k].shape, b[k].shape)
        for m in range(a[k].shape[0]):
            fl = max(float(b[k][m].abs().pow(2).sum().sqrt()), set_floor * gnorm[group_of(k)] ** 0.5, 1e-300)
            eg = rel_err(a[k][m], b[k][m], fl)
            ee = rel_err(e[k][m], b[k][m], fl)
            allowed = max(tol, factor * ee)
            if eg / allowed > worst[0]:
                worst = (eg / allowed, k, m, eg, ee)
    assert worst[0] <= 1.0, (f"{worst[1]} mode {worst[2]}: relative L2 {worst[3]:.3e} above max({tol:g}, "
                             f"{factor:g} x storage rounding {worst[4]:.3e})")
    return worst


def oracle_run(wl, nsteps):
    g, ph = Q.grid_physics(wl)
    st = Q.init_state(wl)
    return Q.run(st, g, ph, nsteps)
