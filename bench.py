#!/usr/bin/env python3
"""Benchmark of the QDS + Klein-Gordon field advance on one MI355X.

One step = one full pass of the hot path (background set with cold-plasma
response, Klein-Gordon axion with its source, axion current, regenerated set)
over the 8192 x 256 x 3-mode two-colour axion workload, FP64 complex, inputs
resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--dtype f64|f32] [--workload axion|window|vacuum]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-mode updates/s + % HBM peak (QDS+KG); fwd+adjoint vs fwd time"
HBM_PEAK_GBPS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")


def plane_accesses(wl, kernel, split=True):
    """Complex planes read + written per cell-mode by one launch of each fused
    kernel (their algorithmic bytes).  With the regenerated set the axion
    advance runs in the axion-current kernel:
      kernel 0 (A): reads and writes the background set (T_r^+-, T_theta^+-,
        E_x, B_x and, with plasma, j_x, j_r, j_theta), writes S_a;
      kernel 1 (B): reads and writes the regenerated set, reads the axion current;
      kernel 2 (axion current): reads T^n and T^{n+1} of the background set
        (4 + 4), B_x at t^{n-1/2} and t^{n+1/2}, E_x at t^{n+1/2}, T_a^{n-1/2}
        (2), phi^n and S_a; writes T_a^{n+1/2} (2), phi^{n+1} and j_a (3).
    Without it kernel A also reads and writes the axion (phi, T_a^+-).
    With ``split`` false (the option kernel AX) one launch does the work of
    kernel A and the axion kernel: it reads and writes the background set and
    the axion once and writes j_a (27 planes), and kernel 2 does not run.
    Electromagnetic-only: kernel 0 reads and writes the 6 (or 9) planes, and
    with a prescribed drive reads its j_x^(0) plane for mode 0 (1/M of a plane
    per cell-mode; the drive kernel that writes it is not counted).
    Kernel 3 is the two-step march, per launch (two steps): the regenerated
    set (or the set of an electromagnetic-only run) read and written once and,
    with the regenerated set, the axion current of both steps read."""
    em = 6 + (3 if wl.wp2 else 0)
    if kernel == 3:
        # the two-step march (one launch per two steps): the set read and
        # written once, the axion current (or the drive's mode-0 plane) of
        # both steps read
        return 2 * em + (6 if wl.arem else 0) + (2.0 / wl.nmodes if wl.drive is not None else 0.0)
    if not wl.axion:
        if kernel != 0:
            return 0
        return 2 * em + (1.0 / wl.nmodes if wl.drive is not None else 0.0)
    drv = 1.0 / wl.nmodes if wl.drive is not None else 0.0
    if wl.arem and not split:
        return {0: 2 * (em + 3) + 3 + drv, 1: 2 * em + 3, 2: 0}[kernel]
    if kernel == 0:
        return (2 * em + 1 if wl.arem else 2 * (em + 3)) + drv
    if kernel == 1:
        return (2 * em + 3) if wl.arem else 0
    return 21 if wl.arem else 0


KERNEL_NAMES = {0: "kernel A (background set, axion source)", 1: "kernel B (regenerated set)",
                2: "axion kernel (axion advance, axion current)"}
KERNEL_NAME_AX = "kernel AX (background set, axion source, axion advance, axion current)"
KERNEL_NAME_PAIR = {True: "two-step march of the regenerated set (two steps per launch)",
                    False: "two-step march of the electromagnetic set (two steps per launch)"}
# untimed steps of the library's autotuner: 8 trials, each a pair of steps
# where steps run in pairs
TUNE_STEPS = 16
# untimed steps before the autotuner's trials of the headline solver
TUNE_WARM = 20


def pairs_active(wl, fused, pair=1, kernel_ax=0, overlap=0):
    """Whether qds_step runs this workload in pairs of steps (QDS_OPT_PAIR):
    on the fused kernels, with the regenerated set on the split kernels (no
    moving window, no drive), or without the axion (with or without both)."""
    if not (pair and fused) or overlap:
        return False
    if wl.axion:
        return bool(wl.arem) and not kernel_ax and wl.x_bc != "window" and wl.drive is None
    return True


def workload(name):
    from paper_2609_03550_amd import inputs as I
    if name == "axion":
        return I.axion_two_colour(8192, 256, 6000, 3)
    if name == "window":
        return I.driven_window(4096, 256, 4000)
    if name == "vacuum":
        return I.vacuum_em()
    raise SystemExit(f"unknown workload {name}")


KERNEL_KEYS = {0: "kernel_a", 1: "kernel_b", 2: "axion_current", 3: "kernel_b2"}


def _code_only(text):
    """Source text without comments and with whitespace collapsed."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_digest():
    """Digest of the code (comments aside) of the kernel sources the HBM counters depend on."""
    h = hashlib.sha256()
    for f in ("qds_fused.hip", "qds_current.hip", "qds_current_rows.hpp", "qds_stages.hip", "qds_stage_ops.hpp",
              "qds_kernels.hpp", "qds_common.hpp"):
        with open(os.path.join(ROOT, "paper_2609_03550_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(wl, dtype, kernel, tiles):
    """HBM bytes per launch of one fused kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), if it
    was taken on the current kernel sources for this workload and dtype at the
    same tile height (the halo rows a tile re-reads depend on it)."""
    path = os.path.join(PROFILE_DIR, f"traffic_{wl.name}_{dtype}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_digest") != source_digest() or d.get("workload") != wl.name or d.get("dtype") != dtype:
        return None
    key = KERNEL_KEYS[kernel]
    return d.get("kernels", {}).get(key, {}).get("by_tile", {}).get(str(tiles.get(key)), {}).get("hbm_bytes_per_launch")


def adjoint_ratio(dtype, steps, ckpt):
    """Forward + adjoint against forward alone on the 4096 x 128 x 2-mode axion
    workload: wall time of qds_backward over ``steps`` steps (its checkpointed
    forward sweep, the recomputation of each segment and the adjoint steps, the
    loss being the regenerated mode-1 energy over the last 256 columns) divided
    by the time of ``steps`` plain forward steps from the same initial state."""
    import torch
    from paper_2609_03550_amd import inputs as I
    from paper_2609_03550_amd import qds
    wl = I.adjoint_workload(steps=steps)
    s = qds.Solver(wl, dtype=dtype)
    s.load_pulses()
    f = qds.Solver(wl, dtype=dtype)
    f.load_pulses()
    f.set_option(qds.OPT_TUNE, 1)
    f.step(TUNE_STEPS + 2)          # the forward's autotuner, then warm
    s.set_option(qds.OPT_TUNE, 1)
    # the caller-owned checkpoint pool and lambda buffer are allocated once,
    # as a caller repeating the gradient would keep them
    pool = torch.empty(s.backward_pool_bytes(steps, ckpt), dtype=torch.uint8, device=s.device)
    lam = torch.empty(s.nbytes, dtype=torch.uint8, device=s.device)
    s.backward(40, 20, pool=pool, out=lam)    # tunes on its checkpoint pass; warms the adjoint
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    L, lam, _ = s.backward(steps, ckpt, pool=pool, out=lam)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    return {"workload": wl.name, "steps": steps, "ckpt_every": ckpt, "dtype": dtype, "fwd_s": t_fwd,
            "fwd_adj_s": t_adj, "ratio": t_adj / t_fwd, "loss": L}


def batched_leg(step_scale, graph_steps, count=64):
    """The 64 uneven single-precision instances, each for its own seeded step
    count (500..3000) times ``step_scale``, so that instances finish at
    different steps and the set of running instances changes along the run:
    the batch (one launch per kernel class per step over every running
    instance, tiles from the batch's autotuner) with the whole uneven schedule
    captured as one HIP graph and launched once (``graph_steps`` -1; otherwise
    that many steps per graph), against the same schedule launched without
    graphs and against each instance advanced alone with qds_step (each with
    the tiles its own autotuner chose): in pairs of steps (the library's
    default), and one step at a time (the kernels the batch launches).  The
    graph is captured on an untimed first pass of the schedule and replayed
    on the timed one."""
    import torch
    from paper_2609_03550_amd import inputs as I
    from paper_2609_03550_amd import qds
    wls = I.batched_instances(count, 4)
    steps = [max(1, int(round(wl.steps * step_scale))) for wl in wls]
    bs = []
    for wl in wls:
        s = qds.Solver(wl, dtype="f32")
        s.load_pulses()
        bs.append(s)
    updates = sum(wl.cell_modes * n for wl, n in zip(wls, steps))
    b = qds.Batch(bs)
    b.run(TUNE_STEPS, graph_steps=graph_steps, tune=True)   # the autotuner's trial steps (pairs)
    b.run(steps, graph_steps=graph_steps)              # capture pass
    torch.cuda.synchronize()
    s0 = b.stats()
    t0 = time.perf_counter()
    b.run(steps, graph_steps=graph_steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    s1 = b.stats()
    t0 = time.perf_counter()
    b.run(steps, graph_steps=0)
    torch.cuda.synchronize()
    t_direct = time.perf_counter() - t0
    s2 = b.stats()
    for s in bs:
        s.set_option(qds.OPT_TUNE, 1)      # each instance's own autotuner, untimed
        s.step(TUNE_STEPS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, n in zip(bs, steps):
        s.step(n)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    # one at a time and one step at a time: the kernels the batch launches
    for s in bs:
        s.set_option(qds.OPT_PAIR, 0)
        s.set_option(qds.OPT_TUNE, 1)
        s.step(TUNE_STEPS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, n in zip(bs, steps):
        s.step(n)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    tiles, tuned = b.tiles()
    b.close()
    for s in bs:
        s.close()
    kernel_launches_direct = s2[2] - s1[2]
    return {"instances": count, "dtype": "f32", "steps_per_instance": {"min": min(steps), "max": max(steps),
                                                                        "scale": step_scale},
            "cell_mode_updates": updates, "graph_steps": graph_steps, "tiles": tiles, "tuned": tuned,
            "graph_launches_per_run": s1[0] - s0[0], "kernel_launches_per_run": kernel_launches_direct,
            "batched_updates_per_s": updates / t_batch, "batched_no_graph_updates_per_s": updates / t_direct,
            "one_at_a_time_updates_per_s": updates / t_solo, "speedup": t_solo / t_batch,
            "one_at_a_time_single_steps_updates_per_s": updates / t_single,
            "speedup_vs_single_steps": t_single / t_batch,
            "graph_gain_s": t_direct - t_batch,
            "launch_overhead_us_per_kernel": (t_direct - t_batch) / max(kernel_launches_direct, 1) * 1e6}


def window_leg(steps):
    """The moving-window workload with the prescribed ring drive (4096 x 256 x
    3 modes, electromagnetic only, steps in pairs) in FP64 and FP32: autotuned
    tiles, 10 warm-up steps, ``steps`` timed; the whole step against its
    one-read-one-write byte model (the 9 planes of the set with the plasma)."""
    import torch
    from paper_2609_03550_amd import qds
    wl = workload("window")
    out = {"workload": wl.name, "steps": steps}
    for dt in ("f64", "f32"):
        s = qds.Solver(wl, dtype=dt)
        s.load_pulses()
        s.set_option(qds.OPT_TUNE, 1)
        s.step(TUNE_STEPS)
        s.step(10)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        eb = 16 if dt == "f64" else 8
        nplanes = 9 if wl.wp2 else 6
        out[dt] = {"ms_per_step": ms, "value": wl.cell_modes / (ms / 1e3),
                   "roofline_frac": 2 * nplanes * eb * wl.cell_modes / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS,
                   "pairs_of_steps": pairs_active(wl, s.fused), "tiles": s.tiles()[0]}
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def f32_leg(wl, steps):
    """The same workload in single precision: autotuned tiles, 10 warm-up
    steps, then ``steps`` timed steps; the whole step against its
    one-read-one-write byte model (336 B per cell-mode with every plane)."""
    import torch
    from paper_2609_03550_amd import qds
    s = qds.Solver(wl, dtype="f32")
    s.load_pulses()
    s.set_option(qds.OPT_TUNE, 1)
    s.step(TUNE_STEPS)
    s.step(10)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nplanes = (21 if wl.arem else 12) if wl.axion else (9 if wl.wp2 else 6)
    step_bytes = 2 * nplanes * 8 * wl.cell_modes
    tiles = s.tiles()
    s.close()
    return {"dtype": "f32", "steps": steps, "ms_per_step": ms, "value": wl.cell_modes / (ms / 1e3),
            "unit": "cell-mode updates/s", "roofline_frac": step_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS,
            "tiles": tiles[0]}


def kernel_variants_leg(wl, dtype, steps):
    """The main workload on its launch arrangements: the split kernels in
    pairs of steps (kernel A, the marched axion kernel, twice, then the
    two-step march of the regenerated set; the default), the split kernels
    one step at a time (kernel A, the marched axion kernel, kernel B), the
    same with kernel A of step k+1 on a second stream beside kernel B of
    step k (QDS_OPT_OVERLAP), and the one-pass kernel AX then kernel B
    (QDS_OPT_KERNEL_AX).
    Each solver picks its tiles with its own autotuner on TUNE_STEPS untimed steps,
    then runs 10 untimed and ``steps`` timed steps; the four run twice in
    rotating order and the faster run of each is kept."""
    import torch
    from paper_2609_03550_amd import qds
    names = ("split_pairs", "split", "split_overlap", "ax")
    res = {n: [] for n in names}
    tiles = {}
    for rep in range(2):
        for name in (names if rep == 0 else names[::-1]):
            s = qds.Solver(wl, dtype=dtype)
            s.load_pulses()
            s.set_option(qds.OPT_KERNEL_AX, 1 if name == "ax" else 0)
            s.set_option(qds.OPT_OVERLAP, 1 if name == "split_overlap" else 0)
            s.set_option(qds.OPT_PAIR, 1 if name == "split_pairs" else 0)
            s.set_option(qds.OPT_TUNE, 1)
            s.step(TUNE_STEPS)
            s.step(10)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step(steps)
            e1.record()
            torch.cuda.synchronize()
            res[name].append(e0.elapsed_time(e1) / steps)
            tiles[name] = s.tiles()[0]
            s.close()
    out = {"steps": steps}
    for n in names:
        out[n + "_ms_per_step"] = min(res[n])
        out[n + "_tiles"] = tiles[n]
    out["ax_over_split"] = out["ax_ms_per_step"] / out["split_ms_per_step"]
    out["overlap_over_split"] = out["split_overlap_ms_per_step"] / out["split_ms_per_step"]
    out["pairs_over_split"] = out["split_pairs_ms_per_step"] / out["split_ms_per_step"]
    return out


def theta_leg(steps=20):
    """Axion source and current by the theta-grid transform pair against the
    direct mode convolution on the staged kernels (one thread per point and
    every mode), and the direct convolution on the fused kernels (one
    wavefront per mode, autotuned tiles): 6 and 8 modes of the full physics on
    a 2048 x 64 grid with dr = 8 dx (what the radial stability bound allows
    for 8 modes), FP64, ``steps`` timed steps after 3 untimed (and the
    autotuner's TUNE_STEPS on the fused kernels)."""
    import torch
    from paper_2609_03550_amd import inputs as I
    from paper_2609_03550_amd import qds
    out = {}
    for M in (6, 8):
        p1 = I.Pulse("y", 0.5, 1.0, 12 * I.LAMBDA, 299.8 * I.H, 1100 * I.H)
        p2 = I.Pulse("z", 0.5, 0.8, 12 * I.LAMBDA, 299.8 * I.H, 1100 * I.H)
        wl = I.Workload(f"theta_2048x64x{M}", 2048, 64, M, 0, wp2=5.7407e-5, axion=True, arem=True, ma2=2.325e-4,
                        pulses=(p1, p2), dr=8 * I.H)
        res = {}
        for name, prod, path in (("direct", qds.PRODUCTS_DIRECT, qds.PATH_STAGED),
                                 ("theta", qds.PRODUCTS_THETA, qds.PATH_STAGED),
                                 ("fused_direct", qds.PRODUCTS_DIRECT, qds.PATH_FUSED)):
            s = qds.Solver(wl, dtype="f64", path=path)
            s.set_option(qds.OPT_PRODUCTS, prod)
            s.load_pulses()
            if path == qds.PATH_FUSED:
                s.set_option(qds.OPT_TUNE, 1)
                s.step(TUNE_STEPS)
            s.step(3)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step(steps)
            e1.record()
            torch.cuda.synchronize()
            res[name + "_ms_per_step"] = e0.elapsed_time(e1) / steps
            s.close()
        res["theta_over_direct"] = res["theta_ms_per_step"] / res["direct_ms_per_step"]
        res["fused_direct_over_direct"] = res["fused_direct_ms_per_step"] / res["direct_ms_per_step"]
        out[f"modes_{M}"] = res
    return out


def pic_leg(steps, ppc=2, dtype="f64", sort=True):
    """The coupled PIC loop (Sec. 3.1) in place of the prescribed ring drive:
    the laser of the moving-window workload (4096 x 256 x 3 modes, a0 = 2,
    w0 = 10 lambda, 30 fs) in a cold electron slab of n_e = 1e17 cm^-3 over
    the middle half of the grid and r < 240 dr, ``ppc`` macro-electrons per
    (x, r) cell placed at seeded random positions (uniform in x, in r^2 and in
    theta), on a fixed grid (particles take no moving window).  Each step is
    qds_particles_step (gather, Boris, modal charge-conserving deposit) then
    qds_step with the deposit (fused kernels).  ``steps`` timed coupled steps
    after 8 untimed field steps (the autotuner's trials of the field step's
    tile height) and 3 untimed coupled steps, then the same number of
    particle steps alone."""
    import numpy as np
    import torch
    from paper_2609_03550_amd import inputs as I
    from paper_2609_03550_amd import qds
    base = I.driven_window(4096, 256, 4000)
    wl = base.with_(name="pic_4096x256x3", x_bc="open", drive=None)
    s = qds.Solver(wl, dtype=dtype)
    s.load_pulses()
    rng = np.random.default_rng(17)
    nx, nr = wl.nx, wl.nr
    x_lo, x_hi, r_max = 0.25 * nx * wl.h, 0.75 * nx * wl.h, 240 * wl.dr
    n = int(ppc * (0.5 * nx) * 240)
    x = rng.uniform(x_lo, x_hi, n)
    r = r_max * np.sqrt(rng.uniform(0, 1, n))
    th = rng.uniform(-np.pi, np.pi, n)
    pos = torch.from_numpy(np.stack([x, r * np.cos(th), r * np.sin(th)])).to(s.device).contiguous()
    if sort:
        # by cell, as PIC codes keep their particles: tiles of 8 rows x 16
        # columns (a workgroup's 256 particles at two per cell), x fastest
        # within a tile (the planes' contiguous direction).  A wave's 64
        # particles then sit on 16 consecutive columns of two rows, so each
        # of its gather loads touches a few cache lines (sorted with r fastest,
        # one line per row), and a workgroup's deposit box is 19 x 11 cells
        # (in rows of 128 cells, 131 x 5: about twice the tile values to add)
        tr, tc = 8, 16
        ix = torch.floor(pos[0] / wl.h)
        ir = torch.floor(torch.sqrt(pos[1] ** 2 + pos[2] ** 2) / wl.dr)
        tile = torch.div(ir, tr, rounding_mode="floor") * ((nx + tc - 1) // tc) + torch.div(ix, tc, rounding_mode="floor")
        key = tile * (tr * tc) + torch.remainder(ir, tr) * tc + torch.remainder(ix, tc)
        pos = pos[:, torch.argsort(key)].contiguous()
    u = torch.zeros_like(pos)
    # the coupled loop advances the fields one step per call, with the
    # background set's one-step march: its tile height from the autotuner's
    # 8 single field steps (untimed, before the particles are loaded)
    s.set_option(qds.OPT_PAIR, 0)
    s.set_option(qds.OPT_TUNE, 1)
    s.step(8)
    s.set_option(qds.OPT_PAIR, 1)
    ne = 1e17 / I.NC_CM3                       # density in units of the critical density
    charge = -ne * (x_hi - x_lo) * np.pi * r_max ** 2 / n
    cpl = None
    cpl, _ = s.pic_steps(pos, u, -1.0, charge, 3, cpl)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    cpl, sk = s.pic_steps(pos, u, -1.0, charge, steps, cpl)
    e1.record()
    torch.cuda.synchronize()
    t_all = e0.elapsed_time(e1) / steps
    skipped = sum(int(k.item()) for k in sk)
    planes = s.current_planes()
    e0.record()
    for _ in range(steps):
        s.particles_step(pos, u, -1.0, charge, planes=planes, extrapolate=True, clear=True)
    e1.record()
    torch.cuda.synchronize()
    t_part = e0.elapsed_time(e1) / steps
    fused = s.fused
    s_tiles = s.tiles()[0][0]
    s.close()
    return {"workload": wl.name, "dtype": dtype, "particles": n, "sorted_by_cell": sort, "steps": steps,
            "path": "fused" if fused else "staged",
            "coupled_ms_per_step": t_all, "particle_ms_per_step": t_part, "field_ms_per_step": t_all - t_part,
            "particle_pushes_per_s": n / (t_part / 1e3), "field_cell_mode_updates_per_s": wl.cell_modes / ((t_all - t_part) / 1e3),
            "skipped_particles": skipped, "field_tile_rows": s_tiles}


def stream_reference(nbytes=1 << 31, reps=10):
    """Bandwidth of plain device copies (read + write) and a fill (write only)
    in the same process: torch's copy and fill, and the library's 16-byte-per-
    lane copy (qds_stream_copy) with and without the streaming hint over 65536
    workgroups -- the practical ceiling next to the 8 TB/s peak for kernels
    that both read and write their planes."""
    import torch
    from paper_2609_03550_amd import qds
    dev = torch.device("cuda:0")
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)

    def timed(f):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    stream = torch.cuda.current_stream().cuda_stream
    lib = qds.lib()

    def lib_copy(streaming):
        st = lib.qds_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, streaming, 65536, stream)
        if st != 0:
            raise RuntimeError(f"qds_stream_copy failed ({st})")

    t_copy = timed(lambda: b.copy_(a))
    t_fill = timed(lambda: b.fill_(3))
    t_lib = timed(lambda: lib_copy(0))
    t_nt = timed(lambda: lib_copy(1))
    del a, b
    torch.cuda.empty_cache()
    return {"copy_read_write_gbps": 2 * nbytes / t_copy / 1e9, "fill_write_gbps": nbytes / t_fill / 1e9,
            "lib_copy_read_write_gbps": 2 * nbytes / t_lib / 1e9,
            "lib_streaming_copy_read_write_gbps": 2 * nbytes / t_nt / 1e9, "bytes": nbytes}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, seconds_target=10.0, one_thread_seconds=6.0):
    """The FP64 oracle on this host, as it stands: whole-grid steps of the same
    workload with torch's default intra-op threads until about
    ``seconds_target`` of work (the reported value), then steps of a
    1024-column x-crop of it on one thread (the one-core rate, per update, and
    the linear-scaling ceiling it implies over the cores this process may use)."""
    import torch
    from oracle import qds as Q

    def rate(w, target, max_steps):
        g, ph = Q.grid_physics(w)
        st = Q.init_state(w)
        st = Q.step(st, g, ph)                  # first step outside the timing
        n, t0 = 0, time.perf_counter()
        while True:
            st = Q.step(st, g, ph)
            n += 1
            el = time.perf_counter() - t0
            if el > target or n >= max_steps:
                return w.cell_modes * n / el, n, el

    threads = torch.get_num_threads()
    v, n, el = rate(wl, seconds_target, 20)
    crop = wl.with_(nx=min(wl.nx, 1024))
    torch.set_num_threads(1)
    try:
        v1, n1, el1 = rate(crop, one_thread_seconds, 20)
    finally:
        torch.set_num_threads(threads)
    cores = len(os.sched_getaffinity(0))
    return {"value": v, "unit": "cell-mode updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} whole-grid steps of {wl.name} (FP64 oracle, {threads} intra-op threads, after 1 "
                      f"untimed step), {el:.1f} s; one thread: {n1} steps of a {crop.nx}-column x-crop, {el1:.1f} s",
            "cpu_model": _cpu_model(), "affinity_cores": cores, "one_thread_value": v1,
            "linear_scaling_ceiling": v1 * cores}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--workload", default="axion", choices=["axion", "window", "vacuum"])
    ap.add_argument("--path", type=int, default=0, help="0 auto (fused), 1 staged, 2 fused")
    ap.add_argument("--rows", type=int, default=None)
    ap.add_argument("--tiles", default=None,
                    help="tile heights of kernel A, the axion current, kernel B and the two-step march "
                         "(a,c,b[,p]) instead of the autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="steps of the forward + adjoint timing (0 skips it)")
    ap.add_argument("--ckpt-every", type=int, default=45)
    ap.add_argument("--batched-scale", type=float, default=0.04,
                    help="factor on the 64 instances' seeded step counts (500..3000) for the batched "
                         "comparison (0 skips it)")
    ap.add_argument("--graph-steps", type=int, default=-1,
                    help="steps per HIP graph of the batched leg (-1: the whole uneven schedule as one graph)")
    ap.add_argument("--theta-steps", type=int, default=20,
                    help="steps of the theta-grid vs direct product comparison at 6 and 8 modes (0 skips it)")
    ap.add_argument("--window-steps", type=int, default=100,
                    help="steps of the moving-window workload with the drive, FP64 and FP32 (0 skips it)")
    ap.add_argument("--f32-steps", type=int, default=100,
                    help="steps of the single-precision figure of the same workload (0 skips it)")
    ap.add_argument("--kernel-ax", type=int, default=0,
                    help="1 runs the one-pass kernel AX instead of kernel A and the marched axion kernel "
                         "(QDS_OPT_KERNEL_AX)")
    ap.add_argument("--pair", type=int, default=1,
                    help="1 (default) runs steps in pairs with the two-step march of one set where it applies "
                         "(QDS_OPT_PAIR); 0 one step at a time")
    ap.add_argument("--overlap", type=int, default=0,
                    help="1 runs kernel A of the next step beside the regenerated set (QDS_OPT_OVERLAP)")
    ap.add_argument("--variant-steps", type=int, default=100,
                    help="steps of the comparison of kernel AX with the split kernels, with and without "
                         "the overlap (0 skips it)")
    ap.add_argument("--pic-steps", type=int, default=10,
                    help="steps of the coupled particle-in-cell leg (0 skips it)")
    ap.add_argument("--stream-reference", type=int, default=1,
                    help="1 times plain device copies for the copy-relative roofline fractions (0 skips them)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for the HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the x-slab sharding is a "
              "design, not code); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_03550_amd import qds

    wl = workload(args.workload)
    dev = torch.device("cuda:0")
    s = qds.Solver(wl, dtype=args.dtype, device="cuda:0", path=args.path, rows=args.rows)
    s.load_pulses()
    s.set_option(qds.OPT_KERNEL_AX, args.kernel_ax)
    s.set_option(qds.OPT_OVERLAP, args.overlap)
    s.set_option(qds.OPT_PAIR, args.pair)
    paired = pairs_active(wl, s.fused, args.pair, args.kernel_ax, args.overlap)
    if args.tiles:
        for opt, v in zip((qds.OPT_ROWS_A, qds.OPT_ROWS_CUR, qds.OPT_ROWS_B, qds.OPT_ROWS_PAIR),
                          args.tiles.split(",")):
            s.set_option(opt, int(v))
    elif args.rows is None:
        # tile heights chosen by the library's autotuner on TUNE_STEPS untimed steps of
        # the run, before the warm-up steps; its trials follow TUNE_WARM untimed steps
        # at the default heights, so that they are not timed on a GPU still idle
        s.step(TUNE_WARM)
        s.set_option(qds.OPT_TUNE, 1)
        s.step(TUNE_STEPS)
        torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    s.step(args.warmup)
    torch.cuda.synchronize()

    # the timed region: K steps with nothing between the launches but the
    # launches themselves (events only at its two ends)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    # per-kernel breakdown: a second pass of K steps with a HIP event pair
    # around every launch (the events add a few per cent to each kernel, so
    # this pass is not the headline)
    s.set_option(qds.OPT_TIMING, 1)
    torch.cuda.synchronize()
    e0.record(stream)
    s.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    breakdown_ms = e0.elapsed_time(e1) / args.steps
    kms, kn = s.timing()
    s.set_option(qds.OPT_TIMING, 0)

    ms_per_step = total_ms / args.steps
    cells = wl.cell_modes
    value = cells * args.steps / (total_ms / 1e3)
    eb = 16 if args.dtype == "f64" else 8
    run_tiles = dict(zip(("kernel_a", "axion_current", "kernel_b", "kernel_b2"), s.tiles()[0]))
    kernels = {}
    for q in range(3):
        if not kn[q]:
            continue
        avg = kms[q] / kn[q]
        # the timing slot of a set's two-step march is that of the set
        kind = 3 if paired and q == (1 if wl.arem else 0) else q
        name = KERNEL_NAMES[q] if (s.fused and wl.axion) else ("electromagnetic set" if s.fused else
                                                                 "staged step (all stage kernels)")
        if s.fused and wl.arem and args.kernel_ax and q == 0:
            name = KERNEL_NAME_AX
        if kind == 3:
            name = KERNEL_NAME_PAIR[bool(wl.arem)]
        alg = (plane_accesses(wl, kind, not args.kernel_ax) if s.fused
               else sum(plane_accesses(wl, k, True) for k in range(3))) * eb * cells
        kernels[KERNEL_KEYS[kind]] = {"name": name, "avg_launch_ms": avg, "launches": kn[q],
                                      "steps_per_launch": 2 if kind == 3 else 1,
                                      "plane_passes": alg / eb / cells, "algorithmic_bytes_per_launch": alg,
                                      "achieved_gbps": alg / (avg / 1e3) / 1e9,
                                      "hbm_bytes_per_launch": measured_traffic(wl, args.dtype, kind, run_tiles)
                                      if s.fused else None}
    # the whole step against the one-read-one-write byte model: every state
    # plane read once and written once per step
    nplanes = (21 if wl.arem else 12) if wl.axion else (9 if wl.wp2 else 6)
    step_bytes = 2 * nplanes * eb * cells
    kernel_sum_ms = sum(k["avg_launch_ms"] * k["launches"] for k in kernels.values()) / args.steps
    achieved = step_bytes / (ms_per_step / 1e3) / 1e9
    traffic = None
    if s.fused and all(k["hbm_bytes_per_launch"] is not None for k in kernels.values()):
        traffic = sum(k["hbm_bytes_per_launch"] * k["launches"] for k in kernels.values()) / args.steps
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-mode updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "nr": wl.nr, "modes": wl.nmodes,
                   "physics": "QDS Maxwell + Klein-Gordon axion + regenerated fields + cold plasma"
                   if wl.arem else ("QDS Maxwell + prescribed current, moving window" if wl.drive else "QDS Maxwell"),
                   "path": "fused" if s.fused else "staged", "overlap": bool(args.overlap),
                   "kernels": ("AX, B" if args.kernel_ax else ("A, axion, A, axion, two-step B" if paired
                                                               else "A, axion, B"))
                   if (s.fused and wl.arem) else None,
                   "pairs_of_steps": paired,
                   "parallelism": "single GPU"},
        # the dominant unit is the whole step (its kernels run back to back):
        # algorithmic bytes = every state plane read once and written once
        "roofline": {"bound": "hbm", "kernel": "whole step (" + " + ".join(k["name"] for k in kernels.values()) + ")",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic, "traffic_over_model": traffic / step_bytes if traffic else None,
                     # the measured fraction: HBM bytes (rocprofv3 counters) per step / step time / 8 TB/s
                     "measured_frac": traffic / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBPS if traffic else None,
                     "bytes_per_step": step_bytes, "bytes_per_cell_mode": 2 * nplanes * eb,
                     "step_ms": ms_per_step, "kernel_sum_ms": kernel_sum_ms,
                     "breakdown_pass_step_ms": breakdown_ms},
        "kernels": kernels,
        "fwd_adj_over_fwd": None,
        "tiles": dict(run_tiles, tuned=s.tiles()[1]),
    }
    s_fused = s.fused
    del s
    torch.cuda.empty_cache()
    if args.adjoint_steps > 0:
        adj = adjoint_ratio(args.dtype, args.adjoint_steps, args.ckpt_every)
        out["fwd_adj_over_fwd"] = adj["ratio"]
        out["adjoint"] = adj
        torch.cuda.empty_cache()
        if args.dtype == "f64":
            # the configuration's single-precision variant
            out["adjoint_f32"] = adjoint_ratio("f32", args.adjoint_steps, args.ckpt_every)
            torch.cuda.empty_cache()
    if args.batched_scale > 0:
        out["batched"] = batched_leg(args.batched_scale, args.graph_steps)
        torch.cuda.empty_cache()
    if args.f32_steps > 0 and args.dtype == "f64" and args.workload == "axion":
        out["f32"] = f32_leg(wl, args.f32_steps)
        torch.cuda.empty_cache()
    if args.variant_steps > 0 and wl.arem and s_fused:
        out["kernel_variants"] = kernel_variants_leg(wl, args.dtype, args.variant_steps)
        torch.cuda.empty_cache()
    if args.window_steps > 0 and args.workload == "axion":
        out["window"] = window_leg(args.window_steps)
        torch.cuda.empty_cache()
    if args.theta_steps > 0:
        out["theta_grid_products"] = theta_leg(args.theta_steps)
        torch.cuda.empty_cache()
    if args.pic_steps > 0:
        out["pic"] = pic_leg(args.pic_steps)
        torch.cuda.empty_cache()
    if args.stream_reference:
        out["stream_reference"] = stream_reference()
        out["roofline"]["frac_of_copy"] = achieved / out["stream_reference"]["copy_read_write_gbps"]
        out["roofline"]["frac_of_streaming_copy"] = (achieved /
                                                     out["stream_reference"]["lib_streaming_copy_read_write_gbps"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
