"""Thin ctypes binding of libqds (include/qds.h).

Argument marshalling only: every step of the field advance runs in the HIP
library.  PyTorch supplies the device memory (two state buffers) and the
stream.  Importing this module loads libqds.so and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, Optional

import numpy as np
import torch

from . import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqds.so")

QDS_OK, QDS_EINVAL, QDS_ECFL, QDS_ENOMEM, QDS_EHIP, QDS_EUNSUPPORTED, QDS_ESTATE = range(7)
F64, F32 = 0, 1
X_BC = {"open": 0, "periodic": 1, "window": 2}
R_BC = {"open": 0, "pec": 1}
HAS_PLASMA, HAS_AXION, HAS_AREM = 1, 2, 4
J_NONE, J_RING, J_PARTICLES = 0, 1, 2
P_TRP, P_TRM, P_TTP, P_TTM, P_EX, P_BX, P_JX, P_JR, P_JT = range(9)
P_SET1, P_PHI, P_TAP, P_TAM = 9, 18, 19, 20

OPT_PATH, OPT_ROWS, OPT_TIMING, OPT_TUNE = 1, 2, 3, 4
OPT_ROWS_A, OPT_ROWS_CUR, OPT_ROWS_B = 5, 6, 7       # one kernel's tile height
OPT_PRODUCTS = 8
OPT_OVERLAP = 9
OPT_KERNEL_AX = 10
OPT_PAIR, OPT_ROWS_PAIR = 11, 12                     # two steps per launch of the set's march
OPT_PAIR_A = 13                                      # in pairs, the background set's two-step march too
PRODUCTS_DIRECT, PRODUCTS_THETA = 0, 1
PATH_AUTO, PATH_STAGED, PATH_FUSED = 0, 1, 2


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nr", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("x_bc", ctypes.c_int32), ("r_bc", ctypes.c_int32), ("content", ctypes.c_int32),
                ("dr", ctypes.c_double)]


class Current(ctypes.Structure):
    _fields_ = [("wp2", ctypes.c_double), ("kind", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("amp", ctypes.c_double), ("x0", ctypes.c_double), ("v", ctypes.c_double),
                ("sx", ctypes.c_double), ("r0", ctypes.c_double), ("sr", ctypes.c_double),
                ("noise", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("pjx_prev", ctypes.c_void_p), ("pjx_next", ctypes.c_void_p), ("pjr", ctypes.c_void_p),
                ("pjt", ctypes.c_void_p)]


class Axion(ctypes.Structure):
    _fields_ = [("ma2", ctypes.c_double), ("s_phi", ctypes.c_double), ("s_j", ctypes.c_double),
                ("bext", ctypes.c_double * 6)]


class Loss(ctypes.Structure):
    _fields_ = [("set", ctypes.c_int32), ("mode", ctypes.c_int32), ("x_begin", ctypes.c_int32),
                ("x_end", ctypes.c_int32)]


class Particles(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p), ("uz", ctypes.c_void_p),
                ("q", ctypes.c_void_p), ("count", ctypes.c_int64), ("charge", ctypes.c_double),
                ("qm", ctypes.c_double), ("clear", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class State(ctypes.Structure):
    _fields_ = [("buf", ctypes.c_void_p * 2), ("cur", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("step", ctypes.c_int64), ("window", ctypes.c_int64)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.qds_init.argtypes = [ctypes.POINTER(Grid), i32, dbl, dbl, ctypes.POINTER(vp)]
    lib.qds_init.restype = i32
    lib.qds_state_bytes.argtypes = [vp]
    lib.qds_state_bytes.restype = ctypes.c_size_t
    lib.qds_row_pitch.argtypes = [vp]
    lib.qds_row_pitch.restype = i32
    lib.qds_plane_offset.argtypes = [vp, i32]
    lib.qds_plane_offset.restype = i64
    lib.qds_add_pulse.argtypes = [vp, ctypes.POINTER(State), i32, vp, vp, vp, vp]
    lib.qds_add_pulse.restype = i32
    lib.qds_step.argtypes = [vp, ctypes.POINTER(State), ctypes.POINTER(Current), ctypes.POINTER(Axion), i64, vp]
    lib.qds_step.restype = i32
    lib.qds_destroy.argtypes = [vp]
    lib.qds_destroy.restype = i32
    lib.qds_last_error.argtypes = [vp]
    lib.qds_last_error.restype = ctypes.c_char_p
    lib.qds_version.argtypes = []
    lib.qds_version.restype = ctypes.c_char_p
    lib.qds_set_option.argtypes = [vp, i32, i64]
    lib.qds_set_option.restype = i32
    lib.qds_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.qds_get_timing.restype = i32
    lib.qds_get_tiles.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.qds_get_tiles.restype = i32
    lib.qds_uses_fused.argtypes = [vp]
    lib.qds_uses_fused.restype = i32
    lib.qds_backward_pool_bytes.argtypes = [vp, i64, i64]
    lib.qds_backward_pool_bytes.restype = ctypes.c_size_t
    lib.qds_backward.argtypes = [vp, ctypes.POINTER(State), ctypes.POINTER(Current), ctypes.POINTER(Axion),
                                 ctypes.POINTER(Loss), i64, i64, vp, ctypes.c_size_t, vp,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), vp]
    lib.qds_backward.restype = i32
    lib.qds_dot.argtypes = [vp, vp, vp, vp, vp]
    lib.qds_dot.restype = i32
    lib.qds_loss_eval.argtypes = [vp, vp, ctypes.POINTER(Loss), vp, vp, vp]
    lib.qds_loss_eval.restype = i32
    lib.qds_loss_eval_noalloc.argtypes = [vp, vp, ctypes.POINTER(Loss), vp, vp]
    lib.qds_loss_eval_noalloc.restype = i32
    lib.qds_radial_mu_max.argtypes = [i32, dbl, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.qds_radial_mu_max.restype = i32
    lib.qds_particles_step.argtypes = [vp, ctypes.POINTER(State), i32, ctypes.POINTER(Particles), vp, vp, vp, vp, vp]
    lib.qds_particles_step.restype = i32
    lib.qds_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, i32, i32, vp]
    lib.qds_stream_copy.restype = i32
    lib.qds_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    lib.qds_batch_create.restype = i32
    lib.qds_batch_run.argtypes = [vp, ctypes.POINTER(State), ctypes.POINTER(Current), ctypes.POINTER(Axion),
                                  ctypes.POINTER(i64), i32, i32, vp]
    lib.qds_batch_run.restype = i32
    lib.qds_batch_get_tiles.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.qds_batch_get_tiles.restype = i32
    lib.qds_batch_set_tiles.argtypes = [vp, ctypes.POINTER(i32)]
    lib.qds_batch_set_tiles.restype = i32
    lib.qds_batch_stats.argtypes = [vp, ctypes.POINTER(i64)]
    lib.qds_batch_stats.restype = i32
    lib.qds_batch_last_error.argtypes = [vp]
    lib.qds_batch_last_error.restype = ctypes.c_char_p
    lib.qds_batch_destroy.argtypes = [vp]
    lib.qds_batch_destroy.restype = i32
    return lib


_LIB: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class QDSError(RuntimeError):
    pass


def _check(status: int, handle) -> None:
    if status != QDS_OK:
        msg = lib().qds_last_error(handle).decode()
        raise QDSError(f"libqds status {status}: {msg}")


def _bcheck(status: int, batch) -> None:
    if status != QDS_OK:
        msg = lib().qds_batch_last_error(batch).decode()
        raise QDSError(f"libqds status {status}: {msg}")


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Solver:
    """One QDS field advance on one GPU: a libqds handle plus its two state
    buffers (torch uint8 tensors on the device)."""

    def __init__(self, wl: I.Workload, dtype: str = "f64", device: str = "cuda:0", path: int = PATH_AUTO,
                 rows: Optional[int] = None):
        self.wl = wl
        self.device = torch.device(device)
        self.dtype = dtype
        content = 0
        if wl.wp2 != 0.0:
            content |= HAS_PLASMA
        if wl.axion:
            content |= HAS_AXION
        if wl.arem:
            content |= HAS_AREM
        g = Grid(wl.nx, wl.nr, F64 if dtype == "f64" else F32, X_BC[wl.x_bc], R_BC[wl.r_bc], content, wl.dr)
        h = ctypes.c_void_p()
        _check(lib().qds_init(ctypes.byref(g), wl.nmodes, wl.h, wl.h, ctypes.byref(h)), None)
        self.h = h
        self.nbytes = int(lib().qds_state_bytes(h))
        self.ld = int(lib().qds_row_pitch(h))
        self.bufs = [torch.zeros(self.nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.state = State()
        self.state.buf[0] = self.bufs[0].data_ptr()
        self.state.buf[1] = self.bufs[1].data_ptr()
        self.state.cur = 0
        self.state.step = 0
        self.state.window = 0
        self.cur = self._current()
        self.ax = self._axion()
        self.set_option(OPT_PATH, path)
        if rows is not None:
            self.set_option(OPT_ROWS, rows)

    def set_option(self, key: int, value: int) -> None:
        _check(lib().qds_set_option(self.h, key, int(value)), self.h)

    @property
    def fused(self) -> bool:
        return bool(lib().qds_uses_fused(self.h))

    def tiles(self):
        """Tile heights (rows per workgroup) of kernel A, the axion current,
        kernel B and the two-step march, and whether the autotuner chose them."""
        t = (ctypes.c_int32 * 4)()
        tuned = ctypes.c_int32()
        _check(lib().qds_get_tiles(self.h, t, ctypes.byref(tuned)), self.h)
        return list(t), bool(tuned.value)

    def timing(self):
        """(ms per kernel, launches per kernel) recorded since timing was set;
        index 0 = background set + axion (kernel A), 1 = regenerated set
        (kernel B), 2 = axion current."""
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        _check(lib().qds_get_timing(self.h, ms, n), self.h)
        return list(ms), list(n)

    # -- parameters ---------------------------------------------------------
    def _current(self) -> Current:
        c = Current()
        c.wp2 = self.wl.wp2
        d = self.wl.drive
        if d is None:
            c.kind = J_NONE
        else:
            c.kind = J_RING
            c.amp, c.x0, c.v, c.sx, c.r0, c.sr, c.noise = d.amp, d.x0, d.v, d.sx, d.r0, d.sr, d.noise
            c.seed = d.seed
        return c

    def _axion(self) -> Axion:
        a = Axion()
        a.ma2, a.s_phi, a.s_j = self.wl.ma2, self.wl.s_phi, self.wl.s_j
        for k, z in enumerate(self.wl.bext):
            a.bext[2 * k] = complex(z).real
            a.bext[2 * k + 1] = complex(z).imag
        return a

    # -- state --------------------------------------------------------------
    def load_pulses(self, pulses=None, basis=None) -> None:
        """Add the workload's pulses (sampled at the staggered points) to set 0.
        ``basis`` = (pulse index, coefficient index) loads the derivative of the
        pulse with respect to that envelope coefficient instead."""
        wl = self.wl
        xI = np.arange(wl.nx) * wl.h
        rK = (np.arange(wl.nr) + 0.5) * wl.dr
        rJ = np.arange(wl.nr + 1) * wl.dr
        rG = np.array([(wl.nr + 0.5) * wl.dr])
        plist = [(None, p) for p in (pulses if pulses is not None else wl.pulses)]
        if basis is not None:
            plist = [(basis[1], wl.pulses[basis[0]])]
        for q, p in plist:
            f = p.field if q is None else (lambda x, r, p=p, q=q: p.field_basis(x, r, q))
            fK = torch.from_numpy(np.ascontiguousarray(f(xI[None, :], rK[:, None]))).to(self.device)
            fJ = torch.from_numpy(np.ascontiguousarray(f(xI[None, :], rJ[:, None]))).to(self.device)
            fG = torch.from_numpy(np.ascontiguousarray(f(xI[None, :], rG[:, None])[0])).to(self.device)
            _check(lib().qds_add_pulse(self.h, ctypes.byref(self.state), ord(p.pol), fK.data_ptr(),
                                       fJ.data_ptr(), fG.data_ptr(), _stream_ptr()), self.h)
            torch.cuda.current_stream().synchronize()

    def step(self, n: int = 1, stream=None) -> None:
        _check(lib().qds_step(self.h, ctypes.byref(self.state), ctypes.byref(self.cur),
                              ctypes.byref(self.ax), int(n), _stream_ptr(stream)), self.h)

    @property
    def n(self) -> int:
        return int(self.state.step)

    @property
    def window(self) -> int:
        return int(self.state.window)

    def plane(self, plane: int, which: Optional[int] = None) -> Optional[torch.Tensor]:
        """View of one plane of a state buffer as a complex tensor [M, nr+1, nx]."""
        off = int(lib().qds_plane_offset(self.h, plane))
        if off < 0:
            return None
        b = self.bufs[self.state.cur if which is None else which]
        ebytes = 16 if self.dtype == "f64" else 8
        cdt = torch.complex128 if self.dtype == "f64" else torch.complex64
        M, nr, ld = self.wl.nmodes, self.wl.nr, self.ld
        n = M * (nr + 1) * ld
        v = b[off:off + n * ebytes].view(cdt).view(M, nr + 1, ld)
        return v[..., : self.wl.nx]

    def fields(self) -> Dict[str, torch.Tensor]:
        """Current state as named complex128 CPU tensors (names of the
        state dictionary the oracle uses)."""
        nr = self.wl.nr
        out = {}
        sets = [0, 1] if self.wl.arem else [0]
        for s in sets:
            b = 9 * s
            trp = self.plane(b + P_TRP)
            out[f"Trp{s}"] = trp[:, :nr]
            out[f"Bg{s}"] = trp[:, nr]
            out[f"Trm{s}"] = self.plane(b + P_TRM)[:, :nr]
            out[f"Ttp{s}"] = self.plane(b + P_TTP)
            out[f"Ttm{s}"] = self.plane(b + P_TTM)
            out[f"Ex{s}"] = self.plane(b + P_EX)
            out[f"Bx{s}"] = self.plane(b + P_BX)
            if self.wl.wp2 != 0.0:
                out[f"jx{s}"] = self.plane(b + P_JX)
                out[f"jr{s}"] = self.plane(b + P_JR)[:, :nr]
                out[f"jt{s}"] = self.plane(b + P_JT)
        if self.wl.axion:
            phi = self.plane(P_PHI)
            out["phi"] = phi[:, :nr]
            out["phig"] = phi[:, nr]
            out["Tap"] = self.plane(P_TAP)[:, :nr]
            out["Tam"] = self.plane(P_TAM)[:, :nr]
        return {k: v.to("cpu", torch.complex128) for k, v in out.items()}

    def load_fields(self, f: Dict[str, torch.Tensor]) -> None:
        """Overwrite the current state with named complex tensors (the names
        and shapes fields() returns); rows and planes not named are zeroed.
        Integer entries "n" (step) and "w" (window offset), if present, set
        the state's counters."""
        nr = self.wl.nr
        self.bufs[self.state.cur].zero_()
        cdt = torch.complex128 if self.dtype == "f64" else torch.complex64

        def put(plane, rows, key):
            if key in f:
                v = self.plane(plane)
                v[:, rows] = f[key].to(self.device, cdt)
        sets = [0, 1] if self.wl.arem else [0]
        for s in sets:
            b = 9 * s
            put(b + P_TRP, slice(0, nr), f"Trp{s}")
            put(b + P_TRP, nr, f"Bg{s}")
            put(b + P_TRM, slice(0, nr), f"Trm{s}")
            put(b + P_TTP, slice(None), f"Ttp{s}")
            put(b + P_TTM, slice(None), f"Ttm{s}")
            put(b + P_EX, slice(None), f"Ex{s}")
            put(b + P_BX, slice(None), f"Bx{s}")
            if self.wl.wp2 != 0.0:
                put(b + P_JX, slice(None), f"jx{s}")
                put(b + P_JR, slice(0, nr), f"jr{s}")
                put(b + P_JT, slice(None), f"jt{s}")
        if self.wl.axion:
            put(P_PHI, slice(0, nr), "phi")
            put(P_PHI, nr, "phig")
            put(P_TAP, slice(0, nr), "Tap")
            put(P_TAM, slice(0, nr), "Tam")
        if "n" in f:
            self.state.step = int(f["n"])
        if "w" in f:
            self.state.window = int(f["w"])
        torch.cuda.current_stream().synchronize()

    # -- adjoint ------------------------------------------------------------
    def backward_pool_bytes(self, n_steps: int, ckpt_every: int) -> int:
        """Bytes of the caller-owned work pool of ``backward(n_steps, ckpt_every)``."""
        return int(lib().qds_backward_pool_bytes(self.h, n_steps, ckpt_every))

    def backward(self, n_steps: int, ckpt_every: int, loss_set: int = 1, loss_mode: int = 1,
                 x_begin: Optional[int] = None, x_end: Optional[int] = None, stream=None,
                 pool: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
        """Gradient of the loss (energy of mode ``loss_mode`` of set ``loss_set``
        over columns [x_begin, x_end) after ``n_steps``) with respect to the
        current state, by the library's adjoint with checkpoints every
        ``ckpt_every`` steps.  Returns (loss, lambda0 buffer, (dL/ds_phi, dL/ds_j));
        the state itself is not advanced.  ``pool`` (a uint8 device tensor of at
        least backward_pool_bytes bytes) and ``out`` (a state-sized uint8 device
        tensor for lambda0) let a caller that repeats the call keep its memory;
        by default both are allocated here."""
        wl = self.wl
        lo = Loss(loss_set, loss_mode, max(0, wl.nx - 256) if x_begin is None else x_begin,
                  wl.nx if x_end is None else x_end)
        nbytes = self.backward_pool_bytes(n_steps, ckpt_every)
        if pool is None:
            pool = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        elif pool.dtype != torch.uint8 or pool.device != self.device or pool.numel() < nbytes or not pool.is_contiguous():
            raise ValueError(f"pool must be a contiguous uint8 tensor of at least {nbytes} bytes on {self.device}")
        if out is None:
            lam = torch.zeros(self.nbytes, dtype=torch.uint8, device=self.device)
        elif out.dtype != torch.uint8 or out.device != self.device or out.numel() != self.nbytes or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous uint8 tensor of {self.nbytes} bytes on {self.device}")
        else:
            lam = out
        dlds = (ctypes.c_double * 2)()
        loss = ctypes.c_double()
        cur = Current()
        ctypes.memmove(ctypes.byref(cur), ctypes.byref(self.cur), ctypes.sizeof(Current))
        _check(lib().qds_backward(self.h, ctypes.byref(self.state), ctypes.byref(cur), ctypes.byref(self.ax),
                                  ctypes.byref(lo), int(n_steps), int(ckpt_every), pool.data_ptr(), nbytes,
                                  lam.data_ptr(), dlds, ctypes.byref(loss), _stream_ptr(stream)), self.h)
        del pool
        return loss.value, lam, (dlds[0], dlds[1])

    def loss(self, loss_set: int = 1, loss_mode: int = 1, x_begin: Optional[int] = None,
             x_end: Optional[int] = None) -> float:
        """The backward loss evaluated on the current state (device reduction)."""
        wl = self.wl
        lo = Loss(loss_set, loss_mode, max(0, wl.nx - 256) if x_begin is None else x_begin,
                  wl.nx if x_end is None else x_end)
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        grad = torch.zeros(self.nbytes, dtype=torch.uint8, device=self.device)
        _check(lib().qds_loss_eval(self.h, self.bufs[self.state.cur].data_ptr(), ctypes.byref(lo), out.data_ptr(),
                                   grad.data_ptr(), _stream_ptr()), self.h)
        return float(out.item())

    def current_planes(self):
        """Three zeroed complex planes [M, nr+1, row pitch] (j_x, j_r, j_theta)
        in the state's dtype, for particles_step."""
        cdt = torch.complex128 if self.dtype == "f64" else torch.complex64
        return [torch.zeros(self.wl.nmodes, self.wl.nr + 1, self.ld, dtype=cdt, device=self.device) for _ in range(3)]

    def particles_step(self, pos: torch.Tensor, u: torch.Tensor, qm: float, charge=1.0, planes=None,
                       extrapolate: bool = False, clear: bool = False, stream=None):
        """One particle step in the current fields (qds_particles_step).
        ``pos`` and ``u`` are float64 device tensors [3, n] (rows x, y, z and
        u_x, u_y, u_z), updated in place; ``charge`` a float or a float64
        device tensor [n].  Returns (jx, jr, jt planes, skipped count)."""
        if pos.dtype != torch.float64 or u.dtype != torch.float64 or pos.shape[0] != 3 or u.shape != pos.shape \
                or not pos.is_contiguous() or not u.is_contiguous():
            raise ValueError("pos and u must be contiguous float64 tensors of shape [3, n]")
        planes = self.current_planes() if planes is None else planes
        n = pos.shape[1]
        P = Particles()
        P.x, P.y, P.z = pos[0].data_ptr(), pos[1].data_ptr(), pos[2].data_ptr()
        P.ux, P.uy, P.uz = u[0].data_ptr(), u[1].data_ptr(), u[2].data_ptr()
        if isinstance(charge, torch.Tensor):
            P.q = charge.data_ptr()
        else:
            P.q = None
            P.charge = float(charge)
        P.count = n
        P.qm = float(qm)
        P.clear = 1 if clear else 0
        skipped = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(lib().qds_particles_step(self.h, ctypes.byref(self.state), 1 if extrapolate else 0, ctypes.byref(P),
                                        planes[0].data_ptr(), planes[1].data_ptr(), planes[2].data_ptr(),
                                        skipped.data_ptr(), _stream_ptr(stream)), self.h)
        return planes, skipped

    def pic_steps(self, pos: torch.Tensor, u: torch.Tensor, qm: float, charge, n: int, coupling=None):
        """``n`` coupled PIC steps (Sec. 3.1): per step qds_particles_step in
        the current fields (E_x, B_x extrapolated to t^n once a previous state
        exists) depositing into fresh planes, then qds_step with those
        currents (kind QDS_J_PARTICLES: j_x^n the mean of this and the
        previous step's deposit).  ``coupling`` carries the deposit planes
        between calls; returns it (and the skipped-particle counters)."""
        if coupling is None:
            coupling = {"planes": [self.current_planes(), self.current_planes()], "prev": None, "steps": 0}
        skipped = []
        for _ in range(n):
            new = coupling["planes"][0] if coupling["prev"] is not coupling["planes"][0] else coupling["planes"][1]
            _, sk = self.particles_step(pos, u, qm, charge, planes=new, extrapolate=coupling["steps"] > 0,
                                        clear=True)
            skipped.append(sk)
            J = Current()
            ctypes.memmove(ctypes.byref(J), ctypes.byref(self.cur), ctypes.sizeof(Current))
            J.kind = J_PARTICLES
            J.pjx_prev = coupling["prev"][0].data_ptr() if coupling["prev"] is not None else None
            J.pjx_next, J.pjr, J.pjt = new[0].data_ptr(), new[1].data_ptr(), new[2].data_ptr()
            _check(lib().qds_step(self.h, ctypes.byref(self.state), ctypes.byref(J), ctypes.byref(self.ax), 1,
                                  _stream_ptr()), self.h)
            coupling["prev"] = new
            coupling["steps"] += 1
        return coupling, skipped

    def dot(self, a: torch.Tensor, b: torch.Tensor) -> float:
        """Re sum conj(a) b over two state buffers (device reduction)."""
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(lib().qds_dot(self.h, a.data_ptr(), b.data_ptr(), out.data_ptr(), _stream_ptr()), self.h)
        return float(out.item())

    def buffer_fields(self, buf: torch.Tensor) -> Dict[str, torch.Tensor]:
        """Named complex128 CPU views of an arbitrary state-layout buffer."""
        saved = self.bufs[self.state.cur]
        self.bufs[self.state.cur] = buf
        try:
            return self.fields()
        finally:
            self.bufs[self.state.cur] = saved

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            lib().qds_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NTILES = 12
TILE_A1, TILE_CUR1, TILE_EM0, TILE_EM1, TILE_PAIR0, TILE_PAIR1 = 0, 4, 8, 9, 10, 11


class Batch:
    """Many independent solvers advanced together by qds_batch_run: one launch
    per kernel class per step over all running instances, ``graph_steps``
    steps per captured HIP graph (-1: the whole uneven schedule as one graph)."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        n = len(self.solvers)
        arr = (ctypes.c_void_p * n)(*[s.h.value for s in self.solvers])
        h = ctypes.c_void_p()
        _bcheck(lib().qds_batch_create(arr, n, ctypes.byref(h)), None)
        self.b = h

    def run(self, n_steps, graph_steps: int = 16, tune: bool = False, stream=None) -> None:
        n = len(self.solvers)
        if isinstance(n_steps, int):
            n_steps = [n_steps] * n
        states = (State * n)()
        cur = (Current * n)()
        ax = (Axion * n)()
        for k, s in enumerate(self.solvers):
            ctypes.memmove(ctypes.byref(states[k]), ctypes.byref(s.state), ctypes.sizeof(State))
            ctypes.memmove(ctypes.byref(cur[k]), ctypes.byref(s.cur), ctypes.sizeof(Current))
            ctypes.memmove(ctypes.byref(ax[k]), ctypes.byref(s.ax), ctypes.sizeof(Axion))
        steps = (ctypes.c_int64 * n)(*[int(v) for v in n_steps])
        _bcheck(lib().qds_batch_run(self.b, states, cur, ax, steps, int(graph_steps), 1 if tune else 0,
                                    _stream_ptr(stream)), self.b)
        for k, s in enumerate(self.solvers):
            ctypes.memmove(ctypes.byref(s.state), ctypes.byref(states[k]), ctypes.sizeof(State))

    def tiles(self):
        t = (ctypes.c_int32 * NTILES)()
        tuned = ctypes.c_int32()
        _bcheck(lib().qds_batch_get_tiles(self.b, t, ctypes.byref(tuned)), self.b)
        return list(t), bool(tuned.value)

    def stats(self):
        """(graph launches, graphs instantiated, kernel launches outside graphs,
        kernel launches inside launched graphs) since creation."""
        v = (ctypes.c_int64 * 4)()
        _bcheck(lib().qds_batch_stats(self.b, v), self.b)
        return list(v)

    def set_tiles(self, tiles) -> None:
        t = (ctypes.c_int32 * NTILES)(*[int(v) for v in tiles])
        _bcheck(lib().qds_batch_set_tiles(self.b, t), self.b)

    def close(self) -> None:
        if getattr(self, "b", None):
            lib().qds_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
