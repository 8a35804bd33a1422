"""Thin ctypes binding of libewald.so (C ABI declared in include/ewald.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions keep the C names; a non-OK status raises EwaldError with
the library's message.  Device buffers are passed as integer addresses (for
example ``tensor.data_ptr()``), streams as integer handles
(``torch.cuda.current_stream().cuda_stream``).

`System` and `Batch` are small conveniences over those calls that own the
handles and allocate device buffers with PyTorch.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libewald.so")

EWALD_OK, EWALD_E_ARG, EWALD_E_RCUT, EWALD_E_GCUT, EWALD_E_LATTICE, EWALD_E_NOMEM, EWALD_E_HIP, EWALD_E_STATE = range(8)
EWALD_FP64, EWALD_FP32_MIXED = 0, 1
STATUS_NAMES = {0: "EWALD_OK", 1: "EWALD_E_ARG", 2: "EWALD_E_RCUT", 3: "EWALD_E_GCUT",
                4: "EWALD_E_LATTICE", 5: "EWALD_E_NOMEM", 6: "EWALD_E_HIP", 7: "EWALD_E_STATE"}

# every symbol include/ewald.h declares
EXPORTS = ("ewald_setup", "ewald_sys_query", "ewald_sys_tables", "ewald_sys_candidates",
           "ewald_sys_geometry", "ewald_sys_destroy", "ewald_batch_create", "ewald_batch_layout", "ewald_state_offsets",
           "ewald_batch_destroy", "ewald_energy_batch", "ewald_move_delta_batch",
           "ewald_accept_batch", "ewald_run_moves_batch", "ewald_move_delta_grad_batch",
           "ewald_run_moves_grad_batch", "ewald_step_batch", "ewald_batch_set_tuning",
           "ewald_batch_get_tuning", "ewald_autotune", "ewald_blip_create", "ewald_blip_destroy",
           "ewald_blip_eval_batch", "ewald_timing_enable", "ewald_timing_report", "ewald_last_error")


class EwaldError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class SysDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("lattice", (ctypes.c_double * 3) * 3),
                ("n_fixed", ctypes.c_int), ("fixed_pos", ctypes.POINTER(ctypes.c_double)),
                ("fixed_q", ctypes.POINTER(ctypes.c_double)), ("n_mobile", ctypes.c_int),
                ("mobile_q", ctypes.POINTER(ctypes.c_double)), ("alpha", ctypes.c_double),
                ("g_cut", ctypes.c_double), ("r_cut", ctypes.c_double),
                ("precision", ctypes.c_int), ("refresh_every", ctypes.c_int),
                ("n_jastrow", ctypes.c_int), ("jastrow_a", ctypes.POINTER(ctypes.c_double)),
                ("u_terms", ctypes.c_int), ("u_C", ctypes.c_int), ("u_cutoff", ctypes.c_double),
                ("u_alpha", ctypes.POINTER(ctypes.c_double)), ("mobile_spin", ctypes.POINTER(ctypes.c_int32)),
                ("n_layers", ctypes.c_int), ("layer_z", ctypes.c_double * 2), ("n_mobile_layer0", ctypes.c_int),
                ("fixed_layer", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def load() -> ctypes.CDLL:
    """Load libewald.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    P, c_int, c_size, vp = ctypes.POINTER, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p
    lib.ewald_setup.argtypes = [P(SysDesc), P(vp)]
    lib.ewald_sys_query.argtypes = [vp, P(c_int), P(c_int), P(c_int), P(ctypes.c_double), P(ctypes.c_double)]
    lib.ewald_sys_tables.argtypes = [vp, vp, vp, vp, vp]
    lib.ewald_sys_candidates.argtypes = [vp, P(c_int), vp]
    lib.ewald_sys_geometry.argtypes = [vp, P(c_int), vp]
    lib.ewald_sys_destroy.argtypes = [vp]
    lib.ewald_sys_destroy.restype = None
    lib.ewald_batch_create.argtypes = [P(vp), c_int, P(c_int), c_int, P(vp)]
    lib.ewald_batch_layout.argtypes = [vp, vp, P(c_size)]
    lib.ewald_state_offsets.argtypes = [vp, c_int, P(c_size), P(c_size), P(c_size)]
    lib.ewald_batch_destroy.argtypes = [vp]
    lib.ewald_batch_destroy.restype = None
    lib.ewald_energy_batch.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.ewald_move_delta_batch.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.ewald_accept_batch.argtypes = [vp, vp, vp, vp]
    lib.ewald_run_moves_batch.argtypes = [vp, vp, c_int, vp, vp, vp, vp, vp, vp]
    lib.ewald_move_delta_grad_batch.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ewald_run_moves_grad_batch.argtypes = [vp, vp, c_int, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ewald_step_batch.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ewald_batch_set_tuning.argtypes = [vp, c_int, c_int, c_int, c_int, c_int]
    lib.ewald_batch_get_tuning.argtypes = [vp, P(c_int), P(c_int), P(c_int), P(c_int), P(c_int), P(c_int)]
    lib.ewald_autotune.argtypes = [vp, vp, c_int, ctypes.c_char_p, vp]
    lib.ewald_blip_create.argtypes = [P((ctypes.c_double * 3) * 3), P(c_int * 3), c_int, P(vp)]
    lib.ewald_blip_destroy.argtypes = [vp]
    lib.ewald_blip_destroy.restype = None
    lib.ewald_blip_eval_batch.argtypes = [vp, vp, c_int, vp, vp, vp, vp, vp]
    lib.ewald_timing_enable.argtypes = [c_int]
    lib.ewald_timing_report.argtypes = [ctypes.c_char_p, c_size, c_int]
    lib.ewald_last_error.argtypes = []
    lib.ewald_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("ewald_sys_destroy", "ewald_batch_destroy", "ewald_blip_destroy", "ewald_last_error"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != EWALD_OK:
        raise EwaldError(status, load().ewald_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- raw C calls (same names as the ABI) -----------------------------------

def ewald_setup(dim: int, lattice, mobile_q, alpha: float, g_cut: float, r_cut: float,
                fixed_pos=None, fixed_q=None, precision: int = EWALD_FP64,
                refresh_every: int = 0, jastrow_a=None, u_alpha=None, u_C: int = 0, u_cutoff: float = 0.0,
                mobile_spin=None, layer_z=None, n_mobile_layer0: int = 0, fixed_layer=None) -> int:
    """Returns the ewald_sys* handle as an int.  u_alpha [2][N_u + 1] (with
    u_C, u_cutoff and the mobile particles' spin labels) adds the Jastrow
    two-body polynomial term."""
    lib = load()
    keep = []
    d = SysDesc()
    d.dim = int(dim)
    lat = np.zeros((3, 3))
    lat[:, :] = np.asarray(lattice, dtype=np.float64)[:3, :3]
    for i in range(3):
        for j in range(3):
            d.lattice[i][j] = float(lat[i, j])
    mq = np.ascontiguousarray(mobile_q, dtype=np.float64)
    keep.append(mq)
    d.n_mobile = int(mq.shape[0])
    d.mobile_q = _dp(mq)
    if fixed_q is not None and len(fixed_q) > 0:
        fq = np.ascontiguousarray(fixed_q, dtype=np.float64)
        fp = np.ascontiguousarray(fixed_pos, dtype=np.float64).reshape(-1)
        keep += [fq, fp]
        d.n_fixed = int(fq.shape[0])
        d.fixed_q, d.fixed_pos = _dp(fq), _dp(fp)
    else:
        d.n_fixed = 0
    d.alpha, d.g_cut, d.r_cut = float(alpha), float(g_cut), float(r_cut)
    d.precision = int(precision)
    d.refresh_every = int(refresh_every)
    if jastrow_a is not None:
        ja = np.ascontiguousarray(jastrow_a, dtype=np.float64)
        keep.append(ja)
        d.n_jastrow = int(ja.shape[0])
        d.jastrow_a = _dp(ja)
    else:
        d.n_jastrow = 0
    if u_alpha is not None:
        ua = np.ascontiguousarray(u_alpha, dtype=np.float64).reshape(2, -1)
        keep.append(ua)
        d.u_terms, d.u_C, d.u_cutoff = int(ua.shape[1]), int(u_C), float(u_cutoff)
        d.u_alpha = _dp(ua)
        if mobile_spin is not None:
            sp = np.ascontiguousarray(mobile_spin, dtype=np.int32)
            keep.append(sp)
            d.mobile_spin = sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    else:
        d.u_terms = 0
    if layer_z is not None:
        d.n_layers = 2
        d.layer_z[0], d.layer_z[1] = float(layer_z[0]), float(layer_z[1])
        d.n_mobile_layer0 = int(n_mobile_layer0)
        if fixed_layer is not None and len(fixed_layer) > 0:
            fl = np.ascontiguousarray(fixed_layer, dtype=np.int32)
            keep.append(fl)
            d.fixed_layer = fl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    h = ctypes.c_void_p()
    _check(lib.ewald_setup(ctypes.byref(d), ctypes.byref(h)))
    return int(h.value)


def ewald_sys_query(sys_h: int) -> dict:
    n_g, n_slots, n_sh = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    r_ins, e_c = ctypes.c_double(), ctypes.c_double()
    _check(load().ewald_sys_query(ctypes.c_void_p(sys_h), ctypes.byref(n_g), ctypes.byref(n_slots),
                                  ctypes.byref(n_sh), ctypes.byref(r_ins), ctypes.byref(e_c)))
    return dict(n_g=n_g.value, n_slots=n_slots.value, n_shells=n_sh.value,
                r_inscribed=r_ins.value, e_const=e_c.value)


def ewald_sys_tables(sys_h: int) -> dict:
    q = ewald_sys_query(sys_h)
    ns = q["n_slots"]
    n = np.zeros((ns, 3), dtype=np.int32)
    w = np.zeros(ns)
    ja = np.zeros(ns)
    sh = np.zeros(ns, dtype=np.int32)
    _check(load().ewald_sys_tables(ctypes.c_void_p(sys_h), n.ctypes.data, w.ctypes.data,
                                   ja.ctypes.data, sh.ctypes.data))
    return dict(n=n, weight=w, jastrow=ja, shell=sh)


def ewald_sys_candidates(sys_h: int) -> np.ndarray:
    nc = ctypes.c_int()
    _check(load().ewald_sys_candidates(ctypes.c_void_p(sys_h), ctypes.byref(nc), None))
    out = np.zeros((nc.value, 3))
    _check(load().ewald_sys_candidates(ctypes.c_void_p(sys_h), ctypes.byref(nc), out.ctypes.data))
    return out


def ewald_sys_geometry(sys_h: int):
    """(sublattice index or 0 for the general reduction, box lengths [3])."""
    idx = ctypes.c_int()
    box = np.zeros(3)
    _check(load().ewald_sys_geometry(ctypes.c_void_p(sys_h), ctypes.byref(idx), box.ctypes.data))
    return idx.value, box


def ewald_sys_destroy(sys_h: int) -> None:
    load().ewald_sys_destroy(ctypes.c_void_p(sys_h))


def ewald_batch_create(sys_handles: Sequence[int], walker_sys) -> int:
    lib = load()
    arr = (ctypes.c_void_p * len(sys_handles))(*[ctypes.c_void_p(h) for h in sys_handles])
    ws = np.ascontiguousarray(walker_sys, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib.ewald_batch_create(arr, len(sys_handles), ws.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  int(ws.shape[0]), ctypes.byref(h)))
    return int(h.value)


def ewald_batch_layout(batch_h: int, n_walkers: int):
    offs = np.zeros(n_walkers + 1, dtype=np.uint64)
    sb = ctypes.c_size_t()
    _check(load().ewald_batch_layout(ctypes.c_void_p(batch_h), offs.ctypes.data, ctypes.byref(sb)))
    return offs.astype(np.int64), int(sb.value)


def ewald_state_offsets(batch_h: int, walker: int):
    h, p, r = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().ewald_state_offsets(ctypes.c_void_p(batch_h), int(walker), ctypes.byref(h),
                                      ctypes.byref(p), ctypes.byref(r)))
    return int(h.value), int(p.value), int(r.value)


def ewald_batch_destroy(batch_h: int) -> None:
    load().ewald_batch_destroy(ctypes.c_void_p(batch_h))


def ewald_energy_batch(batch_h, pos_ptr, state_ptr, energy_ptr, jastrow_ptr=0, stream=0) -> None:
    _check(load().ewald_energy_batch(ctypes.c_void_p(batch_h), ctypes.c_void_p(pos_ptr),
                                     ctypes.c_void_p(state_ptr), ctypes.c_void_p(energy_ptr),
                                     ctypes.c_void_p(jastrow_ptr or None), ctypes.c_void_p(stream or None)))


def ewald_move_delta_batch(batch_h, state_ptr, k_ptr, new_pos_ptr, delta_ptr, djastrow_ptr=0, stream=0) -> None:
    _check(load().ewald_move_delta_batch(ctypes.c_void_p(batch_h), ctypes.c_void_p(state_ptr),
                                         ctypes.c_void_p(k_ptr), ctypes.c_void_p(new_pos_ptr),
                                         ctypes.c_void_p(delta_ptr), ctypes.c_void_p(djastrow_ptr or None),
                                         ctypes.c_void_p(stream or None)))


def ewald_accept_batch(batch_h, state_ptr, accept_ptr, stream=0) -> None:
    _check(load().ewald_accept_batch(ctypes.c_void_p(batch_h), ctypes.c_void_p(state_ptr),
                                     ctypes.c_void_p(accept_ptr), ctypes.c_void_p(stream or None)))


def ewald_run_moves_batch(batch_h, state_ptr, n_steps, k_ptr, new_pos_ptr, accept_ptr, delta_ptr,
                          djastrow_ptr=0, stream=0) -> None:
    _check(load().ewald_run_moves_batch(ctypes.c_void_p(batch_h), ctypes.c_void_p(state_ptr), int(n_steps),
                                        ctypes.c_void_p(k_ptr), ctypes.c_void_p(new_pos_ptr),
                                        ctypes.c_void_p(accept_ptr), ctypes.c_void_p(delta_ptr),
                                        ctypes.c_void_p(djastrow_ptr or None), ctypes.c_void_p(stream or None)))


def ewald_move_delta_grad_batch(batch_h, state_ptr, k_ptr, new_pos_ptr, delta_ptr, djastrow_ptr=0, jgrad_ptr=0,
                                jlap_ptr=0, stream=0) -> None:
    _check(load().ewald_move_delta_grad_batch(ctypes.c_void_p(batch_h), ctypes.c_void_p(state_ptr),
                                              ctypes.c_void_p(k_ptr), ctypes.c_void_p(new_pos_ptr),
                                              ctypes.c_void_p(delta_ptr), ctypes.c_void_p(djastrow_ptr or None),
                                              ctypes.c_void_p(jgrad_ptr or None), ctypes.c_void_p(jlap_ptr or None),
                                              ctypes.c_void_p(stream or None)))


def ewald_step_batch(batch_h, state_ptr, accept_prev_ptr, k_ptr, new_pos_ptr, delta_ptr, djastrow_ptr=0,
                     jgrad_ptr=0, jlap_ptr=0, stream=0) -> None:
    _check(load().ewald_step_batch(ctypes.c_void_p(batch_h), ctypes.c_void_p(state_ptr),
                                   ctypes.c_void_p(accept_prev_ptr or None), ctypes.c_void_p(k_ptr),
                                   ctypes.c_void_p(new_pos_ptr), ctypes.c_void_p(delta_ptr),
                                   ctypes.c_void_p(djastrow_ptr or None), ctypes.c_void_p(jgrad_ptr or None),
                                   ctypes.c_void_p(jlap_ptr or None), ctypes.c_void_p(stream or None)))


def ewald_timing_enable(on: bool) -> None:
    _check(load().ewald_timing_enable(1 if on else 0))


def ewald_timing_report(reset: bool = False) -> dict:
    """The per-call timer table: {call: {calls, gpu_calls, gpu_ms_total,
    gpu_ms_mean, host_ms_total}}."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load().ewald_timing_report(buf, len(buf), 1 if reset else 0))
    out = {}
    for line in buf.value.decode().splitlines()[1:]:
        name, calls, gcalls, gms, gmean, hms = line.split()
        out[name] = dict(calls=int(calls), gpu_calls=int(gcalls), gpu_ms_total=float(gms),
                         gpu_ms_mean=float(gmean), host_ms_total=float(hms))
    return out


def ewald_run_moves_grad_batch(batch_h, state_ptr, n_steps, k_ptr, new_pos_ptr, accept_ptr, delta_ptr,
                               djastrow_ptr=0, jgrad_ptr=0, jlap_ptr=0, stream=0) -> None:
    _check(load().ewald_run_moves_grad_batch(ctypes.c_void_p(batch_h), ctypes.c_void_p(state_ptr), int(n_steps),
                                             ctypes.c_void_p(k_ptr), ctypes.c_void_p(new_pos_ptr),
                                             ctypes.c_void_p(accept_ptr), ctypes.c_void_p(delta_ptr),
                                             ctypes.c_void_p(djastrow_ptr or None), ctypes.c_void_p(jgrad_ptr or None),
                                             ctypes.c_void_p(jlap_ptr or None), ctypes.c_void_p(stream or None)))


def ewald_batch_set_tuning(batch_h, threads=0, chunk=0, general_frame=0, waves=0, walkers_per_block=0) -> None:
    _check(load().ewald_batch_set_tuning(ctypes.c_void_p(batch_h), int(threads), int(chunk), int(general_frame),
                                         int(waves), int(walkers_per_block)))


def ewald_batch_get_tuning(batch_h) -> dict:
    v = [ctypes.c_int() for _ in range(6)]
    _check(load().ewald_batch_get_tuning(ctypes.c_void_p(batch_h), *[ctypes.byref(x) for x in v]))
    return dict(threads=v[0].value, chunk=v[1].value, general_frame=v[2].value, fused=v[3].value, waves=v[4].value,
                walkers_per_block=v[5].value)


def ewald_autotune(batch_h, state_ptr, n_moves=32, cache_path=None, stream=0) -> None:
    _check(load().ewald_autotune(ctypes.c_void_p(batch_h), ctypes.c_void_p(state_ptr), int(n_moves),
                                 None if cache_path is None else str(cache_path).encode(),
                                 ctypes.c_void_p(stream or None)))


def ewald_last_error() -> str:
    return load().ewald_last_error().decode()


# ---- conveniences ------------------------------------------------------------

class System:
    """Owns an ewald_sys handle built from a workloads.System."""

    def __init__(self, system, precision: int = EWALD_FP64, refresh_every: int = 0, jastrow_a=None,
                 **override):
        kw = dict(alpha=system.alpha, g_cut=system.g_cut, r_cut=system.r_cut)
        kw.update(override)
        self.system = system
        u = {}
        if getattr(system, "u_alpha", None) is not None:
            u = dict(u_alpha=system.u_alpha, u_C=system.u_C, u_cutoff=system.u_cut,
                     mobile_spin=system.mobile_spin)
        if getattr(system, "layer_z", None) is not None:
            ml = np.asarray(system.mobile_layer)
            n0 = int(np.sum(ml == 0))
            if not (np.all(ml[:n0] == 0) and np.all(ml[n0:] == 1)):
                raise ValueError("mobile particles must be ordered by plane (plane 0 first)")
            u.update(layer_z=system.layer_z, n_mobile_layer0=n0, fixed_layer=system.fixed_layer)
        self.handle = ewald_setup(system.dim, system.lattice, system.mobile_q, kw["alpha"], kw["g_cut"],
                                  kw["r_cut"], fixed_pos=system.fixed_pos, fixed_q=system.fixed_q,
                                  precision=precision, refresh_every=refresh_every, jastrow_a=jastrow_a, **u)
        self.info = ewald_sys_query(self.handle)

    def tables(self):
        return ewald_sys_tables(self.handle)

    def close(self):
        if self.handle:
            ewald_sys_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Walker batch with a torch-allocated state buffer on `device`."""

    def __init__(self, systems: Sequence[System], walker_sys, device="cuda"):
        import torch
        self.systems = list(systems)
        self.walker_sys = np.ascontiguousarray(walker_sys, dtype=np.int32)
        self.n_walkers = int(self.walker_sys.shape[0])
        self.dim = systems[0].system.dim
        self.handle = ewald_batch_create([s.handle for s in systems], self.walker_sys)
        self.pos_offsets, self.state_bytes = ewald_batch_layout(self.handle, self.n_walkers)
        self.state = torch.zeros(self.state_bytes, dtype=torch.uint8, device=device)
        self.device = device

    def stream(self):
        import torch
        return torch.cuda.current_stream().cuda_stream

    def energy(self, pos, energy, jastrow=None):
        ewald_energy_batch(self.handle, pos.data_ptr(), self.state.data_ptr(), energy.data_ptr(),
                           0 if jastrow is None else jastrow.data_ptr(), self.stream())

    def move_delta(self, k, new_pos, delta, djastrow=None):
        ewald_move_delta_batch(self.handle, self.state.data_ptr(), k.data_ptr(), new_pos.data_ptr(),
                               delta.data_ptr(), 0 if djastrow is None else djastrow.data_ptr(), self.stream())

    def accept(self, accept):
        ewald_accept_batch(self.handle, self.state.data_ptr(), accept.data_ptr(), self.stream())

    def step(self, accept_prev, k, new_pos, delta, djastrow=None, jgrad=None, jlap=None):
        ewald_step_batch(self.handle, self.state.data_ptr(), 0 if accept_prev is None else accept_prev.data_ptr(),
                         k.data_ptr(), new_pos.data_ptr(), delta.data_ptr(),
                         0 if djastrow is None else djastrow.data_ptr(), 0 if jgrad is None else jgrad.data_ptr(),
                         0 if jlap is None else jlap.data_ptr(), self.stream())

    def run_moves(self, k, new_pos, accept, delta, djastrow=None):
        ewald_run_moves_batch(self.handle, self.state.data_ptr(), int(k.shape[0]), k.data_ptr(),
                              new_pos.data_ptr(), accept.data_ptr(), delta.data_ptr(),
                              0 if djastrow is None else djastrow.data_ptr(), self.stream())

    def move_delta_grad(self, k, new_pos, delta, djastrow, jgrad, jlap):
        ewald_move_delta_grad_batch(self.handle, self.state.data_ptr(), k.data_ptr(), new_pos.data_ptr(),
                                    delta.data_ptr(), 0 if djastrow is None else djastrow.data_ptr(),
                                    jgrad.data_ptr(), jlap.data_ptr(), self.stream())

    def run_moves_grad(self, k, new_pos, accept, delta, djastrow, jgrad, jlap):
        ewald_run_moves_grad_batch(self.handle, self.state.data_ptr(), int(k.shape[0]), k.data_ptr(),
                                   new_pos.data_ptr(), accept.data_ptr(), delta.data_ptr(),
                                   0 if djastrow is None else djastrow.data_ptr(), jgrad.data_ptr(),
                                   jlap.data_ptr(), self.stream())

    def set_tuning(self, threads=0, chunk=0, general_frame=0, waves=0, walkers_per_block=0):
        ewald_batch_set_tuning(self.handle, threads, chunk, general_frame, waves, walkers_per_block)

    def tuning(self) -> dict:
        return ewald_batch_get_tuning(self.handle)

    def autotune(self, n_moves=32, cache_path=None):
        ewald_autotune(self.handle, self.state.data_ptr(), n_moves, cache_path, self.stream())

    def walker_rho(self, w: int, plane: int = 0) -> np.ndarray:
        """rho of walker w (valid and padding slots) as complex numpy, after a
        sync; plane 1: a layered system's second plane (stored after the first)."""
        _, _, r = ewald_state_offsets(self.handle, w)
        ns = self.systems[self.walker_sys[w]].info["n_slots"]
        r += plane * ns * 16
        raw = self.state[r: r + ns * 16].cpu().numpy().view(np.float64)
        return raw[0::2] + 1j * raw[1::2]

    def walker_header(self, w: int) -> dict:
        h, _, _ = ewald_state_offsets(self.handle, w)
        raw = self.state[h: h + 48].cpu().numpy()
        ints = raw[:16].view(np.int32)
        dbl = raw[16:48].view(np.float64)
        return dict(counter=int(ints[0]), pending_k=int(ints[1]), n_accepts=int(ints[2]),
                    n_refresh=int(ints[3]), pending_s=dbl[:3].copy(), drift_max=float(dbl[3]))

    def walker_positions(self, w: int) -> np.ndarray:
        _, p, _ = ewald_state_offsets(self.handle, w)
        n = self.systems[self.walker_sys[w]].system.n_mobile
        raw = self.state[p: p + n * self.dim * 8].cpu().numpy().view(np.float64)
        return raw.reshape(n, self.dim)

    def close(self):
        if self.handle:
            ewald_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- blip orbitals -------------------------------------------------------------

def ewald_blip_create(lattice, grid, n_orb: int) -> int:
    lat = ((ctypes.c_double * 3) * 3)()
    a = np.asarray(lattice, dtype=np.float64)
    for i in range(3):
        for j in range(3):
            lat[i][j] = float(a[i, j])
    g = (ctypes.c_int * 3)(*[int(x) for x in grid])
    h = ctypes.c_void_p()
    _check(load().ewald_blip_create(ctypes.byref(lat), ctypes.byref(g), int(n_orb), ctypes.byref(h)))
    return int(h.value)


def ewald_blip_destroy(h: int) -> None:
    load().ewald_blip_destroy(ctypes.c_void_p(h))


def ewald_blip_eval_batch(h: int, coef: int, n_points: int, pos: int, val: int, grad: int = 0, lap: int = 0,
                          stream: int = 0) -> None:
    _check(load().ewald_blip_eval_batch(ctypes.c_void_p(h), ctypes.c_void_p(coef), int(n_points),
                                        ctypes.c_void_p(pos), ctypes.c_void_p(val), ctypes.c_void_p(grad or None),
                                        ctypes.c_void_p(lap or None), ctypes.c_void_p(stream or None)))


class Blips:
    """Owns an ewald_blip handle; evaluates orbitals from torch device tensors."""

    def __init__(self, lattice, grid, n_orb: int):
        self.grid = tuple(int(x) for x in grid)
        self.n_orb = int(n_orb)
        self.handle = ewald_blip_create(lattice, self.grid, self.n_orb)

    def eval(self, coef, pos, val, grad=None, lap=None):
        import torch
        n = int(pos.shape[0])
        ewald_blip_eval_batch(self.handle, coef.data_ptr(), n, pos.data_ptr(), val.data_ptr(),
                              0 if grad is None else grad.data_ptr(), 0 if lap is None else lap.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)

    def close(self):
        if self.handle:
            ewald_blip_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
