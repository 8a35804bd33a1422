"""ctypes front end of oracle.c (see that file's header for the mathematics).

Test infrastructure only; see the package docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def lib_path() -> str:
    return _LIB


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    _libs.pop(out, None)
    return out


class _OSys(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("lat", ctypes.c_double * 9),
                ("alpha", ctypes.c_double), ("r_cut", ctypes.c_double),
                ("g_cut", ctypes.c_double), ("n_jastrow", ctypes.c_int),
                ("jastrow_a", ctypes.POINTER(ctypes.c_double)),
                ("n_u", ctypes.c_int), ("u_c", ctypes.c_int), ("u_cut", ctypes.c_double),
                ("u_alpha", ctypes.POINTER(ctypes.c_double)), ("spin", ctypes.POINTER(ctypes.c_int)),
                ("z", ctypes.POINTER(ctypes.c_double))]


_libs = {}


def _load(path: str = _LIB):
    if path not in _libs:
        if path == _LIB and not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, i = ctypes.c_double, ctypes.c_int
        lib.oracle_count_g.argtypes = [P(_OSys), P(i), P(i)]
        lib.oracle_gvectors.argtypes = [P(_OSys), P(d), P(d), P(i)]
        lib.oracle_rho_at.argtypes = [P(_OSys), i, P(d), P(d), i, P(d), P(d)]
        lib.oracle_energy.argtypes = [P(_OSys), i, P(d), P(d), P(d), P(d)]
        lib.oracle_run.argtypes = [P(_OSys), i, i, P(d), P(d), i, P(ctypes.c_int32), P(d),
                                   P(ctypes.c_uint8), P(d), P(d), P(d), P(d), P(d), P(d), P(d)]
        lib.oracle_jastrow_derivs.argtypes = [P(_OSys), i, P(d), P(d), i, P(d), P(d)]
        lib.oracle_run_batch.argtypes = [P(_OSys), i, i, i, P(d), P(d), i, P(ctypes.c_int32),
                                         P(d), P(ctypes.c_uint8), P(d), P(d), P(d), P(d), i]
        lib.oracle_run_batch.restype = i
        lib.oracle_blip_eval.argtypes = [P(d), i, i, i, i, P(d), i, P(d), P(d), P(d), P(d)]
        _libs[path] = lib
    return _libs[path]


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class _Sys:
    """Keeps the ctypes struct and the arrays it points to alive together."""

    def __init__(self, dim, lattice, alpha, r_cut, g_cut, jastrow_a=None, u_alpha=None, u_C=3, u_cut=0.0,
                 spin=None, z=None):
        self.z = None if z is None else np.ascontiguousarray(z, dtype=np.float64)
        self.ja = None if jastrow_a is None else np.ascontiguousarray(jastrow_a, dtype=np.float64)
        self.ua = None if u_alpha is None else np.ascontiguousarray(u_alpha, dtype=np.float64).reshape(2, -1)
        self.spin = None if spin is None else np.ascontiguousarray(spin, dtype=np.int32)
        s = _OSys()
        s.dim = int(dim)
        lat = np.zeros((3, 3))
        lat[:, :] = np.asarray(lattice, dtype=np.float64)[:3, :3]
        for t in range(9):
            s.lat[t] = float(lat.flat[t])
        s.alpha, s.r_cut, s.g_cut = float(alpha), float(r_cut), float(g_cut)
        if self.ja is None:
            s.n_jastrow = 0
            s.jastrow_a = ctypes.POINTER(ctypes.c_double)()
        else:
            s.n_jastrow = int(self.ja.shape[0])
            s.jastrow_a = _ptr(self.ja, ctypes.c_double)
        if self.ua is None or self.spin is None:
            s.n_u, s.u_c, s.u_cut = 0, 0, 0.0
            s.u_alpha = ctypes.POINTER(ctypes.c_double)()
            s.spin = ctypes.POINTER(ctypes.c_int)()
        else:
            s.n_u, s.u_c, s.u_cut = int(self.ua.shape[1]), int(u_C), float(u_cut)
            s.u_alpha = _ptr(self.ua, ctypes.c_double)
            s.spin = _ptr(self.spin, ctypes.c_int)
        s.z = ctypes.POINTER(ctypes.c_double)() if self.z is None else _ptr(self.z, ctypes.c_double)
        self.s = s

    def ref(self):
        return ctypes.byref(self.s)


def spins(system) -> Optional[np.ndarray]:
    """Spin labels of all particles of a walker (mobile first, then the fixed
    ions with -1), or None when the system has no u term."""
    if getattr(system, "u_alpha", None) is None:
        return None
    ms = getattr(system, "mobile_spin", None)
    ms = np.zeros(system.n_mobile, dtype=np.int32) if ms is None else np.asarray(ms, dtype=np.int32)
    return np.concatenate([ms, -np.ones(system.n_fixed, dtype=np.int32)])


def heights(system) -> Optional[np.ndarray]:
    """Heights of all particles of a layered 2D system (mobile first, then the
    fixed ions), or None for a strictly two- or three-dimensional one."""
    lz = getattr(system, "layer_z", None)
    if lz is None:
        return None
    lz = np.asarray(lz, dtype=np.float64)
    ml = np.asarray(system.mobile_layer, dtype=np.int64)
    fl = getattr(system, "fixed_layer", None)
    fl = np.zeros(system.n_fixed, dtype=np.int64) if fl is None else np.asarray(fl, dtype=np.int64)
    return np.concatenate([lz[ml], lz[fl]])


def _mk(system, jastrow_a=None, spin=None, **over):
    kw = dict(dim=system.dim, lattice=system.lattice, alpha=system.alpha,
              r_cut=system.r_cut, g_cut=system.g_cut)
    if getattr(system, "layer_z", None) is not None:
        kw.update(z=heights(system))
    if getattr(system, "u_alpha", None) is not None:
        kw.update(u_alpha=system.u_alpha, u_C=system.u_C, u_cut=system.u_cut,
                  spin=spins(system) if spin is None else spin)
    kw.update(over)
    return _Sys(jastrow_a=jastrow_a, **kw)


def particles(system, mobile_pos: np.ndarray):
    """All particles of one walker, mobile first then the fixed ions: (pos, q)."""
    pos = np.concatenate([np.asarray(mobile_pos, dtype=np.float64).reshape(-1, system.dim),
                          np.asarray(system.fixed_pos, dtype=np.float64).reshape(-1, system.dim)])
    q = np.concatenate([system.mobile_q, system.fixed_q]).astype(np.float64)
    return np.ascontiguousarray(pos), np.ascontiguousarray(q)


def count_g(system, _path=_LIB, **over):
    s = _mk(system, **over)
    n, sh = ctypes.c_int(), ctypes.c_int()
    _load(_path).oracle_count_g(s.ref(), ctypes.byref(n), ctypes.byref(sh))
    return n.value, sh.value


def gvectors(system, _path=_LIB, **over):
    """Full G set: (g [n][3], g2 [n], shell [n])."""
    n, _ = count_g(system, _path, **over)
    s = _mk(system, **over)
    g = np.zeros((n, 3))
    g2 = np.zeros(n)
    sh = np.zeros(n, dtype=np.int32)
    _load(_path).oracle_gvectors(s.ref(), _ptr(g, ctypes.c_double), _ptr(g2, ctypes.c_double),
                            _ptr(sh, ctypes.c_int))
    return g, g2, sh


def rho_at(system, pos, q, g, _path=_LIB):
    s = _mk(system)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((g.shape[0], 2))
    _load(_path).oracle_rho_at(s.ref(), int(q.shape[0]), _ptr(pos, ctypes.c_double),
                          _ptr(q, ctypes.c_double), int(g.shape[0]), _ptr(g, ctypes.c_double),
                          _ptr(out, ctypes.c_double))
    return out[:, 0] + 1j * out[:, 1]


def energy(system, pos, q, jastrow_a: Optional[np.ndarray] = None, _path=_LIB, **over):
    """Energy of one configuration (all particles given explicitly).
    Returns dict(real, recip, self, background, total, jastrow)."""
    s = _mk(system, jastrow_a=jastrow_a, **over)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert s.spin is None or s.spin.shape[0] == q.shape[0], "one spin label per particle"
    assert s.z is None or s.z.shape[0] == q.shape[0], "one height per particle"
    parts = np.zeros(5)
    jas = ctypes.c_double(0.0)
    _load(_path).oracle_energy(s.ref(), int(q.shape[0]), _ptr(pos, ctypes.c_double),
                          _ptr(q, ctypes.c_double), _ptr(parts, ctypes.c_double), ctypes.byref(jas))
    return dict(real=parts[0], recip=parts[1], self=parts[2], background=parts[3],
                total=parts[4], jastrow=jas.value)


def jastrow_derivs(system, pos, q, k, jastrow_a, _path=_LIB, **over):
    """Gradient [dim] and Laplacian of J with respect to particle k (all
    particles given explicitly)."""
    s = _mk(system, jastrow_a=jastrow_a, **over)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert s.spin is None or s.spin.shape[0] == q.shape[0], "one spin label per particle"
    grad = np.zeros(system.dim)
    lap = ctypes.c_double(0.0)
    _load(_path).oracle_jastrow_derivs(s.ref(), int(q.shape[0]), _ptr(pos, ctypes.c_double),
                                       _ptr(q, ctypes.c_double), int(k), _ptr(grad, ctypes.c_double),
                                       ctypes.byref(lap))
    return grad, lap.value


def run(system, mobile_pos, k, new_pos, accept, jastrow_a=None, _path=_LIB, derivs=False, **over):
    """One walker: initial energy then the move sequence.  Returns dict with
    e0 (parts array), j0, delta [S], djas [S], pos_final (mobile), and with
    derivs=True jgrad [S][dim] and jlap [S]: the gradient and Laplacian of J
    with respect to the moved particle at each proposed configuration."""
    s = _mk(system, jastrow_a=jastrow_a, **over)
    pos, q = particles(system, mobile_pos)
    n = int(q.shape[0])
    k = np.ascontiguousarray(k, dtype=np.int32)
    S = int(k.shape[0])
    newp = np.ascontiguousarray(new_pos, dtype=np.float64).reshape(S, system.dim)
    acc = np.ascontiguousarray(accept, dtype=np.uint8)
    e0 = np.zeros(5)
    j0 = ctypes.c_double(0.0)
    delta = np.zeros(S)
    djas = np.zeros(S)
    pf = np.zeros_like(pos)
    jg = np.zeros((S, system.dim)) if derivs else None
    jl = np.zeros(S) if derivs else None
    null = ctypes.POINTER(ctypes.c_double)()
    _load(_path).oracle_run(s.ref(), n, system.n_mobile, _ptr(pos, ctypes.c_double),
                       _ptr(q, ctypes.c_double), S, _ptr(k, ctypes.c_int32),
                       _ptr(newp, ctypes.c_double), _ptr(acc, ctypes.c_uint8),
                       _ptr(e0, ctypes.c_double), ctypes.byref(j0), _ptr(delta, ctypes.c_double),
                       _ptr(djas, ctypes.c_double), _ptr(pf, ctypes.c_double),
                       null if jg is None else _ptr(jg, ctypes.c_double),
                       null if jl is None else _ptr(jl, ctypes.c_double))
    out = dict(e0=e0, energy0=e0[4], j0=j0.value, delta=delta, djas=djas,
               pos_final=pf[: system.n_mobile])
    if derivs:
        out.update(jgrad=jg, jlap=jl)
    return out


def run_batch(system, mobile_pos, k, new_pos, accept, jastrow_a=None, n_threads=0, _path=_LIB):
    """Walkers of one system. mobile_pos [W][n_mobile][dim], k [S][W],
    new_pos [S][W][dim], accept [S][W].  Returns dict(e0 [W][5], j0 [W],
    delta [S][W], djas [S][W], threads)."""
    s = _mk(system, jastrow_a=jastrow_a)
    W = int(mobile_pos.shape[0])
    allp = np.stack([particles(system, mobile_pos[w])[0] for w in range(W)])
    q = particles(system, mobile_pos[0])[1]
    n = int(q.shape[0])
    k = np.ascontiguousarray(k, dtype=np.int32)
    S = int(k.shape[0])
    newp = np.ascontiguousarray(new_pos, dtype=np.float64)
    acc = np.ascontiguousarray(accept, dtype=np.uint8)
    allp = np.ascontiguousarray(allp)
    e0 = np.zeros((W, 5))
    j0 = np.zeros(W)
    delta = np.zeros((S, W))
    djas = np.zeros((S, W))
    used = _load(_path).oracle_run_batch(s.ref(), W, n, system.n_mobile, _ptr(allp, ctypes.c_double),
                                    _ptr(q, ctypes.c_double), S, _ptr(k, ctypes.c_int32),
                                    _ptr(newp, ctypes.c_double), _ptr(acc, ctypes.c_uint8),
                                    _ptr(e0, ctypes.c_double), _ptr(j0, ctypes.c_double),
                                    _ptr(delta, ctypes.c_double), _ptr(djas, ctypes.c_double),
                                    int(n_threads))
    return dict(e0=e0, j0=j0, delta=delta, djas=djas, threads=used)


def blip_eval(lattice, grid, coef, pos, derivs=True, _path=_LIB):
    """Blip orbitals at Cartesian points: coef [n1][n2][n3][n_orb], pos [P][3].
    Returns (val [P][n_orb], grad [P][3][n_orb], lap [P][n_orb]) (the last two
    None without derivs)."""
    lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64)[:3, :3]).reshape(-1)
    n1, n2, n3 = (int(x) for x in grid)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    n_orb = int(coef.shape[-1])
    assert coef.shape == (n1, n2, n3, n_orb)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    P = int(pos.shape[0])
    val = np.zeros((P, n_orb))
    grad = np.zeros((P, 3, n_orb)) if derivs else None
    lap = np.zeros((P, n_orb)) if derivs else None
    null = ctypes.POINTER(ctypes.c_double)()
    _load(_path).oracle_blip_eval(_ptr(lat, ctypes.c_double), n1, n2, n3, n_orb, _ptr(coef, ctypes.c_double), P,
                                  _ptr(pos, ctypes.c_double), _ptr(val, ctypes.c_double),
                                  null if grad is None else _ptr(grad, ctypes.c_double),
                                  null if lap is None else _ptr(lap, ctypes.c_double))
    return val, grad, lap


class Variant:
    """The same front end bound to another build of oracle.c (used by the
    mutation tests, which compile deliberately broken copies)."""

    def __init__(self, so_path: str):
        self.path = so_path

    def count_g(self, system, **over):
        return count_g(system, self.path, **over)

    def gvectors(self, system, **over):
        return gvectors(system, self.path, **over)

    def rho_at(self, system, pos, q, g):
        return rho_at(system, pos, q, g, self.path)

    def energy(self, system, pos, q, jastrow_a=None, **over):
        return energy(system, pos, q, jastrow_a, self.path, **over)

    def run(self, system, mobile_pos, k, new_pos, accept, jastrow_a=None, derivs=False, **over):
        return run(system, mobile_pos, k, new_pos, accept, jastrow_a, self.path, derivs, **over)

    def jastrow_derivs(self, system, pos, q, k, jastrow_a, **over):
        return jastrow_derivs(system, pos, q, k, jastrow_a, self.path, **over)

    def run_batch(self, system, mobile_pos, k, new_pos, accept, jastrow_a=None, n_threads=0):
        return run_batch(system, mobile_pos, k, new_pos, accept, jastrow_a, n_threads, self.path)

    def blip_eval(self, lattice, grid, coef, pos, derivs=True):
        return blip_eval(lattice, grid, coef, pos, derivs, self.path)

    particles = staticmethod(particles)
