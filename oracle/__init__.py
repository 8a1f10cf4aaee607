"""CPU FP64 oracle for the direct-sum N-body method (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it.

Every function follows one passage of the paper (Zhu, "N-body Simulations of
the Solar System with CPU-based Parallel Methods"):

* ``accel``    Eq. (1), the direct sum, ascending j, sqrt and divide.
* ``verlet``   Eqs. (3)-(4), velocity Verlet taken literally.
* ``energy``   Sec. 2: conserved total energy as the accuracy measure.
* ``momenta``  linear / angular momentum, invariants of Eq. (1).
* ``accel_targets``  Eq. (1) for a list of targets.
* ``euler``    the first-order scheme of Sec. 2 (negative control).
* ``rk4``      the classical fourth-order Runge-Kutta method Sec. 2 names.
* ``vjp``      Jacobian-transpose of Eq. (1) from its blocks.
* ``adjoint``  reverse mode through the literal Eqs. (3)-(4) map.
* ``tangent``  forward mode (dual numbers) through the same map.

Each function is pinned by ``tests/test_oracle.py`` and
``tests/test_oracle_mutations.py`` to something other than itself (closed
forms, invariants, extended precision, worked examples, finite differences,
independent derivations); none is left unpinned.

All arrays are float64 structure-of-arrays: ``pos[3, n]``, ``vel[3, n]``,
``mass[n]``.  The C source is ``oracle.c``; :func:`build` compiles it with gcc
(-O2 -fopenmp -ffp-contract=off, no fast-math).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.c_double
_I64 = ctypes.c_int64
_P = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` next to the source."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_get_threads.restype = ctypes.c_int
    lib.oracle_accel.argtypes = [_I64, _D, _P, _P, _P]
    lib.oracle_accel_targets.argtypes = [_I64, _D, _P, _P, _P, _I64, _P]
    lib.oracle_verlet.argtypes = [_I64, _D, _D, _I64, _P, _P, _P, _P]
    lib.oracle_verlet.restype = ctypes.c_int
    lib.oracle_euler.argtypes = [_I64, _D, _D, _I64, _P, _P, _P]
    lib.oracle_euler.restype = ctypes.c_int
    lib.oracle_rk4.argtypes = [_I64, _D, _D, _I64, _P, _P, _P]
    lib.oracle_rk4.restype = ctypes.c_int
    lib.oracle_energy.argtypes = [_I64, _D, _P, _P, _P, _P]
    lib.oracle_momenta.argtypes = [_I64, _P, _P, _P, _P, _P]
    lib.oracle_vjp.argtypes = [_I64, _D, _P, _P, _P, _P, _P]
    lib.oracle_adjoint.argtypes = [_I64, _D, _D, _I64, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.oracle_adjoint.restype = ctypes.c_int
    lib.oracle_tangent.argtypes = [_I64, _D, _D, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.oracle_tangent.restype = ctypes.c_int
    _lib = lib
    return lib


class use_library:
    """Context manager that routes this module's calls to another build of
    the oracle (the mutation tests load deliberately broken copies)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = None
        real = _LIB
        globals()["_LIB"] = self.path
        try:
            _load()
        finally:
            globals()["_LIB"] = real
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _c(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(k: int) -> None:
    _load().oracle_set_threads(int(k))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def accel(pos, mass, G):
    """Eq. (1) accelerations, shape (3, n)."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    pos = _c(pos, (3, n))
    acc = np.empty((3, n))
    lib.oracle_accel(n, G, _ptr(pos), _ptr(mass), _ptr(acc))
    return acc


def accel_targets(pos, mass, G, idx):
    """Eq. (1) for the targets ``idx`` only; returns (3, len(idx))."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    pos = _c(pos, (3, n))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise IndexError("target index out of range")
    out = np.empty((idx.size, 3))
    lib.oracle_accel_targets(n, G, _ptr(pos), _ptr(mass), _ptr(idx), idx.size, _ptr(out))
    return np.ascontiguousarray(out.T)


def verlet(pos, vel, mass, G, dt, steps, trajectory=False):
    """Run Eqs. (3)-(4) for ``steps`` steps; returns (pos, vel[, traj])."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    p = _c(pos, (3, n)).copy()
    v = _c(vel, (3, n)).copy()
    traj = np.empty((steps + 1, 3, n)) if trajectory else None
    rc = lib.oracle_verlet(n, G, dt, int(steps), _ptr(p), _ptr(v), _ptr(mass),
                           _ptr(traj) if trajectory else None)
    if rc != 0:
        raise MemoryError("oracle_verlet allocation failed")
    return (p, v, traj) if trajectory else (p, v)


def euler(pos, vel, mass, G, dt, steps):
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    p = _c(pos, (3, n)).copy()
    v = _c(vel, (3, n)).copy()
    if lib.oracle_euler(n, G, dt, int(steps), _ptr(p), _ptr(v), _ptr(mass)) != 0:
        raise MemoryError("oracle_euler allocation failed")
    return p, v


def rk4(pos, vel, mass, G, dt, steps):
    """Classical fourth-order Runge-Kutta for ``steps`` steps; returns (pos, vel)."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    p = _c(pos, (3, n)).copy()
    v = _c(vel, (3, n)).copy()
    if lib.oracle_rk4(n, G, dt, int(steps), _ptr(p), _ptr(v), _ptr(mass)) != 0:
        raise MemoryError("oracle_rk4 allocation failed")
    return p, v


def energy(pos, vel, mass, G):
    """(kinetic, potential, total), Neumaier-compensated."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    out = np.empty(3)
    lib.oracle_energy(n, G, _ptr(_c(pos, (3, n))), _ptr(_c(vel, (3, n))), _ptr(mass), _ptr(out))
    return float(out[0]), float(out[1]), float(out[2])


def momenta(pos, vel, mass):
    """(P[3], L[3]) total linear and angular momentum."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    P = np.empty(3)
    L = np.empty(3)
    lib.oracle_momenta(n, _ptr(_c(pos, (3, n))), _ptr(_c(vel, (3, n))), _ptr(mass), _ptr(P), _ptr(L))
    return P, L


def vjp(pos, mass, u, G):
    """(J^T u [3, n], M^T u [n]) for the accelerations of Eq. (1)."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    out_r = np.empty((3, n))
    out_m = np.empty(n)
    lib.oracle_vjp(n, G, _ptr(_c(pos, (3, n))), _ptr(mass), _ptr(_c(u, (3, n))),
                   _ptr(out_r), _ptr(out_m))
    return out_r, out_m


def adjoint(pos0, vel0, mass, G, dt, steps, lam_r, lam_v):
    """(dL/dr0, dL/dv0, dL/dm) given dL/dr_n and dL/dv_n."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    gr = np.empty((3, n))
    gv = np.empty((3, n))
    gm = np.empty(n)
    rc = lib.oracle_adjoint(n, G, dt, int(steps), _ptr(_c(pos0, (3, n))), _ptr(_c(vel0, (3, n))),
                            _ptr(mass), _ptr(_c(lam_r, (3, n))), _ptr(_c(lam_v, (3, n))),
                            _ptr(gr), _ptr(gv), _ptr(gm))
    if rc != 0:
        raise MemoryError("oracle_adjoint allocation failed")
    return gr, gv, gm


def tangent(pos0, vel0, mass, G, dt, steps, dpos0, dvel0, dmass):
    """(r_n, v_n, dr_n, dv_n): forward-mode derivative along a direction."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    outs = [np.empty((3, n)) for _ in range(4)]
    rc = lib.oracle_tangent(n, G, dt, int(steps), _ptr(_c(pos0, (3, n))), _ptr(_c(vel0, (3, n))),
                            _ptr(mass), _ptr(_c(dpos0, (3, n))), _ptr(_c(dvel0, (3, n))),
                            _ptr(_c(dmass, (n,))), *[_ptr(o) for o in outs])
    if rc != 0:
        raise MemoryError("oracle_tangent allocation failed")
    return tuple(outs)


def timed_verlet(pos, vel, mass, G, dt, steps):
    """Wall time (s) of ``verlet`` on the host's cores, excluding set-up."""
    lib = _load()
    mass = _c(mass)
    n = mass.shape[0]
    p = _c(pos, (3, n)).copy()
    v = _c(vel, (3, n)).copy()
    t0 = time.perf_counter()
    lib.oracle_verlet(n, G, dt, int(steps), _ptr(p), _ptr(v), _ptr(mass), None)
    return time.perf_counter() - t0, p, v
