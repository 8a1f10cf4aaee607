"""Python entry points with the names of the C ABI (include/nbody.h).

All state is float64 torch tensors on the GPU in structure-of-arrays form:
``pos`` and ``vel`` of shape (3, n), ``mass`` of shape (n,).  Work is
enqueued on the current torch stream.  Each function only checks and
marshals arguments; the computation happens in libnbody.so.
"""
from __future__ import annotations

import ctypes
import json

import torch

from . import _capi as C
from ._capi import NBODY_FP64, NBODY_SPLIT, NBODY_SPLIT_COMPENSATED

_PREC = {"fp64": NBODY_FP64, "split": NBODY_SPLIT, "compensated": NBODY_SPLIT_COMPENSATED,
         NBODY_FP64: NBODY_FP64, NBODY_SPLIT: NBODY_SPLIT,
         NBODY_SPLIT_COMPENSATED: NBODY_SPLIT_COMPENSATED}
_PREC_NAME = {NBODY_FP64: "fp64", NBODY_SPLIT: "split", NBODY_SPLIT_COMPENSATED: "compensated"}

#: 3e17 kg in solar masses (1 Msun = 1.98847e30 kg): the small-body class
#: boundary for the split form in AU / day / Msun units.
SMALL_MASS_MSUN = 3e17 / 1.98847e30


def _prec(p) -> int:
    try:
        return _PREC[p]
    except KeyError:
        raise ValueError(f"precision must be 'fp64', 'split' or 'compensated', got {p!r}") from None


def _state(t: torch.Tensor, name: str, n: int | None = None, planes: int = 3) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (no CPU path exists)")
    want = (planes, n) if planes > 1 else (n,)
    if n is not None and tuple(t.shape) != want:
        raise ValueError(f"{name} must have shape {want}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _mass(mass: torch.Tensor) -> int:
    _state(mass, "mass", planes=1)
    if mass.dim() != 1 or mass.shape[0] < 1:
        raise ValueError("mass must be a non-empty 1-D tensor")
    return int(mass.shape[0])


def _same_device(*ts):
    d = ts[0].device
    for t in ts[1:]:
        if t.device != d:
            raise ValueError("all tensors must be on one device")
    return d


def _small(precision: int, small_mass):
    if precision != NBODY_FP64:
        return float(SMALL_MASS_MSUN if small_mass is None else small_mass)
    return 0.0


def accel(pos, mass, G, precision="fp64", small_mass=None, out=None):
    """Eq. (1) accelerations at ``pos``; returns a (3, n) tensor."""
    n = _mass(mass)
    _state(pos, "pos", n)
    dev = _same_device(pos, mass)
    p = _prec(precision)
    if out is None:
        out = torch.empty((3, n), dtype=torch.float64, device=dev)
    _state(out, "out", n)
    lib = C.load()
    nb = C.workspace_bytes(C.OP_ACCEL, n, precision=p)
    ws = C.workspace(nb, dev)
    st = lib.nbody_accel(pos.data_ptr(), None, mass.data_ptr(), n, float(G), 0.0, 0,
                         out.data_ptr(), p, _small(p, small_mass), ws.data_ptr(), ws.numel(),
                         C.stream_handle(dev))
    C.check(st, "nbody_accel")
    return out


def accel_shard(pos, mass, G, t0, nt, out=None):
    """FP64 Eq. (1) accelerations of bodies t0 .. t0 + nt - 1 from all n
    sources (one GPU's share of the targets); returns a (3, nt) tensor."""
    n = _mass(mass)
    _state(pos, "pos", n)
    dev = _same_device(pos, mass)
    t0, nt = int(t0), int(nt)
    if out is None:
        out = torch.empty((3, max(nt, 1)), dtype=torch.float64, device=dev)
    _state(out, "out", max(nt, 1))
    lib = C.load()
    ws = C.workspace(C.workspace_bytes(C.OP_ACCEL_SHARD, n), dev)
    st = lib.nbody_accel_shard(pos.data_ptr(), mass.data_ptr(), n, float(G), t0, nt,
                               out.data_ptr(), ws.data_ptr(), ws.numel(), C.stream_handle(dev))
    C.check(st, "nbody_accel_shard")
    return out


def verlet_run(pos, vel, mass, G, dt, steps, precision="fp64", small_mass=None):
    """Advances (pos, vel) in place by ``steps`` velocity-Verlet steps
    (Eqs. (3)-(4)); returns (pos, vel)."""
    n = _mass(mass)
    _state(pos, "pos", n)
    _state(vel, "vel", n)
    dev = _same_device(pos, vel, mass)
    p = _prec(precision)
    steps = int(steps)
    lib = C.load()
    nb = C.workspace_bytes(C.OP_RUN, n, steps=steps, precision=p)
    ws = C.workspace(nb, dev)
    st = lib.nbody_verlet_run(pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), n, float(G),
                              float(dt), steps, p, _small(p, small_mass), ws.data_ptr(),
                              ws.numel(), C.stream_handle(dev))
    C.check(st, "nbody_verlet_run")
    return pos, vel


def rk4_run(pos, vel, mass, G, dt, steps, precision="fp64", small_mass=None):
    """Advances (pos, vel) in place by ``steps`` classical fourth-order
    Runge-Kutta steps (four evaluations of Eq. (1) per step); returns
    (pos, vel)."""
    n = _mass(mass)
    _state(pos, "pos", n)
    _state(vel, "vel", n)
    dev = _same_device(pos, vel, mass)
    p = _prec(precision)
    steps = int(steps)
    lib = C.load()
    ws = C.workspace(C.workspace_bytes(C.OP_RK4, n, steps=steps, precision=p), dev)
    st = lib.nbody_rk4_run(pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), n, float(G),
                           float(dt), steps, p, _small(p, small_mass), ws.data_ptr(), ws.numel(),
                           C.stream_handle(dev))
    C.check(st, "nbody_rk4_run")
    return pos, vel


def verlet_adjoint(pos0, vel0, mass, G, dt, steps, checkpoint_every, grad_posT, grad_velT):
    """Discrete adjoint of an FP64 run: returns (dL/dr0, dL/dv0, dL/dm, r_T, v_T)
    given dL/dr_T and dL/dv_T."""
    n = _mass(mass)
    for t, name in ((pos0, "pos0"), (vel0, "vel0"), (grad_posT, "grad_posT"),
                    (grad_velT, "grad_velT")):
        _state(t, name, n)
    dev = _same_device(pos0, vel0, mass, grad_posT, grad_velT)
    steps = int(steps)
    K = int(checkpoint_every)
    gr = torch.empty((3, n), dtype=torch.float64, device=dev)
    gv = torch.empty_like(gr)
    gm = torch.empty((n,), dtype=torch.float64, device=dev)
    pT = torch.empty_like(gr)
    vT = torch.empty_like(gr)
    lib = C.load()
    nb = C.workspace_bytes(C.OP_ADJOINT, n, steps=steps, checkpoint_every=max(K, 1))
    ws = C.workspace(nb, dev)
    st = lib.nbody_verlet_adjoint(pos0.data_ptr(), vel0.data_ptr(), mass.data_ptr(), n, float(G),
                                  float(dt), steps, K, grad_posT.data_ptr(), grad_velT.data_ptr(),
                                  gr.data_ptr(), gv.data_ptr(), gm.data_ptr(), pT.data_ptr(),
                                  vT.data_ptr(), ws.data_ptr(), ws.numel(), C.stream_handle(dev))
    C.check(st, "nbody_verlet_adjoint")
    return gr, gv, gm, pT, vT


def checkpoint_shape(n, steps, checkpoint_every):
    """Shape of the checkpoint tensor of verlet_checkpoints: one (r, v)
    record every K steps plus the final state."""
    K = int(checkpoint_every)
    return ((int(steps) + K - 1) // K + 1, 6, int(n))


def verlet_checkpoints(pos0, vel0, mass, G, dt, steps, checkpoint_every):
    """The forward half of verlet_adjoint: runs ``steps`` FP64 steps from
    (pos0, vel0) and returns (r_T, v_T, checkpoints), checkpoints a device
    tensor of checkpoint_shape(...) for verlet_adjoint_from_checkpoints."""
    n = _mass(mass)
    _state(pos0, "pos0", n)
    _state(vel0, "vel0", n)
    dev = _same_device(pos0, vel0, mass)
    steps, K = int(steps), int(checkpoint_every)
    ck = torch.empty(checkpoint_shape(n, steps, max(K, 1)), dtype=torch.float64, device=dev)
    pT = torch.empty((3, n), dtype=torch.float64, device=dev)
    vT = torch.empty_like(pT)
    lib = C.load()
    ws = C.workspace(C.workspace_bytes(C.OP_ADJOINT_SWEEP, n, steps=steps,
                                       checkpoint_every=max(K, 1)), dev)
    st = lib.nbody_verlet_checkpoints(pos0.data_ptr(), vel0.data_ptr(), mass.data_ptr(), n,
                                      float(G), float(dt), steps, K, ck.data_ptr(), pT.data_ptr(),
                                      vT.data_ptr(), ws.data_ptr(), ws.numel(),
                                      C.stream_handle(dev))
    C.check(st, "nbody_verlet_checkpoints")
    return pT, vT, ck


def verlet_adjoint_from_checkpoints(checkpoints, mass, G, dt, steps, checkpoint_every,
                                    grad_posT, grad_velT):
    """The reverse half of verlet_adjoint: (dL/dr0, dL/dv0, dL/dm) from the
    checkpoints of verlet_checkpoints (same masses, G, dt, steps, K)."""
    n = _mass(mass)
    steps, K = int(steps), int(checkpoint_every)
    if not isinstance(checkpoints, torch.Tensor) or checkpoints.dtype != torch.float64 or \
            tuple(checkpoints.shape) != checkpoint_shape(n, steps, max(K, 1)) or \
            not checkpoints.is_contiguous() or checkpoints.device.type != "cuda":
        raise ValueError("checkpoints must be the contiguous float64 GPU tensor of "
                         "verlet_checkpoints for these sizes")
    for t, name in ((grad_posT, "grad_posT"), (grad_velT, "grad_velT")):
        _state(t, name, n)
    dev = _same_device(checkpoints, mass, grad_posT, grad_velT)
    gr = torch.empty((3, n), dtype=torch.float64, device=dev)
    gv = torch.empty_like(gr)
    gm = torch.empty((n,), dtype=torch.float64, device=dev)
    lib = C.load()
    ws = C.workspace(C.workspace_bytes(C.OP_ADJOINT_SWEEP, n, steps=steps,
                                       checkpoint_every=max(K, 1)), dev)
    st = lib.nbody_verlet_adjoint_from_checkpoints(checkpoints.data_ptr(), mass.data_ptr(), n,
                                                   float(G), float(dt), steps, K,
                                                   grad_posT.data_ptr(), grad_velT.data_ptr(),
                                                   gr.data_ptr(), gv.data_ptr(), gm.data_ptr(),
                                                   ws.data_ptr(), ws.numel(), C.stream_handle(dev))
    C.check(st, "nbody_verlet_adjoint_from_checkpoints")
    return gr, gv, gm


def verlet_run_batched(pos, vel, mass, offsets, G, dt, steps, precision="fp64", small_mass=None):
    """Advances many independent systems (concatenated SoA, system k owns
    bodies offsets[k]:offsets[k+1]) in place."""
    n = _mass(mass)
    _state(pos, "pos", n)
    _state(vel, "vel", n)
    dev = _same_device(pos, vel, mass)
    offs = [int(x) for x in offsets]
    ns = len(offs) - 1
    if ns < 1 or offs[-1] != n:
        raise ValueError("offsets must have num_systems+1 entries ending at n")
    p = _prec(precision)
    arr = (ctypes.c_int64 * len(offs))(*offs)
    lib = C.load()
    nb = C.workspace_bytes(C.OP_BATCHED, n, num_systems=ns, steps=int(steps), precision=p)
    ws = C.workspace(nb, dev)
    st = lib.nbody_verlet_run_batched(pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), arr, ns,
                                      float(G), float(dt), int(steps), p, _small(p, small_mass),
                                      ws.data_ptr(), ws.numel(), C.stream_handle(dev))
    C.check(st, "nbody_verlet_run_batched")
    return pos, vel


def energy(pos, vel, mass, G):
    """(kinetic, potential, total) as a device tensor of 3 doubles."""
    n = _mass(mass)
    _state(pos, "pos", n)
    _state(vel, "vel", n)
    dev = _same_device(pos, vel, mass)
    out = torch.empty(3, dtype=torch.float64, device=dev)
    lib = C.load()
    nb = C.workspace_bytes(C.OP_ENERGY, n)
    ws = C.workspace(nb, dev)
    st = lib.nbody_energy(pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), n, float(G),
                          out.data_ptr(), ws.data_ptr(), ws.numel(), C.stream_handle(dev))
    C.check(st, "nbody_energy")
    return out


def momenta(pos, vel, mass):
    """(Px, Py, Pz, Lx, Ly, Lz) as a device tensor of 6 doubles."""
    n = _mass(mass)
    _state(pos, "pos", n)
    _state(vel, "vel", n)
    dev = _same_device(pos, vel, mass)
    out = torch.empty(6, dtype=torch.float64, device=dev)
    st = C.load().nbody_momenta(pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), n,
                                out.data_ptr(), C.stream_handle(dev))
    C.check(st, "nbody_momenta")
    return out


def get_flags(device=None, clear=False) -> int:
    """Flags of the last runs on this device and the current stream (their
    shared workspace; bit 0: non-finite value produced).  Synchronises the
    current stream."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ws = C.workspace(256, dev)
    v = ctypes.c_int32(0)
    st = C.load().nbody_get_flags(ws.data_ptr(), C.stream_handle(dev), int(bool(clear)),
                                  ctypes.byref(v))
    C.check(st, "nbody_get_flags")
    return int(v.value)


def get_tile(kind, precision, n):
    t = C.Tile()
    C.check(C.load().nbody_get_tile(int(kind), _prec(precision), int(n), ctypes.byref(t)),
            "nbody_get_tile")
    return t.as_dict()


def set_tile(kind, precision, n, targets_per_lane, waves, chunks, variant=0):
    t = C.Tile(int(targets_per_lane), int(waves), int(chunks), int(variant))
    C.check(C.load().nbody_set_tile(int(kind), _prec(precision), int(n), ctypes.byref(t)),
            "nbody_set_tile")


# Tile shapes chosen by the autotuner in this process, for save_tuning():
# (kind, precision, n) -> tile dict.
_tuned = {}


def save_tuning(path):
    """Writes the tile shapes the autotuner chose in this process to a JSON
    file (device name, library version and one entry per tuned size), which
    load_tuning() installs in a later process."""
    entries = [{"kind": k, "precision": p, "n": n, "tile": t} for (k, p, n), t in _tuned.items()]
    doc = {"library": version(), "device": torch.cuda.get_device_name(), "entries": entries}
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)


def load_tuning(path, strict_device=True):
    """Installs tile shapes from a save_tuning() file; returns how many.
    With strict_device, a file written on another device or library version
    is ignored (returns 0)."""
    with open(path) as fh:
        doc = json.load(fh)
    if strict_device and (doc.get("device") != torch.cuda.get_device_name()
                          or doc.get("library") != version()):
        return 0
    count = 0
    for e in doc.get("entries", []):
        t = e["tile"]
        set_tile(e["kind"], e["precision"], e["n"], t["targets_per_lane"], t["waves"],
                 t["chunks"], t["variant"])
        _tuned[(e["kind"], e["precision"], e["n"])] = t
        count += 1
    return count


def autotune(pos, mass, G, precision="fp64", kind=0, small_mass=None):
    """Times candidate tile shapes on this data, keeps the fastest for n's
    size class; returns (tile dict, ms per pass)."""
    n = _mass(mass)
    _state(pos, "pos", n)
    dev = _same_device(pos, mass)
    p = _prec(precision)
    op = C.OP_ACCEL if kind == 0 else C.OP_ADJOINT
    nb = C.workspace_bytes(op, n, steps=1, precision=p)
    ws = C.workspace(nb, dev)
    t = C.Tile()
    ms = ctypes.c_double(0)
    st = C.load().nbody_autotune(int(kind), p, pos.data_ptr(), mass.data_ptr(), n, float(G),
                                 _small(p, small_mass), ws.data_ptr(), ws.numel(),
                                 C.stream_handle(dev), ctypes.byref(t), ctypes.byref(ms))
    C.check(st, "nbody_autotune")
    _tuned[(int(kind), _PREC_NAME[p], n)] = t.as_dict()
    return t.as_dict(), float(ms.value)


def autotune_batched(pos, mass, offsets, G, precision="fp64", small_mass=None):
    """Autotunes the ensemble's force pass; returns (tile dict, ms per pass)."""
    n = _mass(mass)
    _state(pos, "pos", n)
    dev = _same_device(pos, mass)
    offs = [int(x) for x in offsets]
    ns = len(offs) - 1
    if ns < 1 or offs[-1] != n:
        raise ValueError("offsets must have num_systems+1 entries ending at n")
    p = _prec(precision)
    arr = (ctypes.c_int64 * len(offs))(*offs)
    ws = C.workspace(C.workspace_bytes(C.OP_BATCHED, n, num_systems=ns, steps=1, precision=p), dev)
    t = C.Tile()
    ms = ctypes.c_double(0)
    st = C.load().nbody_autotune_batched(p, pos.data_ptr(), mass.data_ptr(), arr, ns, float(G),
                                         _small(p, small_mass), ws.data_ptr(), ws.numel(),
                                         C.stream_handle(dev), ctypes.byref(t), ctypes.byref(ms))
    C.check(st, "nbody_autotune_batched")
    _tuned[(2, _PREC_NAME[p], 0)] = t.as_dict()
    return t.as_dict(), float(ms.value)


def time_force(pos, mass, G, precision="fp64", kind=0, reps=50, small_mass=None):
    """Average ms of one force pass (HIP events on the current stream)."""
    n = _mass(mass)
    _state(pos, "pos", n)
    dev = _same_device(pos, mass)
    p = _prec(precision)
    op = C.OP_ACCEL if kind == 0 else C.OP_ADJOINT
    ws = C.workspace(C.workspace_bytes(op, n, steps=1, precision=p), dev)
    ms = ctypes.c_double(0)
    st = C.load().nbody_time_force(int(kind), p, pos.data_ptr(), mass.data_ptr(), n, float(G),
                                   _small(p, small_mass), int(reps), ws.data_ptr(), ws.numel(),
                                   C.stream_handle(dev), ctypes.byref(ms))
    C.check(st, "nbody_time_force")
    return float(ms.value)


def reset_caches():
    """Drops the library's captured graphs, ensemble work lists and tile
    table (tuned shapes included)."""
    C.load().nbody_reset_caches()
    _tuned.clear()


def version() -> str:
    return C.load().nbody_version().decode()
