"""ctypes binding of libnbody.so (include/nbody.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels.  PyTorch supplies device memory (tensor data pointers) and the
stream (``torch.cuda.current_stream()``).  There is no CPU fallback: if the
library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # first: the library then binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbody.so")

NBODY_OK, NBODY_EINVAL, NBODY_EUNSUPPORTED, NBODY_EWORKSPACE, NBODY_EHIP = range(5)
NBODY_FP64, NBODY_SPLIT, NBODY_SPLIT_COMPENSATED = 0, 1, 2
(OP_ACCEL, OP_RUN, OP_ADJOINT, OP_BATCHED, OP_ENERGY, OP_RK4, OP_ADJOINT_SWEEP,
 OP_ACCEL_SHARD) = range(8)

EXPORTS = (
    "nbody_workspace_bytes", "nbody_accel", "nbody_accel_shard", "nbody_verlet_run",
    "nbody_verlet_run_static",
    "nbody_rk4_run",
    "nbody_verlet_adjoint", "nbody_verlet_checkpoints", "nbody_verlet_adjoint_from_checkpoints",
    "nbody_verlet_run_batched", "nbody_energy", "nbody_momenta", "nbody_get_flags",
    "nbody_get_tile", "nbody_set_tile", "nbody_autotune", "nbody_autotune_batched",
    "nbody_time_force", "nbody_reset_caches",
    "nbody_last_error", "nbody_version",
)


class NBodyError(RuntimeError):
    """A library call failed (HIP error, unsupported size, short workspace)."""


class Tile(ctypes.Structure):
    _fields_ = [("targets_per_lane", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("chunks", ctypes.c_int32), ("variant", ctypes.c_int32)]

    def as_dict(self):
        return {"targets_per_lane": self.targets_per_lane, "waves": self.waves,
                "chunks": self.chunks, "variant": self.variant}


_lib = None
_lock = threading.Lock()
_P = ctypes.c_void_p
_D = ctypes.c_double
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t


def load():
    """Loads libnbody.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2112_15079_amd.build` (no CPU fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        lib.nbody_workspace_bytes.restype = _SZ
        lib.nbody_workspace_bytes.argtypes = [_I32, _I64, _I32, _I64, _I64, _I32]
        lib.nbody_accel.restype = _I32
        lib.nbody_accel.argtypes = [_P, _P, _P, _I64, _D, _D, _I64, _P, _I32, _D, _P, _SZ, _P]
        lib.nbody_accel_shard.restype = _I32
        lib.nbody_accel_shard.argtypes = [_P, _P, _I64, _D, _I64, _I64, _P, _P, _SZ, _P]
        lib.nbody_verlet_run.restype = _I32
        lib.nbody_verlet_run.argtypes = [_P, _P, _P, _I64, _D, _D, _I64, _I32, _D, _P, _SZ, _P]
        lib.nbody_verlet_run_static.restype = _I32
        lib.nbody_verlet_run_static.argtypes = [_P, _P, _P, _I64, _D, _D, _I64, _I32, _D, _P]
        lib.nbody_rk4_run.restype = _I32
        lib.nbody_rk4_run.argtypes = [_P, _P, _P, _I64, _D, _D, _I64, _I32, _D, _P, _SZ, _P]
        lib.nbody_verlet_adjoint.restype = _I32
        lib.nbody_verlet_adjoint.argtypes = [_P, _P, _P, _I64, _D, _D, _I64, _I64, _P, _P, _P,
                                             _P, _P, _P, _P, _P, _SZ, _P]
        lib.nbody_verlet_checkpoints.restype = _I32
        lib.nbody_verlet_checkpoints.argtypes = [_P, _P, _P, _I64, _D, _D, _I64, _I64, _P, _P,
                                                 _P, _P, _SZ, _P]
        lib.nbody_verlet_adjoint_from_checkpoints.restype = _I32
        lib.nbody_verlet_adjoint_from_checkpoints.argtypes = [_P, _P, _I64, _D, _D, _I64, _I64,
                                                              _P, _P, _P, _P, _P, _P, _SZ, _P]
        lib.nbody_verlet_run_batched.restype = _I32
        lib.nbody_verlet_run_batched.argtypes = [_P, _P, _P, _P, _I32, _D, _D, _I64, _I32, _D,
                                                 _P, _SZ, _P]
        lib.nbody_energy.restype = _I32
        lib.nbody_energy.argtypes = [_P, _P, _P, _I64, _D, _P, _P, _SZ, _P]
        lib.nbody_momenta.restype = _I32
        lib.nbody_momenta.argtypes = [_P, _P, _P, _I64, _P, _P]
        lib.nbody_get_flags.restype = _I32
        lib.nbody_get_flags.argtypes = [_P, _P, _I32, ctypes.POINTER(_I32)]
        lib.nbody_get_tile.restype = _I32
        lib.nbody_get_tile.argtypes = [_I32, _I32, _I64, ctypes.POINTER(Tile)]
        lib.nbody_set_tile.restype = _I32
        lib.nbody_set_tile.argtypes = [_I32, _I32, _I64, ctypes.POINTER(Tile)]
        lib.nbody_autotune.restype = _I32
        lib.nbody_autotune.argtypes = [_I32, _I32, _P, _P, _I64, _D, _D, _P, _SZ, _P,
                                       ctypes.POINTER(Tile), ctypes.POINTER(_D)]
        lib.nbody_autotune_batched.restype = _I32
        lib.nbody_autotune_batched.argtypes = [_I32, _P, _P, _P, _I32, _D, _D, _P, _SZ, _P,
                                               ctypes.POINTER(Tile), ctypes.POINTER(_D)]
        lib.nbody_time_force.restype = _I32
        lib.nbody_time_force.argtypes = [_I32, _I32, _P, _P, _I64, _D, _D, _I32, _P, _SZ, _P,
                                         ctypes.POINTER(_D)]
        lib.nbody_reset_caches.restype = None
        lib.nbody_reset_caches.argtypes = []
        lib.nbody_last_error.restype = ctypes.c_char_p
        lib.nbody_version.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def last_error() -> str:
    return load().nbody_last_error().decode()


def check(status: int, what: str) -> None:
    if status == NBODY_OK:
        return
    msg = f"{what}: {last_error()} (status {status})"
    if status == NBODY_EINVAL:
        raise ValueError(msg)
    raise NBodyError(msg)


def stream_handle(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


# ----------------------------------------------------------------------------
# workspace: one growing, zero-initialised buffer per (device, stream)

_ws = {}


def workspace(nbytes: int, device) -> torch.Tensor:
    """A 256-byte-aligned device buffer of at least nbytes, one per (device,
    current stream): calls on one stream are ordered and share it, calls on
    different streams get different buffers and do not race.  A buffer that
    grows is replaced; the old one goes back to torch's allocator in the
    order of its stream's work, the only stream that used it (the library's
    own second stream in the adjoint is ordered before the caller's stream
    returns)."""
    dev = torch.device(device)
    index = dev.index if dev.index is not None else torch.cuda.current_device()
    key = (index, torch.cuda.current_stream(index).cuda_stream)
    buf = _ws.get(key)
    if buf is None or buf.numel() < nbytes:
        with torch.cuda.device(index):
            buf = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=dev)
        if buf.data_ptr() % 256:
            raise NBodyError("device allocation is not 256-byte aligned")
        _ws[key] = buf
    return buf


def workspace_bytes(op: int, n: int, num_systems: int = 1, steps: int = 0,
                    checkpoint_every: int = 1, precision: int = NBODY_FP64) -> int:
    b = load().nbody_workspace_bytes(op, n, num_systems, steps, checkpoint_every, precision)
    if b == 0:
        raise ValueError(f"invalid workspace request (op={op}, n={n}, systems={num_systems}, "
                         f"steps={steps}, checkpoint_every={checkpoint_every})")
    return b
