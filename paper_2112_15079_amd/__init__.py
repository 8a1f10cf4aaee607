"""Direct-sum Solar-System N-body on AMD Instinct MI355X (gfx950).

Eq. (1) of Zhu, "N-body Simulations of the Solar System with CPU-based
Parallel Methods", evaluated every step inside the velocity-Verlet integrator
of Eqs. (3)-(4), as hand-written HIP kernels behind the C ABI of
``include/nbody.h``; this package is its Python binding.

    from paper_2112_15079_amd import accel, verlet_run, verlet_adjoint, \
        verlet_run_batched, energy, momenta, VerletRun
"""
from .nbody import (SMALL_MASS_MSUN, accel, accel_shard, autotune, autotune_batched, energy, get_flags, get_tile,
                    load_tuning, momenta, reset_caches, rk4_run, save_tuning, set_tile,
                    time_force, verlet_adjoint, verlet_adjoint_from_checkpoints, verlet_checkpoints,
                    verlet_run, verlet_run_batched, version)
from .autograd import VerletRun, verlet

__all__ = [
    "accel", "accel_shard", "verlet_run", "rk4_run", "verlet_adjoint", "verlet_checkpoints",
    "verlet_adjoint_from_checkpoints", "verlet_run_batched", "energy", "momenta",
    "get_flags", "get_tile", "set_tile", "autotune", "autotune_batched", "save_tuning",
    "load_tuning", "time_force", "reset_caches", "version", "VerletRun", "verlet",
    "SMALL_MASS_MSUN",
]
