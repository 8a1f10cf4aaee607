"""The C-ABI library on the host: it loads, exports every symbol the header
declares, sizes workspaces, and rejects bad arguments before any GPU work.
No kernel is launched here (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")

C = pytest.importorskip("paper_2112_15079_amd._capi")


def _lib():
    if not os.path.exists(C.LIB_PATH):
        pytest.skip("libnbody.so not built (run __graft_entry__.build())")
    return C.load()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = _declared()
    for want in ("nbody_accel", "nbody_verlet_run", "nbody_verlet_adjoint",
                 "nbody_verlet_run_batched", "nbody_workspace_bytes", "nbody_last_error"):
        assert want in names
    assert set(names) == set(C.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.nbody_version().decode().startswith("nbody-gfx950")


def test_workspace_sizes():
    lib = _lib()
    ws = lambda *a: lib.nbody_workspace_bytes(*a)
    a = ws(C.OP_ACCEL, 10425, 1, 0, 1, C.NBODY_FP64)
    assert a >= 64 * 3 * 10425 * 8          # chunk partials
    assert ws(C.OP_ACCEL, 10425, 1, 0, 1, C.NBODY_SPLIT) > a
    assert ws(C.OP_RUN, 1, 1, 5, 1, C.NBODY_FP64) > 0
    adj = ws(C.OP_ADJOINT, 2079, 1, 36500, 100, C.NBODY_FP64)
    assert adj >= 366 * 6 * 2079 * 8 + 100 * 3 * 2079 * 8
    assert ws(C.OP_BATCHED, 2_000_000, 512, 1000, 1, C.NBODY_FP64) > 0
    # single systems up to 131,072 bodies hold one partial per 256-body range
    # for the each-pair-once pass (512 slots at 131,072), beyond that 2^22 / n
    assert ws(C.OP_RUN, 131072, 1, 5, 1, C.NBODY_FP64) >= 512 * 3 * 131072 * 8
    assert ws(C.OP_RUN, 131073, 1, 5, 1, C.NBODY_FP64) < 64 * 3 * 131073 * 8
    # the pair-once passes at 10,425 bodies: 41 ranges and, with the last
    # round split into halves, 2 x 3 extra slots (47); the force pass writes
    # three planes per slot, the transpose-Jacobian pass four
    assert ws(C.OP_RUN, 10425, 1, 5, 1, C.NBODY_FP64) >= 47 * 3 * 10425 * 8
    assert ws(C.OP_ADJOINT, 10425, 1, 10, 5, C.NBODY_FP64) >= 47 * 4 * 10425 * 8
    assert ws(C.OP_ADJOINT_SWEEP, 10425, 1, 10, 5, C.NBODY_FP64) >= 47 * 4 * 10425 * 8
    # RK4: the run's buffers plus stage velocity and two slope sums
    assert ws(C.OP_RK4, 10425, 1, 5, 1, C.NBODY_FP64) >= ws(C.OP_RUN, 10425, 1, 5, 1, C.NBODY_FP64) \
        + 3 * 3 * 10425 * 8
    # invalid requests return 0
    assert ws(C.OP_ACCEL, 0, 1, 0, 1, C.NBODY_FP64) == 0
    assert ws(C.OP_ADJOINT, 10, 1, 10, 0, C.NBODY_FP64) == 0
    assert ws(9, 10, 1, 0, 1, C.NBODY_FP64) == 0
    assert ws(C.OP_ACCEL, 10, 1, 0, 1, 7) == 0


FAKE = ctypes.c_void_p(0x10000)   # never dereferenced: validation fails first


def test_accel_rejects_bad_arguments():
    lib = _lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    # null pos
    assert lib.nbody_accel(None, None, FAKE, 10, 1.0, 0.0, 0, FAKE, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    assert "null" in C.last_error()
    # n < 1
    assert lib.nbody_accel(FAKE, None, FAKE, 0, 1.0, 0.0, 0, FAKE, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    # non-finite G
    assert lib.nbody_accel(FAKE, None, FAKE, 5, float("nan"), 0.0, 0, FAKE, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    # unknown precision
    assert lib.nbody_accel(FAKE, None, FAKE, 5, 1.0, 0.0, 0, FAKE, 3, 0.0, ws, big, None) == C.NBODY_EINVAL
    # negative split threshold
    assert lib.nbody_accel(FAKE, None, FAKE, 5, 1.0, 0.0, 0, FAKE, 1, -1.0, ws, big, None) == C.NBODY_EINVAL
    # null output
    assert lib.nbody_accel(FAKE, None, FAKE, 5, 1.0, 0.0, 0, None, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    # workspace missing / short / misaligned
    assert lib.nbody_accel(FAKE, None, FAKE, 5, 1.0, 0.0, 0, FAKE, 0, 0.0, None, big, None) == C.NBODY_EWORKSPACE
    assert lib.nbody_accel(FAKE, None, FAKE, 5, 1.0, 0.0, 0, FAKE, 0, 0.0, ws, 16, None) == C.NBODY_EWORKSPACE
    assert lib.nbody_accel(FAKE, None, FAKE, 5, 1.0, 0.0, 0, FAKE, 0, 0.0,
                           ctypes.c_void_p(0x100010), big, None) == C.NBODY_EINVAL
    # too many bodies
    assert lib.nbody_accel(FAKE, None, FAKE, (1 << 30) + 1, 1.0, 0.0, 0, FAKE, 0, 0.0, ws, big,
                           None) == C.NBODY_EUNSUPPORTED


def test_run_rejects_bad_arguments():
    lib = _lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    assert lib.nbody_verlet_run(FAKE, None, FAKE, 5, 1.0, 0.1, 3, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    assert lib.nbody_verlet_run(FAKE, FAKE, FAKE, 5, 1.0, 0.1, -1, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    assert lib.nbody_verlet_run(FAKE, FAKE, FAKE, 5, 1.0, float("inf"), 3, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    # steps = 0 is a valid no-op (returns before any launch)
    assert lib.nbody_verlet_run(FAKE, FAKE, FAKE, 5, 1.0, 0.1, 0, 0, 0.0, ws, big, None) == C.NBODY_OK


def test_rk4_rejects_bad_arguments():
    lib = _lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    assert lib.nbody_rk4_run(FAKE, None, FAKE, 5, 1.0, 0.1, 3, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    assert lib.nbody_rk4_run(FAKE, FAKE, FAKE, 5, 1.0, 0.1, -1, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    assert lib.nbody_rk4_run(FAKE, FAKE, FAKE, 5, 1.0, float("nan"), 3, 0, 0.0, ws, big, None) == C.NBODY_EINVAL
    assert lib.nbody_rk4_run(FAKE, FAKE, FAKE, 5, 1.0, 0.1, 3, 3, 0.0, ws, big, None) == C.NBODY_EINVAL
    assert lib.nbody_rk4_run(FAKE, FAKE, FAKE, 5, 1.0, 0.1, 3, 0, 0.0, ws, 64, None) == C.NBODY_EWORKSPACE
    assert lib.nbody_rk4_run(FAKE, FAKE, FAKE, 5, 1.0, 0.1, 0, 0, 0.0, ws, big, None) == C.NBODY_OK


def test_adjoint_rejects_bad_arguments():
    lib = _lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    args = [FAKE, FAKE, FAKE, 5, 1.0, 0.1, 10, 0, FAKE, FAKE, FAKE, FAKE, FAKE, None, None, ws, big, None]
    assert lib.nbody_verlet_adjoint(*args) == C.NBODY_EINVAL       # checkpoint_every = 0
    args[7] = 5
    args[8] = None
    assert lib.nbody_verlet_adjoint(*args) == C.NBODY_EINVAL       # null cotangent


def test_batched_rejects_bad_offsets():
    lib = _lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    bad = [(0, 5, 5, 9), (1, 5, 9), (0, 7, 4)]
    for offs in bad:
        arr = (ctypes.c_int64 * len(offs))(*offs)
        st = lib.nbody_verlet_run_batched(FAKE, FAKE, FAKE, arr, len(offs) - 1, 1.0, 0.1, 10, 0,
                                          0.0, ws, big, None)
        assert st == C.NBODY_EINVAL, offs
    assert lib.nbody_verlet_run_batched(FAKE, FAKE, FAKE, None, 1, 1.0, 0.1, 10, 0, 0.0, ws, big,
                                        None) == C.NBODY_EINVAL


def test_tile_table():
    lib = _lib()
    lib.nbody_reset_caches()
    t = C.Tile()
    # defaults: each pair once (variant 5) up to 131,072 bodies, from 4,096
    # (FP64) or 8,000 (split), one-way passes on either side
    for prec, n, variant in [(0, 4095, 1), (0, 4096, 5), (0, 10425, 5), (0, 40000, 5),
                             (0, 131072, 5), (0, 131073, 0), (1, 7999, 0), (1, 8000, 5),
                             (1, 10425, 5), (1, 131072, 5), (1, 131073, 0)]:
        assert lib.nbody_get_tile(0, prec, n, ctypes.byref(t)) == C.NBODY_OK
        assert t.variant == variant, (prec, n, t.variant)
    assert lib.nbody_get_tile(0, 0, 10425, ctypes.byref(t)) == C.NBODY_OK
    assert (t.targets_per_lane, t.waves, t.chunks) == (4, 4, 1)
    want = C.Tile(4, 2, 7, 0)
    assert lib.nbody_set_tile(0, 0, 10425, ctypes.byref(want)) == C.NBODY_OK
    assert lib.nbody_get_tile(0, 0, 10425, ctypes.byref(t)) == C.NBODY_OK
    assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == (4, 2, 7, 0)
    assert lib.nbody_set_tile(0, 0, 10425, ctypes.byref(C.Tile(1, 2, 9, 1))) == C.NBODY_OK
    assert lib.nbody_get_tile(0, 0, 10425, ctypes.byref(t)) == C.NBODY_OK
    assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == (1, 2, 9, 1)
    assert lib.nbody_set_tile(0, 0, 10425, ctypes.byref(C.Tile(1, 2, 9, 3))) == C.NBODY_EINVAL
    # the adjoint pass defaults to scalar operands, 2 waves, up to 64 source
    # chunks of >= 16 bodies, within the workspace's chunk cap; from 4,500 to
    # 131,072 bodies to each pair once in the (4, 4) shape
    for n, want in ((20, (1, 2, 1, 1)), (100, (1, 2, 6, 1)), (2079, (1, 2, 64, 1)),
                    (4499, (1, 2, 64, 1)), (4500, (4, 4, 1, 5)), (131072, (4, 4, 1, 5)),
                    (131073, (1, 2, 31, 1))):
        assert lib.nbody_get_tile(1, 0, n, ctypes.byref(t)) == C.NBODY_OK
        assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == want, n
    # it takes variants 0 (LDS tiles), 1 (scalar operands) and 5 (each pair
    # once, the force pass's shapes, one chunk, up to 131,072 bodies)
    assert lib.nbody_set_tile(1, 0, 100, ctypes.byref(C.Tile(1, 1, 1, 1))) == C.NBODY_OK
    assert lib.nbody_get_tile(1, 0, 100, ctypes.byref(t)) == C.NBODY_OK and t.variant == 1
    assert lib.nbody_set_tile(1, 0, 100, ctypes.byref(C.Tile(1, 1, 1, 2))) == C.NBODY_EINVAL
    for shape in ((1, 4), (2, 2), (2, 4), (4, 4)):
        assert lib.nbody_set_tile(1, 0, 5000, ctypes.byref(C.Tile(*shape, 1, 5))) == C.NBODY_OK
        assert lib.nbody_get_tile(1, 0, 5000, ctypes.byref(t)) == C.NBODY_OK
        assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == (*shape, 1, 5)
    assert lib.nbody_set_tile(1, 0, 5000, ctypes.byref(C.Tile(4, 2, 1, 5))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(1, 0, 5000, ctypes.byref(C.Tile(2, 4, 2, 5))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(1, 0, 131073, ctypes.byref(C.Tile(2, 4, 1, 5))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(2, 0, 0, ctypes.byref(C.Tile(2, 1, 16, 1))) == C.NBODY_OK
    assert lib.nbody_get_tile(2, 0, 0, ctypes.byref(t)) == C.NBODY_OK and t.variant == 1
    assert lib.nbody_set_tile(3, 0, 10, ctypes.byref(C.Tile(1, 1, 1, 0))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(0, 0, 10425, ctypes.byref(C.Tile(3, 1, 1, 0))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(0, 0, 10425, ctypes.byref(C.Tile(1, 1, 65, 0))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(1, 0, 100, ctypes.byref(C.Tile(4, 1, 1, 0))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(0, 7, 100, ctypes.byref(C.Tile(1, 1, 1, 0))) == C.NBODY_EINVAL
    assert lib.nbody_get_tile(0, -1, 100, ctypes.byref(t)) == C.NBODY_EINVAL
    lib.nbody_reset_caches()


def test_tile_table_single_workgroup_variant():
    """Variant 3 (one workgroup runs whole steps): the heuristic for small
    systems, and the shapes and sizes it accepts."""
    lib = _lib()
    lib.nbody_reset_caches()
    t = C.Tile()
    for prec in (0, 1):
        assert lib.nbody_get_tile(0, prec, 131, ctypes.byref(t)) == C.NBODY_OK
        # as many slices as 1024 lanes allow: 1024 // 131 = 7
        assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == (1, 16, 7, 3)
        assert lib.nbody_get_tile(0, prec, 193, ctypes.byref(t)) == C.NBODY_OK
        assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == (1, 8, 1, 4)
        assert lib.nbody_get_tile(0, prec, 600, ctypes.byref(t)) == C.NBODY_OK and t.variant < 3
    assert lib.nbody_get_tile(0, 0, 16, ctypes.byref(t)) == C.NBODY_OK and t.chunks == 16
    assert lib.nbody_get_tile(1, 0, 131, ctypes.byref(t)) == C.NBODY_OK and t.variant == 1
    assert lib.nbody_get_tile(2, 0, 0, ctypes.byref(t)) == C.NBODY_OK and t.variant != 3
    assert lib.nbody_set_tile(0, 0, 400, ctypes.byref(C.Tile(1, 16, 2, 3))) == C.NBODY_OK
    assert lib.nbody_get_tile(0, 0, 400, ctypes.byref(t)) == C.NBODY_OK
    assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == (1, 16, 2, 3)
    assert lib.nbody_set_tile(0, 0, 512, ctypes.byref(C.Tile(1, 16, 1, 3))) == C.NBODY_OK
    # 513 shares 512's size class: the stored variant-3 shape is not used above 512
    assert lib.nbody_set_tile(0, 0, 513, ctypes.byref(C.Tile(1, 16, 1, 3))) == C.NBODY_EINVAL
    assert lib.nbody_get_tile(0, 0, 513, ctypes.byref(t)) == C.NBODY_OK and t.variant != 3
    for bad in [(1, 8, 4, 3), (2, 16, 4, 3), (1, 16, 0, 3), (1, 16, 65, 3), (1, 1, 1, 4)]:
        assert lib.nbody_set_tile(0, 0, 131, ctypes.byref(C.Tile(*bad))) == C.NBODY_EINVAL, bad
    assert lib.nbody_set_tile(1, 0, 131, ctypes.byref(C.Tile(1, 16, 4, 3))) == C.NBODY_EINVAL
    # variant 4 (force pass and step fused): tpl 1 or 2, waves 2..8, one chunk, kind 0
    assert lib.nbody_set_tile(0, 0, 3000, ctypes.byref(C.Tile(2, 8, 1, 4))) == C.NBODY_OK
    assert lib.nbody_get_tile(0, 0, 3000, ctypes.byref(t)) == C.NBODY_OK and t.variant == 4
    for bad in [(1, 16, 1, 4), (4, 2, 1, 4), (1, 1, 1, 4), (1, 2, 2, 4)]:
        assert lib.nbody_set_tile(0, 0, 3000, ctypes.byref(C.Tile(*bad))) == C.NBODY_EINVAL, bad
    assert lib.nbody_set_tile(1, 0, 3000, ctypes.byref(C.Tile(1, 2, 1, 4))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(2, 0, 0, ctypes.byref(C.Tile(1, 2, 1, 4))) == C.NBODY_EINVAL
    assert lib.nbody_set_tile(2, 0, 0, ctypes.byref(C.Tile(1, 16, 4, 3))) == C.NBODY_EINVAL
    # variant 5 (each pair once): single systems of up to 131,072 bodies (512
    # ranges of partials), (1, 4), (2, 2), (2, 4) or (4, 4), one chunk
    for good in [(1, 4, 1, 5), (2, 2, 1, 5), (2, 4, 1, 5), (4, 4, 1, 5)]:
        assert lib.nbody_set_tile(0, 0, 10425, ctypes.byref(C.Tile(*good))) == C.NBODY_OK, good
        assert lib.nbody_get_tile(0, 0, 10425, ctypes.byref(t)) == C.NBODY_OK
        assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == good
    for bad in [(2, 4, 4, 5), (1, 4, 2, 5), (1, 8, 1, 5), (1, 2, 1, 5), (4, 1, 1, 5), (4, 2, 1, 5)]:
        assert lib.nbody_set_tile(0, 0, 10425, ctypes.byref(C.Tile(*bad))) == C.NBODY_EINVAL, bad
    assert lib.nbody_set_tile(0, 1, 10425, ctypes.byref(C.Tile(4, 4, 1, 5))) == C.NBODY_OK
    for kind, prec, n in [(1, 0, 131073), (0, 0, 131073), (0, 1, 131073)]:
        assert lib.nbody_set_tile(kind, prec, n, ctypes.byref(C.Tile(1, 4, 1, 5))) == C.NBODY_EINVAL
    # ensembles take it too (a plan with a system of more than 40 ranges falls
    # back to the heuristic tile)
    for prec in (0, 1):
        assert lib.nbody_set_tile(2, prec, 0, ctypes.byref(C.Tile(4, 4, 1, 5))) == C.NBODY_OK
        assert lib.nbody_get_tile(2, prec, 0, ctypes.byref(t)) == C.NBODY_OK and t.variant == 5
    lib.nbody_reset_caches()


def test_python_wrapper_rejects_cpu_tensors():
    torch = pytest.importorskip("torch")
    _lib()
    import paper_2112_15079_amd as nb
    pos = torch.zeros(3, 4, dtype=torch.float64)
    mass = torch.ones(4, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU"):
        nb.accel(pos, mass, 1.0)
    with pytest.raises(TypeError):
        nb.accel(pos, mass.float(), 1.0)
    with pytest.raises(ValueError):
        nb.accel(pos, mass, 1.0, precision="fp16")


def test_compensated_split_form_host_rules():
    """Precision 2 (the split form with FP64-refined factors and Kahan-
    compensated FP32 light terms) runs in the each-pair-once pass only: its
    tile is variant 5 at every size, other variants are refused, and systems
    beyond 131,072 bodies are refused before anything is enqueued."""
    lib = _lib()
    lib.nbody_reset_caches()
    t = C.Tile()
    for n in (1, 10, 131, 600, 10425, 131072):
        assert lib.nbody_get_tile(0, C.NBODY_SPLIT_COMPENSATED, n, ctypes.byref(t)) == C.NBODY_OK
        assert (t.targets_per_lane, t.waves, t.chunks, t.variant) == (4, 4, 1, 5), n
    assert lib.nbody_get_tile(2, C.NBODY_SPLIT_COMPENSATED, 0, ctypes.byref(t)) == C.NBODY_OK
    assert t.variant == 5
    for bad in [(1, 2, 9, 1), (1, 16, 2, 3), (1, 8, 1, 4), (2, 1, 3, 0)]:
        assert lib.nbody_set_tile(0, C.NBODY_SPLIT_COMPENSATED, 10425,
                                  ctypes.byref(C.Tile(*bad))) == C.NBODY_EINVAL, bad
    assert lib.nbody_set_tile(0, C.NBODY_SPLIT_COMPENSATED, 10425,
                              ctypes.byref(C.Tile(2, 4, 1, 5))) == C.NBODY_OK
    assert lib.nbody_get_tile(0, C.NBODY_SPLIT_COMPENSATED, 10425, ctypes.byref(t)) == C.NBODY_OK
    assert (t.targets_per_lane, t.waves, t.variant) == (2, 4, 5)
    lib.nbody_reset_caches()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    for fn, args in (("nbody_accel", (FAKE, None, FAKE, 131073, 1.0, 0.0, 0, FAKE, 2, 0.0)),
                     ("nbody_verlet_run", (FAKE, FAKE, FAKE, 131073, 1.0, 0.1, 10, 2, 0.0)),
                     ("nbody_rk4_run", (FAKE, FAKE, FAKE, 131073, 1.0, 0.1, 10, 2, 0.0))):
        assert getattr(lib, fn)(*args, ws, big, None) == C.NBODY_EUNSUPPORTED, fn
        assert "compensated" in C.last_error()
    # a negative threshold is refused as for the split form
    assert lib.nbody_accel(FAKE, None, FAKE, 5, 1.0, 0.0, 0, FAKE, 2, -1.0, ws, big,
                           None) == C.NBODY_EINVAL
    ws_bytes = lib.nbody_workspace_bytes
    for op in (C.OP_ACCEL, C.OP_RUN, C.OP_RK4, C.OP_BATCHED):
        assert ws_bytes(op, 10425, 1, 0, 1, C.NBODY_SPLIT_COMPENSATED) == \
            ws_bytes(op, 10425, 1, 0, 1, C.NBODY_SPLIT) > 0


def test_static_scratch_run_validates_first():
    """nbody_verlet_run_static: bad arguments and runs whose scratch would
    exceed the static array are refused before anything touches the device;
    zero steps is a no-op."""
    lib = _lib()
    run = lib.nbody_verlet_run_static
    assert run(FAKE, None, FAKE, 10, 1.0, 0.1, 5, 0, 0.0, None) == C.NBODY_EINVAL
    assert run(FAKE, FAKE, FAKE, 10, 1.0, 0.1, -1, 0, 0.0, None) == C.NBODY_EINVAL
    assert run(FAKE, FAKE, FAKE, 10, 1.0, 0.1, 5, 3, 0.0, None) == C.NBODY_EINVAL
    assert run(FAKE, FAKE, FAKE, 10, float("inf"), 0.1, 5, 0, 0.0, None) == C.NBODY_EINVAL
    for prec in (0, 1, 2):
        assert run(FAKE, FAKE, FAKE, 40000, 1.0, 0.1, 5, prec, 0.0, None) == C.NBODY_EUNSUPPORTED
        assert "static scratch" in C.last_error()
    assert run(FAKE, FAKE, FAKE, 10, 1.0, 0.1, 0, 0, 0.0, None) == C.NBODY_OK


def test_split_adjoint_validates_first():
    lib = _lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    ck = lib.nbody_verlet_checkpoints
    rev = lib.nbody_verlet_adjoint_from_checkpoints
    assert ck(FAKE, FAKE, FAKE, 10, 1.0, 0.1, 5, 2, None, None, None, ws, big, None) == C.NBODY_EINVAL
    assert ck(FAKE, None, FAKE, 10, 1.0, 0.1, 5, 2, FAKE, None, None, ws, big, None) == C.NBODY_EINVAL
    assert ck(FAKE, FAKE, FAKE, 10, 1.0, 0.1, 5, 0, FAKE, None, None, ws, big, None) == C.NBODY_EINVAL
    assert ck(FAKE, FAKE, FAKE, 10, 1.0, 0.1, 5, 2, FAKE, None, None, ws, 64, None) == C.NBODY_EWORKSPACE
    assert rev(None, FAKE, 10, 1.0, 0.1, 5, 2, FAKE, FAKE, FAKE, FAKE, FAKE, ws, big, None) == C.NBODY_EINVAL
    assert rev(FAKE, FAKE, 10, 1.0, 0.1, 5, 2, None, FAKE, FAKE, FAKE, FAKE, ws, big, None) == C.NBODY_EINVAL
    assert rev(FAKE, FAKE, 10, 1.0, 0.1, -1, 2, FAKE, FAKE, FAKE, FAKE, FAKE, ws, big, None) == C.NBODY_EINVAL
    wsb = lib.nbody_workspace_bytes
    # the sweep's workspace is the adjoint's without its checkpoints
    full = wsb(C.OP_ADJOINT, 2079, 1, 36500, 100, 0)
    sweep = wsb(C.OP_ADJOINT_SWEEP, 2079, 1, 36500, 100, 0)
    assert 0 < sweep < full and full - sweep >= 366 * 6 * 2079 * 8
    assert wsb(C.OP_ADJOINT_SWEEP, 10, 1, 5, 0, 0) == 0


def test_target_share_validates_first():
    """nbody_accel_shard: a share of the targets must be a non-empty part of
    [0, n); bad arguments and short workspaces are refused before any device
    work.  Its workspace is sized for FP64 and one system only."""
    lib = _lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    sh = lib.nbody_accel_shard
    assert sh(None, FAKE, 10, 1.0, 0, 5, FAKE, ws, big, None) == C.NBODY_EINVAL
    assert sh(FAKE, FAKE, 10, 1.0, 0, 5, None, ws, big, None) == C.NBODY_EINVAL
    assert sh(FAKE, FAKE, 0, 1.0, 0, 1, FAKE, ws, big, None) == C.NBODY_EINVAL
    assert sh(FAKE, FAKE, 10, float("nan"), 0, 5, FAKE, ws, big, None) == C.NBODY_EINVAL
    for t0, nt in ((-1, 5), (0, 0), (6, 5), (10, 1), (0, 11), (9, -3)):
        assert sh(FAKE, FAKE, 10, 1.0, t0, nt, FAKE, ws, big, None) == C.NBODY_EINVAL, (t0, nt)
        assert "targets" in C.last_error()
    assert sh(FAKE, FAKE, 10, 1.0, 0, 10, FAKE, None, big, None) == C.NBODY_EWORKSPACE
    assert sh(FAKE, FAKE, 10, 1.0, 0, 10, FAKE, ws, 64, None) == C.NBODY_EWORKSPACE
    wsb = lib.nbody_workspace_bytes
    # 64 chunk partials of every body, the G m plane and the work list
    assert wsb(C.OP_ACCEL_SHARD, 131072, 1, 0, 1, 0) >= 64 * 3 * 131072 * 8 + 131072 * 8
    assert wsb(C.OP_ACCEL_SHARD, 131072, 1, 0, 1, 1) == 0
    assert wsb(C.OP_ACCEL_SHARD, 131072, 2, 0, 1, 0) == 0


def test_oracle_and_hip_path_share_no_code():
    """The oracle and the HIP path are independent: no source of the library
    (kernels, C ABI, binding, header) names the oracle, and the oracle's
    sources name nothing of the library."""
    lib_dirs = [os.path.join(ROOT, "paper_2112_15079_amd", "csrc"),
                os.path.join(ROOT, "paper_2112_15079_amd"), os.path.join(ROOT, "include")]
    for d in lib_dirs:
        for f in os.listdir(d):
            if f.endswith((".hip", ".hpp", ".h", ".py")):
                assert "oracle" not in open(os.path.join(d, f)).read().lower(), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h", ".py")):
            src = open(os.path.join(ROOT, "oracle", f)).read()
            for name in ("paper_2112_15079_amd", "csrc", "nbody.h", "libnbody", "hip_runtime",
                         "hipMalloc", "hipLaunch", "__global__"):
                assert name not in src, (f, name)
